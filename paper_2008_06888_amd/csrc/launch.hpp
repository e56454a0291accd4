// Host launch wrappers of the HIP kernels (defined next to the kernels).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "potts.hpp"

namespace tt {

// threads: at least 2^tb of every item's pass; lds: at least 4 * 2^t bytes of every item's pass
// (2 * 2^t for dtype 2: int16 couplings and state, k_pass16).
// t0 / t1 (optional, created events): receive the kernel's own start and end times.
// ng (dtype 2 only): groups of 16 entries per thread, 1, or 2 with threads =
// 2^(tb - 1) of every item's pass (tb >= 7).
hipError_t launch_pass(const PassItem* items, int n_items, int64_t n_wg, int threads, size_t lds, int dtype,
                       hipStream_t stream, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr, int ng = 1,
                       bool z2 = false);
int reduce_log2_chunks(int w);
// state16: the items' states are int16 (int16 couplings), else float32
hipError_t launch_reduce(const RedItem* items, int n_items, int64_t n_chunks, float* pv, uint64_t* pi,
                         hipStream_t stream, bool partials_ready = false, bool state16 = false);
hipError_t launch_backward(const BwdItem* items, int n_items, int dtype, hipStream_t stream);

hipError_t launch_tgemm(int batch, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, int64_t sA,
                        const float* B, int64_t ldb, int64_t sB, float* C, int64_t ldc, int64_t sC,
                        hipStream_t stream);

// chimera row chain (energy or counting) and backward finish
hipError_t launch_chain(const ChainItem* item, int64_t n_blocks, int dtype, bool count, hipStream_t stream);
hipError_t launch_chim_finish(const ChimFinishItem* item, int batch, int dtype, hipStream_t stream);

// counting path: state entries (x, n mod p_r), r < nres (r = 3: modulo 2^64);
// residues come out as 4 words per instance (unused planes 0)
hipError_t launch_count_pass(const DevPass& P, const DevOp* ops, const int32_t* J, const int32_t* h,
                             int64_t jst, int64_t hst, const float* xin, const uint64_t* nin, float* xout,
                             uint64_t* nout, int64_t sst, int batch, int nres, bool z2, hipStream_t stream);
int count_reduce_log2_chunks(int w);
hipError_t launch_count_reduce(const float* x, const uint64_t* nplanes, int64_t sst, int w, uint64_t free_mask,
                               int batch, int nres, bool z2, float* pv, uint64_t* pn, int64_t* energy,
                               uint64_t* residues, hipStream_t stream);

// 3-state Potts sweep: one pass over `batch` instances of 3^W entries (sst)
// in place (low: the pass's tile digits are slots 0 .. t-1); n == nullptr: energy only, else nres residue planes of
// batch * sst entries each
hipError_t launch_potts_pass(const PottsPass* pass, int t, bool low, int64_t threads, const void* J, int64_t jst,
                             int dtype,
                             float* x, uint64_t* n, int nres, int64_t sst, int batch, hipStream_t s);
int64_t potts_reduce_chunk(int64_t combos);
// final maximum (and count): energy H* (double), energy2 2H* (int64), res
// [batch][4] residues; each output may be null; pv / pn hold batch * chunks
// partials (chunks from potts_reduce_chunk)
hipError_t launch_potts_reduce(const PottsReduce* red, int64_t combos, const float* x, const uint64_t* n, int nres,
                               int64_t sst, int batch, float* pv, uint64_t* pn, double* energy, int64_t* energy2,
                               uint64_t* res, hipStream_t s);

// configurations by finite differences of the fields: the n + 1 perturbed
// copies of one instance, then sigma, E* and Eq. (1) of sigma from their energies
hipError_t launch_fd_build(const float* J, const float* h, int64_t m, int n, float delta, float* Jb, float* hb,
                           hipStream_t s);
hipError_t launch_fd_sigma(const double* E, const float* J, const float* h, const int32_t* edges, int64_t m, int n,
                           int8_t* sigma, double* energy, double* e_sigma, hipStream_t s);

// sliced plans: index tables (device int32) that reduce an instance to its
// 2^s slices; reduced instance r is instance r >> s with the fixed spins set
// to the bits of r & (2^s - 1) (bit j = 1 <-> fixed spin j at sigma = -1)
struct SliceArgs {
  int32_t s;                  // fixed spins
  int32_t n, nr;              // spins of the graph and of the reduced graph
  int32_t n_inner;            // bonds between two fixed spins
  int64_t m, mr;              // edges of the graph and of the reduced graph
  const int32_t* spins;       // [s] spin of fixed index j
  const int32_t* keep;        // [nr] reduced spin -> spin
  const int32_t* emap;        // [mr] reduced edge -> edge
  const int32_t* cross_ptr;   // [nr + 1] per reduced spin, its bonds to fixed spins:
  const int32_t* cross_bit;   //   fixed index j of the other end
  const int32_t* cross_edge;  //   and the edge
  const int32_t* inner_a;     // [n_inner] fixed indices of both ends, and the edge
  const int32_t* inner_b;
  const int32_t* inner_edge;
};
// reduced couplings Jr, fields hr and constant energies c of n_red reduced
// instances starting at r0 (kpick == nullptr), or of the slices kpick[b] of
// instances b = r0 .. r0 + n_red - 1; h may be null (zero fields); dtype 0
// float32, 1 int32, 2 int16
hipError_t launch_slice_build(const SliceArgs& A, int64_t r0, int n_red, const int32_t* kpick, int dtype,
                              const void* J, const void* h, void* Jr, void* hr, double* c, hipStream_t s);
// energy[b] = min over the slices of instance b of Er + c, kbest[b] the first
// minimising slice (either output may be null)
hipError_t launch_slice_min(const double* Er, const double* c, int s, int batch, double* energy, int32_t* kbest,
                            hipStream_t st);
// sigma of each instance from the ground state sr of its chosen slice, and
// the gradients dJ = -sigma_i sigma_j, dh = -sigma_i (either may be null)
hipError_t launch_slice_pick(const SliceArgs& A, int batch, const int8_t* sr, const int32_t* kbest,
                             const int32_t* edges, int8_t* sigma, float* dJ, float* dh, hipStream_t s);

// workspace of the allocation-free contraction: its size, and the current
// device's address of it
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
hipError_t noalloc_scratch(void** ptr);

// input check: status[i] for the n_inst instances of the items (CHK_* flags)
hipError_t launch_check(const CheckArgs& a, int64_t n_inst, uint32_t* status, hipStream_t stream);

}  // namespace tt
