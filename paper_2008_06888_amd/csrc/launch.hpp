// Host launch wrappers of the HIP kernels (defined next to the kernels).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "potts.hpp"

namespace tt {

// threads: at least 2^tb of every item's pass; lds: at least 4 * 2^t bytes of every item's pass.
// t0 / t1 (optional, created events): receive the kernel's own start and end times.
hipError_t launch_pass(const PassItem* items, int n_items, int64_t n_wg, int threads, size_t lds, int dtype,
                       hipStream_t stream, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
int reduce_log2_chunks(int w);
hipError_t launch_reduce(const RedItem* items, int n_items, int64_t n_chunks, float* pv, uint64_t* pi,
                         hipStream_t stream, bool partials_ready = false);
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
                             uint64_t* nout, int64_t sst, int batch, int nres, hipStream_t stream);
int count_reduce_log2_chunks(int w);
hipError_t launch_count_reduce(const float* x, const uint64_t* nplanes, int64_t sst, int w, uint64_t free_mask,
                               int batch, int nres, float* pv, uint64_t* pn, int64_t* energy, uint64_t* residues,
                               hipStream_t stream);

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

// workspace of the allocation-free contraction: its size, and the current
// device's address of it
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
hipError_t noalloc_scratch(void** ptr);

// input check: status[i] for the n_inst instances of the items (CHK_* flags)
hipError_t launch_check(const CheckArgs& a, int64_t n_inst, uint32_t* status, hipStream_t stream);

}  // namespace tt
