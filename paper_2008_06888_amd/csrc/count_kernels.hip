// HIP kernels (gfx950) of the counting sweep: every state entry is the tuple
// (x, n) of Eq. (4), x the tropical number (negative energy) and n the number
// of configurations attaining it. The tropical product with a leaf tensor
// (count 1) keeps n; the tropical sum keeps the n of the larger x and adds
// the n's when the x's are equal. n is carried as three residues modulo the
// primes p_r = 2^61 - 1, 2^61 - 31, 2^61 - 45 (exact recombination by CRT on
// the host), and, for graphs of more than 182 spins (where g may reach the
// product of the primes), a fourth residue modulo 2^64 (plain wrap-around
// arithmetic) that the host compares with the CRT value. x is an exact
// integer held in float32 (|x| < 2^24 is checked by the caller), so every
// equality test of Eq. (4) is exact.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "device_mem.hpp"
#include "plan.hpp"

namespace tt {

constexpr int CNT = 256;        // reductions
constexpr int CNT_PASS = 1024;  // count passes: 16 waves hide the LDS latency of the per-op sweeps
constexpr int NRES = 4;   // residue planes at most (the fourth: modulo 2^64)
constexpr int CNT_MAX_OPS = 64;   // ops of one pass (the partitioner's bound)
constexpr int CNT_MAX_T = 12;     // tile bits at most (the count tile option's bound)
constexpr int CNT_PER_THREAD = (1 << CNT_MAX_T) / CNT_PASS;   // tile entries per thread at most

// modulus 0 stands for 2^64
__device__ __constant__ uint64_t c_mod[NRES] = {(1ull << 61) - 1, (1ull << 61) - 31, (1ull << 61) - 45, 0};

// The modulus of residue plane r as a compile-time constant (r known at
// compile time after unrolling): no memory read in the inner loops.
__host__ __device__ constexpr uint64_t mod_of(int r) {
  return r == 0 ? (1ull << 61) - 1 : r == 1 ? (1ull << 61) - 31 : r == 2 ? (1ull << 61) - 45 : 0ull;
}

__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t p) {
  const uint64_t s = a + b;   // a, b < p < 2^61: no overflow; p = 0: modulo 2^64
  return (p != 0 && s >= p) ? s - p : s;
}

__device__ __forceinline__ int cbit(uint8_t enc, uint32_t i, uint64_t base) {
  return enc < SLOT_FIXED ? (int)((i >> enc) & 1u) : (int)((base >> (enc - SLOT_FIXED)) & 1ull);
}

__device__ __forceinline__ void cbuild_deposit(const uint8_t* R, int t, uint64_t* lo, uint64_t* hi) {
  for (int j = threadIdx.x; j < 256; j += blockDim.x) {
    uint64_t a = 0, b = 0;
    for (int k = 0; k < 8; ++k) {
      if (k < t && ((j >> k) & 1)) a |= 1ull << R[k];
      if (k + 8 < t && ((j >> k) & 1)) b |= 1ull << R[k + 8];
    }
    lo[j] = a;
    hi[j] = b;
  }
}

// State layout per instance: x plane [sst] float, then residue planes
// n[r][sst] uint64 (sst = 2^W entries per plane, 2^(W-1) for half-state
// plans). With z2 (h = 0: every state is even under flipping all of its
// bits) only entries whose top address bit is 0 are stored, an entry with
// the top bit set is read at the complement address, and only the tiles
// whose tile-id bit z2_skip is 0 run: each writes its outputs at their
// stored addresses, which cover those of the complementary tile too.
__global__ __launch_bounds__(CNT_PASS) void k_count_pass(DevPass P, const DevOp* __restrict__ ops,
                                                    const int32_t* __restrict__ J, const int32_t* __restrict__ h,
                                                    int64_t jst, int64_t hst, const float* __restrict__ xin,
                                                    const uint64_t* __restrict__ nin, float* __restrict__ xout,
                                                    uint64_t* __restrict__ nout, int64_t sst, int log2_tiles,
                                                    int nres, int z2) {
  extern __shared__ uint64_t csm[];
  const uint32_t size = 1u << P.t;
  uint64_t* tn = csm;                                        // [nres][size]
  float* tx = reinterpret_cast<float*>(csm + nres * size);   // [size]
  __shared__ uint64_t dep_lo[256], dep_hi[256];
  __shared__ DevOp s_op[CNT_MAX_OPS];
  __shared__ float s_val[CNT_MAX_OPS];
  const int64_t inst = (int64_t)blockIdx.x >> log2_tiles;
  const uint64_t tile_id = z2_tile((uint64_t)blockIdx.x & ((1ull << log2_tiles) - 1ull), z2 ? P.z2_skip : -1);
  uint64_t base = 0;
  for (int k = 0; k < P.n_free; ++k) base |= ((tile_id >> k) & 1ull) << P.fre[k];
  cbuild_deposit(P.R, P.t, dep_lo, dep_hi);
  // the pass's ops and their couplings / fields, read once per tile and all
  // at the same time (a dependent read per op would stall every op)
  const int32_t* Jrow = J + inst * jst;
  const int32_t* hrow = h ? h + inst * hst : nullptr;
  for (int o = threadIdx.x; o < P.n_ops; o += CNT_PASS) {
    const DevOp op = ops[P.op_begin + o];
    s_op[o] = op;
    s_val[o] = (op.kind == OP_GATE || op.kind == OP_DIAG) ? (float)Jrow[op.param]
               : (op.kind == OP_FIELD && hrow)              ? (float)hrow[op.param]
                                                            : 0.f;
  }
  __syncthreads();
  const uint64_t in_mask = (1ull << P.in_w) - 1ull;
  const float* xs = xin + inst * sst;
  const uint64_t* ns = nin + inst * sst * nres;
  {
    // every load of the thread's entries (at most CNT_PER_THREAD) is issued
    // before the first is written to LDS, so the tile arrives in one round
    // trip instead of one per entry
    float xv[CNT_PER_THREAD];
    uint64_t nv[CNT_PER_THREAD][NRES];
#pragma unroll
    for (int k = 0; k < CNT_PER_THREAD; ++k) {
      const uint32_t i = threadIdx.x + (uint32_t)k * CNT_PASS;
      xv[k] = 0.f;
#pragma unroll
      for (int r = 0; r < NRES; ++r) nv[k][r] = 1ull;
      if (i < size && !P.init) {
        uint64_t idx = (base | dep_lo[i & 255u] | dep_hi[i >> 8]) & in_mask;
        if (z2) idx = z2_addr(idx, P.in_w);
        xv[k] = xs[idx];
#pragma unroll
        for (int r = 0; r < NRES; ++r)
          if (r < nres) nv[k][r] = ns[r * sst + idx];
      }
    }
#pragma unroll
    for (int k = 0; k < CNT_PER_THREAD; ++k) {
      const uint32_t i = threadIdx.x + (uint32_t)k * CNT_PASS;
      if (i < size) {
        tx[i] = xv[k];
#pragma unroll
        for (int r = 0; r < NRES; ++r)
          if (r < nres) tn[r * size + i] = nv[k][r];
      }
    }
  }
  __syncthreads();
  for (int o = 0; o < P.n_ops; ++o) {
    const DevOp op = s_op[o];
    if (op.kind == OP_GATE || op.kind == OP_CUT) {
      const float Jv = s_val[o];
      const int b = op.a;
      const uint32_t lowmask = (1u << b) - 1u;
      // the thread's pairs (at most two): every LDS read of both issued
      // before the updates, the residue planes and their moduli unrolled at
      // compile time
      constexpr int PP = CNT_PER_THREAD / 2;
      uint32_t j0[PP], j1[PP];
      float a0[PP], a1[PP];
      uint64_t n0[PP][NRES], n1[PP][NRES];
#pragma unroll
      for (int q = 0; q < PP; ++q) {
        const uint32_t p = threadIdx.x + (uint32_t)q * CNT_PASS;
        j0[q] = ((p & ~lowmask) << 1) | (p & lowmask);
        j1[q] = j0[q] | (1u << b);
        if (p < (size >> 1)) {
          a0[q] = tx[j0[q]];
          a1[q] = tx[j1[q]];
#pragma unroll
          for (int r = 0; r < NRES; ++r)
            if (r < nres) {
              n0[q][r] = tn[r * size + j0[q]];
              n1[q][r] = tn[r * size + j1[q]];
            }
        }
      }
#pragma unroll
      for (int q = 0; q < PP; ++q) {
        const uint32_t p = threadIdx.x + (uint32_t)q * CNT_PASS;
        if (p >= (size >> 1)) continue;
        const float c00 = a0[q] + Jv, c10 = a1[q] - Jv, c01 = a0[q] - Jv, c11 = a1[q] + Jv;
        tx[j0[q]] = fmaxf(c00, c10);
        tx[j1[q]] = fmaxf(c01, c11);
#pragma unroll
        for (int r = 0; r < NRES; ++r)
          if (r < nres) {
            const uint64_t both = addmod(n0[q][r], n1[q][r], mod_of(r));
            tn[r * size + j0[q]] = c00 > c10 ? n0[q][r] : (c10 > c00 ? n1[q][r] : both);
            tn[r * size + j1[q]] = c01 > c11 ? n0[q][r] : (c11 > c01 ? n1[q][r] : both);
          }
      }
      __syncthreads();
    } else if (op.kind == OP_DIAG || op.kind == OP_FIELD) {
      const float v = s_val[o];
      const bool diag = op.kind == OP_DIAG;
      float xv[CNT_PER_THREAD];
#pragma unroll
      for (int k = 0; k < CNT_PER_THREAD; ++k) {
        const uint32_t i = threadIdx.x + (uint32_t)k * CNT_PASS;
        if (i < size) xv[k] = tx[i];
      }
#pragma unroll
      for (int k = 0; k < CNT_PER_THREAD; ++k) {
        const uint32_t i = threadIdx.x + (uint32_t)k * CNT_PASS;
        if (i < size) {
          const int s = diag ? (cbit(op.a, i, base) ^ cbit(op.b, i, base)) : cbit(op.a, i, base);
          tx[i] = xv[k] + (s ? -v : v);
        }
      }
      __syncthreads();
    }
  }
  float* xd = xout + inst * sst;
  uint64_t* nd = nout + inst * sst * nres;
#pragma unroll
  for (int k = 0; k < CNT_PER_THREAD; ++k) {
    const uint32_t i = threadIdx.x + (uint32_t)k * CNT_PASS;
    if (i >= size) continue;
    uint64_t idx = base | dep_lo[i & 255u] | dep_hi[i >> 8];
    if ((idx >> P.out_w) != 0) continue;
    if (z2) idx = z2_addr(idx, P.out_w);
    // non-temporal: the next pass reads the state from memory
    __builtin_nontemporal_store(tx[i], &xd[idx]);
#pragma unroll
    for (int r = 0; r < NRES; ++r)
      if (r < nres) __builtin_nontemporal_store(tn[r * size + i], &nd[r * sst + idx]);
  }
}

// final reduction: x* = max x, n* = sum of n over entries with x = x* (Eq. 4)
__device__ float cblock_max(float v) {
  __shared__ float sh[CNT / 64];
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = sh[0];
  for (int k = 1; k < CNT / 64; ++k) r = fmaxf(r, sh[k]);
  __syncthreads();
  return r;
}

__device__ uint64_t cblock_summod(uint64_t v, uint64_t p) {
  __shared__ uint64_t sh[CNT / 64];
  for (int off = 32; off > 0; off >>= 1) v = addmod(v, __shfl_xor(v, off, 64), p);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t r = sh[0];
  for (int k = 1; k < CNT / 64; ++k) r = addmod(r, sh[k], p);
  __syncthreads();
  return r;
}

// Slots that are free after the last op hold copies of every configuration
// (their two halves are equal), so only entries with those bits zero count.
// Half-state plans (z2) read every entry at its stored address.
__global__ __launch_bounds__(CNT) void k_count_reduce1(const float* __restrict__ x, const uint64_t* __restrict__ nr,
                                                       int64_t sst, int w, int log2_chunks, uint64_t free_mask,
                                                       int nres, int z2, float* __restrict__ pv,
                                                       uint64_t* __restrict__ pn) {
  const int64_t inst = (int64_t)blockIdx.x >> log2_chunks;
  const uint64_t chunk = (uint64_t)blockIdx.x & ((1ull << log2_chunks) - 1ull);
  const uint64_t len = 1ull << (w - log2_chunks);
  const float* xs = x + inst * sst;
  const uint64_t* ns = nr + inst * sst * nres;
  float mx = -INFINITY;
  const int zw = z2 ? w : 0;
  for (uint64_t k = threadIdx.x; k < len; k += CNT) mx = fmaxf(mx, xs[z2_addr(chunk * len + k, zw)]);
  mx = cblock_max(mx);
  for (int r = 0; r < NRES; ++r) {
    if (r >= nres) {
      if (threadIdx.x == 0) pn[blockIdx.x * NRES + r] = 0;
      continue;
    }
    uint64_t acc = 0;
    for (uint64_t k = threadIdx.x; k < len; k += CNT) {
      const uint64_t idx = chunk * len + k, at = z2_addr(idx, zw);
      if ((idx & free_mask) == 0 && xs[at] == mx) acc = addmod(acc, ns[r * sst + at], c_mod[r]);
    }
    acc = cblock_summod(acc, c_mod[r]);
    if (threadIdx.x == 0) pn[blockIdx.x * NRES + r] = acc;
  }
  if (threadIdx.x == 0) pv[blockIdx.x] = mx;
}

// partials and residues: NRES words per chunk / instance (unused planes 0)
__global__ __launch_bounds__(CNT) void k_count_reduce2(const float* __restrict__ pv, const uint64_t* __restrict__ pn,
                                                       int log2_chunks, int64_t* __restrict__ energy,
                                                       uint64_t* __restrict__ residues) {
  const int64_t inst = blockIdx.x;
  const int64_t nc = 1ll << log2_chunks;
  float mx = -INFINITY;
  for (int64_t k = threadIdx.x; k < nc; k += CNT) mx = fmaxf(mx, pv[inst * nc + k]);
  mx = cblock_max(mx);
  for (int r = 0; r < NRES; ++r) {
    uint64_t acc = 0;
    for (int64_t k = threadIdx.x; k < nc; k += CNT)
      if (pv[inst * nc + k] == mx) acc = addmod(acc, pn[(inst * nc + k) * NRES + r], c_mod[r]);
    acc = cblock_summod(acc, c_mod[r]);
    if (threadIdx.x == 0) residues[inst * NRES + r] = acc;
  }
  if (threadIdx.x == 0) energy[inst] = -(int64_t)mx;
}

int count_reduce_log2_chunks(int w) {
  int c = w - 12;
  if (c < 0) c = 0;
  if (c > 10) c = 10;
  return c;
}

hipError_t launch_count_pass(const DevPass& P, const DevOp* ops, const int32_t* J, const int32_t* h, int64_t jst,
                             int64_t hst, const float* xin, const uint64_t* nin, float* xout, uint64_t* nout,
                             int64_t sst, int batch, int nres, bool z2, hipStream_t stream) {
  if (nres < 3 || nres > NRES || P.n_ops > CNT_MAX_OPS || P.t > CNT_MAX_T) return hipErrorInvalidValue;
  const size_t lds = ((size_t)1 << P.t) * (sizeof(float) + nres * sizeof(uint64_t));
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_count_pass),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // half-state plans run half of the tiles (all of them when no fixed slot
  // reaches the output)
  const int run_bits = P.n_free - ((z2 && P.z2_skip >= 0) ? 1 : 0);
  const uint64_t grid = (uint64_t)batch << run_bits;
  if (grid >= (1ull << 31)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_count_pass, dim3((uint32_t)grid), dim3(CNT_PASS), lds, stream, P, ops, J, h, jst, hst, xin, nin,
                     xout, nout, sst, run_bits, nres, z2 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_count_reduce(const float* x, const uint64_t* nplanes, int64_t sst, int w, uint64_t free_mask,
                               int batch, int nres, bool z2, float* pv, uint64_t* pn, int64_t* energy,
                               uint64_t* residues, hipStream_t stream) {
  if (nres < 3 || nres > NRES) return hipErrorInvalidValue;
  const int lc = count_reduce_log2_chunks(w);
  hipLaunchKernelGGL(k_count_reduce1, dim3((uint32_t)((uint64_t)batch << lc)), dim3(CNT), 0, stream, x, nplanes, sst,
                     w, lc, free_mask, nres, z2 ? 1 : 0, pv, pn);
  hipLaunchKernelGGL(k_count_reduce2, dim3((uint32_t)batch), dim3(CNT), 0, stream, pv, pn, lc, energy, residues);
  return hipGetLastError();
}

}  // namespace tt
