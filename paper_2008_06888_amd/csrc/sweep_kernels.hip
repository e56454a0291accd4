// HIP kernels (gfx950) of the tropical sweep: energy passes, final
// reduction and the argmax-routing backward walk.
//
// A pass applies a run of operations (see plan.hpp) to the state tensor.
// Each workgroup owns one tile: the 2^t state entries that share the values
// of every non-resident slot. The tile is staged in LDS, every operation of
// the run is applied there, and the tile is written back, so one pass costs
// one read and one write of the state per run of up to t gate bits.
//
// Arithmetic is the max-plus semiring of Eq. (2): the tropical product is a
// float add, the tropical sum a float max. Bond entries follow the sign
// convention of Sec. II: the bond matrix is [[J, -J], [-J, J]] with index 0
// <-> sigma = +1, so the state holds negative energies and its final maximum
// is -E*.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "plan.hpp"

namespace tt {

constexpr int NT = 256;   // threads per workgroup

__device__ __forceinline__ int bit_of(uint8_t enc, uint32_t i, uint64_t base) {
  return enc < SLOT_FIXED ? (int)((i >> enc) & 1u) : (int)((base >> (enc - SLOT_FIXED)) & 1ull);
}

template <typename IT>
__device__ __forceinline__ float ldv(const IT* p, int64_t k) {
  return (float)p[k];
}

// Builds the two 256-entry lookup tables that scatter a tile index (t <= 16
// bits) onto the slots R of the state index.
__device__ __forceinline__ void build_deposit(const uint8_t* R, int t, uint64_t* lo, uint64_t* hi) {
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

__device__ __forceinline__ uint64_t tile_base(const DevPass& P, uint64_t tile_id) {
  uint64_t base = 0;
  for (int k = 0; k < P.n_free; ++k) base |= ((tile_id >> k) & 1ull) << P.fre[k];
  return base;
}

// Applies ops [0, n_ops) of a pass to an LDS tile of 2^t floats.
// REC: record the argmax decision of every GATE / CUT for every output entry
// (bit i of row op.dec), ties resolving to the first argument.
template <bool REC, typename IT>
__device__ void apply_ops(float* tile, uint32_t* dec, int t, uint64_t base, const DevOp* ops,
                          int n_ops, const IT* Jrow, const IT* hrow) {
  const uint32_t size = 1u << t;
  const uint32_t half = size >> 1;
  const int tid = threadIdx.x;
  for (int o = 0; o < n_ops; ++o) {
    const DevOp op = ops[o];
    if (op.kind == OP_GATE || op.kind == OP_CUT) {
      const float J = op.kind == OP_GATE ? ldv(Jrow, op.param) : 0.f;
      const int b = op.a;
      const uint32_t lowmask = (1u << b) - 1u;
      for (uint32_t p = tid; p < half; p += NT) {
        const uint32_t i0 = ((p & ~lowmask) << 1) | (p & lowmask);
        const uint32_t i1 = i0 | (1u << b);
        const float a0 = tile[i0], a1 = tile[i1];
        // new index 0: from old 0 with +J, from old 1 with -J; new index 1: the reverse
        const float c00 = a0 + J, c10 = a1 - J;
        const float c01 = a0 - J, c11 = a1 + J;
        tile[i0] = fmaxf(c00, c10);
        tile[i1] = fmaxf(c01, c11);
        if (REC) {
          uint32_t* row = dec + (size_t)op.dec * ((size + 31u) >> 5);
          if (c10 > c00) atomicOr(&row[i0 >> 5], 1u << (i0 & 31));
          if (c11 > c01) atomicOr(&row[i1 >> 5], 1u << (i1 & 31));
        }
      }
      __syncthreads();
    } else if (op.kind == OP_DIAG) {
      const float J = ldv(Jrow, op.param);
      for (uint32_t i = tid; i < size; i += NT) {
        const int s = bit_of(op.a, i, base) ^ bit_of(op.b, i, base);
        tile[i] += s ? -J : J;
      }
      __syncthreads();
    } else if (op.kind == OP_FIELD) {
      const float hv = ldv(hrow, op.param);
      for (uint32_t i = tid; i < size; i += NT) {
        tile[i] += bit_of(op.a, i, base) ? -hv : hv;
      }
      __syncthreads();
    }
    // OP_INTRO: the new slot was free, i.e. constant along its bit: nothing to do
  }
}

template <typename IT>
__global__ __launch_bounds__(NT) void k_sweep_pass(DevPass P, const DevOp* __restrict__ ops,
                                                   const IT* __restrict__ J, const IT* __restrict__ h,
                                                   int64_t jst, int64_t hst, const float* __restrict__ in,
                                                   float* __restrict__ out, int64_t sst, int log2_tiles) {
  extern __shared__ float tile[];
  __shared__ uint64_t dep_lo[256], dep_hi[256];
  const int64_t inst = (int64_t)blockIdx.x >> log2_tiles;
  const uint64_t tile_id = (uint64_t)blockIdx.x & ((1ull << log2_tiles) - 1ull);
  const uint64_t base = tile_base(P, tile_id);
  build_deposit(P.R, P.t, dep_lo, dep_hi);
  __syncthreads();
  const uint32_t size = 1u << P.t;
  const uint64_t in_mask = (1ull << P.in_w) - 1ull;
  const float* src = in + inst * sst;
  for (uint32_t i = threadIdx.x; i < size; i += NT) {
    const uint64_t idx = base | dep_lo[i & 255u] | dep_hi[i >> 8];
    tile[i] = P.init ? 0.f : src[idx & in_mask];
  }
  __syncthreads();
  apply_ops<false, IT>(tile, nullptr, P.t, base, ops + P.op_begin, P.n_ops, J + inst * jst,
                       h ? h + inst * hst : nullptr);
  float* dst = out + inst * sst;
  for (uint32_t i = threadIdx.x; i < size; i += NT) {
    const uint64_t idx = base | dep_lo[i & 255u] | dep_hi[i >> 8];
    if ((idx >> P.out_w) == 0) dst[idx] = tile[i];
  }
}

// ---------------------------------------------------------------------------
// final reduction: max over the state and its lowest index (Sec. II: the
// contraction with the product state (0, 0)^n of App. A)
// ---------------------------------------------------------------------------

struct VI {
  float v;
  uint64_t i;
};

__device__ __forceinline__ VI vi_best(VI a, VI b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

__device__ VI block_best(VI x) {
  __shared__ float sv[NT / 64];
  __shared__ uint64_t si[NT / 64];
  for (int off = 32; off > 0; off >>= 1) {
    VI y;
    y.v = __shfl_xor(x.v, off, 64);
    y.i = __shfl_xor(x.i, off, 64);
    x = vi_best(x, y);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    sv[w] = x.v;
    si[w] = x.i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < NT / 64; ++k) x = vi_best(x, VI{sv[k], si[k]});
    sv[0] = x.v;
    si[0] = x.i;
  }
  __syncthreads();
  VI r{sv[0], si[0]};
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(NT) void k_reduce_stage1(const float* __restrict__ st, int64_t sst, int w,
                                                      int log2_chunks, float* __restrict__ pv,
                                                      uint64_t* __restrict__ pi) {
  const int64_t inst = (int64_t)blockIdx.x >> log2_chunks;
  const uint64_t chunk = (uint64_t)blockIdx.x & ((1ull << log2_chunks) - 1ull);
  const uint64_t len = 1ull << (w - log2_chunks);
  const float* s = st + inst * sst;
  VI best{-INFINITY, ~0ull};
  for (uint64_t k = threadIdx.x; k < len; k += NT) {
    const uint64_t idx = chunk * len + k;
    best = vi_best(best, VI{s[idx], idx});
  }
  best = block_best(best);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = best.v;
    pi[blockIdx.x] = best.i;
  }
}

__global__ __launch_bounds__(NT) void k_reduce_stage2(const float* __restrict__ pv,
                                                      const uint64_t* __restrict__ pi, int log2_chunks,
                                                      double* __restrict__ energy,
                                                      uint64_t* __restrict__ arg) {
  const int64_t inst = blockIdx.x;
  const int64_t nc = 1ll << log2_chunks;
  VI best{-INFINITY, ~0ull};
  for (int64_t k = threadIdx.x; k < nc; k += NT) best = vi_best(best, VI{pv[inst * nc + k], pi[inst * nc + k]});
  best = block_best(best);
  if (threadIdx.x == 0) {
    if (energy) energy[inst] = -(double)best.v;
    if (arg) arg[inst] = best.i;
  }
}

// ---------------------------------------------------------------------------
// backward: argmax routing (Sec. IV, caching intermediates and backtracking;
// the first argument wins ties). One workgroup per instance walks the passes
// in reverse; for each pass it reloads the tile holding the selected entry
// from that pass's input, recomputes the pass recording every decision, and
// routes the selected index back through the pass's ops.
// ---------------------------------------------------------------------------

constexpr int MAX_SPINS = 8192;

template <typename IT>
__global__ __launch_bounds__(NT) void k_sweep_backward(
    const DevPass* __restrict__ passes, int n_passes, const DevOp* __restrict__ ops,
    const DevSpin* __restrict__ spins, const IT* __restrict__ J, const IT* __restrict__ h, int64_t jst,
    int64_t hst, const float* const* __restrict__ ckpt, int64_t sst, const uint64_t* __restrict__ final_idx,
    const int32_t* __restrict__ final_slot_spin, int final_w, const int32_t* __restrict__ edges, int n,
    int64_t m, int8_t* __restrict__ sigma, float* __restrict__ dJ, float* __restrict__ dh, int max_t) {
  extern __shared__ float smem[];
  float* tile = smem;
  uint32_t* dec = reinterpret_cast<uint32_t*>(smem + (1u << max_t));
  __shared__ uint64_t dep_lo[256], dep_hi[256];
  __shared__ int8_t s_sh[MAX_SPINS];
  __shared__ uint64_t sh_idx, sh_base;
  const int64_t inst = blockIdx.x;
  const int tid = threadIdx.x;
  const IT* Jrow = J + inst * jst;
  const IT* hrow = h ? h + inst * hst : nullptr;
  for (int v = tid; v < n; v += NT) s_sh[v] = 0;
  __syncthreads();
  if (tid == 0) {
    const uint64_t idx = final_idx[inst];
    for (int c = 0; c < final_w; ++c) {
      const int sp = final_slot_spin[c];
      if (sp >= 0) s_sh[sp] = (int8_t)((idx >> c) & 1ull);
    }
    sh_idx = idx;
  }
  __syncthreads();
  for (int p = n_passes - 1; p >= 0; --p) {
    const DevPass P = passes[p];
    const uint32_t size = 1u << P.t;
    const uint32_t words = (size + 31u) >> 5;
    build_deposit(P.R, P.t, dep_lo, dep_hi);
    for (uint32_t k = tid; k < (uint32_t)P.n_dec * words; k += NT) dec[k] = 0u;
    if (tid == 0) {
      uint64_t rmask = 0;
      for (int k = 0; k < P.t; ++k) rmask |= 1ull << P.R[k];
      sh_base = sh_idx & ~rmask & ((1ull << P.w_max) - 1ull);
    }
    __syncthreads();
    const uint64_t base = sh_base;
    const uint64_t in_mask = (1ull << P.in_w) - 1ull;
    const float* src = ckpt[p];
    for (uint32_t i = tid; i < size; i += NT) {
      const uint64_t idx = base | dep_lo[i & 255u] | dep_hi[i >> 8];
      tile[i] = P.init ? 0.f : src[inst * sst + (idx & in_mask)];
    }
    __syncthreads();
    apply_ops<true, IT>(tile, dec, P.t, base, ops + P.op_begin, P.n_ops, Jrow, hrow);
    __syncthreads();
    if (tid == 0) {
      const uint64_t idx = sh_idx;
      uint32_t i = 0;
      for (int k = 0; k < P.t; ++k) i |= (uint32_t)((idx >> P.R[k]) & 1ull) << k;
      uint64_t b = base;
      for (int o = P.n_ops - 1; o >= 0; --o) {
        const DevOp op = ops[P.op_begin + o];
        if (op.kind == OP_GATE || op.kind == OP_CUT) {
          const uint32_t d = (dec[(size_t)op.dec * words + (i >> 5)] >> (i & 31u)) & 1u;
          s_sh[spins[P.op_begin + o].old_spin] = (int8_t)d;
          i = (i & ~(1u << op.a)) | (d << op.a);
        } else if (op.kind == OP_INTRO) {
          if (op.a < SLOT_FIXED) i &= ~(1u << op.a);
          else b &= ~(1ull << (op.a - SLOT_FIXED));
        }
      }
      uint64_t idx_in = b;
      for (int k = 0; k < P.t; ++k) idx_in |= (uint64_t)((i >> k) & 1u) << P.R[k];
      sh_idx = idx_in & in_mask;
    }
    __syncthreads();
  }
  for (int v = tid; v < n; v += NT) {
    const float sg = s_sh[v] ? -1.f : 1.f;
    sigma[inst * n + v] = (int8_t)(s_sh[v] ? -1 : 1);
    if (dh) dh[inst * n + v] = -sg;
  }
  if (dJ) {
    for (int64_t e = tid; e < m; e += NT) {
      const int a = edges[2 * e], c = edges[2 * e + 1];
      const float sa = s_sh[a] ? -1.f : 1.f, sc = s_sh[c] ? -1.f : 1.f;
      dJ[inst * m + e] = -(sa * sc);
    }
  }
}

// ---------------------------------------------------------------------------
// host launch wrappers (kernels are launched from this translation unit)
// ---------------------------------------------------------------------------

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_sweep_pass(const DevPass& P, const DevOp* ops, int dtype, const void* J, const void* h,
                             int64_t jst, int64_t hst, const float* in, float* out, int64_t sst, int batch,
                             hipStream_t stream) {
  const size_t lds = sizeof(float) << P.t;
  const int log2_tiles = P.n_free;
  const uint64_t grid = (uint64_t)batch << log2_tiles;
  if (grid >= (1ull << 31)) return hipErrorInvalidConfiguration;
  if (dtype == 0) {
    hipError_t e = allow_lds(k_sweep_pass<float>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_pass<float>, dim3((uint32_t)grid), dim3(NT), lds, stream, P, ops,
                       (const float*)J, (const float*)h, jst, hst, in, out, sst, log2_tiles);
  } else {
    hipError_t e = allow_lds(k_sweep_pass<int32_t>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_pass<int32_t>, dim3((uint32_t)grid), dim3(NT), lds, stream, P, ops,
                       (const int32_t*)J, (const int32_t*)h, jst, hst, in, out, sst, log2_tiles);
  }
  return hipGetLastError();
}

int reduce_log2_chunks(int w) {
  // chunks of at least 2^12 entries, at most 2^10 chunks per instance
  int c = w - 12;
  if (c < 0) c = 0;
  if (c > 10) c = 10;
  return c;
}

hipError_t launch_reduce(const float* st, int64_t sst, int w, int batch, float* pv, uint64_t* pi,
                         double* energy, uint64_t* arg, hipStream_t stream) {
  const int lc = reduce_log2_chunks(w);
  hipLaunchKernelGGL(k_reduce_stage1, dim3((uint32_t)((uint64_t)batch << lc)), dim3(NT), 0, stream, st, sst,
                     w, lc, pv, pi);
  hipLaunchKernelGGL(k_reduce_stage2, dim3((uint32_t)batch), dim3(NT), 0, stream, pv, pi, lc, energy, arg);
  return hipGetLastError();
}

size_t backward_lds_bytes(int max_t, int max_dec) {
  const size_t words = (((size_t)1 << max_t) + 31) / 32;   // decision row: whole 32-bit words
  return (sizeof(float) << max_t) + (size_t)max_dec * words * sizeof(uint32_t);
}

hipError_t launch_sweep_backward(const DevPass* passes, int n_passes, const DevOp* ops, const DevSpin* spins,
                                 int dtype, const void* J, const void* h, int64_t jst, int64_t hst,
                                 const float* const* ckpt, int64_t sst, const uint64_t* final_idx,
                                 const int32_t* final_slot_spin, int final_w, const int32_t* edges, int n,
                                 int64_t m, int8_t* sigma, float* dJ, float* dh, int max_t, int max_dec,
                                 int batch, hipStream_t stream) {
  const size_t lds = backward_lds_bytes(max_t, max_dec);
  if (dtype == 0) {
    hipError_t e = allow_lds(k_sweep_backward<float>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_backward<float>, dim3(batch), dim3(NT), lds, stream, passes, n_passes, ops, spins,
                       (const float*)J, (const float*)h, jst, hst, ckpt, sst, final_idx, final_slot_spin,
                       final_w, edges, n, m, sigma, dJ, dh, max_t);
  } else {
    hipError_t e = allow_lds(k_sweep_backward<int32_t>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_backward<int32_t>, dim3(batch), dim3(NT), lds, stream, passes, n_passes, ops,
                       spins, (const int32_t*)J, (const int32_t*)h, jst, hst, ckpt, sst, final_idx,
                       final_slot_spin, final_w, edges, n, m, sigma, dJ, dh, max_t);
  }
  return hipGetLastError();
}

}  // namespace tt
