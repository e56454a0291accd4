// HIP kernels (gfx950) of the 3-state Potts sweep (App. C): passes over a
// 3^W state of negative doubled energies, energy only or with (x, n) tuples
// (Eq. 4) whose counts are residues modulo the three count primes (and a
// plane modulo 2^64 as the exactness guard), and the final maximum / count.
//
// A thread owns the 3^T entries of one assignment of the non-tile digits
// (T tile digits, compile-time) in registers: every op of the pass is a
// compile-time loop over those entries, dispatched on its tile digit(s) by a
// uniform branch. No LDS. The non-tile digits of the lowest slots vary
// fastest across threads, so a wave's loads of one register are one run of
// consecutive entries whenever the four lowest slots are non-tile digits.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_mem.hpp"
#include "launch.hpp"
#include "potts.hpp"

namespace tt {

namespace {

constexpr int PT = 256;   // threads per workgroup

__host__ __device__ constexpr int ipow3(int k) { return k == 0 ? 1 : 3 * ipow3(k - 1); }
__host__ __device__ constexpr int digit(int i, int r) { return (i / ipow3(r)) % 3; }

constexpr uint64_t P0 = (1ull << 61) - 1, P1 = (1ull << 61) - 31, P2 = (1ull << 61) - 45;
__device__ __forceinline__ uint64_t prime(int r) { return r == 0 ? P0 : (r == 1 ? P1 : P2); }

// (a + b) mod p for a, b < p < 2^61; plane 3 is modulo 2^64 (plain wraparound)
template <int R>
__device__ __forceinline__ uint64_t addm(uint64_t a, uint64_t b) {
  if constexpr (R == 3) {
    return a + b;
  } else {
    const uint64_t p = R == 0 ? P0 : (R == 1 ? P1 : P2);
    const uint64_t s = a + b;
    return s >= p ? s - p : s;
  }
}

// ---- energy ops on the register tile -------------------------------------
template <int T, int D>
__device__ __forceinline__ void gate(float (&v)[ipow3(T)], float ceq, float cne) {
  constexpr int S = ipow3(D);
#pragma unroll
  for (int c = 0; c < ipow3(T) / 3; ++c) {
    const int i0 = (c / S) * 3 * S + (c % S);
    const float a0 = v[i0], a1 = v[i0 + S], a2 = v[i0 + 2 * S];
    const float m12 = fmaxf(a1, a2), m02 = fmaxf(a0, a2), m01 = fmaxf(a0, a1);
    v[i0] = fmaxf(a0 + ceq, m12 + cne);
    v[i0 + S] = fmaxf(a1 + ceq, m02 + cne);
    v[i0 + 2 * S] = fmaxf(a2 + ceq, m01 + cne);
  }
}

template <int T, int D>
__device__ __forceinline__ void cut(float (&v)[ipow3(T)]) {
  constexpr int S = ipow3(D);
#pragma unroll
  for (int c = 0; c < ipow3(T) / 3; ++c) {
    const int i0 = (c / S) * 3 * S + (c % S);
    const float m = fmaxf(fmaxf(v[i0], v[i0 + S]), v[i0 + 2 * S]);
    v[i0] = m;
    v[i0 + S] = m;
    v[i0 + 2 * S] = m;
  }
}

template <int T, int A, int B>
__device__ __forceinline__ void diag(float (&v)[ipow3(T)], float ceq, float cne) {
#pragma unroll
  for (int i = 0; i < ipow3(T); ++i) v[i] += digit(i, A) == digit(i, B) ? ceq : cne;
}

// ---- counting ops: (x, n) tuples, n in NR residue planes -------------------
template <int NR>
struct Cnt {
  uint64_t r[NR];
};

template <int NR, int R = 0>
__device__ __forceinline__ void cnt_add_if(Cnt<NR>& acc, bool hit, const Cnt<NR>& x) {
  if constexpr (R < NR) {
    acc.r[R] = addm<R>(acc.r[R], hit ? x.r[R] : 0ull);
    cnt_add_if<NR, R + 1>(acc, hit, x);
  }
}

template <int T, int NR, int D>
__device__ __forceinline__ void cgate(float (&v)[ipow3(T)], Cnt<NR> (&n)[ipow3(T)], float ceq, float cne) {
  constexpr int S = ipow3(D);
#pragma unroll
  for (int c = 0; c < ipow3(T) / 3; ++c) {
    const int i0 = (c / S) * 3 * S + (c % S);
    const float a[3] = {v[i0], v[i0 + S], v[i0 + 2 * S]};
    const Cnt<NR> m[3] = {n[i0], n[i0 + S], n[i0 + 2 * S]};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      float cand[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) cand[k] = a[k] + (k == b ? ceq : cne);
      const float y = fmaxf(fmaxf(cand[0], cand[1]), cand[2]);
      Cnt<NR> acc;
#pragma unroll
      for (int r = 0; r < NR; ++r) acc.r[r] = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) cnt_add_if<NR>(acc, cand[k] == y, m[k]);
      v[i0 + b * S] = y;
      n[i0 + b * S] = acc;
    }
  }
}

template <int T, int NR, int D>
__device__ __forceinline__ void ccut(float (&v)[ipow3(T)], Cnt<NR> (&n)[ipow3(T)]) {
  constexpr int S = ipow3(D);
#pragma unroll
  for (int c = 0; c < ipow3(T) / 3; ++c) {
    const int i0 = (c / S) * 3 * S + (c % S);
    const float a[3] = {v[i0], v[i0 + S], v[i0 + 2 * S]};
    const float y = fmaxf(fmaxf(a[0], a[1]), a[2]);
    Cnt<NR> acc;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc.r[r] = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) cnt_add_if<NR>(acc, a[k] == y, n[i0 + k * S]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[i0 + k * S] = y;
      n[i0 + k * S] = acc;
    }
  }
}

// ---- dispatch on the op's tile digit(s) (uniform branches) -----------------
template <int T, int NR, bool COUNT, int D>
__device__ __forceinline__ void gate_d(float (&v)[ipow3(T)], Cnt<NR> (&n)[ipow3(T)], float ceq, float cne) {
  if constexpr (D < T) {
    if constexpr (COUNT) cgate<T, NR, D>(v, n, ceq, cne);
    else gate<T, D>(v, ceq, cne);
  }
}

template <int T, int NR, bool COUNT, int D>
__device__ __forceinline__ void cut_d(float (&v)[ipow3(T)], Cnt<NR> (&n)[ipow3(T)]) {
  if constexpr (D < T) {
    if constexpr (COUNT) ccut<T, NR, D>(v, n);
    else cut<T, D>(v);
  }
}

template <int T, int A, int B>
__device__ __forceinline__ void diag_ab(float (&v)[ipow3(T)], float ceq, float cne) {
  if constexpr (B < T) diag<T, A, B>(v, ceq, cne);
}

template <int T, int NR, bool COUNT>
__device__ __forceinline__ void apply_op(int kind, int a, int b, float ceq, float cne, float (&v)[ipow3(T)],
                                         Cnt<NR> (&n)[ipow3(T)]) {
  if (kind == OP_GATE) {
    switch (a) {
      case 0: gate_d<T, NR, COUNT, 0>(v, n, ceq, cne); break;
      case 1: gate_d<T, NR, COUNT, 1>(v, n, ceq, cne); break;
      case 2: gate_d<T, NR, COUNT, 2>(v, n, ceq, cne); break;
      default: gate_d<T, NR, COUNT, 3>(v, n, ceq, cne); break;
    }
  } else if (kind == OP_CUT) {
    switch (a) {
      case 0: cut_d<T, NR, COUNT, 0>(v, n); break;
      case 1: cut_d<T, NR, COUNT, 1>(v, n); break;
      case 2: cut_d<T, NR, COUNT, 2>(v, n); break;
      default: cut_d<T, NR, COUNT, 3>(v, n); break;
    }
  } else {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    switch (lo * 4 + hi) {
      case 1: diag_ab<T, 0, 1>(v, ceq, cne); break;
      case 2: diag_ab<T, 0, 2>(v, ceq, cne); break;
      case 6: diag_ab<T, 1, 2>(v, ceq, cne); break;
      case 3: diag_ab<T, 0, 3>(v, ceq, cne); break;
      case 7: diag_ab<T, 1, 3>(v, ceq, cne); break;
      default: diag_ab<T, 2, 3>(v, ceq, cne); break;
    }
  }
}

// Coupling of edge e of instance `inst` as a float (int32 couplings are exact
// below 2^24; the call checks sum |J| < 2^23).
__device__ __forceinline__ float coupling(const void* J, int64_t jst, int inst, int e, int dtype) {
  if (dtype == 0) return as_const(static_cast<const float*>(J))[(int64_t)inst * jst + e];
  return (float)as_const(static_cast<const int32_t*>(J))[(int64_t)inst * jst + e];
}

// LOW passes (tile = slots 0 .. T-1): thread t of a workgroup owns the run
// [base + t 3^T, base + (t + 1) 3^T) and the workgroup one contiguous block;
// direct loads would send each lane of a wave to its own cache line, so the
// block goes through LDS in three chunks (the entries c 3^(T-1) .. (c + 1)
// 3^(T-1) - 1 of every run): coalesced loads of the chunk into LDS, then each
// thread takes its part (stride 3^(T-1) words across lanes: odd, so the lanes
// of a wave hit distinct banks), and the reverse for the stores; one plane at
// a time. A chunk's buffer (a third of the block) leaves room for several
// workgroups per CU.
template <int T>
constexpr int low_chunk() {
  return T >= 2 ? ipow3(T - 1) : ipow3(T);
}
template <int T>
constexpr int low_chunks() {
  return ipow3(T) / low_chunk<T>();
}

// Chunk c of the block: global entry of LDS word e (thread e / EC's run).
template <int T>
__device__ __forceinline__ int64_t low_addr(int64_t base, int e, int c) {
  constexpr int E = ipow3(T), EC = low_chunk<T>();
  return base + (int64_t)(e / EC) * E + c * EC + (e % EC);
}

// Chunk c of plane `src` into LDS (words below nvalid), every load of the
// thread issued before the first store.
template <int T, typename V>
__device__ __forceinline__ void low_fill(V* lds, const gptr<V> src, int64_t base, int c, int nvalid) {
  constexpr int EC = low_chunk<T>();
  V t[EC];
#pragma unroll
  for (int k = 0; k < EC; ++k) {
    const int e = (int)threadIdx.x + k * PT;
    t[k] = e < nvalid ? __builtin_nontemporal_load(&src[low_addr<T>(base, e, c)]) : V(0);
  }
#pragma unroll
  for (int k = 0; k < EC; ++k) {
    const int e = (int)threadIdx.x + k * PT;
    if (e < nvalid) lds[e] = t[k];
  }
}
// Chunk c from LDS to plane `dst`, every LDS read issued before the stores.
template <int T, typename V>
__device__ __forceinline__ void low_drain(const V* lds, gptr<V> dst, int64_t base, int c, int nvalid) {
  constexpr int EC = low_chunk<T>();
  V t[EC];
#pragma unroll
  for (int k = 0; k < EC; ++k) {
    const int e = (int)threadIdx.x + k * PT;
    t[k] = e < nvalid ? lds[e] : V(0);
  }
#pragma unroll
  for (int k = 0; k < EC; ++k) {
    const int e = (int)threadIdx.x + k * PT;
    if (e < nvalid) __builtin_nontemporal_store(t[k], &dst[low_addr<T>(base, e, c)]);
  }
}

template <int T, int NR, bool COUNT, bool LOW>
__global__ __launch_bounds__(PT) void k_potts_pass(const PottsPass* __restrict__ pass, const void* __restrict__ J,
                                                   int64_t jst, int dtype, float* __restrict__ x,
                                                   uint64_t* __restrict__ nst, int64_t sst, int64_t plane) {
  constexpr int E = ipow3(T);
  const cptr<PottsPass> P = as_const(pass);
  const int64_t threads = P->threads;
  const int64_t gid0 = (int64_t)blockIdx.x * PT;
  const int64_t gid = gid0 + threadIdx.x;
  if (!LOW && gid >= threads) return;   // (LOW workgroups stay whole for their barriers)
  const int inst = (int)blockIdx.y;
  const gptr<float> X = as_global(x);
  const gptr<uint64_t> N = as_global(nst);
  float v[E];
  Cnt<NR> n[E];
  const bool init = P->init != 0;
  if constexpr (LOW) {
    extern __shared__ float lds_f[];
    uint64_t* lds_u = reinterpret_cast<uint64_t*>(lds_f);
    constexpr int EC = low_chunk<T>(), NC = low_chunks<T>();
    const int64_t base = (int64_t)inst * sst + gid0 * E;
    const int64_t left = threads - gid0;
    const int nvalid = (int)((left < PT ? left : PT) * EC);   // words of a chunk
    const int mine = (int)threadIdx.x * EC;
    if (init) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        v[i] = 0.f;
        if constexpr (COUNT) {
#pragma unroll
          for (int r = 0; r < NR; ++r) n[i].r[r] = 1;
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        if (c) __syncthreads();
        low_fill<T>(lds_f, X, base, c, nvalid);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < EC; ++i) v[c * EC + i] = lds_f[mine + i];
      }
      if constexpr (COUNT) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            __syncthreads();
            low_fill<T>(lds_u, N + r * plane, base, c, nvalid);
            __syncthreads();
#pragma unroll
            for (int i = 0; i < EC; ++i) n[c * EC + i].r[r] = lds_u[mine + i];
          }
        }
      }
    }
    const int nops = P->n_ops;
    for (int o = 0; o < nops; ++o) {
      const int kind = P->ops[o].kind, a = P->ops[o].a, b = P->ops[o].b, e = P->ops[o].edge;
      const float Jv = kind == OP_CUT ? 0.f : coupling(J, jst, inst, e, dtype);
      apply_op<T, NR, COUNT>(kind, a, b, -2.f * Jv, Jv, v, n);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < EC; ++i) lds_f[mine + i] = v[c * EC + i];
      __syncthreads();
      low_drain<T>(lds_f, X, base, c, nvalid);
    }
    if constexpr (COUNT) {
#pragma unroll
      for (int r = 0; r < NR; ++r) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          __syncthreads();
#pragma unroll
          for (int i = 0; i < EC; ++i) lds_u[mine + i] = n[c * EC + i].r[r];
          __syncthreads();
          low_drain<T>(lds_u, N + r * plane, base, c, nvalid);
        }
      }
    }
    return;
  } else {
    // this thread's non-tile digits -> base entry
    int64_t off = (int64_t)inst * sst;
    {
      uint64_t g = (uint64_t)gid;
      const int nnt = P->n_nt;
      for (int r = 0; r < nnt; ++r) {
        const uint64_t q = g / 3u;
        off += (int64_t)(g - 3u * q) * P->nt_st[r];
        g = q;
      }
    }
    // tile entry i sits at off + lo[i % 3^TL] + hi[i / 3^TL]: the offsets of the
    // low and high tile digits (32 bits: an instance has at most 3^20 entries)
    constexpr int TL = T / 2, TH = T - TL;
    uint32_t lo[ipow3(TL)], hi[ipow3(TH)];
    {
      uint32_t st[T];
#pragma unroll
      for (int r = 0; r < T; ++r) st[r] = (uint32_t)P->tile_st[r];
#pragma unroll
      for (int i = 0; i < ipow3(TL); ++i) {
        lo[i] = 0;
#pragma unroll
        for (int r = 0; r < TL; ++r) lo[i] += (uint32_t)digit(i, r) * st[r];
      }
#pragma unroll
      for (int i = 0; i < ipow3(TH); ++i) {
        hi[i] = 0;
#pragma unroll
        for (int r = 0; r < TH; ++r) hi[i] += (uint32_t)digit(i, r) * st[TL + r];
      }
    }
    auto addr = [&](int i) { return off + (int64_t)(lo[i % ipow3(TL)] + hi[i / ipow3(TL)]); };
    if (init) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        v[i] = 0.f;
        if constexpr (COUNT) {
#pragma unroll
          for (int r = 0; r < NR; ++r) n[i].r[r] = 1;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int64_t a = addr(i);
        v[i] = __builtin_nontemporal_load(&X[a]);
        if constexpr (COUNT) {
#pragma unroll
          for (int r = 0; r < NR; ++r) n[i].r[r] = __builtin_nontemporal_load(&N[a + r * plane]);
        }
      }
    }
    const int nops = P->n_ops;
    for (int o = 0; o < nops; ++o) {
      const int kind = P->ops[o].kind, a = P->ops[o].a, b = P->ops[o].b, e = P->ops[o].edge;
      const float Jv = kind == OP_CUT ? 0.f : coupling(J, jst, inst, e, dtype);
      apply_op<T, NR, COUNT>(kind, a, b, -2.f * Jv, Jv, v, n);
    }
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int64_t a = addr(i);
      __builtin_nontemporal_store(v[i], &X[a]);
      if constexpr (COUNT) {
#pragma unroll
        for (int r = 0; r < NR; ++r) __builtin_nontemporal_store(n[i].r[r], &N[a + r * plane]);
      }
    }
  }
}

// ---- final maximum and count ---------------------------------------------
// Stage 1: workgroup (c, inst) takes the live-digit combinations
// [c chunk, (c + 1) chunk) of its instance: maximum, and with counting the
// residue sums of the entries attaining it. Partials: pv [inst][chunks],
// pn [inst][chunks][4].
template <bool COUNT>
__global__ __launch_bounds__(PT) void k_potts_reduce1(const PottsReduce* __restrict__ red, const float* __restrict__ x,
                                                      const uint64_t* __restrict__ nst, int64_t sst, int64_t plane,
                                                      int nres, int64_t chunk, float* __restrict__ pv,
                                                      uint64_t* __restrict__ pn) {
  const cptr<PottsReduce> R = as_const(red);
  const int inst = (int)blockIdx.y;
  const int64_t combos = R->combos;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < combos ? lo + chunk : combos;
  const int nl = R->n_live;
  const cptr<float> X = as_const(x);
  const cptr<uint64_t> Nn = as_const(nst);
  float best = -INFINITY;
  uint64_t c[4] = {0, 0, 0, 0};
  const bool contig = R->contig != 0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += PT) {
    int64_t a = (int64_t)inst * sst;
    if (contig) {
      a += k;
    } else {
      uint64_t g = (uint64_t)k;
      for (int r = 0; r < nl; ++r) {
        const uint64_t q = g / 3u;
        a += (int64_t)(g - 3u * q) * R->st[r];
        g = q;
      }
    }
    const float val = X[a];
    if (COUNT) {
      if (val > best) {
        best = val;
        for (int r = 0; r < 4; ++r) c[r] = 0;
      }
      if (val == best)
        for (int r = 0; r < nres; ++r) {
          const uint64_t s = c[r] + Nn[a + r * plane];
          c[r] = (r < 3 && s >= prime(r)) ? s - prime(r) : s;
        }
    } else {
      best = fmaxf(best, val);
    }
  }
  __shared__ float sv[PT];
  __shared__ uint64_t sc[PT][4];
  sv[threadIdx.x] = best;
  for (int r = 0; r < 4; ++r) sc[threadIdx.x][r] = c[r];
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = -INFINITY;
    for (int k = 0; k < PT; ++k) b = fmaxf(b, sv[k]);
    uint64_t t[4] = {0, 0, 0, 0};
    if (COUNT)
      for (int k = 0; k < PT; ++k)
        if (sv[k] == b)
          for (int r = 0; r < nres; ++r) {
            const uint64_t s = t[r] + sc[k][r];
            t[r] = (r < 3 && s >= prime(r)) ? s - prime(r) : s;
          }
    const int64_t idx = (int64_t)inst * gridDim.x + blockIdx.x;
    pv[idx] = b;
    for (int r = 0; r < 4; ++r) pn[idx * 4 + r] = t[r];
  }
}

// Stage 2: one thread per instance combines its partials. energy: H* as a
// double (= -max / 2); energy2 (may be null): 2H* as int64 (integer
// couplings); res (may be null): [inst][4] residues.
__global__ void k_potts_reduce2(const float* __restrict__ pv, const uint64_t* __restrict__ pn, int64_t chunks,
                                int batch, int nres, double* __restrict__ energy, int64_t* __restrict__ energy2,
                                uint64_t* __restrict__ res) {
  const int inst = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (inst >= batch) return;
  float b = -INFINITY;
  for (int64_t k = 0; k < chunks; ++k) b = fmaxf(b, pv[(int64_t)inst * chunks + k]);
  uint64_t t[4] = {0, 0, 0, 0};
  for (int64_t k = 0; k < chunks; ++k) {
    const int64_t idx = (int64_t)inst * chunks + k;
    if (pv[idx] != b) continue;
    for (int r = 0; r < nres; ++r) {
      const uint64_t s = t[r] + pn[idx * 4 + r];
      t[r] = (r < 3 && s >= prime(r)) ? s - prime(r) : s;
    }
  }
  if (energy) energy[inst] = -0.5 * (double)b;
  if (energy2) energy2[inst] = -(int64_t)b;
  if (res)
    for (int r = 0; r < 4; ++r) res[(int64_t)inst * 4 + r] = t[r];
}

template <int T, int NR, bool COUNT>
hipError_t launch_t(const PottsPass* pass, bool low, int64_t threads, const void* J, int64_t jst, int dtype, float* x,
                    uint64_t* n, int64_t sst, int64_t plane, int batch, hipStream_t s) {
  const dim3 grid((uint32_t)((threads + PT - 1) / PT), (uint32_t)batch);
  if (!low) {
    hipLaunchKernelGGL((k_potts_pass<T, NR, COUNT, false>), grid, dim3(PT), 0, s, pass, J, jst, dtype, x, n, sst,
                       plane);
    return hipGetLastError();
  }
  constexpr size_t lds = (size_t)PT * low_chunk<T>() * (COUNT ? sizeof(uint64_t) : sizeof(float));
  static bool raised = false;   // one flag per instantiation
  if (!raised) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_potts_pass<T, NR, COUNT, true>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    raised = true;
  }
  hipLaunchKernelGGL((k_potts_pass<T, NR, COUNT, true>), grid, dim3(PT), lds, s, pass, J, jst, dtype, x, n, sst, plane);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_potts_pass(const PottsPass* pass, int t, bool low, int64_t threads, const void* J, int64_t jst, int dtype,
                             float* x, uint64_t* n, int nres, int64_t sst, int batch, hipStream_t s) {
  if (batch < 1 || batch > 65535 || threads < 1 || (threads + PT - 1) / PT >= (1ll << 31))
    return hipErrorInvalidConfiguration;
  const int64_t plane = (int64_t)batch * sst;
  if (!n) {
    switch (t) {
      case 1: return launch_t<1, 1, false>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      case 2: return launch_t<2, 1, false>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      case 3: return launch_t<3, 1, false>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      case 4: return launch_t<4, 1, false>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      default: return hipErrorInvalidConfiguration;
    }
  }
  if (nres == 3) {
    switch (t) {
      case 1: return launch_t<1, 3, true>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      case 2: return launch_t<2, 3, true>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      case 3: return launch_t<3, 3, true>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      default: return hipErrorInvalidConfiguration;
    }
  }
  if (nres == 4) {
    switch (t) {
      case 1: return launch_t<1, 4, true>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      case 2: return launch_t<2, 4, true>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      case 3: return launch_t<3, 4, true>(pass, low, threads, J, jst, dtype, x, n, sst, plane, batch, s);
      default: return hipErrorInvalidConfiguration;
    }
  }
  return hipErrorInvalidConfiguration;
}

int64_t potts_reduce_chunk(int64_t combos) {
  // at most 1024 chunks per instance, at least 2^14 combinations each
  int64_t c = (combos + 1023) / 1024;
  return c < (1 << 14) ? (1 << 14) : c;
}

hipError_t launch_potts_reduce(const PottsReduce* red, int64_t combos, const float* x, const uint64_t* n, int nres,
                               int64_t sst, int batch, float* pv, uint64_t* pn, double* energy, int64_t* energy2,
                               uint64_t* res, hipStream_t s) {
  if (batch < 1 || batch > 65535 || combos < 1) return hipErrorInvalidConfiguration;
  const int64_t chunk = potts_reduce_chunk(combos);
  const int64_t chunks = (combos + chunk - 1) / chunk;
  const int64_t plane = (int64_t)batch * sst;
  const dim3 grid((uint32_t)chunks, (uint32_t)batch);
  if (n)
    hipLaunchKernelGGL(k_potts_reduce1<true>, grid, dim3(PT), 0, s, red, x, n, sst, plane, nres, chunk, pv, pn);
  else
    hipLaunchKernelGGL(k_potts_reduce1<false>, grid, dim3(PT), 0, s, red, x, n, sst, plane, nres, chunk, pv, pn);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_potts_reduce2, dim3((uint32_t)((batch + 63) / 64)), dim3(64), 0, s, pv, pn, chunks, batch,
                     n ? nres : 0, energy, energy2, res);
  return hipGetLastError();
}

}  // namespace tt
