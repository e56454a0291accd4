// HIP kernels (gfx950) of sliced contractions. Splitting the sum of Eq. (1)
// by the values of s fixed spins turns every bond between a fixed spin and a
// free one into a field on the free spin, and the bonds and fields among the
// fixed spins into a constant: each of the 2^s assignments (slices) is an
// instance of the reduced graph with fields, and E* is the minimum over the
// slices of their ground-state energies plus the constants. The slices are
// contracted as batches of the reduced plan; these kernels build those
// batches and combine their results.
//
// Reduced instance r is slice k = r & (2^s - 1) of instance b = r >> s; bit j
// of k is fixed spin j (1 <-> sigma = -1, as every index here).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_mem.hpp"
#include "launch.hpp"

namespace tt {

namespace {

constexpr int SLT = 256;

// One workgroup row per reduced instance (blockIdx.y), workgroups along x
// stride over its edges and spins.
template <typename T>
__global__ __launch_bounds__(SLT) void k_slice_build(SliceArgs A, int64_t r0, const int32_t* __restrict__ kpick,
                                                     const T* __restrict__ J, const T* __restrict__ h,
                                                     T* __restrict__ Jr, T* __restrict__ hr, double* __restrict__ c) {
  const int64_t loc = blockIdx.y;
  int64_t b;
  uint32_t k;
  if (kpick) {
    b = r0 + loc;
    k = (uint32_t)kpick[b];
  } else {
    const int64_t r = r0 + loc;
    b = r >> A.s;
    k = (uint32_t)(r & ((1ll << A.s) - 1));
  }
  const cptr<T> Jb = as_const(J) + b * A.m;
  const cptr<T> hb = h ? as_const(h) + b * A.n : cptr<T>(nullptr);
  const gptr<T> Jo = as_global(Jr) + loc * A.mr;
  const gptr<T> ho = as_global(hr) + loc * A.nr;
  const cptr<int32_t> emap = as_const(A.emap), keep = as_const(A.keep);
  const cptr<int32_t> xptr = as_const(A.cross_ptr), xbit = as_const(A.cross_bit), xedge = as_const(A.cross_edge);
  const int64_t step = (int64_t)gridDim.x * SLT;
  for (int64_t e = (int64_t)blockIdx.x * SLT + threadIdx.x; e < A.mr; e += step) Jo[e] = Jb[emap[e]];
  for (int64_t v = (int64_t)blockIdx.x * SLT + threadIdx.x; v < A.nr; v += step) {
    // J sigma_i sigma_j with sigma_j fixed is a field J sigma_j on spin i
    T f = hb ? hb[keep[v]] : T(0);
    for (int32_t q = xptr[v]; q < xptr[v + 1]; ++q) {
      const T jv = Jb[xedge[q]];
      f += ((k >> xbit[q]) & 1u) ? -jv : jv;
    }
    ho[v] = f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the slice's constant: Eq. (1) restricted to the fixed spins
    double e = 0.0;
    const cptr<int32_t> ia = as_const(A.inner_a), ib = as_const(A.inner_b), ie = as_const(A.inner_edge);
    for (int32_t q = 0; q < A.n_inner; ++q) {
      const bool sa = (k >> ia[q]) & 1u, sb = (k >> ib[q]) & 1u;
      e -= (sa == sb) ? (double)Jb[ie[q]] : -(double)Jb[ie[q]];
    }
    if (hb) {
      const cptr<int32_t> sp = as_const(A.spins);
      for (int j = 0; j < A.s; ++j) e -= ((k >> j) & 1u) ? -(double)hb[sp[j]] : (double)hb[sp[j]];
    }
    c[loc] = e;
  }
}

__global__ void k_slice_min(const double* __restrict__ Er, const double* __restrict__ c, int s, int batch,
                            double* __restrict__ energy, int32_t* __restrict__ kbest) {
  const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= batch) return;
  const int64_t ns = 1ll << s;
  double best = Er[(int64_t)b * ns] + c[(int64_t)b * ns];
  int32_t kb = 0;
  for (int64_t k = 1; k < ns; ++k) {
    const double v = Er[(int64_t)b * ns + k] + c[(int64_t)b * ns + k];
    if (v < best) {
      best = v;
      kb = (int32_t)k;
    }
  }
  if (energy) energy[b] = best;
  if (kbest) kbest[b] = kb;
}

// One workgroup per instance; the assembled configuration is held in LDS
// (n <= 8192) for the gradients.
__global__ __launch_bounds__(SLT) void k_slice_pick(SliceArgs A, const int8_t* __restrict__ sr,
                                                    const int32_t* __restrict__ kbest,
                                                    const int32_t* __restrict__ edges, int8_t* __restrict__ sigma,
                                                    float* __restrict__ dJ, float* __restrict__ dh) {
  __shared__ int8_t sl[8192];
  const int64_t b = blockIdx.x;
  const uint32_t k = (uint32_t)kbest[b];
  const cptr<int8_t> src = as_const(sr) + b * A.nr;
  const cptr<int32_t> keep = as_const(A.keep), sp = as_const(A.spins);
  for (int v = threadIdx.x; v < A.nr; v += SLT) sl[keep[v]] = src[v];
  for (int j = threadIdx.x; j < A.s; j += SLT) sl[sp[j]] = ((k >> j) & 1u) ? -1 : 1;
  __syncthreads();
  const gptr<int8_t> sg = as_global(sigma) + b * A.n;
  for (int v = threadIdx.x; v < A.n; v += SLT) sg[v] = sl[v];
  if (dh) {
    const gptr<float> o = as_global(dh) + b * A.n;
    for (int v = threadIdx.x; v < A.n; v += SLT) o[v] = sl[v] < 0 ? 1.f : -1.f;
  }
  if (dJ) {
    const cptr<int32_t> ed = as_const(edges);
    const gptr<float> o = as_global(dJ) + b * A.m;
    for (int64_t e = threadIdx.x; e < A.m; e += SLT) o[e] = (sl[ed[2 * e]] == sl[ed[2 * e + 1]]) ? -1.f : 1.f;
  }
}

}  // namespace

hipError_t launch_slice_build(const SliceArgs& A, int64_t r0, int n_red, const int32_t* kpick, int dtype,
                              const void* J, const void* h, void* Jr, void* hr, double* c, hipStream_t s) {
  if (n_red < 1 || n_red > 65535 || A.s < 1 || A.s > 16) return hipErrorInvalidConfiguration;
  const int64_t big = A.mr > A.nr ? A.mr : A.nr;
  int64_t gx = (big + SLT - 1) / SLT;
  gx = gx < 1 ? 1 : (gx > 64 ? 64 : gx);
  const dim3 grid((uint32_t)gx, (uint32_t)n_red);
  if (dtype == 2)
    hipLaunchKernelGGL(k_slice_build<int16_t>, grid, dim3(SLT), 0, s, A, r0, kpick, static_cast<const int16_t*>(J),
                       static_cast<const int16_t*>(h), static_cast<int16_t*>(Jr), static_cast<int16_t*>(hr), c);
  else if (dtype == 0)
    hipLaunchKernelGGL(k_slice_build<float>, grid, dim3(SLT), 0, s, A, r0, kpick, static_cast<const float*>(J),
                       static_cast<const float*>(h), static_cast<float*>(Jr), static_cast<float*>(hr), c);
  else
    hipLaunchKernelGGL(k_slice_build<int32_t>, grid, dim3(SLT), 0, s, A, r0, kpick, static_cast<const int32_t*>(J),
                       static_cast<const int32_t*>(h), static_cast<int32_t*>(Jr), static_cast<int32_t*>(hr), c);
  return hipGetLastError();
}

hipError_t launch_slice_min(const double* Er, const double* c, int s, int batch, double* energy, int32_t* kbest,
                            hipStream_t st) {
  if (batch < 1 || s < 1 || s > 16) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_slice_min, dim3((uint32_t)((batch + 63) / 64)), dim3(64), 0, st, Er, c, s, batch, energy,
                     kbest);
  return hipGetLastError();
}

hipError_t launch_slice_pick(const SliceArgs& A, int batch, const int8_t* sr, const int32_t* kbest,
                             const int32_t* edges, int8_t* sigma, float* dJ, float* dh, hipStream_t s) {
  if (batch < 1 || A.n > 8192) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_slice_pick, dim3((uint32_t)batch), dim3(SLT), 0, s, A, sr, kbest, edges, sigma, dJ, dh);
  return hipGetLastError();
}

}  // namespace tt
