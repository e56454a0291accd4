// HIP kernels (gfx950) of the configuration paths that re-run the forward
// contraction instead of walking it back (Sec. IV): the batch of field-
// perturbed copies of one instance for finite differences, the ground state
// read off their energies, and Eq. (1) of a configuration on the device.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_mem.hpp"
#include "launch.hpp"

namespace tt {

namespace {

constexpr int CT = 256;

// Copy k (k = 0 .. n) of the instance: the couplings, and the fields with
// h_{k-1} raised by delta (copy 0 unperturbed); h may be null (zero fields).
__global__ __launch_bounds__(CT) void k_fd_build(const float* __restrict__ J, const float* __restrict__ h, int64_t m,
                                                 int n, float delta, float* __restrict__ Jb, float* __restrict__ hb) {
  const int k = (int)blockIdx.y;
  const gptr<float> Jo = as_global(Jb) + (int64_t)k * m;
  const gptr<float> ho = as_global(hb) + (int64_t)k * n;
  for (int64_t e = (int64_t)blockIdx.x * CT + threadIdx.x; e < m; e += (int64_t)gridDim.x * CT) Jo[e] = J[e];
  for (int64_t i = (int64_t)blockIdx.x * CT + threadIdx.x; i < n; i += (int64_t)gridDim.x * CT)
    ho[i] = (h ? h[i] : 0.f) + (i == k - 1 ? delta : 0.f);
}

// E(h + delta e_i) = E* - delta sigma_i while the ground state stays the
// same: sigma_i = +1 when the perturbed energy is below E*. Then Eq. (1) of
// the result (one workgroup, float64 sums) for the consistency check.
__global__ __launch_bounds__(CT) void k_fd_sigma(const double* __restrict__ E, const float* __restrict__ J,
                                                 const float* __restrict__ h, const int32_t* __restrict__ edges,
                                                 int64_t m, int n, int8_t* __restrict__ sigma,
                                                 double* __restrict__ energy, double* __restrict__ e_sigma) {
  const double e0 = E[0];
  __shared__ int8_t s[8192];
  for (int i = threadIdx.x; i < n; i += CT) {
    const int8_t v = E[i + 1] < e0 ? 1 : -1;
    s[i] = v;
    sigma[i] = v;
  }
  __syncthreads();
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < m; e += CT) acc -= (double)J[e] * s[edges[2 * e]] * s[edges[2 * e + 1]];
  if (h)
    for (int i = threadIdx.x; i < n; i += CT) acc -= (double)h[i] * s[i];
  __shared__ double part[CT];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = CT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *energy = e0;
    *e_sigma = part[0];
  }
}

}  // namespace

hipError_t launch_fd_build(const float* J, const float* h, int64_t m, int n, float delta, float* Jb, float* hb,
                           hipStream_t s) {
  if (n < 1 || n > 8192 || n + 1 > 65535) return hipErrorInvalidConfiguration;
  const int64_t big = m > n ? m : n;
  const uint32_t gx = (uint32_t)((big + CT - 1) / CT < 64 ? (big + CT - 1) / CT : 64);
  hipLaunchKernelGGL(k_fd_build, dim3(gx > 0 ? gx : 1, (uint32_t)(n + 1)), dim3(CT), 0, s, J, h, m, n, delta, Jb, hb);
  return hipGetLastError();
}

hipError_t launch_fd_sigma(const double* E, const float* J, const float* h, const int32_t* edges, int64_t m, int n,
                           int8_t* sigma, double* energy, double* e_sigma, hipStream_t s) {
  if (n < 1 || n > 8192) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_fd_sigma, dim3(1), dim3(CT), 0, s, E, J, h, edges, m, n, sigma, energy, e_sigma);
  return hipGetLastError();
}

}  // namespace tt
