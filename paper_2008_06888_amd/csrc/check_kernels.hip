// HIP kernel (gfx950) that checks the inputs of a contraction call before
// its passes run: every coupling and field must be finite (Eq. 1 is a finite
// energy), and with integer couplings every state value must stay exact in
// the float32 state, which holds for S = sum |J_ij| + sum |h_i| < 2^24 since
// every entry of the tropical state is a signed sum of a subset of the
// couplings and fields.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "device_mem.hpp"
#include "launch.hpp"

namespace tt {

constexpr int CHK_T = 256;

// The exponent field of a float32 is all ones exactly for inf and NaN. Tested
// on the bits, since the library is built with -fno-honor-nans.
__device__ __forceinline__ uint32_t nonfinite_f32(uint32_t bits) {
  return (bits & 0x7f800000u) == 0x7f800000u ? 1u : 0u;
}

// One workgroup per instance: the item holding instance blockIdx.x is found
// by its first status index (items are in instance order).
__global__ __launch_bounds__(CHK_T) void k_check_inputs(CheckArgs a, uint32_t* __restrict__ status) {
  int it = 0;
  while (it + 1 < a.n && (int64_t)blockIdx.x >= a.it[it + 1].first) ++it;
  const CheckItem& I = a.it[it];
  const int64_t b = (int64_t)blockIdx.x - I.first;
  if (b >= I.batch) return;
  uint32_t bad = 0;
  uint64_t S = 0;
  const bool f32 = I.dtype == 0;
  for (int part = 0; part < 2; ++part) {
    const void* base = part == 0 ? I.J : I.h;
    const int64_t len = part == 0 ? I.m : I.n;
    const int64_t st = part == 0 ? I.jst : I.hst;
    if (!base) continue;
    if (I.dtype == 2) {   // int16
      const cptr<int16_t> row = as_const(static_cast<const int16_t*>(base)) + b * st;
      for (int64_t k = threadIdx.x; k < len; k += CHK_T) {
        const int64_t v = row[k];
        S += (uint64_t)(v < 0 ? -v : v);
      }
      continue;
    }
    const cptr<uint32_t> row = as_const(static_cast<const uint32_t*>(base)) + b * st;
    for (int64_t k = threadIdx.x; k < len; k += CHK_T) {
      const uint32_t w = row[k];
      if (f32) {
        bad |= nonfinite_f32(w);
      } else {
        const int64_t v = (int64_t)(int32_t)w;
        S += (uint64_t)(v < 0 ? -v : v);
      }
    }
  }
  // wave reductions (OR of the flags, sum of |values|), then across waves
  for (int off = 32; off > 0; off >>= 1) {
    bad |= (uint32_t)__shfl_xor((int)bad, off, 64);
    S += (uint64_t)__shfl_xor((long long)S, off, 64);
  }
  __shared__ uint32_t sb[CHK_T / 64];
  __shared__ uint64_t ss[CHK_T / 64];
  if ((threadIdx.x & 63) == 0) {
    sb[threadIdx.x >> 6] = bad;
    ss[threadIdx.x >> 6] = S;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < CHK_T / 64; ++w) {
      bad |= sb[w];
      S += ss[w];
    }
    uint32_t st = bad ? CHK_NONFINITE : 0u;
    if (!f32 && S >= (uint64_t)I.limit) st |= CHK_RANGE;
    status[I.first + b] = st;
  }
}

hipError_t launch_check(const CheckArgs& a, int64_t n_inst, uint32_t* status, hipStream_t stream) {
  if (a.n < 1 || a.n > CHECK_ITEMS || n_inst < 1 || n_inst >= (1ll << 31)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_check_inputs, dim3((uint32_t)n_inst), dim3(CHK_T), 0, stream, a, status);
  return hipGetLastError();
}

}  // namespace tt
