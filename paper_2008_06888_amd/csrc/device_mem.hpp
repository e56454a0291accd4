// Address spaces for device code (HIP kernels only).
#pragma once
#include <cstdint>

#include "device.hpp"

namespace tt {

// Launch tables, encoded programs and inputs are read-only while a kernel
// runs: read through the constant address space, so uniform fields come in
// by scalar loads (through the scalar cache) and the rest by global loads.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

// A whole record read from the constant address space, word by word.
template <typename T>
__device__ __forceinline__ T ldc(cptr<T> p) {
  static_assert(sizeof(T) % 4 == 0, "records are read as 32-bit words");
  T r;
  uint32_t* d = reinterpret_cast<uint32_t*>(&r);
  const cptr<uint32_t> w = (cptr<uint32_t>)(p);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) d[k] = w[k];
  return r;
}

// Device memory written by a kernel: the global address space (no flat
// accesses, whose completion also holds back LDS waits).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)(p);
}

// LDS records reached through pointers: the local address space (ds_*
// accesses instead of flat ones).
using LFloat = __attribute__((address_space(3))) float;
using LByte = __attribute__((address_space(3))) char;

using LShort = __attribute__((address_space(3))) short;

// The int16 at an LDS byte address (same condition as lds_at).
__device__ __forceinline__ LShort& lds16_at(uint32_t addr) {
  return *(LShort*)(uintptr_t)(addr);
}

// Half-state plans (h = 0): the tile index of a run tile k (tile-id bit
// `skip` at 0), and the stored (canonical) address of an entry: the
// complement of every address bit when the top one is set.
__device__ __forceinline__ uint64_t z2_tile(uint64_t k, int skip) {
  return skip < 0 ? k : (((k >> skip) << (skip + 1)) | (k & ((1ull << skip) - 1ull)));
}
__device__ __forceinline__ uint64_t z2_addr(uint64_t a, int w) {
  return (w > 0 && ((a >> (w - 1)) & 1ull)) ? a ^ ((1ull << w) - 1ull) : a;
}

// The float at an LDS byte address. Only for kernels without static LDS,
// whose dynamic region starts at address 0 (their launchers check it).
__device__ __forceinline__ LFloat& lds_at(uint32_t addr) {
  return *(LFloat*)(uintptr_t)(addr);
}

}  // namespace tt
