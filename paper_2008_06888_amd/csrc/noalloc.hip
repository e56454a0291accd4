// Fixed device workspace of the allocation-free entry point
// (tt_contract_noalloc): one file-scope device array per GPU, sized once at
// build time, whose device address is looked up once per device.
//
// In host code the array's name is only a host-side stand-in for the symbol;
// kernels and copies always receive the address obtained here.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <map>
#include <mutex>

#include "launch.hpp"

namespace tt {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of its copy of `scratch`
}  // namespace

// Address of the current device's copy of the workspace (looked up on the
// first call per device, with that device current).
hipError_t noalloc_scratch(void** ptr) {
  int device = 0;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    it = g_scratch_ptr.emplace(device, p).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

}  // namespace tt
