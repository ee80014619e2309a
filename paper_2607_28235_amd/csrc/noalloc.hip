// Static device scratch of the allocation-free V-cycle (r3mg_vcycle_noalloc).
//
// The array lives in the library's code object: every GPU that loads the library holds its own copy, at its own
// address, until the process ends.  Host code never passes the array's name to a kernel (in host code it is a
// host-side stand-in, not a device address): scratch_device_ptr() looks the device address up once per device
// with hipGetSymbolAddress, with that device current, and every kernel argument and fill uses that address.
// All calls on one GPU share the array, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "noalloc.h"
#include "r3mg_internal.h"

namespace r3mg {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// zero `words` 16-byte words (grid-stride)
__global__ __launch_bounds__(256) void k_zero16(uint4* p, int64_t words) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256) p[i] = z;
}

}  // namespace

void* scratch_device_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error{R3MG_ERR_INVALID, "device index out of range for the scratch"};
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess || cur != dev)
      throw Error{R3MG_ERR_INVALID, "the scratch of device " + std::to_string(dev) + " is looked up with it current"};
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      throw Error{R3MG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

void scratch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t words = (int64_t)((bytes + 15) / 16);
  if (words == 0) return;
  int64_t g = (words + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_zero16, dim3((unsigned)g), dim3(256), 0, s, static_cast<uint4*>(p), words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{R3MG_ERR_HIP, std::string("k_zero16: ") + hipGetErrorString(e)};
}

}  // namespace r3mg
