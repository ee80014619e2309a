// Small device/host helpers shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

namespace r3mg {
namespace hiputil {

constexpr int kXcd = 8;  // MI355X: 8 accelerator complex dies, workgroups dispatched round-robin

// Logical block index with XCD-contiguous chunks: consecutive logical blocks (adjacent rows, spatially close
// in the R-tree order) run on the same XCD and share its L2.  The grid must be kXcd * ceil(nlog / kXcd).
__device__ inline int xcd_block(int nlog) {
  int per = (nlog + kXcd - 1) / kXcd;
  int lb = (int)(blockIdx.x % kXcd) * per + (int)(blockIdx.x / kXcd);
  return lb < nlog ? lb : -1;
}
inline int xcd_grid(int nlog) { return kXcd * ((nlog + kXcd - 1) / kXcd); }

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace hiputil
}  // namespace r3mg
