// Loads of tables a kernel only reads, at workgroup-uniform addresses.
#pragma once

#include <hip/hip_runtime.h>

namespace tnvan {

// Through the constant address space the load becomes a scalar load (one per
// wave, into scalar registers), and what is derived from it stays scalar
// (loop bounds, offsets, branches).  Only for tables that are written
// between launches, never by the kernel that reads them.
template <typename T>
__device__ inline T uload(const T *p) {
  T v;
  __builtin_memcpy(&v, (const __attribute__((address_space(4))) T *)p, sizeof(T));
  return v;
}

}  // namespace tnvan
