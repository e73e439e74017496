// Wave-level helpers shared by the chain kernels (64-lane CDNA waves).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tnvan {

// Orders the wave's LDS writes before later reads by other lanes of the same
// wave: LDS instructions of one wave execute in issue order, so it is enough
// that the compiler keeps memory operations on their side of this point.
__device__ inline void wsync() { __builtin_amdgcn_wave_barrier(); }

// Data-parallel-primitive moves inside rows of 16 lanes (no LDS traffic).
template <int CTRL>
__device__ inline float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL,
                                                            0xF, 0xF, false));
}
// sum / max over the 16 lanes of a row, result in every lane of the row:
// swap neighbours, swap pairs, mirror the half rows, mirror the row
__device__ inline float row16_sum(float v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  return v;
}
__device__ inline float row16_max(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x141>(v));
  v = fmaxf(v, dpp<0x140>(v));
  return v;
}

// Exponent e with m * 2^-e in [0.5, 1) for a finite positive m (clamped so
// that 2^-e stays a normal number); the scale factor 2^-e itself.
__device__ inline int expo32(float m) {
  const int E = (int)((__float_as_uint(m) >> 23) & 0xffu);
  const int e = E - 126;
  return e > 126 ? 126 : e;
}
__device__ inline float pow2neg(int e) { return __uint_as_float((uint32_t)(127 - e) << 23); }

}  // namespace tnvan
