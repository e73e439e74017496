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

// max / sum over the four rows of a column (lanes l, l ^ 16, l ^ 32, l ^ 48),
// result in every lane, with the row swaps of CDNA4 (register moves, no LDS):
// swapping rows 2,3 of one copy with rows 0,1 of another pairs rows (0,2) and
// (1,3); swapping odd rows of one copy with even rows of another then pairs
// (0,1) and (2,3).  Both orders of a sum agree, so every lane gets the same bits.
__device__ inline float rows4_max(float v) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = fmaxf(__uint_as_float(p[0]), __uint_as_float(p[1]));
  const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(q[0]), __uint_as_float(q[1]));
}
__device__ inline float rows4_sum(float v) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
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
