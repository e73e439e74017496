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

// Width-set spins of one sample as a bit mask (bit w set: s_w = -1), up to
// 128 spins; the chain kernels read a spin with a uniform index w.
struct SpinBits {
  uint32_t m[4];
  __device__ float sigma(int w) const {
    const uint32_t word = w < 32 ? m[0] : w < 64 ? m[1] : w < 96 ? m[2] : m[3];
    return ((word >> (w & 31)) & 1u) ? -1.f : 1.f;
  }
};

// spins s[0..nw) (+-1 bytes); a sample past the batch reads as all +1
__device__ inline SpinBits load_bits(const int8_t *s, int nw, bool valid) {
  SpinBits b;
  b.m[0] = b.m[1] = b.m[2] = b.m[3] = 0u;
  if (!valid) return b;
  for (int w0 = 0; w0 < nw; w0 += 4) {
    uint32_t v = 0u;
    if ((nw & 3) == 0 && (reinterpret_cast<uintptr_t>(s) & 3) == 0) {
      v = *reinterpret_cast<const uint32_t *>(s + w0);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (w0 + k < nw) v |= (uint32_t)(uint8_t)s[w0 + k] << (8 * k);
    }
    // sign bit of each byte
    const uint32_t nib = ((v >> 7) & 1u) | ((v >> 14) & 2u) | ((v >> 21) & 4u) | ((v >> 28) & 8u);
    const uint32_t sh = nib << (w0 & 31);
    const int wd = w0 >> 5;
    b.m[0] |= wd == 0 ? sh : 0u;
    b.m[1] |= wd == 1 ? sh : 0u;
    b.m[2] |= wd == 2 ? sh : 0u;
    b.m[3] |= wd == 3 ? sh : 0u;
  }
  return b;
}

// The same mask from 16-byte loads, all issued before any is used (a
// per-lane caller would otherwise wait for each load in turn): rows of nw
// bytes, nw a multiple of 16 and at most 16 NL, 16-byte aligned.  Loads past
// the row reread its start (in bounds) and are ignored.
template <int NL>
__device__ inline SpinBits load_bits16(const int8_t *s, int nw) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  u4 v[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) v[k] = *reinterpret_cast<const u4 *>(s + (16 * k < nw ? 16 * k : 0));
  SpinBits b;
  b.m[0] = b.m[1] = b.m[2] = b.m[3] = 0u;
#pragma unroll
  for (int k = 0; k < NL; ++k)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const uint32_t x = v[k][d];
      const uint32_t nib = ((x >> 7) & 1u) | ((x >> 14) & 2u) | ((x >> 21) & 4u) | ((x >> 28) & 8u);
      const int w0 = 16 * k + 4 * d;
      if (16 * k < nw) b.m[w0 >> 5] |= nib << (w0 & 31);
    }
  return b;
}

// a sample's spins (nw <= 128) by the fastest form its row allows
__device__ inline SpinBits load_bits_row(const int8_t *s, int nw) {
  if ((nw & 15) == 0 && (reinterpret_cast<uintptr_t>(s) & 15) == 0) {
    if (nw <= 32) return load_bits16<2>(s, nw);
    if (nw <= 64) return load_bits16<4>(s, nw);
    return load_bits16<8>(s, nw);
  }
  return load_bits(s, nw, true);
}

}  // namespace tnvan
