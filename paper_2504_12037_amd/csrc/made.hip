// Masked autoregressive network q (Sec. 3, Eqs. 6-8), the free-energy
// estimator and REINFORCE weights (Eqs. 9-10) and the Adam update.
//
// Network: positions i = 1..n of the width set, hidden units k with degree
// m(k) = 1 + (k mod (n-1));  a_k = b1_k + sum_{j<=m(k)} W1[k,j] s_j,
// logit_i = b2_i + sum_{m(k)<i} W2[i,k] tanh(a_k) + sum_{j<i} W0[i,j] s_j,
// q(s_i=+1 | s_<i) = sigmoid(logit_i).  The masks are applied by index tests,
// never stored.  Parameters are float32 in the flat layout
// W1 [H,n], b1 [H], W2 [n,H], b2 [n], W0 [n,n].
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>

#include "launch.h"
#include "uload.h"
#include "wave.h"

namespace tnvan {

namespace {

__device__ inline int degree(int k, int n) { return 1 + (k % (n - 1)); }

// parameters of an instance: W1, b1, W2, b2, W0, then D - 1 deeper layers
__device__ inline int64_t made_pc(const MadeInst &m) {
  return (int64_t)m.H * m.n + m.H + (int64_t)m.n * m.H + m.n + (int64_t)m.n * m.n +
         (int64_t)(m.D - 1) * ((int64_t)m.H * m.H + m.H);
}

template <typename real> __device__ inline real rexp(real x);
template <> __device__ inline float rexp<float>(float x) { return expf(x); }
template <> __device__ inline double rexp<double>(double x) { return exp(x); }
template <typename real> __device__ inline real rlog1p(real x);
template <> __device__ inline float rlog1p<float>(float x) { return log1pf(x); }
template <> __device__ inline double rlog1p<double>(double x) { return log1p(x); }
template <typename real> __device__ inline real rlog(real x);
template <> __device__ inline float rlog<float>(float x) { return logf(x); }
template <> __device__ inline double rlog<double>(double x) { return log(x); }
template <typename real> __device__ inline real rtanh(real x);
template <> __device__ inline float rtanh<float>(float x) { return tanhf(x); }
template <> __device__ inline double rtanh<double>(double x) { return tanh(x); }

// log sigmoid(z), stable for both signs
template <typename real> __device__ inline real log_sigmoid(real z) {
  return z >= 0 ? -rlog1p<real>(rexp<real>(-z)) : z - rlog1p<real>(rexp<real>(z));
}
template <typename real> __device__ inline real sigmoid(real z) {
  return z >= 0 ? (real)1 / ((real)1 + rexp<real>(-z))
                : rexp<real>(z) / ((real)1 + rexp<real>(z));
}

// Short FP32 forms for the matrix-core kernels (hardware exp2/log2 and a
// fast reciprocal; a few ulp, far inside the sampling tie band and the
// gradient tolerance): tanh from exp(-2|x|), sigmoid, and log sigmoid.
__device__ inline float ftanh(float x) {
  const float t = __expf(-2.f * fabsf(x));
  return copysignf((1.f - t) * __builtin_amdgcn_rcpf(1.f + t), x);
}
__device__ inline float fsigmoid(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }
// 1 + e^-|x| lies in (1, 2]: the hardware log2 needs no range handling
__device__ inline float flogsigmoid(float x) {
  return fminf(x, 0.f) - 0.69314718055994531f * __builtin_amdgcn_logf(1.f + __expf(-fabsf(x)));
}

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64-bit
// multiplies with word swaps and key xors; Weyl key schedule.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

constexpr int kFreeStage = 2048;   // W-W couplings staged in LDS by the free-energy kernel
constexpr int kFreeLanes = 4;      // lanes per sample in the free-energy kernel
constexpr int KH = 16;    // hidden units per lane
constexpr int KN = 32;    // width-set positions per lane

// Parameter views with row strides.  With kLDS a block first copies the
// parameters of its instance into LDS: for the sampler W1 is stored
// transposed ([n][H], lanes owning consecutive hidden units read consecutive
// words); for the row kernel every matrix keeps its orientation with its rows
// padded by one word so that lanes walking down a column hit distinct banks.
struct MadeView {
  const float *W1;   // [H][ld1] (or transposed [n][ld1])
  const float *b1, *W2, *b2, *W0;
  int ld1, ld2, ld0;
};

// LDS bytes of the staged parameters (padded layout, the larger of the two)
__host__ __device__ inline size_t made_stage_bytes(int n, int H) {
  return (size_t)(H * (n + 1) + n * (H + 1) + n * (n + 1) + H + n) * 4;
}

__device__ inline MadeView made_view(const float *p, int n, int H) {
  MadeView v;
  v.W1 = p;
  v.b1 = p + (int64_t)H * n;
  v.W2 = v.b1 + H;
  v.b2 = v.W2 + (int64_t)n * H;
  v.W0 = v.b2 + n;
  v.ld1 = n; v.ld2 = H; v.ld0 = n;
  return v;
}

__device__ inline MadeView made_stage(const MadeView g, int n, int H, float *s, bool transpose_w1) {
  MadeView v;
  v.ld1 = transpose_w1 ? H : n + 1;
  v.ld2 = transpose_w1 ? H : H + 1;
  v.ld0 = transpose_w1 ? n : n + 1;
  const int rows1 = transpose_w1 ? n : H;
  float *W1 = s, *W2 = W1 + (size_t)rows1 * v.ld1, *W0 = W2 + (size_t)n * v.ld2,
        *b1 = W0 + (size_t)n * v.ld0, *b2 = b1 + H;
  for (int i = threadIdx.x; i < n * H; i += blockDim.x) {
    if (transpose_w1) {
      const int j = i / H, k = i - j * H;     // W1t[j][k] = W1[k][j]
      W1[(size_t)j * v.ld1 + k] = g.W1[(int64_t)k * n + j];
    } else {
      const int k = i / n, j = i - k * n;
      W1[(size_t)k * v.ld1 + j] = g.W1[i];
    }
    const int ii = i / H, k = i - ii * H;
    W2[(size_t)ii * v.ld2 + k] = g.W2[i];
  }
  for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
    const int ii = i / n, j = i - ii * n;
    W0[(size_t)ii * v.ld0 + j] = g.W0[i];
  }
  for (int i = threadIdx.x; i < H; i += blockDim.x) b1[i] = g.b1[i];
  for (int i = threadIdx.x; i < n; i += blockDim.x) b2[i] = g.b2[i];
  __syncthreads();
  v.W1 = W1; v.b1 = b1; v.W2 = W2; v.b2 = b2; v.W0 = W0;
  return v;
}

// One group of L lanes per sample; lane l owns hidden units k = l + L*kk and
// positions j = l + L*jj.  Spins are drawn one position after the other.
// A block runs `reps` rounds of 256/L samples of one instance.
template <typename real, bool kLDS>
__global__ __launch_bounds__(256) void sample_kernel(SampleArgs<real> a) {
  extern __shared__ __align__(16) char smem[];
  const int q = uload(a.blk_inst + blockIdx.x);
  const MadeInst mi = uload(a.mi + q);
  const int L = mi.L;
  const int grp = threadIdx.x / L, l = threadIdx.x % L;
  const int n = mi.n, Hs = mi.H, H = (n >= 2) ? mi.H : 0;
  MadeView w = made_view(a.params + mi.param_off, n, Hs);
  if (kLDS) w = made_stage(w, n, Hs, reinterpret_cast<float *>(smem), true);
  const uint32_t step = a.step_ctr ? (uint32_t)a.step_ctr[q] : 0u;
  int dg[KH];
#pragma unroll
  for (int kk = 0; kk < KH; ++kk) {
    const int k = l + L * kk;
    dg[kk] = k < H ? degree(k, n) : 0;
  }
  for (int rep = 0; rep < a.reps; ++rep) {
    const int64_t b = uload(a.blk_start + blockIdx.x) + (int64_t)rep * a.spb + grp;
    const bool live = grp < a.spb && b < mi.B;
    real av[KH], hv[KH], sv[KN];
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
      const int k = l + L * kk;
      av[kk] = (k < H) ? (real)w.b1[k] : (real)0;
      hv[kk] = 0;
    }
#pragma unroll
    for (int jj = 0; jj < KN; ++jj) sv[jj] = 0;
    real lq = 0;
    const int64_t bs = live ? b : 0;
    const float *u = a.uniforms ? a.uniforms + mi.spin_off + bs * n : nullptr;
    int8_t *so = a.spins + mi.spin_off + bs * n;
    uint32_t pw[4] = {0, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
      real part = 0;
#pragma unroll
      for (int kk = 0; kk < KH; ++kk) {
        const int k = l + L * kk;
        if (k < H && dg[kk] <= i) part += (real)w.W2[(int64_t)i * w.ld2 + k] * hv[kk];
      }
#pragma unroll
      for (int jj = 0; jj < KN; ++jj) {
        const int j = l + L * jj;
        if (j < i) part += (real)w.W0[(int64_t)i * w.ld0 + j] * sv[jj];
      }
      for (int off = L >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
      const real logit = part + (real)w.b2[i];
      float ui;
      if (u) {
        ui = live ? u[i] : 0.5f;
      } else {
        if ((i & 3) == 0) {
          pw[0] = (uint32_t)(i >> 2); pw[1] = (uint32_t)b; pw[2] = step; pw[3] = (uint32_t)q;
          philox4x32_10(pw, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
        }
        ui = (float)(pw[i & 3] >> 8) * 5.9604644775390625e-08f;
      }
      const real p = sigmoid<real>(logit);
      const real si = ((real)ui < p) ? (real)1 : (real)-1;
      lq += log_sigmoid<real>(si * logit);
      if (l == (i % L)) {
        const int jw = i / L;
#pragma unroll
        for (int jj = 0; jj < KN; ++jj)
          if (jj == jw) sv[jj] = si;
        if (live) so[i] = (int8_t)(si > 0 ? 1 : -1);
      }
#pragma unroll
      for (int kk = 0; kk < KH; ++kk) {
        const int k = l + L * kk;
        if (k < H) {
          const int m = dg[kk];
          if (m >= i + 1) {
            const float wk = kLDS ? w.W1[(int64_t)i * w.ld1 + k] : w.W1[(int64_t)k * n + i];
            av[kk] += (real)wk * si;
            if (m == i + 1) hv[kk] = rtanh<real>(av[kk]);
          }
        }
      }
    }
    if (live && l == 0) a.logq[mi.sample_off + b] = lq;
  }
}

// Deeper networks (D > 1): layer l >= 2 has a^l_k' = b^l_k' + sum over
// units k of layer l - 1 with m(k) <= m(k') of W^l[k', k] h^{l-1}_k; the
// logits read layer D.  Its parameters follow W0: (W^l [H, H], b^l [H]).
__device__ inline const float *deep_layer(const float *p, int n, int H, int l) {
  // W^l of layer l = 2..D (its bias follows it)
  return p + (int64_t)H * n + H + (int64_t)n * H + n + (int64_t)n * n +
         (int64_t)(l - 2) * ((int64_t)H * H + H);
}

// One wave per sample (four per block, one instance per block row).  A unit
// of layer 1 with degree m is complete once position m - 1 is drawn; a unit
// of layer l then gets the newly completed units of layer l - 1 (those of
// degree m: k = m - 1 + t (n - 1)) and is complete when its own degree is
// reached.  Lane l owns units l + 64 kk of every layer (pre-activations in
// registers) and positions l + 64 jj (spins in registers); completed tanh
// values go to the wave's own slice of LDS, read by the wave after a wave
// barrier (the four waves of a block never wait for each other).
constexpr int kDeepKK = kDeepMaxH / 64, kDeepJJ = kDeepMaxN / 64;
template <typename real>
__global__ __launch_bounds__(256) void sample_deep_kernel(SampleArgs<real> a) {
  __shared__ real hs[4][kDeepMaxD][kDeepMaxH];
  const int q = blockIdx.y, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const MadeInst mi = a.mi[q];
  if ((int64_t)blockIdx.x * 4 >= mi.B) return;   // uniform over the block
  const int64_t b = (int64_t)blockIdx.x * 4 + wv;
  const bool live = b < mi.B;
  const int64_t bs = live ? b : 0;
  const int n = mi.n, H = n >= 2 ? mi.H : 0, D = H > 0 ? mi.D : 1;
  const float *P = a.params + mi.param_off;
  const MadeView w = made_view(P, n, mi.H);
  const uint32_t step = a.step_ctr ? (uint32_t)a.step_ctr[q] : 0u;
  real acc[kDeepMaxD][kDeepKK], sv[kDeepJJ];
  int dg[kDeepKK];
#pragma unroll
  for (int kk = 0; kk < kDeepKK; ++kk) {
    const int k = lane + 64 * kk;
    dg[kk] = k < H ? degree(k, n) : 0;
#pragma unroll
    for (int l = 0; l < kDeepMaxD; ++l) {
      const float *bl = l == 0 ? w.b1 : deep_layer(P, n, mi.H, l + 1) + (int64_t)mi.H * mi.H;
      acc[l][kk] = (k < H && l < D) ? (real)bl[k] : (real)0;
    }
  }
#pragma unroll
  for (int jj = 0; jj < kDeepJJ; ++jj) sv[jj] = 0;
  const float *u = a.uniforms ? a.uniforms + mi.spin_off + bs * n : nullptr;
  int8_t *so = a.spins + mi.spin_off + bs * n;
  uint32_t pw[4] = {0, 0, 0, 0};
  real lq = 0;
  for (int i = 0; i < n; ++i) {
    // logit_i from the last layer's completed units and the earlier spins
    real part = 0;
#pragma unroll
    for (int kk = 0; kk < kDeepKK; ++kk) {
      const int k = lane + 64 * kk;
      if (k < H && dg[kk] <= i) part += (real)w.W2[(int64_t)i * mi.H + k] * hs[wv][D - 1][k];
    }
#pragma unroll
    for (int jj = 0; jj < kDeepJJ; ++jj) {
      const int j = lane + 64 * jj;
      if (j < i) part += (real)w.W0[(int64_t)i * n + j] * sv[jj];
    }
    // the wave's sum in registers (row sums, then the four rows) in FP32
    if constexpr (sizeof(real) == 4) {
      part = rows4_sum(row16_sum(part));
    } else {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    }
    const real logit = part + (real)w.b2[i];
    float ui;
    if (u) {
      ui = live ? u[i] : 0.5f;
    } else {
      if ((i & 3) == 0) {
        pw[0] = (uint32_t)(i >> 2); pw[1] = (uint32_t)bs; pw[2] = step; pw[3] = (uint32_t)q;
        philox4x32_10(pw, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
      }
      ui = (float)(pw[i & 3] >> 8) * 5.9604644775390625e-08f;
    }
    const real p = sigmoid<real>(logit);
    const real si = ((real)ui < p) ? (real)1 : (real)-1;
    lq += log_sigmoid<real>(si * logit);
#pragma unroll
    for (int jj = 0; jj < kDeepJJ; ++jj)
      if (lane + 64 * jj == i) sv[jj] = si;
    if (lane == 0 && live) so[i] = (int8_t)(si > 0 ? 1 : -1);
    // layer 1: the new spin, and the units it completes
#pragma unroll
    for (int kk = 0; kk < kDeepKK; ++kk) {
      const int k = lane + 64 * kk;
      if (k < H && dg[kk] >= i + 1) {
        acc[0][kk] += (real)w.W1[(int64_t)k * n + i] * si;
        if (dg[kk] == i + 1) hs[wv][0][k] = rtanh<real>(acc[0][kk]);
      }
    }
    // deeper layers: the units of degree i + 1 just completed below (each
    // wave reads only its own sample's slice of LDS, in order: a wave
    // barrier keeps the writes before the reads)
    for (int l = 1; l < D; ++l) {
      wsync();
      const float *Wl = deep_layer(P, n, mi.H, l + 1);
#pragma unroll
      for (int kk = 0; kk < kDeepKK; ++kk) {
        const int k2 = lane + 64 * kk;
        if (k2 < H && dg[kk] >= i + 1) {
          if (i + 1 <= n - 1)
            for (int k = i; k < H; k += n - 1)
              acc[l][kk] += (real)Wl[(int64_t)k2 * mi.H + k] * hs[wv][l - 1][k];
          if (dg[kk] == i + 1) hs[wv][l][k2] = rtanh<real>(acc[l][kk]);
        }
      }
    }
    wsync();
  }
  if (live && lane == 0) a.logq[mi.sample_off + b] = lq;
}

// The same sampler for small deeper networks (every instance |W| <= 128 and
// H <= 64): 16 lanes per sample, four samples per wave and sixteen per
// block, so that four times as many independent position chains are in
// flight.  Lane c of a sample owns units c + 16 kk and positions c + 16 jj;
// the logit is the 16-lane row sum.  Each sample's completed tanh values go
// to its own slice of LDS, read by its own lanes after a wave barrier.
constexpr int kD16KK = kDeep16MaxH / 16, kD16JJ = kDeep16MaxN / 16;
template <typename real>
__global__ __launch_bounds__(256) void sample_deep16_kernel(SampleArgs<real> a) {
  __shared__ real hs[16][kDeepMaxD][kDeep16MaxH];
  const int q = blockIdx.y, lane = threadIdx.x & 63, c = lane & 15;
  const int slot = threadIdx.x >> 4;   // the block's sample 0..15
  const MadeInst mi = uload(a.mi + q);
  if ((int64_t)blockIdx.x * 16 >= mi.B) return;   // uniform over the block
  const int64_t b = (int64_t)blockIdx.x * 16 + slot;
  const bool live = b < mi.B;
  const int64_t bs = live ? b : 0;
  const int n = mi.n, H = n >= 2 ? mi.H : 0, D = H > 0 ? mi.D : 1;
  const float *P = a.params + mi.param_off;
  const MadeView w = made_view(P, n, mi.H);
  const uint32_t step = a.step_ctr ? (uint32_t)a.step_ctr[q] : 0u;
  real acc[kDeepMaxD][kD16KK], sv[kD16JJ];
  int dg[kD16KK];
#pragma unroll
  for (int kk = 0; kk < kD16KK; ++kk) {
    const int k = c + 16 * kk;
    dg[kk] = k < H ? degree(k, n) : 0;
#pragma unroll
    for (int l = 0; l < kDeepMaxD; ++l) {
      const float *bl = l == 0 ? w.b1 : deep_layer(P, n, mi.H, l + 1) + (int64_t)mi.H * mi.H;
      acc[l][kk] = (k < H && l < D) ? (real)bl[k] : (real)0;
    }
  }
#pragma unroll
  for (int jj = 0; jj < kD16JJ; ++jj) sv[jj] = 0;
  const float *u = a.uniforms ? a.uniforms + mi.spin_off + bs * n : nullptr;
  int8_t *so = a.spins + mi.spin_off + bs * n;
  uint32_t pw[4] = {0, 0, 0, 0};
  real lq = 0;
  for (int i = 0; i < n; ++i) {
    // logit_i from the last layer's completed units and the earlier spins
    real part = 0;
#pragma unroll
    for (int kk = 0; kk < kD16KK; ++kk) {
      const int k = c + 16 * kk;
      if (k < H && dg[kk] <= i) part += (real)w.W2[(int64_t)i * mi.H + k] * hs[slot][D - 1][k];
    }
#pragma unroll
    for (int jj = 0; jj < kD16JJ; ++jj) {
      const int j = c + 16 * jj;
      if (j < i) part += (real)w.W0[(int64_t)i * n + j] * sv[jj];
    }
    // the sample's sum over its 16 lanes
    if constexpr (sizeof(real) == 4) {
      part = row16_sum(part);
    } else {
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) part += __shfl_xor(part, off, 16);
    }
    const real logit = part + (real)w.b2[i];
    float ui;
    if (u) {
      ui = live ? u[i] : 0.5f;
    } else {
      if ((i & 3) == 0) {
        pw[0] = (uint32_t)(i >> 2); pw[1] = (uint32_t)bs; pw[2] = step; pw[3] = (uint32_t)q;
        philox4x32_10(pw, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
      }
      ui = (float)(pw[i & 3] >> 8) * 5.9604644775390625e-08f;
    }
    const real p = sigmoid<real>(logit);
    const real si = ((real)ui < p) ? (real)1 : (real)-1;
    lq += log_sigmoid<real>(si * logit);
#pragma unroll
    for (int jj = 0; jj < kD16JJ; ++jj)
      if (c + 16 * jj == i) sv[jj] = si;
    if (c == 0 && live) so[i] = (int8_t)(si > 0 ? 1 : -1);
    // layer 1: the new spin, and the units it completes
#pragma unroll
    for (int kk = 0; kk < kD16KK; ++kk) {
      const int k = c + 16 * kk;
      if (k < H && dg[kk] >= i + 1) {
        acc[0][kk] += (real)w.W1[(int64_t)k * n + i] * si;
        if (dg[kk] == i + 1) hs[slot][0][k] = rtanh<real>(acc[0][kk]);
      }
    }
    // deeper layers: the units of degree i + 1 just completed below
    for (int l = 1; l < D; ++l) {
      wsync();
      const float *Wl = deep_layer(P, n, mi.H, l + 1);
#pragma unroll
      for (int kk = 0; kk < kD16KK; ++kk) {
        const int k2 = c + 16 * kk;
        if (k2 < H && dg[kk] >= i + 1) {
          if (i + 1 <= n - 1)
            for (int k = i; k < H; k += n - 1)
              acc[l][kk] += (real)Wl[(int64_t)k2 * mi.H + k] * hs[slot][l - 1][k];
          if (dg[kk] == i + 1) hs[slot][l][k2] = rtanh<real>(acc[l][kk]);
        }
      }
    }
    wsync();
  }
  if (live && c == 0) a.logq[mi.sample_off + b] = lq;
}

constexpr int kDeepRows = 4096;                // rb H of one block round
constexpr int kDeepND = kDeepRows / 256;       // per-thread entries of one layer's dh

// Rows of the REINFORCE backward for deeper networks: per sample every
// layer's h^l, the logits, dlogit = w ((1+s)/2 - sigmoid), and back through
// the layers da^l = (dh^l) (1 - (h^l)^2) with dh^D = dlogit . W2m and
// dh^{l-1} = da^l . W^l m.  Rows of rb samples per block round, in LDS with
// rows padded by one entry.  Items run sample-fastest, so the rb samples of
// a round share each weight read; the masked sums walk the units of each
// run of |W| - 1 (degree 1 + t for the t-th unit of a run) without a
// per-unit test, in ascending order as every sum here.
template <typename real>
__global__ __launch_bounds__(256) void rows_deep_kernel(RowArgs<real> a, int rb) {
  extern __shared__ __align__(16) char smem[];
  const MadeInst mi = a.mi;
  const int n = mi.n, Hs = mi.H, H = n >= 2 ? mi.H : 0, D = H > 0 ? mi.D : 1;
  const int DH = D * Hs;
  const int ln = n + 1, lh = DH + 1, ld = Hs + 1;
  const float *P = a.params + mi.param_off;
  const MadeView w = made_view(P, n, Hs);
  real *ss = reinterpret_cast<real *>(smem);   // [rb][n + 1]
  real *hh = ss + (size_t)rb * ln;              // [rb][D H + 1]
  real *dl = hh + (size_t)rb * lh;              // [rb][n + 1]
  real *d0 = dl + (size_t)rb * ln;              // [rb][H + 1]: dh of the current layer
  const double Fq = a.stats[0];
  const double invB = 1.0 / (double)mi.B;
  const int64_t c0 = (int64_t)blockIdx.x * a.chunk;
  const int64_t c1 = (c0 + a.chunk) < mi.B ? (c0 + a.chunk) : mi.B;
  for (int64_t r0 = c0; r0 < c1; r0 += rb) {
    const int nr = (int)((c1 - r0) < rb ? (c1 - r0) : rb);
    for (int i = threadIdx.x; i < rb * n; i += blockDim.x) {
      const int r = i / n, j = i - r * n;
      ss[r * ln + j] = r < nr ? (real)a.spins[r0 * n + i] : (real)0;
    }
    __syncthreads();
    // forward through the layers
    for (int i = threadIdx.x; i < rb * Hs; i += blockDim.x) {
      const int k = i / rb, r = i - k * rb;
      real acc = 0;
      if (k < H) {
        acc = (real)w.b1[k];
        const int m = degree(k, n);
        for (int j = 0; j < m; ++j) acc += (real)w.W1[(int64_t)k * n + j] * ss[r * ln + j];
        acc = rtanh<real>(acc);
      }
      hh[(size_t)r * lh + k] = acc;
    }
    __syncthreads();
    for (int l = 2; l <= D; ++l) {
      const float *Wl = deep_layer(P, n, Hs, l), *bl = Wl + (int64_t)Hs * Hs;
      for (int i = threadIdx.x; i < rb * Hs; i += blockDim.x) {
        const int k2 = i / rb, r = i - k2 * rb;
        real acc = 0;
        if (k2 < H) {
          acc = (real)bl[k2];
          const int m2 = degree(k2, n);
          const real *hp = hh + (size_t)r * lh + (size_t)(l - 2) * Hs;
          // units k with degree(k, n) <= m2
          for (int base = 0; base < H; base += n - 1) {
            const int e = m2 < H - base ? m2 : H - base;
            for (int t = 0; t < e; ++t)
              acc += (real)Wl[(int64_t)k2 * Hs + base + t] * hp[base + t];
          }
          acc = rtanh<real>(acc);
        }
        hh[(size_t)r * lh + (size_t)(l - 1) * Hs + k2] = acc;
      }
      __syncthreads();
    }
    // logits and dlogit
    for (int i = threadIdx.x; i < rb * n; i += blockDim.x) {
      const int ii = i / rb, r = i - ii * rb;
      const real *hD = hh + (size_t)r * lh + (size_t)(D - 1) * Hs;
      real z = (real)w.b2[ii];
      // units k with degree(k, n) <= ii
      for (int base = 0; base < H; base += n - 1) {
        const int e = ii < H - base ? ii : H - base;
        for (int t = 0; t < e; ++t) z += (real)w.W2[(int64_t)ii * Hs + base + t] * hD[base + t];
      }
      for (int j = 0; j < ii; ++j) z += (real)w.W0[(int64_t)ii * n + j] * ss[r * ln + j];
      const real sv = ss[r * ln + ii];
      const real wt = r < nr ? (real)((a.f[mi.sample_off + r0 + r] - Fq) * invB) : (real)0;
      const real d = wt * (((real)1 + sv) * (real)0.5 - sigmoid<real>(z));
      dl[r * ln + ii] = d;
      if (r < nr) {
        a.dlogit[(r0 + r) * n + ii] = d;
        a.sf[(r0 + r) * n + ii] = sv;
      }
    }
    __syncthreads();
    // back through the layers: dh^D from the logits, then W^l down
    for (int i = threadIdx.x; i < rb * Hs; i += blockDim.x) {
      const int k = i / rb, r = i - k * rb;
      real acc = 0;
      if (k < H) {
        const int m = degree(k, n);
        for (int ii = m; ii < n; ++ii) acc += dl[r * ln + ii] * (real)w.W2[(int64_t)ii * Hs + k];
      }
      d0[r * ld + k] = acc;
    }
    __syncthreads();
    for (int l = D; l >= 1; --l) {
      // da^l = dh^l (1 - h^2), written out with h^l
      for (int i = threadIdx.x; i < rb * Hs; i += blockDim.x) {
        const int k = i / rb, r = i - k * rb;
        const real hk = hh[(size_t)r * lh + (size_t)(l - 1) * Hs + k];
        const real da = d0[r * ld + k] * ((real)1 - hk * hk);
        d0[r * ld + k] = da;
        if (r < nr) {
          a.hid[(r0 + r) * DH + (int64_t)(l - 1) * Hs + k] = hk;
          a.da[(r0 + r) * DH + (int64_t)(l - 1) * Hs + k] = da;
        }
      }
      __syncthreads();
      if (l == 1) break;
      // dh^{l-1}[k] = sum over k2 with m(k2) >= m(k) of da^l[k2] W^l[k2, k],
      // kept per thread until every thread has read d0
      const float *Wl = deep_layer(P, n, Hs, l);
      // (rb H <= kDeepRows: at most kDeepND entries per thread)
      real nd[kDeepND];
      int c = 0;
      for (int i = threadIdx.x; i < rb * Hs && c < kDeepND; i += blockDim.x, ++c) {
        const int k = i / rb, r = i - k * rb;
        real acc = 0;
        if (k < H) {
          const int m = degree(k, n);
          // units k2 with degree(k2, n) = 1 + t >= m: t from m - 1 in each run
          for (int base = 0; base < H; base += n - 1) {
            const int e = (n - 1) < H - base ? (n - 1) : H - base;
            for (int t = m - 1; t < e; ++t)
              acc += d0[r * ld + base + t] * (real)Wl[(int64_t)(base + t) * Hs + k];
          }
        }
        nd[c] = acc;
      }
      __syncthreads();
      c = 0;
      for (int i = threadIdx.x; i < rb * Hs && c < kDeepND; i += blockDim.x, ++c) {
        const int k = i / rb, r = i - k * rb;
        d0[r * ld + k] = nd[c];
      }
      __syncthreads();
    }
  }
}

// Columns of W0 for the one-layer sampler: w0t[i][k] = W0[k][i] for k > i,
// 0 on and above the diagonal (whatever the parameters hold there, as the
// masks of Eq. 7 require).  32x32 tiles through LDS, both sides coalesced.
__global__ __launch_bounds__(256) void w0t_kernel(const MadeInst *mis, const float *params,
                                                  const int64_t *w0t_off, float *w0t) {
  const MadeInst mi = mis[blockIdx.z];
  const int n = mi.n;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  if (r0 >= n || c0 >= n) return;
  const float *W0 = made_view(params + mi.param_off, n, mi.H).W0;
  float *T = w0t + w0t_off[blockIdx.z];
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int k = r0 + y, i = c0 + tx;   // W0[k][i]
    tile[y][tx] = (k < n && i < n && k > i) ? W0[(int64_t)k * n + i] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int i = c0 + y, k = r0 + tx;   // T[i][k]
    if (i < n && k < n) T[(int64_t)i * n + k] = tile[tx][y];
  }
}

// Ancestral sampling for one-layer nets (H = 0: logit_i = b_i + sum_{j<i}
// W0[i][j] s_j, Eq. 7), one wave per sample.  Lane l owns positions
// l + 64 m (m < NM).  Their logits start at b and take the rank-1 update
// W0[:, i] s_i as soon as s_i is drawn, so position i's logit is complete
// when its turn comes; entries on and above the diagonal are zero, so it
// stays fixed afterwards.  The draw s_i = +1 iff u_i < sigmoid(logit_i) is
// taken as logit_i > ln(u_i / (1 - u_i)), with the right side formed by
// the owning lane before the block of 64 positions starts: the sequential
// part of a step is one compare in lane i, one read of that lane and the
// rank-1 update.  ln q is summed from the final logits after each block.
// The four waves of a workgroup share the columns of W0: chunks of 16
// columns are staged in LDS (two buffers, the next chunk loaded while the
// current one is used).  Waves past the batch run along (the barriers need
// them) and store nothing.
constexpr int kH0Chunk = 16;
template <typename real, int NM>
__global__ __launch_bounds__(256) void sample_h0_kernel(SampleArgs<real> a) {
  const int q = blockIdx.y;
  const MadeInst mi = a.mi[q];
  if ((int64_t)blockIdx.x * 4 >= mi.B) return;   // the whole block
  const int n = mi.n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + wave;
  const bool live = b < mi.B;
  const int64_t bs = live ? b : 0;
  const float *b2 = made_view(a.params + mi.param_off, n, mi.H).b2;
  const float *T = a.w0t + a.w0t_off[q];
  constexpr int RS = 64 * NM;                     // LDS row stride
  constexpr int PER = kH0Chunk * RS / 256;        // staged floats per thread
  __shared__ float buf[2][kH0Chunk * RS];
  const int n_chunks = (n + kH0Chunk - 1) / kH0Chunk;
  float st[PER];
  auto fetch = [&](int c) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int e = threadIdx.x + 256 * j, r = c * kH0Chunk + e / RS, k = e % RS;
      st[j] = (r < n && k < n) ? T[(int64_t)r * n + k] : 0.f;
    }
  };
  auto put = [&](int c) {
#pragma unroll
    for (int j = 0; j < PER; ++j) buf[c & 1][threadIdx.x + 256 * j] = st[j];
  };
  fetch(0);
  put(0);
  __syncthreads();
  real z[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) z[m] = (lane + 64 * m < n) ? (real)b2[lane + 64 * m] : (real)0;
  const uint32_t step = a.step_ctr ? (uint32_t)a.step_ctr[q] : 0u;
  const float *u = a.uniforms ? a.uniforms + mi.spin_off + bs * n : nullptr;
  int8_t *so = a.spins + mi.spin_off + bs * n;
  real lq = 0;
#pragma unroll
  for (int mb = 0; mb < NM; ++mb) {
    if (64 * mb >= n) break;
    const int pos = 64 * mb + lane;
    // the threshold of this lane's position: ln(u / (1 - u)) of its uniform
    // (given, or Philox word pos & 3 of counter pos >> 2)
    float ul;
    if (u) {
      ul = pos < n ? u[pos] : 0.5f;
    } else {
      uint32_t pw[4] = {(uint32_t)(pos >> 2), (uint32_t)bs, step, (uint32_t)q};
      philox4x32_10(pw, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
      const uint32_t wd = (pos & 3) == 0 ? pw[0] : (pos & 3) == 1 ? pw[1] : (pos & 3) == 2 ? pw[2] : pw[3];
      ul = (float)(wd >> 8) * 5.9604644775390625e-08f;
    }
    const real uu = (real)ul;
    const real thr = rlog<real>(uu) - rlog1p<real>(-uu);   // -inf at u = 0: always +1
    for (int c4 = 0; c4 < 4; ++c4) {
      const int c = 4 * mb + c4;
      if (c >= n_chunks) break;
      if (c + 1 < n_chunks) fetch(c + 1);
      const float *cb = buf[c & 1] + lane;
      // the columns of a group of four positions are read from LDS while
      // the previous group is drawn (two register sets used in turn)
      float wa[4][NM], wb[4][NM];
      (void)wb;
      auto rows = [&](int g, float (&w)[4][NM]) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int m = 0; m < NM; ++m) w[r][m] = cb[(g + r) * RS + 64 * m];
      };
      auto group = [&](int g, const float (&w)[4][NM]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int il = kH0Chunk * c4 + g + r;
          if (64 * mb + il < n) {
            const float d = z[mb] > thr ? 1.f : -1.f;
            const real si = (real)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(d), il));
#pragma unroll
            for (int m = 0; m < NM; ++m) z[m] += (real)w[r][m] * si;
          }
        }
      };
      static_assert(kH0Chunk == 16, "four groups of four positions per chunk");
      if constexpr (NM <= 4) {
        rows(0, wa);
        rows(4, wb);
        group(0, wa);
        rows(8, wa);
        group(4, wb);
        rows(12, wb);
        group(8, wa);
        group(12, wb);
      } else {
        // wide width sets: one register set (two would spill)
#pragma unroll 1
        for (int g = 0; g < kH0Chunk; g += 4) {
          rows(g, wa);
          group(g, wa);
        }
      }
      if (c + 1 < n_chunks) put(c + 1);
      __syncthreads();
    }
    // the block's logits are final: spins, their ln q terms and (for the
    // REINFORCE backward of the same parameters) q(s_i = +1 | s_<i)
    if (pos < n) {
      const real sv = z[mb] > thr ? (real)1 : (real)-1;
      lq += log_sigmoid<real>(sv * z[mb]);
      if (live) {
        so[pos] = (int8_t)(sv > 0 ? 1 : -1);
        if (a.sig) a.sig[mi.spin_off + bs * n + pos] = sigmoid<real>(z[mb]);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) lq += __shfl_xor(lq, off, 64);
  if (live && lane == 0) a.logq[mi.sample_off + b] = lq;
}

// Per-sample rows of the log-prob pass and the REINFORCE backward:
// The batched form: block b belongs to the last job whose first block is
// at most b (a search over the prefix sums); inside its job it is the block
// of the same index in the one-job launch's grid.
__device__ inline int job_of(const int32_t *lo, int nj, int b) {
  int a = 0, z = nj - 1;
  while (a < z) {
    const int mid = (a + z + 1) >> 1;
    if (uload(lo + mid) <= b) a = mid;
    else z = mid - 1;
  }
  return a;
}

// a, tanh(a), logits, dlogit = w ((1+s)/2 - sigmoid(logit)) with the weight
// w_b = (f_b - F_q) / B, and da = (dlogit . W2m) (1 - tanh^2).  Block `blk`
// of an instance walks its chunk of samples in rounds of RB, with the
// parameters staged in LDS (kLDS).  Items run sample-fastest: the RB samples
// of a round share each weight (one LDS or cache line per 16 lanes), and the
// per-sample rows in LDS are padded by one entry against bank conflicts.
// Every sum runs in ascending index order.
constexpr int RB = 16;
template <typename real, bool kLDS>
__device__ inline void rows_block(const RowArgs<real> &a, int64_t blk, char *smem) {
  const MadeInst mi = a.mi;
  const int n = mi.n, H = (n >= 2) ? mi.H : 0, Hs = mi.H;
  MadeView w = made_view(a.params + mi.param_off, n, Hs);
  size_t woff = 0;
  if (kLDS) {
    w = made_stage(w, n, Hs, reinterpret_cast<float *>(smem), false);
    woff = (made_stage_bytes(n, Hs) + 15) & ~(size_t)15;
  }
  const int ln = n + 1, lh = Hs + 1;
  real *ss = reinterpret_cast<real *>(smem + woff);  // [RB][n + 1]
  real *hh = ss + RB * ln;                           // [RB][H + 1]
  real *dl = hh + RB * lh;                           // [RB][n + 1]
  const double Fq = a.stats[0];
  const double invB = 1.0 / (double)mi.B;
  const int64_t c0 = blk * a.chunk;
  const int64_t c1 = (c0 + a.chunk) < mi.B ? (c0 + a.chunk) : mi.B;
  for (int64_t r0 = c0; r0 < c1; r0 += RB) {
    const int nr = (int)((c1 - r0) < RB ? (c1 - r0) : RB);
    const int8_t *sp = a.spins + r0 * n;
    for (int i = threadIdx.x; i < RB * n; i += blockDim.x) {
      const int r = i / n, j = i - r * n;
      ss[r * ln + j] = r < nr ? (real)sp[i] : (real)0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < RB * Hs; i += blockDim.x) {
      const int k = i / RB, r = i - k * RB;
      real acc = 0;
      if (k < H) {
        acc = (real)w.b1[k];
        const int m = degree(k, n);
        for (int j = 0; j < m; ++j) acc += (real)w.W1[(int64_t)k * w.ld1 + j] * ss[r * ln + j];
        acc = rtanh<real>(acc);
      }
      hh[r * lh + k] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < RB * n; i += blockDim.x) {
      const int ii = i / RB, r = i - ii * RB;
      real z = (real)w.b2[ii];
      // the units k with degree(k, n) = 1 + k mod (n - 1) <= ii: in every
      // run of n - 1 units, the first ii
      for (int base = 0; base < H; base += n - 1) {
        const int e = ii < H - base ? ii : H - base;
        for (int t = 0; t < e; ++t)
          z += (real)w.W2[(int64_t)ii * w.ld2 + base + t] * hh[r * lh + base + t];
      }
      for (int j = 0; j < ii; ++j) z += (real)w.W0[(int64_t)ii * w.ld0 + j] * ss[r * ln + j];
      const real s = ss[r * ln + ii];
      const real wt = r < nr ? (real)((a.f[mi.sample_off + r0 + r] - Fq) * invB) : (real)0;
      const real d = wt * (((real)1 + s) * (real)0.5 - sigmoid<real>(z));
      dl[r * ln + ii] = d;
      if (r < nr) {
        a.dlogit[(r0 + r) * n + ii] = d;
        a.sf[(r0 + r) * n + ii] = s;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < RB * Hs; i += blockDim.x) {
      const int k = i / RB, r = i - k * RB;
      if (r < nr) {
        real acc = 0;
        const real hk = hh[r * lh + k];
        if (k < H) {
          const int m = degree(k, n);
          for (int ii = m; ii < n; ++ii)
            acc += dl[r * ln + ii] * (real)w.W2[(int64_t)ii * w.ld2 + k];
        }
        a.hid[(r0 + r) * Hs + k] = hk;
        a.da[(r0 + r) * Hs + k] = acc * ((real)1 - hk * hk);
      }
    }
    __syncthreads();
  }
}

// Every instance's rows in one launch: the block finds its job (a search
// over the jobs' first blocks) and runs that instance's block of the same
// index.
template <typename real, bool kLDS>
__global__ __launch_bounds__(1024) void rows_batch_kernel(RowBatch<real> b) {
  extern __shared__ __align__(16) char smem[];
  const int j = job_of(b.lo, b.n_jobs, blockIdx.x);
  const RowJob J = uload(b.jobs + j);
  RowArgs<real> a{};
  a.mi = uload(b.mi + J.q);
  a.params = b.params;
  a.spins = b.spins + a.mi.spin_off;
  a.f = b.f;
  a.stats = b.stats + 4 * (int64_t)J.q;
  a.chunk = J.chunk;
  a.hid = b.hid + J.hoff;
  a.da = b.da + J.hoff;
  a.dlogit = b.dlogit + J.doff;
  a.sf = b.sf + J.doff;
  rows_block<real, kLDS>(a, (int64_t)blockIdx.x - uload(b.lo + j), smem);
}

// The rows of the REINFORCE backward for one-layer nets: dlogit = w_b
// ((1 + s) / 2 - q(s_i = +1 | s_<i)) with the conditionals the sampler
// stored for these spins, and the spins as real; one thread per entry.
template <typename real>
__global__ __launch_bounds__(256) void rows_h0_kernel(RowArgs<real> a) {
  const MadeInst mi = a.mi;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = mi.n;
  if (e >= mi.B * n) return;
  const int64_t r = e / n;
  const real s = (real)a.spins[e];
  const real wt = (real)((a.f[mi.sample_off + r] - a.stats[0]) / (double)mi.B);
  a.dlogit[e] = wt * (((real)1 + s) * (real)0.5 - a.sig[e]);
  a.sf[e] = s;
}

// part[ks][m][n] = sum over batch rows of slice ks of X[b, m] * Y[b, n]
constexpr int TM = 32, TN = 32, TK = 32;
template <typename real>
__device__ inline void atb_block(const real *X, int ldx, const real *Y, int ldy, int64_t B, int M,
                                 int N, real *part, int ksplit, int bx, int by, int ks) {
  __shared__ real xs[TK][TM + 1];
  __shared__ real ys[TK][TN + 1];
  const int m0 = bx * TM, n0 = by * TN;
  const int64_t chunk = (B + ksplit - 1) / ksplit;
  const int64_t bb0 = (int64_t)ks * chunk;
  const int64_t bb1 = (bb0 + chunk) < B ? (bb0 + chunk) : B;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;   // 2x2 outputs each
  real acc[2][2] = {{0, 0}, {0, 0}};
  for (int64_t k0 = bb0; k0 < bb1; k0 += TK) {
    for (int i = threadIdx.x; i < TK * TM; i += 256) {
      const int kk = i / TM, mm = i % TM;
      const int64_t bi = k0 + kk;
      xs[kk][mm] = (bi < bb1 && m0 + mm < M) ? X[bi * ldx + m0 + mm] : (real)0;
      ys[kk][mm] = (bi < bb1 && n0 + mm < N) ? Y[bi * ldy + n0 + mm] : (real)0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < TK; ++kk) {
      const real x0 = xs[kk][ty * 2], x1 = xs[kk][ty * 2 + 1];
      const real y0 = ys[kk][tx * 2], y1 = ys[kk][tx * 2 + 1];
      acc[0][0] += x0 * y0; acc[0][1] += x0 * y1;
      acc[1][0] += x1 * y0; acc[1][1] += x1 * y1;
    }
    __syncthreads();
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const int m = m0 + ty * 2 + i, nn = n0 + tx * 2 + j;
      if (m < M && nn < N) part[((int64_t)ks * M + m) * N + nn] = acc[i][j];
    }
}

// out[m*ldo + n] = mask(m, n) * sum_ks part[ks][m][n]
// mask kinds: 0 none, 1 W2 (n > deg(k)... (row i, col k): i+1 > deg(k)),
//             2 W0 (col j < row i), 3 W1 (row k, col j): j+1 <= deg(k),
//             4 deeper layers (row k', col k): deg(k) <= deg(k')
// one output idx of the batch sum C = X^T Y: the slices in order, then the
// mask of its matrix
template <typename real>
__device__ inline void atb_finish_one(const real *part, int ksplit, int M, int N, float *out,
                                      int ldo, int mask_kind, int nW, int64_t idx) {
  const int64_t tot = (int64_t)M * N;
  const int m = (int)(idx / N), nn = (int)(idx % N);
  // loads in batches of 8 (independent), additions in slice order
  double acc = 0;
  int k = 0;
  for (; k + 8 <= ksplit; k += 8) {
    real v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(k + j) * tot + idx];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += (double)v[j];
  }
  for (; k < ksplit; ++k) acc += (double)part[(int64_t)k * tot + idx];
  bool keep = true;
  if (mask_kind == 1) keep = nW >= 2 && (m + 1) > degree(nn, nW);
  else if (mask_kind == 2) keep = nn < m;
  else if (mask_kind == 3) keep = nW >= 2 && (nn + 1) <= degree(m, nW);
  else if (mask_kind == 4) keep = nW >= 2 && degree(nn, nW) <= degree(m, nW);
  out[(int64_t)m * ldo + nn] = keep ? (float)acc : 0.0f;
}

// column m of batch slice ks
template <typename real>
__device__ inline void colsum_one(const real *X, int ldx, int64_t B, int M, real *part,
                                  int ksplit, int m, int ks) {
  const int64_t chunk = (B + ksplit - 1) / ksplit;
  const int64_t b0 = (int64_t)ks * chunk;
  const int64_t b1 = (b0 + chunk) < B ? (b0 + chunk) : B;
  real acc = 0;
  int64_t b = b0;
  // loads in batches of 8 (independent), additions in row order
  for (; b + 8 <= b1; b += 8) {
    real v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = X[(b + k) * ldx + m];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += v[k];
  }
  for (; b < b1; ++b) acc += X[b * ldx + m];
  part[(int64_t)ks * M + m] = acc;
}

template <typename real>
__device__ inline void colsum_finish_one(const real *part, int ksplit, int M, float *out, int m) {
  // loads in batches of 8 (independent), additions in slice order
  double acc = 0;
  int k = 0;
  for (; k + 8 <= ksplit; k += 8) {
    real v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(k + j) * M + m];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += (double)v[j];
  }
  for (; k < ksplit; ++k) acc += (double)part[(int64_t)k * M + m];
  out[m] = (float)acc;
}

template <typename real>
__global__ __launch_bounds__(256) void batch_atb_kernel(BatchSums<real> a) {
  const int b = blockIdx.x, j = job_of(a.atb_lo, a.n_atb, b);
  const AtbJob<real> J = uload(a.atb + j);
  const int t = b - uload(a.atb_lo + j);
  const int tm = (J.M + TM - 1) / TM, tn = (J.N + TN - 1) / TN;
  atb_block<real>(J.X, J.ldx, J.Y, J.ldy, J.B, J.M, J.N, a.part + J.part_off, J.ks, t % tm,
                  (t / tm) % tn, t / (tm * tn));
}
template <typename real>
__global__ __launch_bounds__(256) void batch_atb_finish(BatchSums<real> a) {
  const int b = blockIdx.x, j = job_of(a.atb_flo, a.n_atb, b);
  const AtbJob<real> J = uload(a.atb + j);
  const int64_t idx = (int64_t)(b - uload(a.atb_flo + j)) * blockDim.x + threadIdx.x;
  if (idx < (int64_t)J.M * J.N)
    atb_finish_one<real>(a.part + J.part_off, J.ks, J.M, J.N, J.out, J.ldo, J.mask, J.nW, idx);
}
template <typename real>
__global__ __launch_bounds__(256) void batch_col_kernel(BatchSums<real> a) {
  const int b = blockIdx.x, j = job_of(a.col_lo, a.n_col, b);
  const ColJob<real> J = uload(a.col + j);
  const int t = b - uload(a.col_lo + j), cm = (J.M + 255) / 256;
  const int m = (t % cm) * 256 + threadIdx.x;
  if (m < J.M) colsum_one<real>(J.X, J.ldx, J.B, J.M, a.part + J.part_off, J.ks, m, t / cm);
}
template <typename real>
__global__ __launch_bounds__(256) void batch_col_finish(BatchSums<real> a) {
  const int b = blockIdx.x, j = job_of(a.col_flo, a.n_col, b);
  const ColJob<real> J = uload(a.col + j);
  const int m = (b - uload(a.col_flo + j)) * 256 + threadIdx.x;
  if (m < J.M) colsum_finish_one<real>(a.part + J.part_off, J.ks, J.M, J.out, m);
}

// f_b = E_1 - logZ_R / beta + ln q / beta (FP64, Eqs. 4 and 9) per sample and
// per-block sums of f, f^2, Etilde and ln q / beta; every instance of the
// batch in one launch (grid.y = instance).
// F_q = mean f, its standard error, mean effective energy and mean ln q / beta
// (Eq. 9) from the batch sums of f, f^2, the effective energy and ln q / beta
__device__ inline void free_stats(const double sm[4], int64_t B, double *out) {
  const double Bd = (double)B;
  const double Fq = sm[0] / Bd;
  double var = B > 1 ? (sm[1] - Bd * Fq * Fq) / (Bd - 1.0) : 0.0;
  if (var < 0.0) var = 0.0;
  out[0] = Fq;
  out[1] = sqrt(var / Bd);
  out[2] = sm[2] / Bd;
  out[3] = sm[3] / Bd;
}

template <typename real>
__global__ __launch_bounds__(256) void free_f_kernel(FreeArgs<real> a) {
  __shared__ double sh[4][256];
  const int q = blockIdx.y, tid = threadIdx.x;
  const InstDesc D = a.inst[q];
  const MadeInst mi = a.mi[q];
  // an instance without samples this step: a zero statistics row, and its
  // step counter stays (its parameters and moments do not move either)
  if (mi.B <= 0) {
    if (blockIdx.x == 0 && tid < 4 && a.stats) a.stats[4 * q + tid] = 0.0;
    return;
  }
  const double beta = D.beta;
  const int32_t *wa = a.ww_a + D.ww_off, *wb = a.ww_b + D.ww_off;
  const double *wJ = a.ww_J + D.ww_off, *hW = a.hW + a.hw_off[q];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // per-sample inputs: spins (as a bit mask when n <= 128), logZ and ln q.
  // logZ is either given or log_const plus the chain partials in chain
  // order, then the unary sums (the order of launch_chain_sum), loaded 16 at
  // a time with every load of a batch in flight together
  struct In {
    SpinBits sb;
    double lz, lq;
  };
  const bool bits = mi.n <= 128;
  auto inputs = [&](int64_t b, bool first) {
    In r;
    if (bits) r.sb = load_bits_row(a.spins + mi.spin_off + b * mi.n, mi.n);
    r.lz = r.lq = 0.0;
    if (!first) return r;
    const int64_t g = mi.sample_off + b;
    r.lq = (double)a.logq[g];
    if (a.cpart) {
      const int nch = a.cinst[q].n_chains, nf = (D.nr + kUnaryChunk - 1) / kUnaryChunk;
      const int tot = nch + nf;
      const double *cp = a.cpart + a.cpart_off[q] + b, *fa = a.fabp + a.f_off[q] + b;
      double lz = D.log_const;
      for (int c0 = 0; c0 < tot; c0 += 16) {
        double v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int c = c0 + j;
          const double *src = c < nch ? cp + (int64_t)c * mi.B
                              : c < tot ? fa + (int64_t)(c - nch) * mi.B
                              : nch > 0 ? cp : fa;
          v[j] = *src;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (c0 + j < tot) lz += v[j];
      }
      r.lz = lz;
    } else {
      r.lz = a.logz[g];
    }
    return r;
  };
  // kFreeLanes lanes per sample: each sums every kFreeLanes-th E_1 term,
  // then a butterfly (the same sum on every lane of the group); the first
  // lane of the group reads the sample's other inputs and forms f
  const int part = tid % kFreeLanes;
  const int64_t b0 = ((int64_t)blockIdx.x * blockDim.x + tid) / kFreeLanes,
                bstride = (int64_t)gridDim.x * blockDim.x / kFreeLanes;
  // the first sample's inputs are requested before the tables are staged,
  // so that both are one memory round trip
  In cur;
  if (mi.B > 0) cur = inputs(b0 < mi.B ? b0 : 0, part == 0);
  // the first kFreeStage W-W couplings (endpoints packed in one word) and
  // the W fields staged in LDS once per block: the per-sample loops then
  // read them without a memory round trip per batch of terms
  __shared__ int32_t s_ab[kFreeStage];
  __shared__ double s_J[kFreeStage], s_h[128];
  const int nst = min(D.n_ww, kFreeStage);
  for (int k = tid; k < nst; k += blockDim.x) {
    s_ab[k] = wa[k] | (wb[k] << 16);
    s_J[k] = wJ[k];
  }
  for (int k = tid; k < mi.n && k < 128; k += blockDim.x) s_h[k] = hW[k];
  __syncthreads();
  const double ib = 1.0 / beta;
  // (every lane of a group walks the same samples: the loop trip count and
  // the butterfly are uniform over the group)
  for (int64_t b = b0; b < mi.B; b += bstride) {
    if (b != b0) cur = inputs(b, part == 0);
    double e1 = 0.0;
    if (bits) {
      // the +-1 products are exact
      const SpinBits &sb = cur.sb;
#pragma unroll 4
      for (int k = part; k < nst; k += kFreeLanes) {
        const int ab = s_ab[k];
        const double j = s_J[k];
        e1 -= sb.sigma(ab & 0xffff) * sb.sigma(ab >> 16) > 0.f ? j : -j;
      }
      for (int k = nst + part; k < D.n_ww; k += kFreeLanes) {
        const double j = wJ[k];
        e1 -= sb.sigma(wa[k]) * sb.sigma(wb[k]) > 0.f ? j : -j;
      }
#pragma unroll 4
      for (int k = part; k < mi.n; k += kFreeLanes) e1 -= sb.sigma(k) > 0.f ? s_h[k] : -s_h[k];
    } else {
      // width sets beyond the mask: spin bytes, the staged couplings first
      // (the same terms in the same order as above)
      const int8_t *s = a.spins + mi.spin_off + b * mi.n;
#pragma unroll 4
      for (int k = part; k < nst; k += kFreeLanes) {
        const int ab = s_ab[k];
        e1 -= s_J[k] * (double)s[ab & 0xffff] * (double)s[ab >> 16];
      }
      for (int k = nst + part; k < D.n_ww; k += kFreeLanes)
        e1 -= wJ[k] * (double)s[wa[k]] * (double)s[wb[k]];
#pragma unroll 4
      for (int k = part; k < mi.n; k += kFreeLanes) e1 -= hW[k] * (double)s[k];
    }
#pragma unroll
    for (int o = 1; o < kFreeLanes; o <<= 1) e1 += __shfl_xor(e1, o, 64);
    if (part == 0) {
      const double et = e1 - cur.lz * ib;
      const double lqb = cur.lq * ib;
      const double f = et + lqb;
      a.f[mi.sample_off + b] = f;
      if (a.nonfinite && !__builtin_isfinite(f)) a.nonfinite[q] = 1;
      acc[0] += f; acc[1] += f * f; acc[2] += et; acc[3] += lqb;
    }
  }
  for (int c = 0; c < 4; ++c) sh[c][tid] = acc[c];
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st)
      for (int c = 0; c < 4; ++c) sh[c][tid] += sh[c][tid + st];
    __syncthreads();
  }
  // block sums, component-major: part[q][c][block]
  if (tid == 0)
    for (int c = 0; c < 4; ++c) a.part[((int64_t)q * 4 + c) * gridDim.x + blockIdx.x] = sh[c][0];
  // the step's sampler (the counter's only earlier reader) has run: the
  // step counter advances here, and the optimiser then reads the step's own
  // number (an atomic add whose result is unused: nothing waits for a load)
  if (blockIdx.x == 0 && tid == 0 && a.step_ctr) atomicAdd(a.step_ctr + q, 1);
  if (!a.finish) return;
  // the last block of the instance (completion ticket) forms the statistics
  // from the block sums: thread k holds block k, then a fixed tree
  __shared__ int last;
  if (tid == 0) {
    __threadfence();
    const int prev = atomicAdd(a.done + q, 1);
    last = prev == (int)gridDim.x - 1;
    if (last) atomicExch(a.done + q, 0);
  }
  __syncthreads();
  if (!last || mi.B <= 0) return;
  __threadfence();
  for (int c = 0; c < 4; ++c)
    sh[c][tid] = tid < (int)gridDim.x
                     ? __hip_atomic_load(a.part + ((int64_t)q * 4 + c) * gridDim.x + tid,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : 0.0;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st)
      for (int c = 0; c < 4; ++c) sh[c][tid] += sh[c][tid + st];
    __syncthreads();
  }
  if (tid != 0) return;
  const double sm[4] = {sh[0][0], sh[1][0], sh[2][0], sh[3][0]};
  free_stats(sm, mi.B, a.stats + 4 * q);
}

// E_1(s_W) = -sum_{W-W edges} J s_i s_j - sum_{i in W} h_i s_i (Eq. 4) of
// every sample, one thread per sample (the couplings are read by every
// thread of a block at the same index: one cache line per term)
__global__ __launch_bounds__(256) void e1_kernel(E1Args a) {
  const int q = blockIdx.y;
  const MadeInst mi = a.mi[q];
  const InstDesc D = a.inst[q];
  const int32_t *wa = a.ww_a + D.ww_off, *wb = a.ww_b + D.ww_off;
  const double *wJ = a.ww_J + D.ww_off, *hW = a.hW + a.hw_off[q];
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < mi.B;
       b += (int64_t)gridDim.x * blockDim.x) {
    const int8_t *s = a.spins + mi.spin_off + b * mi.n;
    double e1 = 0.0;
    for (int k = 0; k < D.n_ww; ++k) e1 -= wJ[k] * (double)(s[wa[k]] * s[wb[k]]);
    for (int k = 0; k < mi.n; ++k) e1 -= hW[k] * (double)s[k];
    a.e1[mi.sample_off + b] = e1;
  }
}

// Adam (Kingma & Ba; beta1 = 0.9, beta2 = 0.999, eps = 1e-8) on one
// parameter, with the bias corrections c1 = 1 - 0.9^t, c2 = 1 - 0.999^t of
// step t taken in FP64.  Masked parameters have zero gradient, so they and
// their moments never move.
__device__ inline void adam_one(float gi, float &p, float &m, float &v, double c1, double c2,
                                float lr) {
  m = 0.9f * m + 0.1f * gi;
  v = 0.999f * v + 0.001f * gi * gi;
  const double mh = (double)m / c1, vh = (double)v / c2;
  p = (float)((double)p - (double)lr * mh / (sqrt(vh) + 1e-8));
}

__device__ inline void pack_scatter(float *P, int n, int Hs, int npt, int64_t i, float v);

// Adam for every instance in one launch (grid.y = instance), on the flat
// gradient buffer.  The step counter already counts this step (the
// free-energy kernel advanced it).  With pack set, each updated parameter
// is also written into the packed operand tables (pack_scatter), which then
// stay current.
__global__ __launch_bounds__(256) void adam_step_kernel(OptArgs a) {
  const int q = blockIdx.y;
  const MadeInst mi = a.mi[q];
  // an instance without samples this step keeps its parameters and moments
  if (mi.B <= 0) return;
  const int64_t pc = made_pc(mi);
  float *P = a.params + mi.param_off, *M = a.m + mi.param_off, *V = a.v + mi.param_off;
  const float *G = a.grad + mi.param_off;
  const double t = (double)a.step_ctr[q];
  const double c1 = 1.0 - pow(0.9, t), c2 = 1.0 - pow(0.999, t);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < pc;
       i += (int64_t)gridDim.x * blockDim.x) {
    float p = P[i], m = M[i], v = V[i];
    adam_one(G[i], p, m, v, c1, c2, a.lr);
    M[i] = m;
    V[i] = v;
    P[i] = p;
    if (a.pack) pack_scatter(a.pack + mi.pack_off, mi.n, mi.H, a.npt, i, p);
  }
}

// ---------------------------------------------------------------------------
// Exact slicing (Sec. 2, Eqs. 3-4): every configuration of the width set W is
// one sample.  slice_spins_kernel writes configurations c0 .. c0 + n - 1
// (spin i of configuration x is -1 where bit i of x is set, else +1);
// slice_lse_kernel forms t = -beta E_1(s) + logZ_R(s) per configuration and
// a per-block log-sum-exp pair (max m, sum of exp(t - m)), in FP64 and in a
// fixed order; slice_final_kernel merges the pairs in order into
// logZ = m + ln(sum) and F = -logZ / beta.
__global__ void slice_spins_kernel(int8_t *spins, int nw, int64_t c0, int64_t nbytes) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nbytes;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / nw;
    const int i = (int)(e - b * nw);
    spins[e] = (((c0 + b) >> i) & 1) ? (int8_t)-1 : (int8_t)1;
  }
}

__device__ inline void lse_merge(double &m, double &s, double m2, double s2) {
  if (s2 == 0.0) return;
  if (s == 0.0) { m = m2; s = s2; return; }
  const double M = m > m2 ? m : m2;
  s = s * exp(m - M) + s2 * exp(m2 - M);
  m = M;
}

__global__ __launch_bounds__(256) void slice_lse_kernel(SliceArgs a) {
  __shared__ double sm[256], ss[256];
  const int tid = threadIdx.x;
  const InstDesc D = a.inst[a.q];
  const int32_t *wa = a.ww_a + D.ww_off, *wb = a.ww_b + D.ww_off;
  const double *wJ = a.ww_J + D.ww_off, *hW = a.hW + a.hw_off[a.q];
  double m = 0.0, s = 0.0;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + tid; b < a.n; b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = a.c0 + b;
    double e1 = 0.0;
    for (int k = 0; k < D.n_ww; ++k) {
      const bool neg = (((x >> wa[k]) ^ (x >> wb[k])) & 1) != 0;   // s_a s_b = -1
      e1 -= neg ? -wJ[k] : wJ[k];
    }
    for (int k = 0; k < D.nw; ++k) e1 -= ((x >> k) & 1) ? -hW[k] : hW[k];
    lse_merge(m, s, -D.beta * e1 + a.logz[b], 1.0);
  }
  sm[tid] = m;
  ss[tid] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      double m1 = sm[tid], s1 = ss[tid];
      lse_merge(m1, s1, sm[tid + st], ss[tid + st]);
      sm[tid] = m1;
      ss[tid] = s1;
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.part[2 * (a.pass * (int64_t)gridDim.x + blockIdx.x)] = sm[0];
    a.part[2 * (a.pass * (int64_t)gridDim.x + blockIdx.x) + 1] = ss[0];
  }
}

__global__ __launch_bounds__(256) void slice_final_kernel(const double *part, int64_t count,
                                                          double beta, double *out) {
  __shared__ double sm[256], ss[256];
  const int tid = threadIdx.x;
  double m = 0.0, s = 0.0;
  for (int64_t k = tid; k < count; k += 256) lse_merge(m, s, part[2 * k], part[2 * k + 1]);
  sm[tid] = m;
  ss[tid] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      double m1 = sm[tid], s1 = ss[tid];
      lse_merge(m1, s1, sm[tid + st], ss[tid + st]);
      sm[tid] = m1;
      ss[tid] = s1;
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double lz = sm[0] + log(ss[0]);
    out[0] = lz;
    out[1] = -lz / beta;
  }
}

// ---------------------------------------------------------------------------
// Moments of p from samples of q.  The W-marginal of p is exp(-beta E_1)
// Z_R / Z, so a sample's weight p / q is exp(-beta f_b) up to a constant
// (f_b of Eq. 9); normalised over the instance's batch, w_b.  The adjoint
// with g_b = w_b / beta then sums w_b times the conditional moments of the
// remainder (dh = beta sum g_b <r>, dJ = beta sum g_b <x x>);
// obs_w_kernel adds the width-set moments, sum_b w_b s_i and
// sum_b w_b s_a s_b.  Every sum is FP64 in a fixed order.
constexpr int kObsThreads = 1024;
__device__ inline double block_reduce(double v, double *sh, bool is_max) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int st = kObsThreads / 2; st > 0; st >>= 1) {
    if (t < st) sh[t] = is_max ? fmax(sh[t], sh[t + st]) : sh[t] + sh[t + st];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
__global__ __launch_bounds__(kObsThreads) void obs_weights_kernel(ObsArgs a) {
  __shared__ double sh[kObsThreads];
  const int q = blockIdx.x;
  const MadeInst mi = a.mi[q];
  const double beta = a.inst[q].beta;
  const double *f = a.f + mi.sample_off;
  double m = -INFINITY;
  for (int64_t b = threadIdx.x; b < mi.B; b += kObsThreads) m = fmax(m, -beta * f[b]);
  m = block_reduce(m, sh, true);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t b = threadIdx.x; b < mi.B; b += kObsThreads) {
    const double e = exp(-beta * f[b] - m);
    s1 += e;
    s2 += e * e;
  }
  s1 = block_reduce(s1, sh, false);
  s2 = block_reduce(s2, sh, false);
  for (int64_t b = threadIdx.x; b < mi.B; b += kObsThreads)
    a.g[mi.sample_off + b] = exp(-beta * f[b] - m) / (s1 * beta);
  if (threadIdx.x == 0) a.ess[q] = mi.B > 0 ? s1 * s1 / s2 : 0.0;
}
// block (output o, instance q): o < |W| the magnetisation of W vertex o,
// else W-W edge o - |W|
__global__ __launch_bounds__(kObsThreads) void obs_w_kernel(ObsArgs a) {
  __shared__ double sh[kObsThreads];
  const int q = blockIdx.y, o = blockIdx.x;
  const InstDesc D = a.inst[q];
  const MadeInst mi = a.mi[q];
  if (o >= D.nw + D.n_ww) return;
  const bool vert = o < D.nw;
  const int i0 = vert ? o : a.ww_a[D.ww_off + o - D.nw], i1 = vert ? -1 : a.ww_b[D.ww_off + o - D.nw];
  const double beta = D.beta;
  const int8_t *s = a.spins + mi.spin_off;
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < mi.B; b += kObsThreads) {
    const double x = (double)s[b * D.nw + i0] * (i1 >= 0 ? (double)s[b * D.nw + i1] : 1.0);
    acc += beta * a.g[mi.sample_off + b] * x;
  }
  acc = block_reduce(acc, sh, false);
  if (threadIdx.x != 0) return;
  if (vert) a.mag[a.spin_base[q] + a.wv[a.hw_off[q] + o]] = acc;
  else a.corr[a.edge_base[q] + a.ww_e[D.ww_off + o - D.nw]] = acc;
}

// ---------------------------------------------------------------------------
// Matrix-core sampler (FP32).  A wave draws 16 samples.  Logits z and spins
// of the wave's samples live in the R-layout of the chain kernels (lane l
// holds positions 16 t + 4 (l >> 4) + r of sample l & 15).  After position i
// is drawn, the hidden units of degree i + 1 are complete: their
// activations are one 16x16x4 product over the spins drawn so far, and
// their tanh values (plus the direct W0 term of s_i in slot 15) are folded
// into every later logit by a second product.  Both products read
// parameters repacked into operand order by made_pack_kernel.
//
// Packed layout per instance (floats, NPT position tiles):
//   PA  [n][NPT][64][4]  W1[k(i, l & 15)][16 t + 4 (l >> 4) + r], j <= i
//   PZ  [n][NPT][64][4]  slot u = 4 (l >> 4) + r:  W2[16 t + (l & 15)][k(i, u)]
//                        for u < 15, W0[16 t + (l & 15)][i] for u = 15
//                        (zero unless the output position is > i)
//   PB1 [n][64][4]       b1[k(i, 4 (l >> 4) + r)]
//   PB2 [NPT][64][4]     b2[16 t + 4 (l >> 4) + r]
// with k(i, u) = i + (n - 1) u the u-th hidden unit of degree i + 1.

__host__ __device__ inline int64_t msample_floats(int n, int npt) {
  return (int64_t)n * npt * 512 + (int64_t)n * 256 + (int64_t)npt * 256;
}
// sampler tables, then the masked matrices of the fused backward:
//   W2T [H][n]  W2[pos][k] where deg(k) <= pos, else 0 (transposed)
//   W1m [H][n]  W1[k][j] where j < deg(k), else 0
//   W2m [n][H]  W2[pos][k] where deg(k) <= pos, else 0
// (padded to 64 floats)
__host__ __device__ inline int64_t mpack_floats(int n, int npt, int H) {
  return msample_floats(n, npt) + (3 * (int64_t)H * n + 63) / 64 * 64;
}

__global__ void made_pack_kernel(const MadeInst *mi, const float *params, float *pack, int npt) {
  const MadeInst m = mi[blockIdx.y];
  const int n = m.n, Hs = m.H, H = n >= 2 ? m.H : 0;
  const float *W1 = params + m.param_off, *b1 = W1 + (int64_t)Hs * n, *W2 = b1 + Hs,
              *b2 = W2 + (int64_t)n * Hs, *W0 = b2 + n;
  const int64_t sa = (int64_t)n * npt * 256, sb = (int64_t)n * 256;
  const int64_t tsamp = msample_floats(n, npt);
  const int64_t hn = (int64_t)Hs * n;
  const int64_t total = tsamp + 3 * hn;
  float *P = pack + m.pack_off;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    if (idx >= tsamp) {
      const int64_t e = idx - tsamp, part = e / (hn > 0 ? hn : 1), f = e - part * hn;
      if (part == 0) {          // W2T
        const int k = (int)(f / n), pos = (int)(f % n);
        if (k < H && 1 + k % (n - 1) <= pos) v = W2[(int64_t)pos * Hs + k];
      } else if (part == 1) {   // W1m
        const int k = (int)(f / n), j = (int)(f % n);
        if (k < H && j < 1 + k % (n - 1)) v = W1[f];
      } else {                  // W2m
        const int pos = (int)(f / Hs), k = (int)(f % Hs);
        if (k < H && 1 + k % (n - 1) <= pos) v = W2[f];
      }
    } else if (idx < 2 * sa) {
      const int64_t e = idx < sa ? idx : idx - sa;
      const int r = (int)(e & 3), lane = (int)((e >> 2) & 63);
      const int t = (int)((e >> 8) % npt), i = (int)((e >> 8) / npt);
      const int ls = lane & 15, lg = lane >> 4;
      if (idx < sa) {
        const int k = i + (n - 1) * ls, j = 16 * t + 4 * lg + r;
        if (i < n - 1 && ls < 15 && k < H && j <= i) v = W1[(int64_t)k * n + j];
      } else {
        const int u = 4 * lg + r, ip = 16 * t + ls;
        if (ip < n && ip > i) {
          if (u == 15) {
            v = W0[(int64_t)ip * n + i];
          } else {
            const int k = i + (n - 1) * u;
            if (i < n - 1 && k < H) v = W2[(int64_t)ip * Hs + k];
          }
        }
      }
    } else if (idx < 2 * sa + sb) {
      const int64_t e = idx - 2 * sa;
      const int r = (int)(e & 3), lane = (int)((e >> 2) & 63), i = (int)(e >> 8);
      const int u = 4 * (lane >> 4) + r, k = i + (n - 1) * u;
      if (i < n - 1 && u < 15 && k < H) v = b1[k];
    } else {
      const int64_t e = idx - 2 * sa - sb;
      const int r = (int)(e & 3), lane = (int)((e >> 2) & 63), t = (int)(e >> 8);
      const int pos = 16 * t + 4 * (lane >> 4) + r;
      if (pos < n) v = b2[pos];
    }
    P[idx] = v;
  }
}

// Parameter i of an instance (flat index into W1, b1, W2, b2, W0) written
// into every slot of the packed tables that made_pack_kernel fills from it:
// the inverse of that kernel's gather.  Slots it leaves zero never hold a
// parameter, so after one full pack these writes keep the tables equal to a
// fresh pack of the current parameters.
__device__ inline void pack_scatter(float *P, int n, int Hs, int npt, int64_t i, float v) {
  const int H = n >= 2 ? Hs : 0;
  const int64_t hn = (int64_t)Hs * n, sa = (int64_t)n * npt * 256, sb = (int64_t)n * 256;
  const int64_t tsamp = msample_floats(n, npt);
  // slot r of lane l in position tile t of step i0
  auto at = [&](int i0, int t, int l, int r) { return (((int64_t)i0 * npt + t) * 64 + l) * 4 + r; };
  if (i < hn) {                          // W1[k][j], j below the degree of k
    const int k = (int)(i / n), j = (int)(i % n);
    if (k >= H) return;
    const int i0 = k % (n - 1), u = k / (n - 1);
    if (j > i0) return;
    P[tsamp + hn + i] = v;               // W1m
    if (u < 15) P[at(i0, j >> 4, 16 * ((j & 15) >> 2) + u, j & 3)] = v;   // PA
    return;
  }
  i -= hn;
  if (i < Hs) {                          // b1[k]: one slot per sample lane
    const int k = (int)i;
    if (k >= H) return;
    const int i0 = k % (n - 1), u = k / (n - 1);
    if (u >= 15) return;
    for (int ls = 0; ls < 16; ++ls) P[2 * sa + ((int64_t)i0 * 64 + 16 * (u >> 2) + ls) * 4 + (u & 3)] = v;
    return;
  }
  i -= Hs;
  if (i < hn) {                          // W2[pos][k], pos above the degree of k
    const int pos = (int)(i / Hs), k = (int)(i % Hs);
    if (k >= H) return;
    const int i0 = k % (n - 1), u = k / (n - 1);
    if (pos <= i0) return;
    P[tsamp + (int64_t)k * n + pos] = v;     // W2T
    P[tsamp + 2 * hn + i] = v;               // W2m
    if (u < 15) P[sa + at(i0, pos >> 4, 16 * (u >> 2) + (pos & 15), u & 3)] = v;   // PZ
    return;
  }
  i -= hn;
  if (i < n) {                           // b2[pos]: one slot per sample lane
    const int pos = (int)i;
    for (int ls = 0; ls < 16; ++ls)
      P[2 * sa + sb + ((int64_t)(pos >> 4) * 64 + 16 * ((pos & 15) >> 2) + ls) * 4 + (pos & 3)] = v;
    return;
  }
  i -= n;                                // W0[ip][i0], ip > i0: PZ slot 15
  const int ip = (int)(i / n), i0 = (int)(i % n);
  if (ip <= i0) return;
  P[sa + at(i0, ip >> 4, 48 + (ip & 15), 3)] = v;
}

template <int NPT, bool kU>
__global__ __launch_bounds__(256) void msample_kernel(MSampleArgs a) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, ls = lane & 15, lg = lane >> 4;
  const int task = blockIdx.x * 4 + wave;
  if (task >= a.n_tasks) return;
  const int q = a.task_inst[task];
  const MadeInst mi = a.mi[q];
  const int n = mi.n;
  const int64_t b = a.task_start[task] + ls;
  const bool live = b < mi.B;
  const int64_t sa = (int64_t)n * NPT * 64;   // in f4 units
  const f4 *PA = reinterpret_cast<const f4 *>(a.pack + mi.pack_off) + lane;
  const f4 *PZ = PA + sa;
  const f4 *PB1 = PZ + sa;
  const f4 *PB2 = PB1 + (int64_t)n * 64;
  const uint32_t step = a.step_ctr ? (uint32_t)a.step_ctr[q] : 0u;
  f4 z[NPT];
  float sp[NPT][4];
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    z[t] = PB2[t * 64];
#pragma unroll
    for (int r = 0; r < 4; ++r) sp[t][r] = 0.f;
  }
  float lq = 0.f;
  uint32_t pw[4] = {0u, 0u, 0u, 0u};
  const float *u = kU ? a.uniforms + mi.spin_off + (live ? b : 0) * n : nullptr;
  // lanes past the batch end read row 0 (in bounds) and ignore it
  float pu = kU ? u[0] : 0.5f, qu = 0.5f;
  f4 pa[NPT], pz[NPT], pb;
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    pa[t] = PA[t * 64];
    pz[t] = PZ[t * 64];
  }
  pb = PB1[0];
  f4 qa[NPT], qz[NPT], qb;
  // one autoregressive position: logit z_i from the lanes that hold it,
  // spin, log q, then the hidden units of degree i + 1 and every later
  // logit; the operands of position i + 1 are loaded meanwhile into the
  // other register set (R = i mod 4 is static after the unroll by four)
  auto position = [&](const int i, auto TC, auto RC, const f4 (&ca)[NPT], const f4 (&cz)[NPT],
                      const f4 &cb, const float cu, f4 (&na)[NPT], f4 (&nz)[NPT], f4 &nb, float &nu) {
    constexpr int ti = decltype(TC)::value, ri = decltype(RC)::value;
    // unconditional (the last position reloads itself), so that the wait
    // for this position's operands can leave the new loads in flight
    const int nx = i + 1 < n ? i + 1 : i;
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
      na[t] = PA[((int64_t)nx * NPT + t) * 64];
      nz[t] = PZ[((int64_t)nx * NPT + t) * 64];
    }
    nb = PB1[(int64_t)nx * 64];
    if (kU) nu = u[nx];
    const int gi = (i >> 2) & 3;
    // hidden pre-activations of the units of degree i + 1: every product
    // that does not hold the new spin is issued before the spin is drawn
    f4 acc = cb;
#pragma unroll
    for (int t = 0; t < NPT; ++t)
      if (t <= ti)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (t != ti || r != ri)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[t][r], sp[t][r], acc, 0, 0, 0);
    float own = z[0][ri];
#pragma unroll
    for (int t = 1; t < NPT; ++t)
      if (t == ti) own = z[t][ri];
    // broadcast from row gi: the other rows add zeros (exact)
    const float zi = rows4_sum(lg == gi ? own : 0.f);
    float ui;
    if (kU) {
      ui = live ? cu : 0.5f;
    } else {
      if (ri == 0) {
        pw[0] = (uint32_t)(i >> 2); pw[1] = (uint32_t)b; pw[2] = step; pw[3] = (uint32_t)q;
        philox4x32_10(pw, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
      }
      ui = (float)(pw[ri] >> 8) * 5.9604644775390625e-08f;
    }
    const float p = fsigmoid(zi);
    const float si = ui < p ? 1.f : -1.f;
    lq += flogsigmoid(si * zi);
    const bool mine = lg == gi;
#pragma unroll
    for (int t = 0; t < NPT; ++t)
      if (t == ti) sp[t][ri] = mine ? si : sp[t][ri];
    // the product holding the new spin (slot ri of tile ti), last
#pragma unroll
    for (int t = 0; t < NPT; ++t)
      if (t == ti) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ca[t][ri], sp[t][ri], acc, 0, 0, 0);
    float h[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = ftanh(acc[r]);
    if (lg == 3) h[3] = si;
    // later logits only: tiles before ti hold positions already drawn
#pragma unroll
    for (int t = 0; t < NPT; ++t)
      if (t >= ti)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          z[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(cz[t][r], h[r], z[t], 0, 0, 0);
  };
  // tile by tile (the tile index static), four positions at a time with no
  // branch between them: a branch between positions makes the compiler wait
  // for every load in flight, the next position's operands included
  auto tile = [&](auto TC) {
    constexpr int t = decltype(TC)::value;
    using R0 = std::integral_constant<int, 0>;
    using R1 = std::integral_constant<int, 1>;
    using R2 = std::integral_constant<int, 2>;
    using R3 = std::integral_constant<int, 3>;
    const int end = n < 16 * t + 16 ? n : 16 * t + 16;
    int i = 16 * t;
    for (; i + 4 <= end; i += 4) {
      position(i, TC, R0{}, pa, pz, pb, pu, qa, qz, qb, qu);
      position(i + 1, TC, R1{}, qa, qz, qb, qu, pa, pz, pb, pu);
      position(i + 2, TC, R2{}, pa, pz, pb, pu, qa, qz, qb, qu);
      position(i + 3, TC, R3{}, qa, qz, qb, qu, pa, pz, pb, pu);
    }
    if (i < end) {
      position(i, TC, R0{}, pa, pz, pb, pu, qa, qz, qb, qu);
      if (i + 1 < end) position(i + 1, TC, R1{}, qa, qz, qb, qu, pa, pz, pb, pu);
      if (i + 2 < end) position(i + 2, TC, R2{}, pa, pz, pb, pu, qa, qz, qb, qu);
    }
  };
  tile(std::integral_constant<int, 0>{});
  if (NPT > 1) tile(std::integral_constant<int, (NPT > 1 ? 1 : 0)>{});
  if (NPT > 2) tile(std::integral_constant<int, (NPT > 2 ? 2 : 0)>{});
  if (NPT > 3) tile(std::integral_constant<int, (NPT > 3 ? 3 : 0)>{});
  if (live) {
    int8_t *so = a.spins + mi.spin_off + b * n;
#pragma unroll
    for (int t = 0; t < NPT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pos = 16 * t + 4 * lg + r;
        if (pos < n) so[pos] = (int8_t)(sp[t][r] > 0.f ? 1 : -1);
      }
    if (lg == 0) a.logq[mi.sample_off + b] = lq;
  }
}

// ---------------------------------------------------------------------------
// Fused REINFORCE backward through q (Eq. 10), FP32 on the matrix cores.
// A workgroup of 4 waves takes 64 samples of one instance.  Each wave first
// computes the rows of its 16 samples in R-layout: a = b1 + W1m s, h = tanh a,
// logits z = b2 + W2m h + W0m s and dlogit = w ((1 + s)/2 - sigmoid z) with
// w = (f_b - F_q) / B, keeping h in registers and writing dlogit and s
// sample-major into LDS.  The hidden units are then taken in passes of
// kMgPass tiles: each wave forms dh = W2m^T dlogit and da = dh (1 - h^2) for
// the pass's tiles and stages h and da sample-major; after a barrier the
// gradient blocks of the pass are products over the 64 samples, each wave
// owning a share of the 16x16 output tiles:  gW2 = dlogit^T h,  gW1 = da^T s
// (and once gW0 = dlogit^T s); the bias gradients are column sums.  Staging a
// pass at a time keeps the LDS of a workgroup small enough for two per CU.
// The workgroup writes its masked partial gradient as one row; mgrad_reduce
// sums the rows of an instance in a fixed order.
constexpr int kMgTiles = 16;    // hidden tiles (H <= 256)
// sched_barrier mask: every instruction kind but vector-memory reads may be
// scheduled across it
constexpr int kNoVmemRead = 0x0001 | 0x0002 | 0x0004 | 0x0008 | 0x0040 | 0x0080 | 0x0400;
constexpr int kMgPass = 4;      // hidden tiles staged per pass

struct MgLayout {
  int ldq, ldn;
  size_t hid, da, dl, sf, end;
};
__host__ __device__ inline MgLayout mg_layout(int npt) {
  MgLayout L;
  L.ldq = 16 * kMgPass + 4;
  L.ldn = 16 * npt + 4;
  L.hid = 0;
  L.da = L.hid + (size_t)64 * L.ldq * 4;
  L.dl = L.da + (size_t)64 * L.ldq * 4;
  L.sf = L.dl + (size_t)64 * L.ldn * 4;
  L.end = L.sf + (size_t)64 * L.ldn * 4;
  return L;
}
// bytes: staged rows plus the degree table (16 * tiles ints)
__host__ __device__ inline size_t mg_bytes(int H, int npt) {
  const int ht = (H + 15) / 16 > 0 ? (H + 15) / 16 : 1;
  return mg_layout(npt).end + (size_t)16 * ht * 4;
}

template <int NPT, int HT>
__global__ __launch_bounds__(256, 2) void mgrad_kernel(MGradArgs a) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int QT = HT < kMgPass ? HT : kMgPass;   // hidden tiles per pass
  constexpr int BM = 4;
  constexpr int B1 = HT < BM ? HT : BM;             // tiles per batch of weight loads
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, ls = lane & 15, lg = lane >> 4;
  const int q = a.task_inst[blockIdx.x];
  const MadeInst mi = a.mi[q];
  const int n = mi.n, Hs = mi.H, H = n >= 2 ? mi.H : 0;
  // HT tiles of 16 hidden units cover the widest instance of the launch;
  // units past an instance's H read as zero
  const int64_t bw = a.task_start[blockIdx.x];
  // F_q from the free-energy kernel's block sums, added in block order (the
  // same value in every workgroup); the instance's first workgroup also
  // writes the step statistics
  // (a fixed order over at most 256 blocks and a fixed tree down to lane 0,
  // then a broadcast)
  double Fq;
  {
    const double *fp = a.fpart + (int64_t)q * 4 * a.fnblk;
    auto bsum = [&](int c) {
      // lane k holds blocks k, k + 64, ... (in that order)
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 256; k += 64) {
        const double x = fp[c * a.fnblk + (lane + k < a.fnblk ? lane + k : 0)];
        v += lane + k < a.fnblk ? x : 0.0;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      return __shfl(v, 0, 64);
    };
    const double s0 = bsum(0);
    Fq = s0 / (double)mi.B;
    if (bw == 0 && wave == 0) {
      const double sm[4] = {s0, bsum(1), bsum(2), bsum(3)};
      if (lane == 0) free_stats(sm, mi.B, a.stats + 4 * q);
    }
  }
  const MgLayout Lm = mg_layout(NPT);
  float *hid = reinterpret_cast<float *>(smem + Lm.hid);
  float *dab = reinterpret_cast<float *>(smem + Lm.da);
  float *dlb = reinterpret_cast<float *>(smem + Lm.dl);
  float *sfb = reinterpret_cast<float *>(smem + Lm.sf);
  int32_t *deg = reinterpret_cast<int32_t *>(smem + Lm.end);
  const float *W1 = a.params + mi.param_off, *b1 = W1 + (int64_t)Hs * n, *W2 = b1 + Hs,
              *b2 = W2 + (int64_t)n * Hs, *W0 = b2 + n;
  const float *W2T = a.pack + mi.pack_off + msample_floats(n, NPT);
  const float *W1m = W2T + (int64_t)Hs * n, *W2m = W1m + (int64_t)Hs * n;
  const int nm1 = n > 1 ? n - 1 : 1;
  // four consecutive parameters p[0..3], zero unless ok; the load itself is
  // unconditional (from the array base when !ok, the buffers are padded),
  // because a load under a lane condition is waited for at its branch join
  auto ld4 = [](const float *base, const float *p, bool ok) {
    const f4 v = *reinterpret_cast<const f4 *>(ok ? p : base);
    return ok ? v : f4{0.f, 0.f, 0.f, 0.f};
  };
  // rows of the wave's 16 samples; every load below is unconditional, at an
  // in-bounds address, so that the loads of a stage are all in flight
  // together (a conditional load is waited for at its branch join)
  const int64_t sb = bw + 16 * wave + ls;
  const bool valid = sb < mi.B;
  const int8_t *spn = a.spins + mi.spin_off + (valid ? sb : 0) * n;   // row 0 past the batch
  float sp[NPT][4];
  if ((n & 3) == 0 && (reinterpret_cast<uintptr_t>(a.spins + mi.spin_off) & 3) == 0) {
    uint32_t wv[NPT];
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
      const int p0 = 16 * t + 4 * lg;
      wv[t] = *reinterpret_cast<const uint32_t *>(spn + (p0 < n ? p0 : 0));
    }
#pragma unroll
    for (int t = 0; t < NPT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pos = 16 * t + 4 * lg + r;
        sp[t][r] = (valid && pos < n) ? (float)(int8_t)(wv[t] >> (8 * r)) : 0.f;
      }
  } else {
    int8_t bv[NPT][4];
#pragma unroll
    for (int t = 0; t < NPT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pos = 16 * t + 4 * lg + r;
        bv[t][r] = spn[pos < n ? pos : 0];
      }
#pragma unroll
    for (int t = 0; t < NPT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pos = 16 * t + 4 * lg + r;
        sp[t][r] = (valid && pos < n) ? (float)bv[t][r] : 0.f;
      }
  }
  const float wt = valid ? (float)((a.f[mi.sample_off + sb] - Fq) / (double)mi.B) : 0.f;
  float h[HT][4];
#pragma unroll
  for (int h0 = 0; h0 < HT; h0 += B1) {
    f4 wl[B1][NPT], bl[B1];
#pragma unroll
    for (int j = 0; j < B1; ++j) {
      const int ka = 16 * (h0 + j) + ls;
#pragma unroll
      for (int t = 0; t < NPT; ++t)
        wl[j][t] = ld4(W1m, W1m + (int64_t)ka * n + 16 * t + 4 * lg, ka < H && 16 * t + 4 * lg < n);
      bl[j] = ld4(b1, b1 + 16 * (h0 + j) + 4 * lg, 16 * (h0 + j) + 4 * lg < H);
    }
    // the batch's loads stay together ahead of its products (the scheduler
    // would otherwise sink each next to its use, one round trip per tile)
    __builtin_amdgcn_sched_barrier(kNoVmemRead);
#pragma unroll
    for (int j = 0; j < B1; ++j) {
      const int ht = h0 + j;
      f4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 16 * ht + 4 * lg + r;
        acc[r] = k < H ? bl[j][r] : 0.f;
      }
#pragma unroll
      for (int t = 0; t < NPT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wl[j][t][r], sp[t][r], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) h[ht][r] = (16 * ht + 4 * lg + r < H) ? ftanh(acc[r]) : 0.f;
    }
  }
  // logits: the NPT position tiles as independent product chains, their
  // weights loaded in batches of B1 hidden tiles
  f4 z[NPT];
  {
    f4 w0[NPT][NPT], bz[NPT];
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      const int pa = 16 * pt + ls;
      bz[pt] = ld4(b2, b2 + 16 * pt + 4 * lg, 16 * pt + 4 * lg < n);
#pragma unroll
      for (int t = 0; t < NPT; ++t)
        w0[pt][t] = ld4(W0, W0 + (int64_t)pa * n + 16 * t + 4 * lg, pa < n && 16 * t + 4 * lg < n);
    }
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt)
#pragma unroll
      for (int r = 0; r < 4; ++r) z[pt][r] = 16 * pt + 4 * lg + r < n ? bz[pt][r] : 0.f;
#pragma unroll
    for (int h0 = 0; h0 < HT; h0 += B1) {
      f4 wz[NPT][B1];
#pragma unroll
      for (int pt = 0; pt < NPT; ++pt) {
        const int pa = 16 * pt + ls;
#pragma unroll
        for (int j = 0; j < B1; ++j)
          wz[pt][j] = ld4(W2m, W2m + (int64_t)pa * Hs + 16 * (h0 + j) + 4 * lg, pa < n && 16 * (h0 + j) + 4 * lg < H);
      }
      __builtin_amdgcn_sched_barrier(kNoVmemRead);
#pragma unroll
      for (int j = 0; j < B1; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int pt = 0; pt < NPT; ++pt)
            z[pt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wz[pt][j][r], h[h0 + j][r], z[pt], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NPT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int pt = 0; pt < NPT; ++pt) {
          const int j = 16 * t + 4 * lg + r, pa = 16 * pt + ls;
          const float wv = j < pa ? w0[pt][t][r] : 0.f;
          z[pt] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv, sp[t][r], z[pt], 0, 0, 0);
        }
  }
  float dl[NPT][4];
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pos = 16 * pt + 4 * lg + r;
      const float s1 = sp[pt][r];
      dl[pt][r] = pos < n ? wt * ((1.f + s1) * 0.5f - fsigmoid(z[pt][r])) : 0.f;
    }
  const int srow = 16 * wave + ls;
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt) {
    *reinterpret_cast<f4 *>(dlb + srow * Lm.ldn + 16 * pt + 4 * lg) =
        f4{dl[pt][0], dl[pt][1], dl[pt][2], dl[pt][3]};
    *reinterpret_cast<f4 *>(sfb + srow * Lm.ldn + 16 * pt + 4 * lg) =
        f4{sp[pt][0], sp[pt][1], sp[pt][2], sp[pt][3]};
  }
  // hidden-unit degrees for the output masks
  for (int k = threadIdx.x; k < 16 * HT; k += blockDim.x) deg[k] = k < H ? 1 + k % nm1 : 1 << 30;
  float *prow = a.part + (int64_t)blockIdx.x * a.pstride;
  const int64_t o_b1 = (int64_t)Hs * n, o_W2 = o_b1 + Hs, o_b2 = o_W2 + (int64_t)n * Hs,
                o_W0 = o_b2 + n;
#pragma unroll
  for (int pass = 0; pass < HT / QT; ++pass) {
    const int hbase = 16 * QT * pass;   // first hidden unit of the pass
    {
      f4 wt2[QT][NPT];
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        const int ka = hbase + 16 * j + ls;
#pragma unroll
        for (int pt = 0; pt < NPT; ++pt)
          wt2[j][pt] = ld4(W2T, W2T + (int64_t)ka * n + 16 * pt + 4 * lg, ka < H && 16 * pt + 4 * lg < n);
      }
      __builtin_amdgcn_sched_barrier(kNoVmemRead);
      if (pass > 0) __syncthreads();   // the previous pass's products are done
#pragma unroll
      for (int j = 0; j < QT; ++j) {
        f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int pt = 0; pt < NPT; ++pt)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(wt2[j][pt][r], dl[pt][r], acc, 0, 0, 0);
        const float *hv = h[QT * pass + j];
        *reinterpret_cast<f4 *>(hid + srow * Lm.ldq + 16 * j + 4 * lg) = f4{hv[0], hv[1], hv[2], hv[3]};
        f4 dv;
#pragma unroll
        for (int r = 0; r < 4; ++r) dv[r] = acc[r] * (1.f - hv[r] * hv[r]);
        *reinterpret_cast<f4 *>(dab + srow * Lm.ldq + 16 * j + 4 * lg) = dv;
      }
    }
    __syncthreads();
    // tiles of the pass: NPT*QT of gW2 (pt, j), QT*NPT of gW1 (j, jt), and
    // in the first pass NPT*NPT of gW0 (pt, jt); wave w takes w, w + 4, ...
    constexpr int n2 = NPT * QT, n1 = QT * NPT;
    const int ntile = n2 + n1 + (pass == 0 ? NPT * NPT : 0);
    for (int tile = wave; tile < ntile; tile += 4) {
      const float *Ab, *Bb;
      int lda, ldb, ai, bj, kind;
      if (tile < n2) {
        kind = 2;
        const int pt = tile / QT, j = tile % QT;
        Ab = dlb; lda = Lm.ldn; ai = 16 * pt;
        Bb = hid; ldb = Lm.ldq; bj = 16 * j;
      } else if (tile < n2 + n1) {
        kind = 1;
        const int e = tile - n2, j = e / NPT, jt = e % NPT;
        Ab = dab; lda = Lm.ldq; ai = 16 * j;
        Bb = sfb; ldb = Lm.ldn; bj = 16 * jt;
      } else {
        kind = 0;
        const int e = tile - n2 - n1, pt = e / NPT, jt = e % NPT;
        Ab = dlb; lda = Lm.ldn; ai = 16 * pt;
        Bb = sfb; ldb = Lm.ldn; bj = 16 * jt;
      }
      // two accumulators (even and odd sample chunks) halve the dependent chain
      f4 acc2[2] = {f4{0.f, 0.f, 0.f, 0.f}, f4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int kc = 0; kc < 16; ++kc) {
        const int s = 4 * kc + lg;
        acc2[kc & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(Ab[s * lda + ai + ls], Bb[s * ldb + bj + ls],
                                                            acc2[kc & 1], 0, 0, 0);
      }
      const f4 acc = acc2[0] + acc2[1];
      // lane holds rows ai + 4 lg + r, column bj + ls of the staged blocks
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ai + 4 * lg + r, col = bj + ls;
        if (kind == 2) {         // gW2[pos][k]: deg(k) <= pos
          const int k = hbase + col;
          if (row < n && k < Hs)
            prow[o_W2 + (int64_t)row * Hs + k] = deg[k] <= row ? acc[r] : 0.f;
        } else if (kind == 1) {  // gW1[k][j]: j < deg(k)
          const int k = hbase + row;
          if (k < Hs && col < n) prow[(int64_t)k * n + col] = col < deg[k] ? acc[r] : 0.f;
        } else {                 // gW0[pos][j]: j < pos
          if (row < n && col < n) prow[o_W0 + (int64_t)row * n + col] = col < row ? acc[r] : 0.f;
        }
      }
    }
    // bias gradients of the pass: column sums over the 64 samples
    for (int k = threadIdx.x; k < 16 * QT; k += blockDim.x) {
      const int kk = hbase + k;
      if (kk >= Hs) continue;
      float acc = 0.f;
      if (kk < H)
        for (int s = 0; s < 64; ++s) acc += dab[s * Lm.ldq + k];
      prow[o_b1 + kk] = acc;
    }
    if (pass == 0)
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        float acc = 0.f;
        for (int s = 0; s < 64; ++s) acc += dlb[s * Lm.ldn + i];
        prow[o_b2 + i] = acc;
      }
  }
}

// ---------------------------------------------------------------------------
// The same fused REINFORCE backward with split-BF16 products (the nets made
// with TNVAN_FLAG_SPLIT_BF16).  Every product is formed on the BF16
// 16x16x32 matrix cores from split operands: x = x_hi + x_lo, each part
// rounded to BF16, and x y ~ x_hi y_hi + x_hi y_lo + x_lo y_hi with FP32
// accumulation; spins are exact in BF16, so products with them take two.
// A lane's K chunk c holds, in element j, index 16 (2c + j/4) + 4 (l >> 4) +
// j % 4 of the contracted dimension, so R-layout registers (spins, h, dlogit)
// are B operands as they are.  A workgroup takes kMg3W waves of 16 samples.
// It stages the first-layer and logit weights once, every load issued
// together, split and in operand order in LDS (one 16-byte read per lane and
// chunk); each backward pass's W2m^T slice is loaded one pass ahead.  The
// gradient blocks contract over the workgroup's samples from operands staged
// feature-major in LDS as BF16 hi and lo rows, eight samples per lane in one
// 16-byte read.  The bias gradients are FP32 sums of the registers (16
// samples per wave, then the waves in order).
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef unsigned int u4w __attribute__((ext_vector_type(4)));
typedef float f4v_t __attribute__((ext_vector_type(4)));
constexpr int kMg3W = 8;        // waves (16 samples each) per workgroup

// LDS of mgrad3_kernel.  The network phase holds the first-layer and logit
// weights, split, in operand order (16 bytes per lane and chunk); the
// backward passes reuse that space for the W2m^T slices of two passes and
// the staged rows.  The degree table follows both.
struct Mg3Layout {
  size_t a1, a2, b1s;                       // network phase
  size_t wt, dlh, dll, st, hh, hl, dah, dal, b2p, b1p;   // backward passes
  size_t deg, end;
};
__host__ __device__ inline Mg3Layout mg3_layout(int npt, int ht, int nw) {
  Mg3Layout L;
  const int nc = (npt + 1) / 2, nch = (ht + 1) / 2, qt = ht < kMgPass ? ht : kMgPass;
  const int kk = 16 * nw + 8;
  size_t o = 0;
  L.a1 = o; o += (size_t)2 * ht * nc * 64 * 16;
  L.a2 = o; o += (size_t)2 * npt * nch * 64 * 16;
  L.b1s = o; o += (size_t)16 * ht * 4;
  const size_t net = o;
  const size_t rp = (size_t)16 * npt * kk * 2, rq = (size_t)16 * qt * kk * 2;
  o = 0;
  L.wt = o; o += (size_t)2 * 2 * qt * nc * 64 * 16;
  L.dlh = o; o += rp;
  L.dll = o; o += rp;
  L.st = o; o += rp;
  L.hh = o; o += rq;
  L.hl = o; o += rq;
  L.dah = o; o += rq;
  L.dal = o; o += rq;
  L.b2p = o; o += (size_t)nw * 16 * npt * 4;
  L.b1p = o; o += (size_t)nw * 16 * qt * 4;
  L.deg = o > net ? o : net;
  L.end = L.deg + (size_t)16 * (ht > 0 ? ht : 1) * 4;
  return L;
}

__device__ inline f4v_t mfma_b(bf8v a, bf8v b, f4v_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// chunk c of R-layout registers x[t][r] (t < NT; zero past NT), split
template <int NT>
__device__ inline void split_c(const float (&x)[NT][4], int c, bf8v &h, bf8v &l) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int t = 2 * c + (j >> 2);
    const float v = t < NT ? x[t < NT ? t : 0][j & 3] : 0.f;
    h[j] = (__bf16)v;
    l[j] = (__bf16)(v - (float)h[j]);
  }
}
// chunk c of R-layout spins (exact in BF16)
template <int NT>
__device__ inline bf8v spin_c(const float (&x)[NT][4], int c) {
  bf8v h;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int t = 2 * c + (j >> 2);
    h[j] = (__bf16)(t < NT ? x[t < NT ? t : 0][j & 3] : 0.f);
  }
  return h;
}

template <int NPT, int HT>
__global__ __launch_bounds__(64 * kMg3W, 8 / kMg3W) void mgrad3_kernel(MGradArgs a) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int NW = kMg3W, NT = 64 * NW;            // waves, threads
  constexpr int KS = 16 * NW + 8;                   // BF16 per staged row (samples + bank spread)
  constexpr int QT = HT < kMgPass ? HT : kMgPass;   // hidden tiles per pass
  constexpr int NC = (NPT + 1) / 2;                 // K chunks over positions
  constexpr int NCH = (HT + 1) / 2;                 // K chunks over hidden units
  constexpr int G1 = (HT * NC * 64 + NT - 1) / NT;    // first-layer operand groups per thread
  constexpr int G2 = (NPT * NCH * 64 + NT - 1) / NT;  // logit operand groups per thread
  constexpr int GT = (QT * NC * 64 + NT - 1) / NT;    // W2m^T operand groups per thread
  extern __shared__ __align__(16) char smem[];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane((int)(tid >> 6));
  const int lane = tid & 63, ls = lane & 15, lg = lane >> 4;
  const int q = a.task_inst[blockIdx.x];
  const MadeInst mi = a.mi[q];
  const int n = mi.n, Hs = mi.H, H = n >= 2 ? mi.H : 0;
  const int64_t bw = a.task_start[blockIdx.x];
  const Mg3Layout Lm = mg3_layout(NPT, HT, NW);
  u4w *A1 = reinterpret_cast<u4w *>(smem + Lm.a1);   // [hi, lo][HT][NC][64]
  u4w *A2 = reinterpret_cast<u4w *>(smem + Lm.a2);   // [hi, lo][NPT][NCH][64]
  float *b1s = reinterpret_cast<float *>(smem + Lm.b1s);
  u4w *WT = reinterpret_cast<u4w *>(smem + Lm.wt);   // [buffer][hi, lo][QT][NC][64]
  __bf16 *dlh = reinterpret_cast<__bf16 *>(smem + Lm.dlh), *dll = reinterpret_cast<__bf16 *>(smem + Lm.dll);
  __bf16 *sT = reinterpret_cast<__bf16 *>(smem + Lm.st);
  __bf16 *hh = reinterpret_cast<__bf16 *>(smem + Lm.hh), *hl = reinterpret_cast<__bf16 *>(smem + Lm.hl);
  __bf16 *dah = reinterpret_cast<__bf16 *>(smem + Lm.dah), *dal = reinterpret_cast<__bf16 *>(smem + Lm.dal);
  float *b2p = reinterpret_cast<float *>(smem + Lm.b2p), *b1p = reinterpret_cast<float *>(smem + Lm.b1p);
  int32_t *deg = reinterpret_cast<int32_t *>(smem + Lm.deg);
  const float *W1 = a.params + mi.param_off, *b1 = W1 + (int64_t)Hs * n, *W2 = b1 + Hs,
              *b2 = W2 + (int64_t)n * Hs, *W0 = b2 + n;
  const float *W2T = a.pack + mi.pack_off + msample_floats(n, NPT);
  const float *W1m = W2T + (int64_t)Hs * n, *W2m = W1m + (int64_t)Hs * n;
  const int nm1 = n > 1 ? n - 1 : 1;
  auto ld4 = [](const float *base, const float *p, bool ok) {
    const f4 v = *reinterpret_cast<const f4 *>(ok ? p : base);
    return ok ? v : f4{0.f, 0.f, 0.f, 0.f};
  };
  // 8 values (two f4) split into BF16 hi and lo, as two 16-byte words
  auto split8 = [](const f4 &x0, const f4 &x1, u4w &hi, u4w &lo) {
    bf8v h, l;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v = j < 4 ? x0[j] : x1[j - 4];
      h[j] = (__bf16)v;
      l[j] = (__bf16)(v - (float)h[j]);
    }
    hi = __builtin_bit_cast(u4w, h);
    lo = __builtin_bit_cast(u4w, l);
  };
  auto as8 = [](const u4w &v) { return __builtin_bit_cast(bf8v, v); };

  // -- the network's weights, staged once per workgroup: every load first --
  // operand group (tile, chunk c, lane l): row 16 tile + (l & 15), elements
  // 16 (2c + j/4) + 4 (l >> 4) + j % 4 of the contracted dimension
  f4 x1[G1][2], x2[G2][2], xb;
#pragma unroll
  for (int i = 0; i < G1; ++i) {
    const int g = tid + NT * i;
    const int ht = g / (NC * 64), c = (g / 64) % NC, l = g % 64;
    const int row = 16 * ht + (l & 15);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int k = 16 * (2 * c + e) + 4 * (l >> 4);
      x1[i][e] = ld4(W1m, W1m + (int64_t)row * n + k, g < HT * NC * 64 && row < H && 2 * c + e < NPT && k < n);
    }
  }
#pragma unroll
  for (int i = 0; i < G2; ++i) {
    const int g = tid + NT * i;
    const int pt = g / (NCH * 64), c = (g / 64) % NCH, l = g % 64;
    const int row = 16 * pt + (l & 15);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int k = 16 * (2 * c + e) + 4 * (l >> 4);
      x2[i][e] = ld4(W2m, W2m + (int64_t)row * Hs + k, g < NPT * NCH * 64 && row < n && 2 * c + e < HT && k < H);
    }
  }
  xb = ld4(b1, b1 + 4 * tid, 4 * tid < H && 4 * tid < 16 * HT);
  // this wave's samples: spins, the direct and bias terms of the logits
  const int64_t sb = bw + 16 * wave + ls;
  const bool valid = sb < mi.B;
  const int8_t *spn = a.spins + mi.spin_off + (valid ? sb : 0) * n;
  uint32_t wv[NPT];
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int p0 = 16 * t + 4 * lg;
    wv[t] = *reinterpret_cast<const uint32_t *>(spn + (p0 < n ? p0 : 0));
  }
  f4 w0[NPT][2 * NC], bz[NPT];
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt) {
    const int pa = 16 * pt + ls;
    bz[pt] = ld4(b2, b2 + 16 * pt + 4 * lg, 16 * pt + 4 * lg < n);
#pragma unroll
    for (int t = 0; t < 2 * NC; ++t)
      w0[pt][t] = t < NPT ? ld4(W0, W0 + (int64_t)pa * n + 16 * t + 4 * lg, pa < n && 16 * t + 4 * lg < n)
                          : f4{0.f, 0.f, 0.f, 0.f};
  }
  const double fv = a.f[mi.sample_off + (valid ? sb : 0)];
  // F_q from the free-energy kernel's block sums (as mgrad_kernel)
  double Fq;
  {
    const double *fp = a.fpart + (int64_t)q * 4 * a.fnblk;
    auto bsum = [&](int c) {
      // lane k holds blocks k, k + 64, ... (in that order)
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 256; k += 64) {
        const double x = fp[c * a.fnblk + (lane + k < a.fnblk ? lane + k : 0)];
        v += lane + k < a.fnblk ? x : 0.0;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      return __shfl(v, 0, 64);
    };
    const double s0 = bsum(0);
    Fq = s0 / (double)mi.B;
    if (bw == 0 && wave == 0) {
      const double sm[4] = {s0, bsum(1), bsum(2), bsum(3)};
      if (lane == 0) free_stats(sm, mi.B, a.stats + 4 * q);
    }
  }
#pragma unroll
  for (int i = 0; i < G1; ++i) {
    const int g = tid + NT * i;
    if (g < HT * NC * 64) split8(x1[i][0], x1[i][1], A1[g], A1[HT * NC * 64 + g]);
  }
#pragma unroll
  for (int i = 0; i < G2; ++i) {
    const int g = tid + NT * i;
    if (g < NPT * NCH * 64) split8(x2[i][0], x2[i][1], A2[g], A2[NPT * NCH * 64 + g]);
  }
  if (4 * tid < 16 * HT) *reinterpret_cast<f4 *>(b1s + 4 * tid) = xb;
  for (int k = tid; k < 16 * HT; k += blockDim.x) deg[k] = k < H ? 1 + k % nm1 : 1 << 30;
  float sp[NPT][4];
#pragma unroll
  for (int t = 0; t < NPT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pos = 16 * t + 4 * lg + r;
      sp[t][r] = (valid && pos < n) ? (float)(int8_t)(wv[t] >> (8 * r)) : 0.f;
    }
  bf8v sc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) sc[c] = spin_c<NPT>(sp, c);
  const float wt = valid ? (float)((fv - Fq) / (double)mi.B) : 0.f;
  __syncthreads();

  // hidden layer: h = tanh(b1 + W1m s), R-layout, 16 units per tile
  float h[HT][4];
#pragma unroll
  for (int ht = 0; ht < HT; ++ht) {
    const f4 bl = *reinterpret_cast<const f4 *>(b1s + 16 * ht + 4 * lg);
    f4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = 16 * ht + 4 * lg + r < H ? bl[r] : 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int g = (ht * NC + c) * 64 + lane;
      acc = mfma_b(as8(A1[g]), sc[c], acc);
      acc = mfma_b(as8(A1[HT * NC * 64 + g]), sc[c], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) h[ht][r] = (16 * ht + 4 * lg + r < H) ? ftanh(acc[r]) : 0.f;
  }
  // logits: z = b2 + W0m s + W2m h, R-layout, 16 positions per tile
  f4 z[NPT];
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt) {
    const int pa = 16 * pt + ls;
#pragma unroll
    for (int r = 0; r < 4; ++r) z[pt][r] = 16 * pt + 4 * lg + r < n ? bz[pt][r] : 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      f4 m0, m1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {   // strictly lower
        m0[r] = 16 * (2 * c) + 4 * lg + r < pa ? w0[pt][2 * c][r] : 0.f;
        m1[r] = 16 * (2 * c + 1) + 4 * lg + r < pa ? w0[pt][2 * c + 1][r] : 0.f;
      }
      u4w hi, lo;
      split8(m0, m1, hi, lo);
      z[pt] = mfma_b(as8(hi), sc[c], z[pt]);
      z[pt] = mfma_b(as8(lo), sc[c], z[pt]);
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    bf8v hb, hs;
    split_c<HT>(h, c, hb, hs);
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
      const int g = (pt * NCH + c) * 64 + lane;
      const bf8v ah = as8(A2[g]), al = as8(A2[NPT * NCH * 64 + g]);
      z[pt] = mfma_b(ah, hb, z[pt]);
      z[pt] = mfma_b(ah, hs, z[pt]);
      z[pt] = mfma_b(al, hb, z[pt]);
    }
  }
  float dl[NPT][4];
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pos = 16 * pt + 4 * lg + r;
      const float s1 = sp[pt][r];
      dl[pt][r] = pos < n ? wt * ((1.f + s1) * 0.5f - fsigmoid(z[pt][r])) : 0.f;
    }
  bf8v dlb[NC], dls[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) split_c<NPT>(dl, c, dlb[c], dls[c]);

  // -- backward passes; W2m^T slices loaded one pass ahead --
  f4 xt[GT][2];
  auto wt_load = [&](int pass) {
#pragma unroll
    for (int i = 0; i < GT; ++i) {
      const int g = tid + NT * i;
      const int j = g / (NC * 64), c = (g / 64) % NC, l = g % 64;
      const int row = 16 * (QT * pass + j) + (l & 15);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int k = 16 * (2 * c + e) + 4 * (l >> 4);
        xt[i][e] = ld4(W2T, W2T + (int64_t)row * n + k, g < QT * NC * 64 && row < H && 2 * c + e < NPT && k < n);
      }
    }
  };
  wt_load(0);
  __syncthreads();   // the network phase's LDS is free
  // staged feature-major: dlogit (hi, lo) and the spins; the bias-2 sums of
  // the wave's 16 samples
  const int srow = 16 * wave + ls;
#pragma unroll
  for (int pt = 0; pt < NPT; ++pt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * pt + 4 * lg + r;
      const __bf16 vh = (__bf16)dl[pt][r];
      dlh[row * KS + srow] = vh;
      dll[row * KS + srow] = (__bf16)(dl[pt][r] - (float)vh);
      sT[row * KS + srow] = (__bf16)sp[pt][r];
      const float bs = row16_sum(dl[pt][r]);
      if (ls == 0) b2p[wave * 16 * NPT + row] = bs;
    }
  float *prow = a.part + (int64_t)blockIdx.x * a.pstride;
  const int64_t o_b1 = (int64_t)Hs * n, o_W2 = o_b1 + Hs, o_b2 = o_W2 + (int64_t)n * Hs,
                o_W0 = o_b2 + n;
  // one staged row chunk: 8 samples (32 c + 8 lg ...) of row r, as BF16
  auto rd = [&](const __bf16 *X, int row, int c) {
    return __builtin_bit_cast(bf8v, *reinterpret_cast<const u4w *>(X + row * KS + 32 * c + 8 * lg));
  };
#pragma unroll
  for (int pass = 0; pass < HT / QT; ++pass) {
    const int hbase = 16 * QT * pass;   // first hidden unit of the pass
    u4w *wb = WT + (pass & 1) * 2 * QT * NC * 64;
#pragma unroll
    for (int i = 0; i < GT; ++i) {
      const int g = tid + NT * i;
      if (g < QT * NC * 64) split8(xt[i][0], xt[i][1], wb[g], wb[QT * NC * 64 + g]);
    }
    if (pass + 1 < HT / QT) wt_load(pass + 1);
    __syncthreads();   // the slice is staged; the previous pass's products are done
#pragma unroll
    for (int j = 0; j < QT; ++j) {
      // dh = W2m^T dlogit, da = dh (1 - h^2)
      f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int g = (j * NC + c) * 64 + lane;
        const bf8v ah = as8(wb[g]), al = as8(wb[QT * NC * 64 + g]);
        acc = mfma_b(ah, dlb[c], acc);
        acc = mfma_b(ah, dls[c], acc);
        acc = mfma_b(al, dlb[c], acc);
      }
      const float *hv = h[QT * pass + j];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * j + 4 * lg + r;
        const float dv = acc[r] * (1.f - hv[r] * hv[r]);
        const __bf16 xh = (__bf16)hv[r], dh = (__bf16)dv;
        hh[row * KS + srow] = xh;
        hl[row * KS + srow] = (__bf16)(hv[r] - (float)xh);
        dah[row * KS + srow] = dh;
        dal[row * KS + srow] = (__bf16)(dv - (float)dh);
        const float bs = row16_sum(dv);
        if (ls == 0) b1p[wave * 16 * QT + row] = bs;
      }
    }
    __syncthreads();
    // tiles of the pass: NPT*QT of gW2 (pt, j), QT*NPT of gW1 (j, jt), and
    // in the first pass NPT*NPT of gW0 (pt, jt); wave w takes w, w + NW, ...
    constexpr int n2 = NPT * QT, n1 = QT * NPT;
    const int ntile = n2 + n1 + (pass == 0 ? NPT * NPT : 0);
    for (int tile = wave; tile < ntile; tile += NW) {
      f4 acc = f4{0.f, 0.f, 0.f, 0.f};
      int ai, bj, kind;
      if (tile < n2) {
        kind = 2;   // gW2 = dlogit^T h
        const int pt = tile / QT, j = tile % QT;
        ai = 16 * pt; bj = 16 * j;
#pragma unroll
        for (int c = 0; c < NW / 2; ++c) {
          const bf8v xh = rd(dlh, ai + ls, c), xl = rd(dll, ai + ls, c);
          const bf8v yh = rd(hh, bj + ls, c), yl = rd(hl, bj + ls, c);
          acc = mfma_b(xh, yh, acc);
          acc = mfma_b(xh, yl, acc);
          acc = mfma_b(xl, yh, acc);
        }
      } else if (tile < n2 + n1) {
        kind = 1;   // gW1 = da^T s
        const int e = tile - n2, j = e / NPT, jt = e % NPT;
        ai = 16 * j; bj = 16 * jt;
#pragma unroll
        for (int c = 0; c < NW / 2; ++c) {
          const bf8v xh = rd(dah, ai + ls, c), xl = rd(dal, ai + ls, c), ys = rd(sT, bj + ls, c);
          acc = mfma_b(xh, ys, acc);
          acc = mfma_b(xl, ys, acc);
        }
      } else {
        kind = 0;   // gW0 = dlogit^T s
        const int e = tile - n2 - n1, pt = e / NPT, jt = e % NPT;
        ai = 16 * pt; bj = 16 * jt;
#pragma unroll
        for (int c = 0; c < NW / 2; ++c) {
          const bf8v xh = rd(dlh, ai + ls, c), xl = rd(dll, ai + ls, c), ys = rd(sT, bj + ls, c);
          acc = mfma_b(xh, ys, acc);
          acc = mfma_b(xl, ys, acc);
        }
      }
      // lane holds rows ai + 4 lg + r, column bj + ls (as mgrad_kernel)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ai + 4 * lg + r, col = bj + ls;
        if (kind == 2) {         // gW2[pos][k]: deg(k) <= pos
          const int k = hbase + col;
          if (row < n && k < Hs)
            prow[o_W2 + (int64_t)row * Hs + k] = deg[k] <= row ? acc[r] : 0.f;
        } else if (kind == 1) {  // gW1[k][j]: j < deg(k)
          const int k = hbase + row;
          if (k < Hs && col < n) prow[(int64_t)k * n + col] = col < deg[k] ? acc[r] : 0.f;
        } else {                 // gW0[pos][j]: j < pos
          if (row < n && col < n) prow[o_W0 + (int64_t)row * n + col] = col < row ? acc[r] : 0.f;
        }
      }
    }
    // bias gradients of the pass: the waves' 16-sample sums in order
    for (int k = tid; k < 16 * QT; k += blockDim.x) {
      const int kk = hbase + k;
      if (kk >= Hs) continue;
      float v = 0.f;
      if (kk < H)
#pragma unroll
        for (int w = 0; w < NW; ++w) v += b1p[w * 16 * QT + k];
      prow[o_b1 + kk] = v;
    }
    if (pass == 0)
      for (int i = tid; i < n; i += blockDim.x) {
        float v = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) v += b2p[w * 16 * NPT + i];
        prow[o_b2 + i] = v;
      }
  }
}

// The REINFORCE gradient (the fixed-order sum of the instance's workgroup
// rows) and the Adam step in one launch.  A block takes 64 parameters of one
// instance (grid.y); its four row quarters sum rows k, k + 4, ... in order in
// FP64, sixteen loads in flight at a time; the quarters are added in order,
// then the parameter's thread stores the gradient, applies Adam and updates
// the packed tables (as adam_step_kernel).
constexpr int kGaRows = 16;   // row loads in flight per thread
__global__ __launch_bounds__(256) void grad_adam_kernel(MGradArgs g, OptArgs o) {
  __shared__ double sh[4][64];
  const int q = blockIdx.y;
  const MadeInst mi = o.mi[q];
  // an instance without samples this step keeps its parameters and moments
  if (mi.B <= 0) return;
  const int64_t pc = made_pc(mi);
  const int pl = threadIdx.x & 63, qr = threadIdx.x >> 6;
  const int64_t i = blockIdx.x * (int64_t)64 + pl;
  const int r0 = g.first_row[q], nr = g.n_rows[q];
  const float *col = g.part + (i < pc ? i : 0);
  double acc = 0.0;
  for (int rb = qr; rb < nr; rb += 4 * kGaRows) {
    float v[kGaRows];
#pragma unroll
    for (int j = 0; j < kGaRows; ++j) {
      const int r = rb + 4 * j;
      v[j] = col[(int64_t)(r0 + (r < nr ? r : 0)) * g.pstride];
    }
#pragma unroll
    for (int j = 0; j < kGaRows; ++j)
      if (rb + 4 * j < nr) acc += (double)v[j];
  }
  sh[qr][pl] = acc;
  __syncthreads();
  if (qr != 0 || i >= pc) return;
  const double t = (double)o.step_ctr[q];
  const double c1 = 1.0 - pow(0.9, t), c2 = 1.0 - pow(0.999, t);
  float *P = o.params + mi.param_off, *M = o.m + mi.param_off, *V = o.v + mi.param_off;
  float p = P[i], m = M[i], v = V[i];
  const float gi = (float)(((sh[0][pl] + sh[1][pl]) + sh[2][pl]) + sh[3][pl]);
  o.grad[mi.param_off + i] = gi;
  adam_one(gi, p, m, v, c1, c2, o.lr);
  M[i] = m;
  V[i] = v;
  P[i] = p;
  if (o.pack) pack_scatter(o.pack + mi.pack_off, mi.n, mi.H, o.npt, i, p);
}

template <int NPT>
void (*pick_mgrad3(int ht))(MGradArgs) {
  switch (ht) {
    case 1: return mgrad3_kernel<NPT, 1>;
    case 2: return mgrad3_kernel<NPT, 2>;
    case 4: return mgrad3_kernel<NPT, 4>;
    case 8: return mgrad3_kernel<NPT, 8>;
    default: return mgrad3_kernel<NPT, 16>;
  }
}

template <int NPT>
void (*pick_mgrad(int ht))(MGradArgs) {
  switch (ht) {
    case 1: return mgrad_kernel<NPT, 1>;
    case 2: return mgrad_kernel<NPT, 2>;
    case 4: return mgrad_kernel<NPT, 4>;
    case 8: return mgrad_kernel<NPT, 8>;
    default: return mgrad_kernel<NPT, 16>;
  }
}

}  // namespace

constexpr size_t kStageMax = 96 * 1024;

size_t made_param_bytes(int n, int H) { return made_stage_bytes(n, H); }
size_t made_stage_max() { return kStageMax; }

int64_t made_pack_floats(int n, int npt, int H) { return mpack_floats(n, npt, H); }
int64_t made_w2t_offset(int n, int npt) { return msample_floats(n, npt); }

size_t mgrad_lds_bytes(int H, int npt, bool split) {
  int ht = 1;
  while (16 * ht < H) ht <<= 1;
  return split ? mg3_layout(npt, ht, kMg3W).end : mg_bytes(16 * ht, npt);
}

hipError_t launch_mgrad(const MGradArgs &a, int npt, hipStream_t st) {
  if (a.n_tasks <= 0) return hipSuccess;
  int ht = 1;
  while (16 * ht < a.hmax) ht <<= 1;
  if (npt > 4 || ht > 16) return hipErrorInvalidValue;
  const size_t lds = mgrad_lds_bytes(a.hmax, npt, a.split != 0);
  void (*k)(MGradArgs) = nullptr;
  if (a.split) {
    // (|W| <= 32: the 4-tile form would spill registers)
    if (npt <= 1) k = pick_mgrad3<1>(ht);
    else if (npt <= 2) k = pick_mgrad3<2>(ht);
    else return hipErrorInvalidValue;
  } else {
    if (npt <= 1) k = pick_mgrad<1>(ht);
    else if (npt <= 2) k = pick_mgrad<2>(ht);
    else k = pick_mgrad<4>(ht);
  }
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(a.n_tasks), dim3(a.split ? 64 * kMg3W : 256), lds, st, a);
  return hipGetLastError();
}

int mgrad_task_samples(bool split) { return split ? 16 * kMg3W : 64; }

hipError_t launch_grad_adam(const MGradArgs &g, const OptArgs &o, int64_t max_pc, hipStream_t st) {
  if (g.n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(grad_adam_kernel, dim3((unsigned)((max_pc + 63) / 64), g.n_inst), dim3(256), 0,
                     st, g, o);
  return hipGetLastError();
}

hipError_t launch_made_pack(const MadeInst *mi, int n_inst, int64_t max_floats, const float *params,
                            float *pack, int npt, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  const int bx = (int)std::min<int64_t>(256, (max_floats + 255) / 256);
  hipLaunchKernelGGL(made_pack_kernel, dim3(std::max(1, bx), n_inst), dim3(256), 0, st, mi, params,
                     pack, npt);
  return hipGetLastError();
}

hipError_t launch_msample(const MSampleArgs &a, int npt, hipStream_t st) {
  if (a.n_tasks <= 0) return hipSuccess;
  const dim3 grid((a.n_tasks + 3) / 4);
  const bool given = a.uniforms != nullptr;
  void (*k)(MSampleArgs);
  if (npt <= 1) k = given ? msample_kernel<1, true> : msample_kernel<1, false>;
  else if (npt <= 2) k = given ? msample_kernel<2, true> : msample_kernel<2, false>;
  else if (npt <= 4) k = given ? msample_kernel<4, true> : msample_kernel<4, false>;
  else return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_sample(const SampleArgs<real> &a, int n_blocks, size_t stage_bytes,
                         hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  if (stage_bytes > 0 && stage_bytes <= kStageMax) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(sample_kernel<real, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)stage_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((sample_kernel<real, true>), dim3(n_blocks), dim3(256), stage_bytes, st, a);
  } else {
    hipLaunchKernelGGL((sample_kernel<real, false>), dim3(n_blocks), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_w0t(const MadeInst *mi, int n_inst, int max_n, const float *params,
                      const int64_t *w0t_off, float *w0t, hipStream_t st) {
  if (n_inst <= 0 || max_n <= 0) return hipSuccess;
  const unsigned t = (unsigned)((max_n + 31) / 32);
  hipLaunchKernelGGL(w0t_kernel, dim3(t, t, n_inst), dim3(256), 0, st, mi, params, w0t_off, w0t);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_sample_h0(const SampleArgs<real> &a, int n_inst, int64_t max_B, int max_n,
                            hipStream_t st) {
  if (n_inst <= 0 || max_B <= 0) return hipSuccess;
  const dim3 grid((unsigned)((max_B + 3) / 4), (unsigned)n_inst);
  if (max_n <= 64)
    hipLaunchKernelGGL((sample_h0_kernel<real, 1>), grid, dim3(256), 0, st, a);
  else if (max_n <= 128)
    hipLaunchKernelGGL((sample_h0_kernel<real, 2>), grid, dim3(256), 0, st, a);
  else if (max_n <= 256)
    hipLaunchKernelGGL((sample_h0_kernel<real, 4>), grid, dim3(256), 0, st, a);
  else if (max_n <= kH0MaxN)
    hipLaunchKernelGGL((sample_h0_kernel<real, 8>), grid, dim3(256), 0, st, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename real>
hipError_t launch_rows_h0(const RowArgs<real> &a, hipStream_t st) {
  const int64_t total = a.mi.B * a.mi.n;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL((rows_h0_kernel<real>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     st, a);
  return hipGetLastError();
}

size_t rows_lds_bytes(int n, int H, size_t real_bytes, bool staged) {
  const size_t rows = real_bytes * (size_t)RB * (2 * ((size_t)n + 1) + H + 1);
  return rows + (staged ? (made_param_bytes(n, H) + 15) & ~(size_t)15 : 0);
}

template <typename real>
hipError_t launch_rows_batch(const RowBatch<real> &a, bool staged, size_t lds_bytes,
                             int threads, hipStream_t st) {
  if (a.n_jobs <= 0 || a.blocks <= 0) return hipSuccess;
  if (threads < 64 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
  const void *k = staged ? reinterpret_cast<const void *>(rows_batch_kernel<real, true>)
                         : reinterpret_cast<const void *>(rows_batch_kernel<real, false>);
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_bytes);
  if (e != hipSuccess) return e;
  if (staged)
    hipLaunchKernelGGL((rows_batch_kernel<real, true>), dim3(a.blocks), dim3(threads), lds_bytes,
                       st, a);
  else
    hipLaunchKernelGGL((rows_batch_kernel<real, false>), dim3(a.blocks), dim3(threads), lds_bytes,
                       st, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_rows_deep(const RowArgs<real> &a, int rb, hipStream_t st) {
  if (a.mi.B <= 0) return hipSuccess;
  if (rb < 1 || (int64_t)rb * a.mi.H > kDeepRows || a.mi.D > kDeepMaxD) return hipErrorInvalidValue;
  const int D = (a.mi.n >= 2 && a.mi.H > 0) ? a.mi.D : 1;
  const size_t lds =
      sizeof(real) * (size_t)rb * (2 * ((size_t)a.mi.n + 1) + (size_t)D * a.mi.H + a.mi.H + 2);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(rows_deep_kernel<real>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t blocks = (a.mi.B + a.chunk - 1) / a.chunk;
  hipLaunchKernelGGL(rows_deep_kernel<real>, dim3((unsigned)blocks), dim3(256), lds, st, a, rb);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_sample_deep(const SampleArgs<real> &a, int n_inst, int64_t max_B, bool small,
                              hipStream_t st) {
  if (n_inst <= 0 || max_B <= 0) return hipSuccess;
  if (small) {
    const int64_t bx = (max_B + 15) / 16;
    if (bx > 0x7fffffff || n_inst > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(sample_deep16_kernel<real>, dim3((unsigned)bx, n_inst), dim3(256), 0, st,
                       a);
    return hipGetLastError();
  }
  const int64_t bx = (max_B + 3) / 4;
  if (bx > 0x7fffffff || n_inst > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sample_deep_kernel<real>, dim3((unsigned)bx, n_inst), dim3(256), 0, st, a);
  return hipGetLastError();
}

void batch_sum_blocks(int M, int N, int ks, int32_t *atb, int32_t *fin) {
  *atb = ((M + TM - 1) / TM) * ((N + TN - 1) / TN) * ks;
  *fin = (int32_t)(((int64_t)M * N + 255) / 256);
}
void batch_col_blocks(int M, int ks, int32_t *col, int32_t *fin) {
  *col = ((M + 255) / 256) * ks;
  *fin = (M + 255) / 256;
}

template <typename real>
hipError_t launch_batch_sums(const BatchSums<real> &a, hipStream_t st) {
  if (a.n_atb > 0 && a.atb_blocks > 0) {
    hipLaunchKernelGGL(batch_atb_kernel<real>, dim3(a.atb_blocks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(batch_atb_finish<real>, dim3(a.atb_fblocks), dim3(256), 0, st, a);
  }
  if (a.n_col > 0 && a.col_blocks > 0) {
    hipLaunchKernelGGL(batch_col_kernel<real>, dim3(a.col_blocks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(batch_col_finish<real>, dim3(a.col_fblocks), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

template <typename real>
hipError_t launch_free(const FreeArgs<real> &a, int n_inst, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(free_f_kernel<real>, dim3(a.nblk, n_inst), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_e1(const E1Args &a, int n_inst, int64_t max_B, hipStream_t st) {
  if (n_inst <= 0 || max_B <= 0) return hipSuccess;
  const int bx = (int)std::min<int64_t>(65535, (max_B + 255) / 256);
  hipLaunchKernelGGL(e1_kernel, dim3(bx, n_inst), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adam_step(const OptArgs &a, int n_inst, int64_t max_pc, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  const int bx = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (max_pc + 255) / 256));
  hipLaunchKernelGGL(adam_step_kernel, dim3(bx, n_inst), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_slice_spins(int8_t *spins, int nw, int64_t c0, int64_t n, hipStream_t st) {
  const int64_t nbytes = n * nw;
  if (nbytes <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (nbytes + 255) / 256);
  hipLaunchKernelGGL(slice_spins_kernel, dim3(blocks), dim3(256), 0, st, spins, nw, c0, nbytes);
  return hipGetLastError();
}

hipError_t launch_slice_lse(const SliceArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(slice_lse_kernel, dim3(kSliceBlocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_slice_final(const double *part, int64_t count, double beta, double *out,
                              hipStream_t st) {
  hipLaunchKernelGGL(slice_final_kernel, dim3(1), dim3(256), 0, st, part, count, beta, out);
  return hipGetLastError();
}

hipError_t launch_obs_weights(const ObsArgs &a, int n_inst, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(obs_weights_kernel, dim3(n_inst), dim3(kObsThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_obs_w(const ObsArgs &a, int n_inst, hipStream_t st) {
  if (n_inst <= 0 || a.max_out <= 0) return hipSuccess;
  hipLaunchKernelGGL(obs_w_kernel, dim3(a.max_out, n_inst), dim3(kObsThreads), 0, st, a);
  return hipGetLastError();
}

template hipError_t launch_sample<float>(const SampleArgs<float> &, int, size_t, hipStream_t);
template hipError_t launch_sample<double>(const SampleArgs<double> &, int, size_t, hipStream_t);
template hipError_t launch_sample_deep<float>(const SampleArgs<float> &, int, int64_t, bool,
                                              hipStream_t);
template hipError_t launch_sample_deep<double>(const SampleArgs<double> &, int, int64_t, bool,
                                               hipStream_t);
template hipError_t launch_rows_deep<float>(const RowArgs<float> &, int, hipStream_t);
template hipError_t launch_rows_deep<double>(const RowArgs<double> &, int, hipStream_t);
template hipError_t launch_sample_h0<float>(const SampleArgs<float> &, int, int64_t, int, hipStream_t);
template hipError_t launch_sample_h0<double>(const SampleArgs<double> &, int, int64_t, int, hipStream_t);
template hipError_t launch_rows_batch<float>(const RowBatch<float> &, bool, size_t, int,
                                             hipStream_t);
template hipError_t launch_rows_batch<double>(const RowBatch<double> &, bool, size_t, int,
                                              hipStream_t);
template hipError_t launch_rows_h0<float>(const RowArgs<float> &, hipStream_t);
template hipError_t launch_rows_h0<double>(const RowArgs<double> &, hipStream_t);
template hipError_t launch_batch_sums<float>(const BatchSums<float> &, hipStream_t);
template hipError_t launch_batch_sums<double>(const BatchSums<double> &, hipStream_t);
template hipError_t launch_free<float>(const FreeArgs<float> &, int, hipStream_t);
template hipError_t launch_free<double>(const FreeArgs<double> &, int, hipStream_t);

}  // namespace tnvan
