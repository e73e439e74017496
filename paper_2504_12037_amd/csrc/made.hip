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

#include "launch.h"

namespace tnvan {

namespace {

__device__ inline int degree(int k, int n) { return 1 + (k % (n - 1)); }

template <typename real> __device__ inline real rexp(real x);
template <> __device__ inline float rexp<float>(float x) { return expf(x); }
template <> __device__ inline double rexp<double>(double x) { return exp(x); }
template <typename real> __device__ inline real rlog1p(real x);
template <> __device__ inline float rlog1p<float>(float x) { return log1pf(x); }
template <> __device__ inline double rlog1p<double>(double x) { return log1p(x); }
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

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64-bit
// multiplies with word swaps and key xors; Weyl key schedule.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
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

constexpr int KH = 16;    // hidden units per lane
constexpr int KN = 32;    // width-set positions per lane

// One group of L lanes per sample; lane l owns hidden units k = l + L*kk and
// positions j = l + L*jj.  Spins are drawn one position after the other.
template <typename real>
__global__ __launch_bounds__(256) void sample_kernel(SampleArgs<real> a) {
  const int q = a.blk_inst[blockIdx.x];
  const MadeInst mi = a.mi[q];
  const int L = mi.L;
  const int grp = threadIdx.x / L, l = threadIdx.x % L;
  const int64_t b = a.blk_start[blockIdx.x] + grp;
  const bool live = grp < a.spb && b < mi.B;
  const int n = mi.n, H = (n >= 2) ? mi.H : 0;
  const float *W1 = a.params + mi.param_off;
  const float *b1 = W1 + (int64_t)mi.H * n;
  const float *W2 = b1 + mi.H;
  const float *b2 = W2 + (int64_t)n * mi.H;
  const float *W0 = b2 + n;
  real av[KH], hv[KH], sv[KN];
#pragma unroll
  for (int kk = 0; kk < KH; ++kk) {
    const int k = l + L * kk;
    av[kk] = (k < H) ? (real)b1[k] : (real)0;
    hv[kk] = 0;
  }
#pragma unroll
  for (int jj = 0; jj < KN; ++jj) sv[jj] = 0;
  real lq = 0;
  const int64_t gs = mi.sample_off + (live ? b : 0);
  const float *u = a.uniforms ? a.uniforms + mi.spin_off + (live ? b : 0) * n : nullptr;
  int8_t *so = a.spins + mi.spin_off + (live ? b : 0) * n;
  uint32_t pw[4] = {0, 0, 0, 0};
  const uint32_t step = a.step_ctr ? (uint32_t)a.step_ctr[q] : 0u;
  for (int i = 0; i < n; ++i) {
    real part = 0;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
      const int k = l + L * kk;
      if (k < H && degree(k, n) <= i) part += (real)W2[(int64_t)i * mi.H + k] * hv[kk];
    }
#pragma unroll
    for (int jj = 0; jj < KN; ++jj) {
      const int j = l + L * jj;
      if (j < i) part += (real)W0[(int64_t)i * n + j] * sv[jj];
    }
    for (int off = L >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    const real logit = part + (real)b2[i];
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
        const int m = degree(k, n);
        if (m >= i + 1) {
          av[kk] += (real)W1[(int64_t)k * n + i] * si;
          if (m == i + 1) hv[kk] = rtanh<real>(av[kk]);
        }
      }
    }
  }
  if (live && l == 0) a.logq[gs] = lq;
}

// Per-sample rows: a, tanh(a), logits, dlogit = w ((1+s)/2 - sigmoid(logit)),
// da = (dlogit . W2m) (1 - tanh^2).  One block of 256 threads per 16 samples.
constexpr int RB = 16;
template <typename real>
__global__ __launch_bounds__(256) void rows_kernel(RowArgs<real> a) {
  extern __shared__ __align__(16) char smem[];
  const MadeInst mi = a.mi;
  const int n = mi.n, H = (n >= 2) ? mi.H : 0, Hs = mi.H;
  real *ss = reinterpret_cast<real *>(smem);         // [RB][n]
  real *hh = ss + RB * n;                            // [RB][H]
  real *dl = hh + RB * Hs;                           // [RB][n]
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const int nr = (int)((mi.B - r0) < RB ? (mi.B - r0) : RB);
  const float *W1 = a.params + mi.param_off;
  const float *b1 = W1 + (int64_t)Hs * n;
  const float *W2 = b1 + Hs;
  const float *b2 = W2 + (int64_t)n * Hs;
  const float *W0 = b2 + n;
  const int8_t *sp = a.spins + mi.spin_off + r0 * n;
  for (int i = threadIdx.x; i < RB * n; i += blockDim.x) {
    const int r = i / n;
    ss[i] = r < nr ? (real)sp[i] : (real)0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < RB * Hs; i += blockDim.x) {
    const int r = i / Hs, k = i % Hs;
    real acc = 0;
    if (k < H) {
      acc = (real)b1[k];
      const int m = degree(k, n);
      for (int j = 0; j < m; ++j) acc += (real)W1[(int64_t)k * n + j] * ss[r * n + j];
      acc = rtanh<real>(acc);
    }
    hh[i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < RB * n; i += blockDim.x) {
    const int r = i / n, ii = i % n;
    real z = (real)b2[ii];
    for (int k = 0; k < H; ++k)
      if (degree(k, n) <= ii) z += (real)W2[(int64_t)ii * Hs + k] * hh[r * Hs + k];
    for (int j = 0; j < ii; ++j) z += (real)W0[(int64_t)ii * n + j] * ss[r * n + j];
    const real s = ss[i];
    const real wt = r < nr ? a.wts[mi.sample_off + r0 + r] : (real)0;
    const real d = wt * (((real)1 + s) * (real)0.5 - sigmoid<real>(z));
    dl[i] = d;
    if (r < nr) {
      a.dlogit[(r0 + r) * n + ii] = d;
      a.sf[(r0 + r) * n + ii] = s;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < RB * Hs; i += blockDim.x) {
    const int r = i / Hs, k = i % Hs;
    if (r >= nr) continue;
    real acc = 0;
    const real hk = hh[i];
    if (k < H) {
      const int m = degree(k, n);
      for (int ii = m; ii < n; ++ii) acc += dl[r * n + ii] * (real)W2[(int64_t)ii * Hs + k];
    }
    a.hid[(r0 + r) * Hs + k] = hk;
    a.da[(r0 + r) * Hs + k] = acc * ((real)1 - hk * hk);
  }
}

// part[ks][m][n] = sum over batch rows of slice ks of X[b, m] * Y[b, n]
constexpr int TM = 32, TN = 32, TK = 32;
template <typename real>
__global__ __launch_bounds__(256) void atb_kernel(const real *X, int ldx, const real *Y,
                                                  int ldy, int64_t B, int M, int N,
                                                  real *part, int ksplit) {
  __shared__ real xs[TK][TM + 1];
  __shared__ real ys[TK][TN + 1];
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN, ks = blockIdx.z;
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
//             2 W0 (col j < row i), 3 W1 (row k, col j): j+1 <= deg(k)
template <typename real>
__global__ void atb_finish(const real *part, int ksplit, int M, int N, float *out,
                           int ldo, int mask_kind, int nW) {
  const int64_t tot = (int64_t)M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < tot;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(idx / N), nn = (int)(idx % N);
    double acc = 0;
    for (int k = 0; k < ksplit; ++k) acc += (double)part[(int64_t)k * tot + idx];
    bool keep = true;
    if (mask_kind == 1) keep = nW >= 2 && (m + 1) > degree(nn, nW);
    else if (mask_kind == 2) keep = nn < m;
    else if (mask_kind == 3) keep = nW >= 2 && (nn + 1) <= degree(m, nW);
    out[(int64_t)m * ldo + nn] = keep ? (float)acc : 0.0f;
  }
}

template <typename real>
__global__ void colsum_kernel(const real *X, int ldx, int64_t B, int M, real *part,
                              int ksplit) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int ks = blockIdx.y;
  if (m >= M) return;
  const int64_t chunk = (B + ksplit - 1) / ksplit;
  const int64_t b0 = (int64_t)ks * chunk;
  const int64_t b1 = (b0 + chunk) < B ? (b0 + chunk) : B;
  real acc = 0;
  for (int64_t b = b0; b < b1; ++b) acc += X[b * ldx + m];
  part[(int64_t)ks * M + m] = acc;
}

template <typename real>
__global__ void colsum_finish(const real *part, int ksplit, int M, float *out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double acc = 0;
  for (int k = 0; k < ksplit; ++k) acc += (double)part[(int64_t)k * M + m];
  out[m] = (float)acc;
}

// f_b = E_1 - logZ_R / beta + ln q / beta (FP64), F_q, its standard error,
// <Etilde>, <ln q>/beta and REINFORCE weights (f_b - F_q) / B.
template <typename real>
__global__ __launch_bounds__(1024) void free_kernel(FreeArgs<real> a) {
  __shared__ double sh[3][1024];
  const int tid = threadIdx.x;
  double s_f = 0, s_e = 0, s_q = 0;
  for (int64_t b = tid; b < a.B; b += blockDim.x) {
    const int8_t *s = a.spins + b * a.nw;
    double e1 = 0;
    for (int k = 0; k < a.n_ww; ++k) e1 -= a.ww_J[k] * (double)s[a.ww_a[k]] * (double)s[a.ww_b[k]];
    for (int k = 0; k < a.nw; ++k) e1 -= a.hW[k] * (double)s[k];
    const double et = e1 - a.logz[b] / a.beta;
    const double lqb = (double)a.logq[b] / a.beta;
    const double f = et + lqb;
    a.f[b] = f;
    s_f += f; s_e += et; s_q += lqb;
  }
  sh[0][tid] = s_f; sh[1][tid] = s_e; sh[2][tid] = s_q;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st) for (int c = 0; c < 3; ++c) sh[c][tid] += sh[c][tid + st];
    __syncthreads();
  }
  const double Fq = sh[0][0] / (double)a.B;
  const double me = sh[1][0] / (double)a.B, mq = sh[2][0] / (double)a.B;
  __syncthreads();
  double v = 0;
  for (int64_t b = tid; b < a.B; b += blockDim.x) {
    const double d = a.f[b] - Fq;
    v += d * d;
    a.wts[b] = (real)(d / (double)a.B);
  }
  sh[0][tid] = v;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if (tid < st) sh[0][tid] += sh[0][tid + st];
    __syncthreads();
  }
  if (tid == 0) {
    const double var = a.B > 1 ? sh[0][0] / (double)(a.B - 1) : 0.0;
    a.stats[0] = Fq;
    a.stats[1] = sqrt(var / (double)a.B);
    a.stats[2] = me;
    a.stats[3] = mq;
  }
}

__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int64_t n,
                            float lr, const int32_t *step_ctr) {
  const double t = (double)(*step_ctr + 1);
  const double c1 = 1.0 - pow(0.9, t), c2 = 1.0 - pow(0.999, t);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const double mh = (double)mi / c1, vh = (double)vi / c2;
    p[i] = (float)((double)p[i] - (double)lr * mh / (sqrt(vh) + 1e-8));
  }
}

__global__ void bump_kernel(int32_t *c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] += 1;
}

}  // namespace

template <typename real>
hipError_t launch_sample(const SampleArgs<real> &a, int n_blocks, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(sample_kernel<real>, dim3(n_blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_rows(const RowArgs<real> &a, hipStream_t st) {
  if (a.mi.B <= 0) return hipSuccess;
  const int blocks = (int)((a.mi.B + RB - 1) / RB);
  const size_t lds = sizeof(real) * (size_t)RB * (2 * a.mi.n + a.mi.H);
  hipLaunchKernelGGL(rows_kernel<real>, dim3(blocks), dim3(256), lds, st, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_atb(const real *X, int ldx, const real *Y, int ldy, int64_t B, int M,
                      int N, real *part, int ksplit, float *out, int ldo, int mask_kind,
                      int nW, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN, ksplit);
  hipLaunchKernelGGL(atb_kernel<real>, grid, dim3(256), 0, st, X, ldx, Y, ldy, B, M, N,
                     part, ksplit);
  int64_t tot = (int64_t)M * N;
  int blocks = (int)((tot + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(atb_finish<real>, dim3(blocks), dim3(256), 0, st, part, ksplit, M, N,
                     out, ldo, mask_kind, nW);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_colsum(const real *X, int ldx, int64_t B, int M, real *part, int ksplit,
                         float *out, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  dim3 grid((M + 255) / 256, ksplit);
  hipLaunchKernelGGL(colsum_kernel<real>, grid, dim3(256), 0, st, X, ldx, B, M, part, ksplit);
  hipLaunchKernelGGL(colsum_finish<real>, dim3((M + 255) / 256), dim3(256), 0, st, part,
                     ksplit, M, out);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_free(const FreeArgs<real> &a, hipStream_t st) {
  hipLaunchKernelGGL(free_kernel<real>, dim3(1), dim3(1024), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int64_t n,
                       float lr, int32_t *step_ctr, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, st, params, grad, m, v, n, lr,
                     step_ctr);
  return hipGetLastError();
}

hipError_t launch_bump(int32_t *step_ctr, int n, hipStream_t st) {
  hipLaunchKernelGGL(bump_kernel, dim3((n + 255) / 256), dim3(256), 0, st, step_ctr, n);
  return hipGetLastError();
}

template hipError_t launch_sample<float>(const SampleArgs<float> &, int, hipStream_t);
template hipError_t launch_sample<double>(const SampleArgs<double> &, int, hipStream_t);
template hipError_t launch_rows<float>(const RowArgs<float> &, hipStream_t);
template hipError_t launch_rows<double>(const RowArgs<double> &, hipStream_t);
template hipError_t launch_atb<float>(const float *, int, const float *, int, int64_t, int, int, float *, int, float *, int, int, int, hipStream_t);
template hipError_t launch_atb<double>(const double *, int, const double *, int, int64_t, int, int, double *, int, float *, int, int, int, hipStream_t);
template hipError_t launch_colsum<float>(const float *, int, int64_t, int, float *, int, float *, hipStream_t);
template hipError_t launch_colsum<double>(const double *, int, int64_t, int, double *, int, float *, hipStream_t);
template hipError_t launch_free<float>(const FreeArgs<float> &, hipStream_t);
template hipError_t launch_free<double>(const FreeArgs<double> &, hipStream_t);

}  // namespace tnvan
