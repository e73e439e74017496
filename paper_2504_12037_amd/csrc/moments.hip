// Conditional mean and variance of the remainder's magnetisation given s_W,
// and the susceptibility estimated from samples of q (Sec. 3: the
// magnetisation and susceptibility of p from the trained network's samples).
//
// With eta = beta H for a uniform field H on R, Z_R(s_W; eta) = sum_r
// exp(-beta E_2(s_W, r) + eta M_R), and
//   d ln Z_R / d eta   = <M_R>,   d^2 ln Z_R / d eta^2 = Var(M_R).
// The field enters the contraction only through the unary factor of each R
// spin, phi(x) -> phi(x) e^{eta s_x}.  Every message is therefore a
// polynomial in eta, and truncated after eta^2 it is carried exactly as a
// jet (c0, c1, c2) of Taylor coefficients: the static transfer tables act
// on each coefficient alike, products of messages multiply jets (dropping
// eta^3 and beyond), and a group state of magnetisation m brings the jet
// (1, m, m^2 / 2).  The closing entry z of each connected part of R then
// gives <M_R> = sum z1 / z0 and Var(M_R) = sum 2 z2 / z0 - (z1 / z0)^2 over
// the parts (independent given s_W).  The same per-step power-of-two
// rescale as the forward kernels applies to all three coefficients.
//
// An instance runs its general step program here (dense grouped steps and
// single-spin steps with full tables; not the wide steps), one thread per
// sample, the jets in device memory as [entry][coefficient][sample] so that
// neighbouring threads touch neighbouring words; instances whose program is
// a set of narrow chains run the same jets on the register-resident chain
// kernels instead (chainr.hip).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"

namespace tnvan {

namespace {

template <typename real>
struct Jet {
  real c0, c1, c2;
};
template <typename real>
__device__ inline Jet<real> jmul(const Jet<real> &a, const Jet<real> &b) {
  return {a.c0 * b.c0, a.c0 * b.c1 + a.c1 * b.c0, a.c0 * b.c2 + a.c1 * b.c1 + a.c2 * b.c0};
}
template <typename real>
__device__ inline Jet<real> jscale(const Jet<real> &a, real s) {
  return {a.c0 * s, a.c1 * s, a.c2 * s};
}

template <typename real>
__device__ inline real rexp(real x);
template <> __device__ inline float rexp<float>(float x) { return expf(x); }
template <> __device__ inline double rexp<double>(double x) { return exp(x); }

// binary exponent e with v 2^-e in [0.5, 1) (0 for v = 0)
template <typename real>
__device__ inline int expo_of(real v) {
  int e = 0;
  (void)frexp(v, &e);
  return e;
}

template <typename real>
__global__ __launch_bounds__(256) void moments_kernel(MomentArgs<real> a) {
  const int q = blockIdx.y;
  if (a.skip && a.skip[q]) return;
  const int64_t B = a.inst_B[q];
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const InstDesc D = a.inst[q];
  const StepDesc *steps = a.steps + D.step_off;
  const int8_t *sp = a.spins + a.inst_spin_off[q] + b * D.nw;
  real *J = a.jarena + a.jar_off[q];
  int32_t *E = a.jexp + a.jexp_off[q];
  const int64_t per = (int64_t)D.arena_fwd;   // scratch jets follow the arena
  auto at = [&](int64_t entry, int c) -> real & { return J[(entry * 3 + c) * B + b]; };
  auto load = [&](int64_t entry) -> Jet<real> { return {at(entry, 0), at(entry, 1), at(entry, 2)}; };
  auto store = [&](int64_t entry, const Jet<real> &v) {
    at(entry, 0) = v.c0;
    at(entry, 1) = v.c1;
    at(entry, 2) = v.c2;
  };
  auto scale_of = [&](int step) -> real { return ldexp((real)1, -E[(int64_t)step * B + b]); };
  const real beta = (real)D.beta;
  double fab = 0.0;
  // unary factor of R position p for spin +1 (k = 0) and -1 (k = 1):
  // fields and W-R couplings, normalised so that the larger is one
  auto phi = [&](int p, real (&ph)[2]) {
    real f = a.hR[D.hr_off + p];
    const int k0 = a.fld_ptr[D.fld_off + p], k1 = a.fld_ptr[D.fld_off + p + 1];
    for (int k = k0; k < k1; ++k) f += a.fld_J[D.fld_nnz_off + k] * (real)sp[a.fld_w[D.fld_nnz_off + k]];
    const real af = beta * (f < 0 ? -f : f);
    const real small = rexp<real>(-2 * af);
    ph[0] = f >= 0 ? (real)1 : small;
    ph[1] = f >= 0 ? small : (real)1;
    fab += (double)af;
  };
  for (int t = 0; t < D.n_steps; ++t) {
    const StepDesc sd = steps[t];
    const int w = sd.w, g = sd.g;
    const real *Tt = a.T + sd.t_off;
    real lmax = 0;
    if (sd.kind == STEP_DENSE) {
      real ph[kMaxG][2];
      for (int j = 0; j < g; ++j) phi(sd.gpos + j, ph[j]);
      int64_t inoff = 0;
      real insc = 1;
      if (sd.n_in) {
        const InputDesc id = a.inputs[sd.in_off];
        inoff = steps[id.step].off_fwd;
        insc = scale_of(id.step);
      }
      // A[x] = d[x] e^{eta m(x)} m_in[x], into the scratch jets
      for (int x = 0; x < (1 << g); ++x) {
        real d = 1;
        int m = 0;
        for (int j = 0; j < g; ++j) {
          const int bit = (x >> j) & 1;
          d *= ph[j][bit];
          m += bit ? -1 : 1;
        }
        Jet<real> A = {d, d * (real)m, d * (real)(m * m) / 2};
        if (sd.n_in) A = jmul(A, jscale(load(inoff + x), insc));
        store(per + x, A);
      }
      for (int o = 0; o < (1 << w); ++o) {
        Jet<real> acc = {0, 0, 0};
        for (int x = 0; x < (1 << g); ++x) {
          const real tx = Tt[(x << w) | o];
          const Jet<real> A = load(per + x);
          acc.c0 += tx * A.c0;
          acc.c1 += tx * A.c1;
          acc.c2 += tx * A.c2;
        }
        store(sd.off_fwd + o, acc);
        lmax = acc.c0 > lmax ? acc.c0 : lmax;
      }
    } else {
      real ph[2];
      phi(sd.gpos, ph);
      for (int o = 0; o < (1 << w); ++o) {
        const real t0 = Tt[o] * ph[0], t1 = Tt[(1 << w) | o] * ph[1];
        // e^{eta s}: (1, s, 1/2) for the eliminated spin s = +1, -1
        Jet<real> p0 = {t0, t0, t0 / 2}, p1 = {t1, -t1, t1 / 2};
        for (int k = 0; k < sd.n_in; ++k) {
          const InputDesc id = a.inputs[sd.in_off + k];
          const int64_t ioff = steps[id.step].off_fwd;
          int i0 = 0;
          if (id.gb_off >= 0) {
            i0 = a.gtab[id.gb_off + o];
          } else {
            for (int bb = 0; bb < id.nbits; ++bb) {
              const int sb = id.src[bb];
              i0 |= (sb < 0 ? 0 : ((o >> sb) & 1)) << bb;
            }
          }
          const real sc = scale_of(id.step);
          p0 = jmul(p0, jscale(load(ioff + i0), sc));
          p1 = jmul(p1, jscale(load(ioff + (i0 | (1 << id.xbit))), sc));
        }
        const Jet<real> out = {p0.c0 + p1.c0, p0.c1 + p1.c1, p0.c2 + p1.c2};
        store(sd.off_fwd + o, out);
        lmax = out.c0 > lmax ? out.c0 : lmax;
      }
    }
    E[(int64_t)t * B + b] = w > 0 ? expo_of(lmax) : 0;
  }
  // ln Z_R and the cumulants from the closing entries
  double lz = D.log_const + fab, m1 = 0.0, v = 0.0;
  int64_t esum = 0;
  for (int t = 0; t < D.n_steps; ++t) {
    const StepDesc sd = steps[t];
    if (sd.w == 0) {
      const Jet<real> z = load(sd.off_fwd);
      const double z0 = (double)z.c0, r1 = (double)z.c1 / z0, r2 = (double)z.c2 / z0;
      lz += log(z0);
      m1 += r1;
      v += 2.0 * r2 - r1 * r1;
    } else {
      esum += E[(int64_t)t * B + b];
    }
  }
  const int64_t g = a.inst_sample_off[q] + b;
  if (a.logz) a.logz[g] = lz + (double)esum * 0.69314718055994530942;
  a.mean[g] = m1;
  a.var[g] = v;
}

// per instance: M_b = M_W(s_b) + <M_R>_b, and with the importance weights
// w_b = beta g_b (g_b = w_b / beta from obs_weights_kernel)
//   <M> = sum w M,  <M^2> = sum w (M^2 + Var(M_R)_b)
// in FP64, a fixed-order tree over the block
constexpr int kSusThreads = 1024;
__global__ __launch_bounds__(kSusThreads) void sus_reduce_kernel(SusArgs a) {
  __shared__ double s1[kSusThreads], s2[kSusThreads];
  const int q = blockIdx.x, t = threadIdx.x;
  const InstDesc D = a.inst[q];
  const int64_t B = a.inst_B[q], off = a.inst_sample_off[q];
  const int8_t *sp = a.spins + a.inst_spin_off[q];
  double acc1 = 0.0, acc2 = 0.0;
  for (int64_t b = t; b < B; b += kSusThreads) {
    int mw = 0;
    for (int k = 0; k < D.nw; ++k) mw += sp[b * D.nw + k];
    const double M = (double)mw + a.mean[off + b];
    const double w = D.beta * a.g[off + b];
    acc1 += w * M;
    acc2 += w * (M * M + a.var[off + b]);
  }
  s1[t] = acc1;
  s2[t] = acc2;
  __syncthreads();
  for (int st = kSusThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      s1[t] += s1[t + st];
      s2[t] += s2[t + st];
    }
    __syncthreads();
  }
  if (t != 0) return;
  const double n = (double)D.n, M1 = s1[0], M2 = s2[0];
  double *o = a.out + 4 * q;
  if (B <= 0) {
    o[0] = o[1] = o[2] = o[3] = 0.0;
    return;
  }
  o[0] = M1 / n;
  o[1] = M2 / (n * n);
  o[2] = D.beta * (M2 - M1 * M1) / n;
  o[3] = a.ess[q];
}

}  // namespace

template <typename real>
hipError_t launch_moments(const MomentArgs<real> &a, int n_inst, int64_t max_B, hipStream_t st) {
  if (n_inst <= 0 || max_B <= 0) return hipSuccess;
  const int64_t bx = (max_B + 255) / 256;
  if (bx > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(moments_kernel<real>, dim3((unsigned)bx, n_inst), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sus_reduce(const SusArgs &a, int n_inst, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(sus_reduce_kernel, dim3(n_inst), dim3(kSusThreads), 0, st, a);
  return hipGetLastError();
}

template hipError_t launch_moments<float>(const MomentArgs<float> &, int, int64_t, hipStream_t);
template hipError_t launch_moments<double>(const MomentArgs<double> &, int, int64_t, hipStream_t);

}  // namespace tnvan
