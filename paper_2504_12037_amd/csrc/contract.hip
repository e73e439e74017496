// Batched conditional log-partition function of the remainder and its
// adjoint (Sec. 2, Eqs. 2-4).
//
// One workgroup (256 threads) contracts a tile of S samples of one instance
// through every elimination step of the compiled program.  Work items of a
// step are (sample, output entry) pairs with the sample index fastest, so a
// thread always serves the same sample and the per-sample state sits in LDS
// as [entry][S] (conflict-free, broadcast reads of the static tables).
//
// Rescaling: a message is stored as computed ("raw"); its per-sample scale
// 2^-e, with e the binary exponent of the largest entry, is kept as the max
// bit pattern of that step (LDS atomic max over positive floats) and applied
// whenever the message is read.  Scaling by a power of two is exact, so the
// contraction result is independent of it; the exponents are summed in FP64
// into log Z.
//
// Adjoint: with mu_t the marginal of message t's scope and m~_t the scaled
// message, rho_t = mu_t / m~_t is written over message t by the step that
// consumed it.  Walking the steps backwards, step t forms for every sample the
// joint weight c(o, x) = rho_t[o] 2^-e_t T[x, o] d[x] prod_k m~_k (a
// probability: it sums to one over (o, x)), from which the marginals of the
// eliminated spins, the correlations of the R-R edges the step consumed and
// the rho of its inputs follow.  Batch sums weighted by the upstream gradient
// are reduced in a fixed order into one partial row per tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "launch.h"
#include "uload.h"

namespace tnvan {

namespace {

constexpr int kThreads = 256;
constexpr int kLogThreads = 8;
constexpr int kWaves = kThreads / 64;
constexpr int kRed = 4;         // values per column reduction pass
constexpr int kJoint = 2;       // output entries per thread and pass of a single-spin step

template <typename real> struct FBits;
template <> struct FBits<float> {
  using U = uint32_t;
  __device__ static U bits(float x) { return __float_as_uint(x); }
  // e with max * 2^-e in [0.5, 1)
  __device__ static int expo(U b) {
    int E = (int)((b >> 23) & 0xffu);
    int e = E - 126;
    return e > 126 ? 126 : e;
  }
  __device__ static float scale(int e) { return __uint_as_float((uint32_t)(127 - e) << 23); }
};
template <> struct FBits<double> {
  using U = unsigned long long;
  __device__ static U bits(double x) { return (U)__double_as_longlong(x); }
  __device__ static int expo(U b) {
    int E = (int)((b >> 52) & 0x7ffull);
    int e = E - 1022;
    return e > 1022 ? 1022 : e;
  }
  __device__ static double scale(int e) {
    return __longlong_as_double((long long)((unsigned long long)(1023 - e) << 52));
  }
};

struct Layout {
  size_t mx, phi, fab, gs, M, C, red, pb, arena, scr, end;
};

__host__ __device__ inline size_t al8(size_t x) { return (x + 7) & ~(size_t)7; }

__host__ __device__ inline Layout make_layout(const InstDesc &D, int S, bool bwd,
                                              bool global_arena, int rs) {
  Layout L{};
  size_t o = 0;
  const int us = rs == 4 ? 4 : 8;
  L.mx = o;  o = al8(o + (size_t)D.n_steps * S * us);
  L.phi = o; o = al8(o + (size_t)D.nr * 2 * S * rs);
  L.fab = o; o = al8(o + (size_t)D.nr * S * rs);
  if (bwd) {
    L.gs = o;  o = al8(o + (size_t)S * rs);
    L.M = o;   o = al8(o + (size_t)D.nr * S * rs);
    L.C = o;   o = al8(o + (size_t)D.n_rr * rs);
    L.red = o; o = al8(o + (size_t)kWaves * kRed * S * rs);
    L.pb = o;  o = al8(o + (size_t)D.pbuf * rs);
  }
  if (!global_arena) {
    L.arena = o; o = al8(o + (size_t)(bwd ? D.arena_all : D.arena_fwd) * S * rs);
    L.scr = o;   o = al8(o + (size_t)(bwd ? D.scr_bwd : D.scr_fwd) * S * rs);
  }
  L.end = o;
  return L;
}

template <typename real>
__device__ inline real rexp(real x);
template <> __device__ inline float rexp<float>(float x) { return expf(x); }
template <> __device__ inline double rexp<double>(double x) { return exp(x); }

// index of the input message entry for output entry o and group state x
// (id in device memory: its scope map is read there, not from a private copy)
__device__ inline int gather_index(const InputDesc *id, int o, int x) {
  int idx = 0;
  for (int b = 0; b < id->nbits; ++b) {
    int sb = id->src[b];
    int bit = sb < 0 ? x : ((o >> sb) & 1);
    idx |= bit << b;
  }
  return idx;
}

// SINGLE steps with at most kFastIn inputs: each input's arena offset,
// gather table, x bit and (per sample) scale are read once per step, and the
// loop over output entries is unrolled over the inputs.  The products are
// formed in the order of the general loop below (same results bit for bit).
constexpr int kFastIn = 4;
template <typename real>
struct FastIn {
  int ioff[kFastIn], xs[kFastIn];
  const uint16_t *gb[kFastIn];
  real sc[kFastIn];
};

template <typename real, bool kBwd>
__device__ inline FastIn<real> fast_inputs(const ContractArgs<real> &a, const StepDesc &sd,
                                           const StepDesc *steps,
                                           const typename FBits<real>::U *mx, int S, int sme) {
  using FB = FBits<real>;
  FastIn<real> f;
#pragma unroll
  for (int k = 0; k < kFastIn; ++k) {
    if (k < sd.n_in) {
      const InputDesc id = uload(a.inputs + sd.in_off + k);
      const StepDesc ps = uload(steps + id.step);
      f.ioff[k] = kBwd ? ps.off_all : ps.off_fwd;
      f.xs[k] = 1 << id.xbit;
      f.gb[k] = a.gtab + id.gb_off;
      f.sc[k] = FB::scale(FB::expo(mx[id.step * S + sme]));
    } else {
      f.ioff[k] = 0;
      f.xs[k] = 0;
      f.gb[k] = a.gtab;
      f.sc[k] = (real)1;
    }
  }
  return f;
}

// the two products of output entry o (eliminated spin +1 and -1), started
// from p0 and p1
template <typename real, int NI>
__device__ inline void fast_pair(const FastIn<real> &f, const real *arena, int S, int sme, int o,
                                 real &p0, real &p1) {
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    const int e = f.ioff[k] + (int)f.gb[k][o];
    p0 *= arena[e * S + sme] * f.sc[k];
    p1 *= arena[(e + f.xs[k]) * S + sme] * f.sc[k];
  }
}

// forward of a SINGLE step: out[o] = sum_x T[x, o] phi[x] prod_k m_k; returns
// this thread's largest output
template <typename real, int NI>
__device__ inline real fast_fwd(const FastIn<real> &f, const real *Tt, int w, real ph0, real ph1,
                                real *arena, int off, int S, int logS, int sme, int tid) {
  real lmax = 0;
  // kJoint entries per pass: every entry's loads before any store
  const int n = S << w;
  for (int i = tid; i < n; i += kJoint * kThreads) {
    real p0[kJoint], p1[kJoint];
    int ov[kJoint];
#pragma unroll
    for (int u = 0; u < kJoint; ++u) {
      const int iu = i + u * kThreads;
      ov[u] = (iu < n ? iu : i) >> logS;
      p0[u] = Tt[ov[u]] * ph0;
      p1[u] = Tt[(1 << w) | ov[u]] * ph1;
      fast_pair<real, NI>(f, arena, S, sme, ov[u], p0[u], p1[u]);
    }
#pragma unroll
    for (int u = 0; u < kJoint; ++u) {
      if (i + u * kThreads >= n) break;
      real acc = 0;
      acc += p0[u];
      acc += p1[u];
      arena[(off + ov[u]) * S + sme] = acc;
      lmax = acc > lmax ? acc : lmax;
    }
  }
  return lmax;
}

// Wide single-spin steps (output scope above kTabW bits, no full table):
// each input's arena offset, split gather tables, x bit and scale, and the
// step's edges (o bit and signed small factor), read once per step.
template <typename real>
struct WideIn {
  int n_in, n_e;
  int ioff[kWideIn], xs[kWideIn];
  const uint32_t *lo[kWideIn];
  const uint32_t *hi[kWideIn];
  real sc[kWideIn];
  int eb[kWideEdges];
  real es[kWideEdges];
};

template <typename real, bool kBwd>
__device__ inline WideIn<real> wide_inputs(const ContractArgs<real> &a, const StepDesc &sd,
                                           const StepDesc *steps,
                                           const typename FBits<real>::U *mx, int S, int sme) {
  using FB = FBits<real>;
  WideIn<real> f;
  f.n_in = sd.n_in;
  f.n_e = sd.n_edge;
#pragma unroll
  for (int k = 0; k < kWideIn; ++k) {
    if (k < sd.n_in) {
      const InputDesc id = uload(a.inputs + sd.in_off + k);
      const StepDesc ps = uload(steps + id.step);
      f.ioff[k] = kBwd ? ps.off_all : ps.off_fwd;
      f.xs[k] = 1 << id.xbit;
      f.lo[k] = a.gtab2 + id.gb_off;
      f.hi[k] = a.gtab2 + id.gb_off + 1024;
      f.sc[k] = FB::scale(FB::expo(mx[id.step * S + sme]));
    } else {
      f.ioff[k] = 0;
      f.xs[k] = 0;
      f.lo[k] = f.hi[k] = a.gtab2;
      f.sc[k] = (real)1;
    }
  }
#pragma unroll
  for (int e = 0; e < kWideEdges; ++e) {
    if (e < sd.n_edge) {
      f.eb[e] = uload(a.edges + sd.edge_off + e).bv;
      f.es[e] = uload(a.esmall + sd.edge_off + e);
    } else {
      f.eb[e] = 0;
      f.es[e] = (real)1;
    }
  }
  return f;
}

// p0 and p1 (output entry o, eliminated spin +1 and -1) times the step's
// transfer factors and the inputs' entries
template <typename real>
__device__ inline void wide_pair(const WideIn<real> &f, const real *arena, int S, int sme, int o,
                                 real &p0, real &p1) {
  real t0 = 1, t1 = 1;
#pragma unroll
  for (int e = 0; e < kWideEdges; ++e)
    if (e < f.n_e) {
      // J s_x s_o > 0: factor 1, else exp(-2 beta |J|); bit 1 <=> spin -1
      const int ob = (o >> f.eb[e]) & 1;
      const bool pos = f.es[e] > (real)0;
      const real sm = pos ? f.es[e] : -f.es[e];
      t0 *= ((ob == 0) == pos) ? (real)1 : sm;
      t1 *= ((ob == 1) == pos) ? (real)1 : sm;
    }
  p0 *= t0;
  p1 *= t1;
#pragma unroll
  for (int k = 0; k < kWideIn; ++k)
    if (k < f.n_in) {
      const int64_t e = (int64_t)f.ioff[k] + (int64_t)(f.lo[k][o & 1023] | f.hi[k][o >> 10]);
      p0 *= arena[e * S + sme] * f.sc[k];
      p1 *= arena[(e + f.xs[k]) * S + sme] * f.sc[k];
    }
}

// One tile of S samples of one instance through every step (forward, or
// forward then reverse), the workgroup's LDS at smem.
template <typename real, bool kGlobal, bool kBwd, bool kWide>
__device__ inline void contract_tile(const ContractArgs<real> &a, const int tile, char *smem) {
  using FB = FBits<real>;
  using U = typename FB::U;
  const int tid = threadIdx.x;
  const int q = uload(a.tile_inst + tile);
  const InstDesc D = uload(a.inst + q);
  const int S = a.S, logS = a.logS;
  const int64_t b0 = uload(a.tile_start + tile);
  const int64_t Bq = uload(a.inst_B + q);
  const int nb = (int)((Bq - b0) < S ? (Bq - b0) : S);
  const int sme = tid & (S - 1);
  const Layout Lo = make_layout(D, S, kBwd, kGlobal, (int)sizeof(real));
  U *mx = reinterpret_cast<U *>(smem + Lo.mx);
  real *phi = reinterpret_cast<real *>(smem + Lo.phi);
  real *fab = reinterpret_cast<real *>(smem + Lo.fab);
  real *arena;
  real *scr;
  if (kGlobal) {
    // one arena per tile, or per resident workgroup (a persistent launch
    // whose batch does not fit device memory at once)
    arena = a.garena + (int64_t)(a.arena_per_block ? (int)blockIdx.x : tile) * a.garena_stride;
    scr = arena + (int64_t)(kBwd ? D.arena_all : D.arena_fwd) * S;
  } else {
    arena = reinterpret_cast<real *>(smem + Lo.arena);
    scr = reinterpret_cast<real *>(smem + Lo.scr);
  }
  const StepDesc *steps = a.steps + D.step_off;
  const int8_t *spq = a.spins + uload(a.inst_spin_off + q);
  const real beta = (real)D.beta;

  for (int i = tid; i < D.n_steps * S; i += kThreads) mx[i] = 0;
  // unary factors of R (fields from h and the fixed width-set spins),
  // normalised so that the larger of the two equals one
  for (int i = tid; i < D.nr * S; i += kThreads) {
    const int p = i >> logS, s = i & (S - 1);
    real f = a.hR[D.hr_off + p];
    if (s < nb) {
      const int8_t *sp = spq + (b0 + s) * D.nw;
      const int k0 = a.fld_ptr[D.fld_off + p], k1 = a.fld_ptr[D.fld_off + p + 1];
      for (int k = k0; k < k1; ++k)
        f += a.fld_J[D.fld_nnz_off + k] * (real)sp[a.fld_w[D.fld_nnz_off + k]];
    }
    const real af = beta * (f < 0 ? -f : f);
    const real small = rexp<real>(-2 * af);
    phi[(2 * p) * S + s] = f >= 0 ? (real)1 : small;       // spin +1
    phi[(2 * p + 1) * S + s] = f >= 0 ? small : (real)1;   // spin -1
    fab[p * S + s] = af;
  }
  __syncthreads();

  // ------------------------------------------------------------ forward
  for (int t = 0; t < D.n_steps; ++t) {
    const StepDesc sd = uload(steps + t);
    const int w = sd.w, g = sd.g;
    const int off = kBwd ? sd.off_all : sd.off_fwd;
    const real *Tt = a.T + (sd.t_off >= 0 ? sd.t_off : 0);
    real lmax = 0;
    if (sd.kind == STEP_DENSE) {
      int inoff = 0;
      real insc = 1;
      if (sd.n_in) {
        const InputDesc id = uload(a.inputs + sd.in_off);
        const StepDesc ps = uload(steps + id.step);
        inoff = kBwd ? ps.off_all : ps.off_fwd;
        insc = FB::scale(FB::expo(mx[id.step * S + sme]));
      }
      for (int i = tid; i < (S << g); i += kThreads) {
        const int x = i >> logS;
        real A = 1;
        for (int j = 0; j < g; ++j) A *= phi[(2 * (sd.gpos + j) + ((x >> j) & 1)) * S + sme];
        if (sd.n_in) A *= arena[(inoff + x) * S + sme] * insc;
        scr[x * S + sme] = A;
      }
      __syncthreads();
      const int nx = 1 << g;
      for (int i = tid; i < (S << w); i += kThreads) {
        const int o = i >> logS;
        real acc = 0;
#pragma unroll 8
        for (int x = 0; x < nx; ++x) acc += Tt[(x << w) | o] * scr[x * S + sme];
        arena[(off + o) * S + sme] = acc;
        lmax = acc > lmax ? acc : lmax;
      }
    } else if (kWide && sd.t_off < 0) {
      // wide step: transfer factors from the edges, split gathers
      const WideIn<real> f = wide_inputs<real, kBwd>(a, sd, steps, mx, S, sme);
      const real ph0 = phi[(2 * sd.gpos) * S + sme], ph1 = phi[(2 * sd.gpos + 1) * S + sme];
      for (int i = tid; i < (S << w); i += kThreads) {
        const int o = i >> logS;
        real p0 = ph0, p1 = ph1;
        wide_pair<real>(f, arena, S, sme, o, p0, p1);
        real acc = 0;
        acc += p0;
        acc += p1;
        arena[((int64_t)off + o) * S + sme] = acc;
        lmax = acc > lmax ? acc : lmax;
      }
    } else if (sd.n_in <= kFastIn) {
      const FastIn<real> f = fast_inputs<real, kBwd>(a, sd, steps, mx, S, sme);
      const real ph0 = phi[(2 * sd.gpos) * S + sme], ph1 = phi[(2 * sd.gpos + 1) * S + sme];
      switch (sd.n_in) {
        case 0: lmax = fast_fwd<real, 0>(f, Tt, w, ph0, ph1, arena, off, S, logS, sme, tid); break;
        case 1: lmax = fast_fwd<real, 1>(f, Tt, w, ph0, ph1, arena, off, S, logS, sme, tid); break;
        case 2: lmax = fast_fwd<real, 2>(f, Tt, w, ph0, ph1, arena, off, S, logS, sme, tid); break;
        case 3: lmax = fast_fwd<real, 3>(f, Tt, w, ph0, ph1, arena, off, S, logS, sme, tid); break;
        default: lmax = fast_fwd<real, 4>(f, Tt, w, ph0, ph1, arena, off, S, logS, sme, tid); break;
      }
    } else {
      for (int i = tid; i < (S << w); i += kThreads) {
        const int o = i >> logS;
        real acc = 0;
        for (int x = 0; x < 2; ++x) {
          real p = Tt[(x << w) | o] * phi[(2 * sd.gpos + x) * S + sme];
          for (int k = 0; k < sd.n_in; ++k) {
            const InputDesc *id = a.inputs + sd.in_off + k;
            const StepDesc ps = steps[id->step];
            const int ioff = kBwd ? ps.off_all : ps.off_fwd;
            const real sc = FB::scale(FB::expo(mx[id->step * S + sme]));
            p *= arena[(ioff + gather_index(id, o, x)) * S + sme] * sc;
          }
          acc += p;
        }
        arena[(off + o) * S + sme] = acc;
        lmax = acc > lmax ? acc : lmax;
      }
    }
    // the step's largest entry per sample: the wave's lanes of one sample
    // first, then one LDS atomic per sample and wave
    for (int sh = S; sh < 64; sh <<= 1) {
      const real o = __shfl_xor(lmax, sh, 64);
      lmax = o > lmax ? o : lmax;
    }
    if ((tid & 63) < S && tid < (S << w)) atomicMax(&mx[t * S + sme], FB::bits(lmax));
    __syncthreads();
  }

  // ln Z_R per sample: the forward kernel's result, and the adjoint's too
  // when it is asked for (its forward sweep is the same arithmetic)
  if (!kBwd || a.logz) {
    for (int s = tid; s < nb; s += kThreads) {
      double acc = D.log_const;
      for (int p = 0; p < D.nr; ++p) acc += (double)fab[p * S + s];
      int64_t esum = 0;
      for (int t = 0; t < D.n_steps; ++t) {
        const StepDesc sd = uload(steps + t);
        if (sd.w == 0) acc += log((double)arena[(int64_t)(kBwd ? sd.off_all : sd.off_fwd) * S + s]);
        else esum += FB::expo(mx[t * S + s]);
      }
      acc += (double)esum * 0.69314718055994530942;
      a.logz[a.inst_sample_off[q] + b0 + s] = acc;
    }
    if (!kBwd) return;
    __syncthreads();
  }

  // ------------------------------------------------------------ reverse
  real *gs = reinterpret_cast<real *>(smem + Lo.gs);
  real *Mg = reinterpret_cast<real *>(smem + Lo.M);
  real *Cw = reinterpret_cast<real *>(smem + Lo.C);
  real *red = reinterpret_cast<real *>(smem + Lo.red);
  real *pb = reinterpret_cast<real *>(smem + Lo.pb);
  for (int s = tid; s < S; s += kThreads)
    gs[s] = s < nb ? (real)a.grad[a.inst_sample_off[q] + b0 + s] : (real)0;
  for (int k = tid; k < D.n_rr; k += kThreads) Cw[k] = 0;
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;

  for (int t = D.n_steps - 1; t >= 0; --t) {
    const StepDesc sd = uload(steps + t);
    const int w = sd.w, g = sd.g;
    const int off = sd.off_all;
    const real *Tt = a.T + (sd.t_off >= 0 ? sd.t_off : 0);
    const real sct = FB::scale(FB::expo(mx[t * S + sme]));
    // adjoint factor of the output entry o for sample sme
    auto rfac = [&](int o) -> real {
      const real v = arena[(off + o) * S + sme];
      if (w == 0) return v > 0 ? (real)1 / v : (real)0;
      return v * sct;
    };
    if (sd.kind == STEP_DENSE) {
      const int nx = 1 << g;
      int inoff = 0;
      real insc = 1;
      if (sd.n_in) {
        const InputDesc id = uload(a.inputs + sd.in_off);
        inoff = uload(steps + id.step).off_all;
        insc = FB::scale(FB::expo(mx[id.step * S + sme]));
      }
      real *sA = scr;                 // [x][S]
      real *sL = scr + nx * S;        // [x][w+1][S], slot w = Lambda
      for (int i = tid; i < (S << g); i += kThreads) {
        const int x = i >> logS;
        real A = 1;
        for (int j = 0; j < g; ++j) A *= phi[(2 * (sd.gpos + j) + ((x >> j) & 1)) * S + sme];
        if (sd.n_in) A *= arena[(inoff + x) * S + sme] * insc;
        real lam = 0;
        real lj[kTabW];
#pragma unroll
        for (int j = 0; j < kTabW; ++j) lj[j] = 0;
        const int no = 1 << w;
#pragma unroll 4
        for (int o = 0; o < no; ++o) {
          const real tr = Tt[(x << w) | o] * rfac(o);
          lam += tr;
#pragma unroll
          for (int j = 0; j < kTabW; ++j)
            if (j < w) lj[j] += ((o >> j) & 1) ? -tr : tr;
        }
        sA[x * S + sme] = A;
#pragma unroll
        for (int j = 0; j < kTabW; ++j)
          if (j < w) sL[(x * (w + 1) + j) * S + sme] = lj[j];
        sL[(x * (w + 1) + w) * S + sme] = lam;
      }
      __syncthreads();
      // rho of the input message: d[x] * Lambda[x]
      if (sd.n_in) {
        for (int i = tid; i < (S << g); i += kThreads) {
          const int x = i >> logS;
          real d = 1;
          for (int j = 0; j < g; ++j) d *= phi[(2 * (sd.gpos + j) + ((x >> j) & 1)) * S + sme];
          arena[(inoff + x) * S + sme] = d * sL[(x * (w + 1) + w) * S + sme];
        }
      }
      // per-sample magnetisation of the eliminated spins
      for (int i = tid; i < S * g; i += kThreads) {
        const int s = i & (S - 1), j = i >> logS;
        real m = 0;
        for (int x = 0; x < nx; ++x) {
          const real c = sA[x * S + s] * sL[(x * (w + 1) + w) * S + s];
          m += ((x >> j) & 1) ? -c : c;
        }
        Mg[(sd.gpos + j) * S + s] = m;
      }
      // gradient-weighted correlations of the R-R edges folded into T:
      // per group state x, P[x][j] = sum_s g_s A_s[x] Lambda_{s,j}[x]
      for (int i = tid; i < nx * (w + 1); i += kThreads) {
        const int x = i / (w + 1), j = i - x * (w + 1);
        real acc = 0;
        for (int s = 0; s < S; ++s) acc += gs[s] * sA[x * S + s] * sL[(x * (w + 1) + j) * S + s];
        pb[i] = acc;
      }
      __syncthreads();
      for (int k = tid; k < sd.n_edge; k += kThreads) {
        const EdgeDesc ed = a.edges[sd.edge_off + k];
        const int ju = ed.bu - w;
        const bool vin = ed.bv >= w;
        const int jv = vin ? ed.bv - w : ed.bv;
        real acc = 0;
        for (int x = 0; x < nx; ++x) {
          real c = vin ? (((x >> jv) & 1) ? -pb[x * (w + 1) + w] : pb[x * (w + 1) + w])
                       : pb[x * (w + 1) + jv];
          acc += ((x >> ju) & 1) ? -c : c;
        }
        Cw[ed.rr] = acc;
      }
      __syncthreads();
    } else {
      // SINGLE: joint weights c(o, x) into scratch [(o*2 + x)][S]
      if (kWide && sd.t_off < 0) {
        const WideIn<real> f = wide_inputs<real, true>(a, sd, steps, mx, S, sme);
        const real ph0 = phi[(2 * sd.gpos) * S + sme], ph1 = phi[(2 * sd.gpos + 1) * S + sme];
        for (int i = tid; i < (S << w); i += kThreads) {
          const int o = i >> logS;
          const real r = rfac(o);
          real p0 = r * ph0, p1 = r * ph1;
          wide_pair<real>(f, arena, S, sme, o, p0, p1);
          scr[(o * 2) * S + sme] = p0;
          scr[(o * 2 + 1) * S + sme] = p1;
        }
      } else if (sd.n_in <= kFastIn) {
        const FastIn<real> f = fast_inputs<real, true>(a, sd, steps, mx, S, sme);
        const real ph0 = phi[(2 * sd.gpos) * S + sme], ph1 = phi[(2 * sd.gpos + 1) * S + sme];
        auto joint = [&](auto ni) {
          constexpr int NI = decltype(ni)::value;
          // kJoint entries per pass: every entry's loads before any store
          const int n = S << w;
          for (int i = tid; i < n; i += kJoint * kThreads) {
            real p0[kJoint], p1[kJoint];
            int ov[kJoint];
#pragma unroll
            for (int u = 0; u < kJoint; ++u) {
              const int iu = i + u * kThreads;
              ov[u] = (iu < n ? iu : i) >> logS;
              const real r = rfac(ov[u]);
              p0[u] = r * Tt[ov[u]] * ph0;
              p1[u] = r * Tt[(1 << w) | ov[u]] * ph1;
              fast_pair<real, NI>(f, arena, S, sme, ov[u], p0[u], p1[u]);
            }
#pragma unroll
            for (int u = 0; u < kJoint; ++u) {
              if (i + u * kThreads >= n) break;
              scr[(ov[u] * 2) * S + sme] = p0[u];
              scr[(ov[u] * 2 + 1) * S + sme] = p1[u];
            }
          }
        };
        switch (sd.n_in) {
          case 0: joint(std::integral_constant<int, 0>{}); break;
          case 1: joint(std::integral_constant<int, 1>{}); break;
          case 2: joint(std::integral_constant<int, 2>{}); break;
          case 3: joint(std::integral_constant<int, 3>{}); break;
          default: joint(std::integral_constant<int, 4>{}); break;
        }
      } else
      for (int i = tid; i < (S << w); i += kThreads) {
        const int o = i >> logS;
        const real r = rfac(o);
        for (int x = 0; x < 2; ++x) {
          real p = r * Tt[(x << w) | o] * phi[(2 * sd.gpos + x) * S + sme];
          for (int k = 0; k < sd.n_in; ++k) {
            const InputDesc *id = a.inputs + sd.in_off + k;
            const StepDesc ps = steps[id->step];
            const real sc = FB::scale(FB::expo(mx[id->step * S + sme]));
            p *= arena[(ps.off_all + gather_index(id, o, x)) * S + sme] * sc;
          }
          scr[(o * 2 + x) * S + sme] = p;
        }
      }
      __syncthreads();
      // rho of every input: marginal of its scope over its scaled value
      for (int k = 0; k < sd.n_in; ++k) {
        const InputDesc id = uload(a.inputs + sd.in_off + k);
        const StepDesc ps = uload(steps + id.step);
        const real sc = FB::scale(FB::expo(mx[id.step * S + sme]));
        const int omask = id.omask;
        const int freem = ((1 << w) - 1) & ~omask;
        // 2^lc lanes share one (entry, sample) sum: each takes one pattern of
        // the lowest lc free bits and walks the others, and the wave adds
        // the lanes' parts (lc aims at two passes of the workgroup; a lane
        // group never leaves its wave)
        int lc = kLogThreads + 1 - logS - id.nbits;
        lc = lc < 0 ? 0 : lc;
        lc = lc < 6 - logS ? lc : 6 - logS;
        lc = lc < __popc(freem) ? lc : __popc(freem);
        int highm = freem;
        for (int b = 0; b < lc; ++b) highm &= highm - 1;
        const int nit = 1 << __popc(highm);
        for (int i = tid; i < (S << (id.nbits + lc)); i += kThreads) {
          const int c = (i >> logS) & ((1 << lc) - 1);
          const int j = i >> (logS + lc);
          // entry j: the eliminated spin's bit, the others deposited in
          // order on the output bits of the scope (both scopes ascend)
          const int x = (j >> id.xbit) & 1;
          int rest = ((j >> (id.xbit + 1)) << id.xbit) | (j & ((1 << id.xbit) - 1));
          int ofix = 0;
          for (int om = omask; om; om &= om - 1) {
            if (rest & 1) ofix |= om & -om;
            rest >>= 1;
          }
          int mm = freem & ~highm;
          for (int b = 0; b < lc; ++b) {
            const int lsb = mm & -mm;
            if ((c >> b) & 1) ofix |= lsb;
            mm ^= lsb;
          }
          // the subsets z of highm in increasing order, four at a time
          const real *col = scr + x * S + sme;
          real m0 = 0, m1 = 0, m2 = 0, m3 = 0;
          int z = 0;
          if (nit >= 4) {
            for (int it = 0; it < nit; it += 4) {
              const int z1 = (z - highm) & highm, z2 = (z1 - highm) & highm;
              const int z3 = (z2 - highm) & highm;
              m0 += col[(int64_t)((ofix | z) * 2) * S];
              m1 += col[(int64_t)((ofix | z1) * 2) * S];
              m2 += col[(int64_t)((ofix | z2) * 2) * S];
              m3 += col[(int64_t)((ofix | z3) * 2) * S];
              z = (z3 - highm) & highm;
            }
          } else {
            for (int it = 0; it < nit; ++it) {
              m0 += col[(int64_t)((ofix | z) * 2) * S];
              z = (z - highm) & highm;
            }
          }
          real mu = (m0 + m1) + (m2 + m3);
          for (int sh = S; sh < (S << lc); sh <<= 1) mu += __shfl_xor(mu, sh, 64);
          if (c == 0) {
            real *slot = &arena[((int64_t)ps.off_all + j) * S + sme];
            const real m = *slot * sc;
            *slot = m > 0 ? mu / m : (real)0;
          }
        }
      }
      // per-sample sums over o: magnetisation of v and its edge correlations
      const int K = 1 + sd.n_edge;
      for (int c0 = 0; c0 < K; c0 += kRed) {
        real v[kRed];
        int ob[kRed];
#pragma unroll
        for (int r = 0; r < kRed; ++r) {
          v[r] = 0;
          const int k = c0 + r;
          ob[r] = (k == 0 || k >= K) ? -1 : uload(a.edges + sd.edge_off + k - 1).bv;
        }
        for (int i = tid; i < (S << w); i += kThreads) {
          const int o = i >> logS;
          const real dlt = scr[(o * 2) * S + sme] - scr[(o * 2 + 1) * S + sme];
#pragma unroll
          for (int r = 0; r < kRed; ++r)
            v[r] += (ob[r] >= 0 && ((o >> ob[r]) & 1)) ? -dlt : dlt;
        }
#pragma unroll
        for (int r = 0; r < kRed; ++r)
          for (int sh = S; sh < 64; sh <<= 1) v[r] += __shfl_xor(v[r], sh, 64);
        if (lane < S) {
#pragma unroll
          for (int r = 0; r < kRed; ++r) red[(wave * kRed + r) * S + lane] = v[r];
        }
        __syncthreads();
        // value r of sample s: the waves' parts added in wave order, read
        // where it is used (no second pass through LDS)
        auto wsum = [&](int i) {
          real sum = 0;
          for (int wv = 0; wv < kWaves; ++wv) sum += red[(wv * kRed) * S + i];
          return sum;
        };
        for (int r = tid; r < kRed; r += kThreads) {
          const int k = c0 + r;
          if (k == 0) {
            // handled below (per sample)
          } else if (k < K) {
            real acc = 0;
            for (int s = 0; s < S; ++s) acc += gs[s] * wsum(r * S + s);
            Cw[a.edges[sd.edge_off + k - 1].rr] = acc;
          }
        }
        if (c0 == 0)
          for (int s = tid; s < S; s += kThreads) Mg[sd.gpos * S + s] = wsum(s);
        __syncthreads();
      }
    }
  }

  // ------------------------------------------------- per-tile partial row
  const int64_t prow = a.inst_partial_off[q] +
                       (int64_t)(tile - a.inst_first_tile[q]) * D.n_partial;
  for (int p = tid; p < D.nr; p += kThreads) {
    real acc = 0;
    for (int s = 0; s < S; ++s) acc += gs[s] * Mg[p * S + s];
    a.partial[prow + p] = acc;
  }
  for (int k = tid; k < D.n_wr; k += kThreads) {
    const int p = a.wr_pos[D.wr_off + k], wi = a.wr_w[D.wr_off + k];
    real acc = 0;
    for (int s = 0; s < nb; ++s)
      acc += gs[s] * (real)spq[(b0 + s) * D.nw + wi] * Mg[p * S + s];
    a.partial[prow + D.nr + k] = acc;
  }
  for (int k = tid; k < D.n_rr; k += kThreads) a.partial[prow + D.nr + D.n_wr + k] = Cw[k];
}

template <typename real, bool kGlobal, bool kBwd, bool kWide>
__global__ __launch_bounds__(kThreads) void contract_kernel(ContractArgs<real> a) {
  extern __shared__ __align__(16) char smem[];
  contract_tile<real, kGlobal, kBwd, kWide>(a, blockIdx.x, smem);
}

// Persistent form: the launch's workgroups take tiles from a device counter
// (a.pq[0]) in tile order (the instances with the costliest samples first)
// until none is left; the last workgroup to leave resets the counter and
// its exit count (a.pq[1]) for the next launch on the stream.
template <typename real, bool kGlobal, bool kBwd, bool kWide>
__global__ __launch_bounds__(kThreads) void contract_pq_kernel(ContractArgs<real> a, int n_tiles) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int next;
  for (;;) {
    __syncthreads();   // every thread has read `next` and left the last tile
    if (threadIdx.x == 0) next = atomicAdd(a.pq, 1);
    __syncthreads();
    const int tile = __builtin_amdgcn_readfirstlane(next);   // the same in every lane
    if (tile >= n_tiles) break;
    contract_tile<real, kGlobal, kBwd, kWide>(a, tile, smem);
  }
  if (threadIdx.x == 0 && atomicAdd(a.pq + 1, 1) == (int)gridDim.x - 1) {
    atomicExch(a.pq, 0);
    atomicExch(a.pq + 1, 0);
  }
}

// Column sums of the per-tile partial rows of every instance (rows in a
// fixed order, FP64): 16 columns x 16 row groups per block.
// Column sums of the partial rows in two passes with a fixed order: block
// (column group, row split, instance) sums its rows for 64 columns (four
// row lanes, then through LDS), then one thread per column adds the splits.
constexpr int kColSplit = 32;
template <typename real>
__global__ __launch_bounds__(256) void vjp_colsum_kernel(VjpArgs a, const real *partial) {
  __shared__ double sh[4][64];
  const int q = blockIdx.z, sp = blockIdx.y;
  const InstDesc D = a.inst[q];
  const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + c;
  const int nt = a.inst_n_tiles[q];
  const int per = (nt + kColSplit - 1) / kColSplit;
  const int r0 = sp * per, r1 = r0 + per < nt ? r0 + per : nt;
  const int64_t pb = a.inst_partial_off[q];
  double acc = 0.0;
  if (k < D.n_partial) {
#pragma unroll 4
    for (int t = r0 + rl; t < r1; t += 4) acc += (double)partial[pb + (int64_t)t * D.n_partial + k];
  }
  sh[rl][c] = acc;
  __syncthreads();
  if (rl == 0 && k < D.n_partial)
    a.part2[((int64_t)q * kColSplit + sp) * a.maxo + a.col_out[a.inst_sum_off[q] + k]] =
        (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
}

// Every output of the adjoint in one launch, one block per instance: dh
// over the instance's vertices and dJ over its edges, each the fixed-order
// sum of its split column sums (stored in output order; 0 for W vertices
// and W-W edges) times beta, and dbeta = sum over outputs of coefficient x
// column sum (per-thread sums in index order, then a fixed tree).
constexpr int kFinishThreads = 1024;
__global__ __launch_bounds__(kFinishThreads) void vjp_finish_kernel(VjpArgs a) {
  __shared__ double sh[kFinishThreads];
  const int q = blockIdx.x;
  const InstDesc D = a.inst[q];
  const int64_t vb = a.inst_spin_base[q], eb = a.inst_edge_base[q];
  const double *p2 = a.part2 + (int64_t)q * kColSplit * a.maxo;
  const double *pc = a.pcoef_out + vb + eb;
  double contrib = 0.0;
  for (int idx = threadIdx.x; idx < D.n + D.n_edges; idx += kFinishThreads) {
    double c[kColSplit];
#pragma unroll
    for (int sp = 0; sp < kColSplit; ++sp) c[sp] = p2[(int64_t)sp * a.maxo + idx];
    const double w = pc[idx];
    double S = 0.0;
#pragma unroll
    for (int sp = 0; sp < kColSplit; ++sp) S += c[sp];
    contrib += w * S;
    if (idx < D.n) a.dh[vb + idx] = D.beta * S;
    else a.dJ[eb + idx - D.n] = D.beta * S;
  }
  sh[threadIdx.x] = contrib;
  __syncthreads();
  for (int st = kFinishThreads / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.dbeta[q] = sh[0];
}


}  // namespace

size_t contract_lds_bytes(const InstDesc &D, int S, bool bwd, bool global_arena,
                          int real_size) {
  return make_layout(D, S, bwd, global_arena, real_size).end;
}

int64_t contract_garena_entries(const InstDesc &D, int S, bool bwd) {
  return (int64_t)((bwd ? D.arena_all : D.arena_fwd) + (bwd ? D.scr_bwd : D.scr_fwd)) * S;
}

template <typename real>
hipError_t launch_contract(const ContractArgs<real> &a, int n_tiles, size_t lds,
                           bool bwd, bool global_arena, hipStream_t st, bool persistent,
                           int max_grid) {
  if (n_tiles <= 0) return hipSuccess;
  if (a.wide && !global_arena) return hipErrorInvalidValue;
  if (persistent) {
    // (nets with wide steps always have their arena in device memory)
    void (*k)(ContractArgs<real>, int);
    if (a.wide) k = bwd ? contract_pq_kernel<real, true, true, true> : contract_pq_kernel<real, true, false, true>;
    else if (bwd) k = global_arena ? contract_pq_kernel<real, true, true, false> : contract_pq_kernel<real, false, true, false>;
    else k = global_arena ? contract_pq_kernel<real, true, false, false> : contract_pq_kernel<real, false, false, false>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    // as many workgroups as are resident at once, at most one per tile
    int dev = 0, cus = 0, per = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
        (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(k),
                                                          kThreads, lds)) != hipSuccess)
      return e;
    int grid = std::max(1, std::min(n_tiles, cus * std::max(per, 1)));
    if (max_grid > 0) grid = std::min(grid, max_grid);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, st, a, n_tiles);
    return hipGetLastError();
  }
  void (*k)(ContractArgs<real>);
  if (a.wide) k = bwd ? contract_kernel<real, true, true, true> : contract_kernel<real, true, false, true>;
  else if (bwd) k = global_arena ? contract_kernel<real, true, true, false> : contract_kernel<real, false, true, false>;
  else k = global_arena ? contract_kernel<real, true, false, false> : contract_kernel<real, false, false, false>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(n_tiles), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_vjp_reduce(const VjpArgs &a, const real *partial, int n_inst, int max_partial,
                             hipStream_t st) {
  if (n_inst <= 0 || max_partial <= 0) return hipSuccess;
  hipLaunchKernelGGL(vjp_colsum_kernel<real>, dim3((max_partial + 63) / 64, kColSplit, n_inst),
                     dim3(256), 0, st, a, partial);
  hipLaunchKernelGGL(vjp_finish_kernel, dim3(n_inst), dim3(kFinishThreads), 0, st, a);
  return hipGetLastError();
}

int vjp_split() { return kColSplit; }


template hipError_t launch_contract<float>(const ContractArgs<float> &, int, size_t, bool, bool, hipStream_t, bool, int);
template hipError_t launch_contract<double>(const ContractArgs<double> &, int, size_t, bool, bool, hipStream_t, bool, int);
template hipError_t launch_vjp_reduce<float>(const VjpArgs &, const float *, int, int, hipStream_t);
template hipError_t launch_vjp_reduce<double>(const VjpArgs &, const double *, int, int, hipStream_t);

}  // namespace tnvan
