// Transfer-matrix form of the conditional contraction on the matrix cores.
//
// A chain of dense steps (a lattice strip eliminated row by row, or the two
// blocks of the SK remainder) is contracted as a product of per-sample
// diagonals and static transfer matrices (Sec. 2, Eqs. 2-4):
//
//   A_0 = d_0,  out_t = A_t . T_t,  A_{t+1} = d_{t+1} * (out_t / 2^e_t)
//
// where A_t is [16 samples x K] and T_t is [K x N].  One wavefront owns one
// chain for 16 samples and never waits for other waves: the products run on
// 16x16x4 FP32 (or 16x16x32 BF16 with FP32 accumulation) MFMA tiles, the
// per-sample power-of-two rescale is a max over the accumulator rows, and
// the next A is written back to the wave's LDS slice in operand order.
//
// The adjoint recomputes the chain from checkpoints kept every k steps in
// LDS and walks back with R_t = rho_t 2^-e_t (rho = marginal / scaled
// message, as in the generic kernel):
//   Lambda_t = R_t . T_t^T                       (MFMA, samples x K)
//   magnetisation of the group spins   sum_x sigma_j(x) A_t Lambda_t
//   R_{t-1} = d_t * Lambda_t / 2^e_{t-1}
//   H_t = (g A_t)^T . R_t                        (MFMA over the 16 samples)
//   edge correlations  sum_{x,o} T_t H_t sigma_u sigma_v
// and writes the gradient-weighted sums of one 16-sample group into one
// partial row (every entry of the row is owned by exactly one chain).
#include <hip/hip_runtime.h>

#include "launch.h"

namespace tnvan {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

constexpr int CW = 16;     // samples per wave
// NTM (template): largest number of 16-wide tiles of K or N in a launch
constexpr int kGM = 8;     // largest group

__device__ inline void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int expo32(float m) {
  const int E = (int)((__float_as_uint(m) >> 23) & 0xffu);
  const int e = E - 126;
  return e > 126 ? 126 : e;
}
__device__ inline float pow2neg(int e) { return __uint_as_float((uint32_t)(127 - e) << 23); }

struct WL {
  int lda;
  size_t phi, lz, es, Aw, gs, raw, ex, M, pb, R0, R1, ck, buf, end;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline WL wave_layout(const ChainInst &C, bool bwd, int kseg) {
  WL L{};
  L.lda = C.kbuf + 4;
  L.buf = al16((size_t)CW * L.lda * 4);
  size_t o = 0;
  L.phi = o; o = al16(o + (size_t)C.npos_max * 2 * CW * 4);
  L.lz = o;  o = al16(o + CW * 8);
  L.es = o;  o = al16(o + CW * 4);
  L.Aw = o;  o += L.buf;
  if (bwd) {
    L.gs = o;  o = al16(o + CW * 4);
    L.raw = o; o = al16(o + CW * 4);
    L.ex = o;  o = al16(o + (size_t)C.max_steps * CW * 4);
    L.M = o;   o = al16(o + (size_t)kGM * CW * 4);
    L.pb = o;  o = al16(o + (size_t)C.pmax * 4);
    L.R0 = o;  o += L.buf;
    L.R1 = o;  o += L.buf;
    const int nc = (C.max_steps + kseg - 1) / kseg + (kseg - 1);
    L.ck = o;  o += (size_t)nc * L.buf;
  }
  L.end = al16(o);
  return L;
}

// One forward step of a chain for the wave's 16 samples: Aout <- scaled
// product times the next step's diagonal.  Returns the per-row exponents.
template <bool kBF, int NTM>
__device__ inline void chain_step(const ChainArgs &a, const ChainStep &cs, const ChainStep &nx,
                                  const float *Ain, float *Aout, int lda, int kbuf,
                                  const float *phi, int pos_lo, int lane, int e[4]) {
  const int ls = lane & 15, lg = lane >> 4;
  const int NT = cs.np >> 4;
  f4 acc[NTM];
#pragma unroll
  for (int nt = 0; nt < NTM; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
  if (!kBF) {
    const float *tp = a.Tp + cs.tp_off + ls;
    for (int kc = 0; kc < (cs.kp >> 2); ++kc) {
      const float av = Ain[ls * lda + 4 * kc + lg];
      const float *tb = tp + (int64_t)(4 * kc + lg) * cs.np;
#pragma unroll
      for (int nt = 0; nt < NTM; ++nt)
        if (nt < NT) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, tb[16 * nt], acc[nt], 0, 0, 0);
    }
  } else {
    const int KC = cs.kb >> 5;
    const u4v *tb = reinterpret_cast<const u4v *>(a.Tb + cs.tb_off);
    for (int kc = 0; kc < KC; ++kc) {
      bf8 av;
      const float *ap = Ain + ls * lda + 32 * kc + 8 * lg;
#pragma unroll
      for (int i = 0; i < 8; ++i) av[i] = (__bf16)ap[i];
#pragma unroll
      for (int nt = 0; nt < NTM; ++nt)
        if (nt < NT) {
          const u4v raw = tb[((int64_t)nt * KC + kc) * 64 + lane];
          const bf8 bv = __builtin_bit_cast(bf8, raw);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
        }
    }
  }
  float m[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int nt = 0; nt < NTM; ++nt)
    if (nt < NT)
#pragma unroll
      for (int r = 0; r < 4; ++r) m[r] = fmaxf(m[r], acc[nt][r]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    for (int off = 1; off < 16; off <<= 1) m[r] = fmaxf(m[r], __shfl_xor(m[r], off, 64));
    e[r] = expo32(m[r]);
  }
  wsync();   // every read of Ain precedes the writes (Aout may alias Ain)
  const int N = 1 << cs.w;
  const int gN = nx.g, poN = nx.gpos - pos_lo;
#pragma unroll
  for (int nt = 0; nt < NTM; ++nt)
    if (nt < NT)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * nt + ls, s = 4 * lg + r;
        float v = 0.f;
        if (o < N) {
          v = acc[nt][r] * pow2neg(e[r]);
          for (int j = 0; j < gN; ++j) v *= phi[((poN + j) * 2 + ((o >> j) & 1)) * CW + s];
        }
        Aout[s * lda + o] = v;
      }
  for (int i = lane; i < CW * (kbuf - cs.np); i += 64) Aout[(i & 15) * lda + cs.np + (i >> 4)] = 0.f;
  wsync();
}

// A_0 = d_0 (columns beyond K are zero)
__device__ inline void chain_first(const ChainStep &cs, float *A, int lda, int kbuf,
                                   const float *phi, int pos_lo, int lane) {
  const int K = 1 << cs.g, po = cs.gpos - pos_lo;
  for (int i = lane; i < CW * kbuf; i += 64) {
    const int s = i & 15, x = i >> 4;
    float v = 0.f;
    if (x < K) {
      v = 1.f;
      for (int j = 0; j < cs.g; ++j) v *= phi[((po + j) * 2 + ((x >> j) & 1)) * CW + s];
    }
    A[s * lda + x] = v;
  }
  wsync();
}

// raw root value sum_x A[s][x] T[x] of sample (lane & 15), on every lane
__device__ inline float chain_root(const ChainArgs &a, const ChainStep &cs, const float *A,
                                   int lda, int lane) {
  const int ls = lane & 15, lg = lane >> 4;
  const int K = 1 << cs.g;
  const float *T = a.Tp + cs.tp_off;
  float part = 0.f;
  for (int x = lg; x < K; x += 4) part += A[ls * lda + x] * T[x];
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part;
}

// unary factors of the chain's positions, normalised to max 1; returns the
// sum of beta |f| of sample (lane & 15)
__device__ inline double chain_phi(const ChainArgs &a, const InstDesc &D, const ChainDesc &cd,
                                   float *phi, int64_t b0, int nb, int lane) {
  double fab = 0.0;
  const int npos = cd.pos_hi - cd.pos_lo;
  const float beta = (float)D.beta;
  for (int i = lane; i < npos * CW; i += 64) {
    const int pl = i >> 4, s = i & 15;
    const int p = cd.pos_lo + pl;
    float f = a.hR[D.hr_off + p];
    if (s < nb) {
      const int8_t *sp = a.spins + (b0 + s) * D.nw;
      const int k0 = a.fld_ptr[D.fld_off + p], k1 = a.fld_ptr[D.fld_off + p + 1];
      for (int k = k0; k < k1; ++k)
        f += a.fld_J[D.fld_nnz_off + k] * (float)sp[a.fld_w[D.fld_nnz_off + k]];
    }
    const float af = beta * fabsf(f);
    const float sm = expf(-2.f * af);
    phi[(pl * 2) * CW + s] = f >= 0.f ? 1.f : sm;
    phi[(pl * 2 + 1) * CW + s] = f >= 0.f ? sm : 1.f;
    fab += (double)af;
  }
  fab += __shfl_xor(fab, 16, 64);
  fab += __shfl_xor(fab, 32, 64);
  wsync();
  return fab;
}

template <bool kBF, int NTM>
__global__ __launch_bounds__(256) void chain_fwd_kernel(ChainArgs a, int wpb) {
  extern __shared__ __align__(16) char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int task = blockIdx.x * wpb + wave;
  if (task >= a.n_tasks) return;
  const int q = a.task_inst[task], c = a.task_chain[task];
  const int64_t b0 = a.task_start[task];
  const InstDesc D = a.inst[q];
  const ChainInst C = a.cinst[q];
  const ChainDesc cd = a.chains[C.chain_off + c];
  const ChainStep *cs = a.csteps + cd.cs_off;
  const int64_t Bq = a.inst_B[q];
  const int nb = (int)((Bq - b0) < CW ? (Bq - b0) : CW);
  const WL L = wave_layout(C, false, 1);
  char *base = smem + (size_t)wave * a.wave_lds;
  float *phi = reinterpret_cast<float *>(base + L.phi);
  int *es = reinterpret_cast<int *>(base + L.es);
  float *A = reinterpret_cast<float *>(base + L.Aw);
  ChainArgs aq = a;
  aq.spins = a.spins + a.inst_spin_off[q];
  const double fab = chain_phi(aq, D, cd, phi, b0, nb, lane);
  chain_first(cs[0], A, L.lda, C.kbuf, phi, cd.pos_lo, lane);
  int esum[4] = {0, 0, 0, 0};
  float raw = 1.f;
  for (int t = 0; t < cd.n_steps; ++t) {
    const ChainStep st = cs[t];
    if (st.w == 0) {
      raw = chain_root(a, st, A, L.lda, lane);
      break;
    }
    int e[4];
    chain_step<kBF, NTM>(a, st, cs[t + 1], A, A, L.lda, C.kbuf, phi, cd.pos_lo, lane, e);
#pragma unroll
    for (int r = 0; r < 4; ++r) esum[r] += e[r];
  }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) es[4 * (lane >> 4) + r] = esum[r];
  }
  wsync();
  if (lane < nb) {
    const double v = fab + (double)es[lane] * 0.69314718055994530942 + log((double)raw);
    a.cpart[a.cpart_off[q] + (int64_t)c * Bq + b0 + lane] = v;
  }
}

template <bool kBF, int NTM>
__global__ __launch_bounds__(256) void chain_bwd_kernel(ChainArgs a, int wpb) {
  extern __shared__ __align__(16) char smem[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int task = blockIdx.x * wpb + wave;
  if (task >= a.n_tasks) return;
  const int ls = lane & 15, lg = lane >> 4;
  const int q = a.task_inst[task], c = a.task_chain[task];
  const int64_t b0 = a.task_start[task];
  const InstDesc D = a.inst[q];
  const ChainInst C = a.cinst[q];
  const ChainDesc cd = a.chains[C.chain_off + c];
  const ChainStep *cs = a.csteps + cd.cs_off;
  const int64_t Bq = a.inst_B[q];
  const int nb = (int)((Bq - b0) < CW ? (Bq - b0) : CW);
  const int kseg = a.kseg;
  const WL L = wave_layout(C, true, kseg);
  const int lda = L.lda, kbuf = C.kbuf;
  char *base = smem + (size_t)wave * a.wave_lds;
  float *phi = reinterpret_cast<float *>(base + L.phi);
  float *Aw = reinterpret_cast<float *>(base + L.Aw);
  float *gs = reinterpret_cast<float *>(base + L.gs);
  float *rawb = reinterpret_cast<float *>(base + L.raw);
  int *ex = reinterpret_cast<int *>(base + L.ex);
  float *Ms = reinterpret_cast<float *>(base + L.M);
  float *pb = reinterpret_cast<float *>(base + L.pb);
  float *Rc = reinterpret_cast<float *>(base + L.R0);
  float *Rn = reinterpret_cast<float *>(base + L.R1);
  auto ck = [&](int i) { return reinterpret_cast<float *>(base + L.ck + (size_t)i * L.buf); };
  const int8_t *spq = a.spins + a.inst_spin_off[q];
  ChainArgs aq = a;
  aq.spins = spq;
  chain_phi(aq, D, cd, phi, b0, nb, lane);
  if (lane < CW) gs[lane] = lane < nb ? (float)a.grad[a.inst_sample_off[q] + b0 + lane] : 0.f;
  const int T = cd.n_steps;
  const int NC = (T + kseg - 1) / kseg;
  const int64_t row = a.inst_partial_off[q] + (b0 / CW) * (int64_t)D.n_partial;
  float *prow = a.partial + row;

  // forward with checkpoints every kseg steps
  chain_first(cs[0], ck(0), lda, kbuf, phi, cd.pos_lo, lane);
  for (int t = 0; t < T; ++t) {
    const ChainStep st = cs[t];
    float *Ain = (t % kseg == 0) ? ck(t / kseg) : Aw;
    if (st.w == 0) {
      const float raw = chain_root(a, st, Ain, lda, lane);
      if (lane < CW) rawb[lane] = raw;
      wsync();
      break;
    }
    float *Aout = ((t + 1) % kseg == 0) ? ck((t + 1) / kseg) : Aw;
    int e[4];
    chain_step<kBF, NTM>(a, st, cs[t + 1], Ain, Aout, lda, kbuf, phi, cd.pos_lo, lane, e);
    if (ls == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) ex[t * CW + 4 * lg + r] = e[r];
    }
    wsync();
  }

  for (int seg = NC - 1; seg >= 0; --seg) {
    const int t0 = seg * kseg;
    const int t1 = (t0 + kseg) < T ? (t0 + kseg) : T;
    auto sbuf = [&](int j) { return j == 0 ? ck(seg) : ck(NC + j - 1); };
    for (int t = t0; t < t1 - 1; ++t) {
      int e[4];
      chain_step<kBF, NTM>(a, cs[t], cs[t + 1], sbuf(t - t0), sbuf(t + 1 - t0), lda, kbuf, phi,
                      cd.pos_lo, lane, e);
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const ChainStep st = cs[t];
      const float *A = sbuf(t - t0);
      const int g = st.g, w = st.w, K = 1 << g;
      const int po = st.gpos - cd.pos_lo;
      const bool has_prev = t > 0;
      float Macc[4][kGM];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < kGM; ++j) Macc[r][j] = 0.f;
      if (w == 0) {
        // closing step: R = 1 / raw, Lambda[s][x] = T[x] R[s]
        const float *Tr = a.Tp + st.tp_off;
        const float rinv = rawb[ls] > 0.f ? 1.f / rawb[ls] : 0.f;
        const float sc = has_prev ? pow2neg(ex[(t - 1) * CW + ls]) : 1.f;
        float mloc[kGM];
#pragma unroll
        for (int j = 0; j < kGM; ++j) mloc[j] = 0.f;
        for (int x = lg; x < st.kp; x += 4) {
          const float lam = x < K ? Tr[x] * rinv : 0.f;
          const float cval = A[ls * lda + x] * lam;
#pragma unroll
          for (int j = 0; j < kGM; ++j)
            if (j < g) mloc[j] += ((x >> j) & 1) ? -cval : cval;
          if (has_prev) {
            float d = 1.f;
            for (int j = 0; j < g; ++j) d *= phi[((po + j) * 2 + ((x >> j) & 1)) * CW + ls];
            Rn[ls * lda + x] = d * lam * sc;
          }
        }
#pragma unroll
        for (int j = 0; j < kGM; ++j) {
          mloc[j] += __shfl_xor(mloc[j], 16, 64);
          mloc[j] += __shfl_xor(mloc[j], 32, 64);
        }
        if (lg == 0) {
#pragma unroll
          for (int j = 0; j < kGM; ++j)
            if (j < g) Ms[j * CW + ls] = mloc[j];
        }
        if (has_prev)
          for (int i = lane; i < CW * (kbuf - st.kp); i += 64) Rn[(i & 15) * lda + st.kp + (i >> 4)] = 0.f;
        // per-state sums for the edges inside the last group
        for (int x = lane; x < K; x += 64) {
          float acc = 0.f;
          for (int s = 0; s < CW; ++s) acc += gs[s] * A[s * lda + x] * Tr[x] * (rawb[s] > 0.f ? 1.f / rawb[s] : 0.f);
          pb[x] = acc;
        }
        wsync();
      } else {
        const int NT = st.np >> 4, KT = st.kp >> 4;
        // Lambda = R . T^T  (samples x K)
        f4 lam[NTM];
#pragma unroll
        for (int xt = 0; xt < NTM; ++xt) lam[xt] = f4{0.f, 0.f, 0.f, 0.f};
        const float *tt = a.Tt + st.tt_off + ls;
        for (int kc = 0; kc < (st.np >> 2); ++kc) {
          const float av = Rc[ls * lda + 4 * kc + lg];
          const float *tb = tt + (int64_t)(4 * kc + lg) * st.kp;
#pragma unroll
          for (int xt = 0; xt < NTM; ++xt)
            if (xt < KT) lam[xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, tb[16 * xt], lam[xt], 0, 0, 0);
        }
        // magnetisations and R of the previous step
        float scp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) scp[r] = has_prev ? pow2neg(ex[(t - 1) * CW + 4 * lg + r]) : 1.f;
#pragma unroll
        for (int xt = 0; xt < NTM; ++xt)
          if (xt < KT)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int x = 16 * xt + ls, s = 4 * lg + r;
              float cval = 0.f, rn = 0.f;
              if (x < K) {
                cval = A[s * lda + x] * lam[xt][r];
                if (has_prev) {
                  float d = 1.f;
                  for (int j = 0; j < g; ++j) d *= phi[((po + j) * 2 + ((x >> j) & 1)) * CW + s];
                  rn = d * lam[xt][r] * scp[r];
                }
              }
#pragma unroll
              for (int j = 0; j < kGM; ++j)
                if (j < g) Macc[r][j] += ((x >> j) & 1) ? -cval : cval;
              if (has_prev) Rn[s * lda + x] = rn;
            }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < kGM; ++j)
            for (int off = 1; off < 16; off <<= 1) Macc[r][j] += __shfl_xor(Macc[r][j], off, 64);
        if (ls == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int j = 0; j < kGM; ++j)
              if (j < g) Ms[j * CW + 4 * lg + r] = Macc[r][j];
        }
        if (has_prev)
          for (int i = lane; i < CW * (kbuf - st.kp); i += 64) Rn[(i & 15) * lda + st.kp + (i >> 4)] = 0.f;
        // H = (g A)^T R over the 16 samples, then per-state partial sums
        if (st.n_edge > 0) {
          const int N = 1 << w;
          const float *Tp = a.Tp + st.tp_off;
          for (int mt = 0; mt < KT; ++mt) {
            float P[4][kGM + 1];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int j = 0; j <= kGM; ++j) P[r][j] = 0.f;
            float ga[4];
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
              const int s = 4 * kc + lg;
              ga[kc] = gs[s] * A[s * lda + 16 * mt + ls];
            }
            for (int nt = 0; nt < NT; ++nt) {
              f4 h = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
              for (int kc = 0; kc < 4; ++kc) {
                const float bv = Rc[(4 * kc + lg) * lda + 16 * nt + ls];
                h = __builtin_amdgcn_mfma_f32_16x16x4f32(ga[kc], bv, h, 0, 0, 0);
              }
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int x = 16 * mt + 4 * lg + r, o = 16 * nt + ls;
                const float G = (x < K && o < N) ? h[r] * Tp[(int64_t)x * st.np + o] : 0.f;
                P[r][kGM] += G;
#pragma unroll
                for (int j = 0; j < kGM; ++j)
                  if (j < w) P[r][j] += ((o >> j) & 1) ? -G : G;
              }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int j = 0; j <= kGM; ++j)
                for (int off = 1; off < 16; off <<= 1) P[r][j] += __shfl_xor(P[r][j], off, 64);
            if (ls == 0) {
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int x = 16 * mt + 4 * lg + r;
                if (x < K) {
#pragma unroll
                  for (int j = 0; j < kGM; ++j)
                    if (j < w) pb[x * (w + 1) + j] = P[r][j];
                  pb[x * (w + 1) + w] = P[r][kGM];
                }
              }
            }
          }
        }
        wsync();
      }
      // edges folded into this step
      for (int k = lane; k < st.n_edge; k += 64) {
        const EdgeDesc ed = a.edges[st.edge_off + k];
        const int ju = ed.bu - w;
        const bool vin = ed.bv >= w;
        const int jv = vin ? ed.bv - w : ed.bv;
        float acc = 0.f;
        for (int x = 0; x < K; ++x) {
          const float v = vin ? (((x >> jv) & 1) ? -pb[x * (w + 1) + w] : pb[x * (w + 1) + w])
                              : pb[x * (w + 1) + jv];
          acc += ((x >> ju) & 1) ? -v : v;
        }
        prow[D.nr + D.n_wr + ed.rr] = acc;
      }
      // gradient-weighted magnetisations and W-R correlations of the group
      for (int j = lane; j < g; j += 64) {
        float acc = 0.f;
        for (int s = 0; s < CW; ++s) acc += gs[s] * Ms[j * CW + s];
        prow[st.gpos + j] = acc;
      }
      for (int j = 0; j < g; ++j) {
        const int p = st.gpos + j;
        const int k0 = a.fld_ptr[D.fld_off + p], k1 = a.fld_ptr[D.fld_off + p + 1];
        for (int k = k0 + lane; k < k1; k += 64) {
          const int wi = a.fld_w[D.fld_nnz_off + k];
          float acc = 0.f;
          for (int s = 0; s < nb; ++s) acc += gs[s] * (float)spq[(b0 + s) * D.nw + wi] * Ms[j * CW + s];
          prow[D.nr + a.fld_wr[D.fld_nnz_off + k]] = acc;
        }
      }
      wsync();
      float *tmp = Rc; Rc = Rn; Rn = tmp;
    }
  }
}

__global__ void chain_sum_kernel(const InstDesc *inst, const ChainInst *cinst,
                                 const int32_t *cis, int n, const int64_t *inst_B,
                                 const int64_t *inst_sample_off, const int64_t *cpart_off,
                                 const double *cpart, double *logz) {
  const int q = cis[blockIdx.y];
  const int64_t B = inst_B[q];
  const int nc = cinst[q].n_chains;
  const double lc = inst[q].log_const;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B;
       b += (int64_t)gridDim.x * blockDim.x) {
    double acc = lc;
    for (int c = 0; c < nc; ++c) acc += cpart[cpart_off[q] + (int64_t)c * B + b];
    logz[inst_sample_off[q] + b] = acc;
  }
}

}  // namespace

int chain_kseg(const ChainInst &C) {
  int k = 1;
  while ((k + 1) * (k + 1) <= C.max_steps) ++k;
  return k;
}

size_t chain_wave_lds(const ChainInst &C, bool bwd, int kseg) {
  return wave_layout(C, bwd, kseg).end;
}

template <int NTM>
void pick_chain_kernel(bool bwd, bool bf, void (**k)(ChainArgs, int)) {
  if (bwd) *k = bf ? chain_bwd_kernel<true, NTM> : chain_bwd_kernel<false, NTM>;
  else *k = bf ? chain_fwd_kernel<true, NTM> : chain_fwd_kernel<false, NTM>;
}

hipError_t launch_chain(const ChainArgs &a, bool bwd, hipStream_t st) {
  if (a.n_tasks <= 0) return hipSuccess;
  int dev = 0, maxlds = 65536;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  int wpb = (int)((size_t)maxlds / (size_t)a.wave_lds);
  if (wpb > 4) wpb = 4;
  if (wpb < 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)wpb * a.wave_lds;
  void (*k)(ChainArgs, int) = nullptr;
  if (a.ntm <= 2) pick_chain_kernel<2>(bwd, a.bf16, &k);
  else if (a.ntm <= 4) pick_chain_kernel<4>(bwd, a.bf16, &k);
  else if (a.ntm <= 16) pick_chain_kernel<16>(bwd, a.bf16, &k);
  else return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int blocks = (a.n_tasks + wpb - 1) / wpb;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * wpb), lds, st, a, wpb);
  return hipGetLastError();
}

hipError_t launch_chain_sum(const InstDesc *inst, const ChainInst *cinst,
                            const int32_t *chain_insts, int n_chain_insts,
                            const int64_t *inst_B, const int64_t *inst_sample_off,
                            const int64_t *cpart_off, const double *cpart, double *logz,
                            hipStream_t st) {
  if (n_chain_insts <= 0) return hipSuccess;
  hipLaunchKernelGGL(chain_sum_kernel, dim3(32, n_chain_insts), dim3(256), 0, st, inst, cinst,
                     chain_insts, n_chain_insts, inst_B, inst_sample_off, cpart_off, cpart,
                     logz);
  return hipGetLastError();
}

}  // namespace tnvan
