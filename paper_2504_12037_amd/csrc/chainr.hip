// Register-resident transfer-matrix kernels for chains of narrow dense steps.
//
// A chain (a lattice strip eliminated row by row, Sec. 2 Eqs. 2-4) is the
// product A_{t+1} = d_{t+1} * (A_t T_t) / 2^e_t over per-sample vectors A_t.
// Here each wave keeps its samples' A_t in registers for the whole chain:
// the product is computed transposed, out^T = T^T A^T, on 16x16x4 FP32 (or
// 16x16x32 BF16) matrix-core tiles, and the output tile layout is exactly
// the operand layout of the next step (program.h, R-layout), so a step is
// table loads (prefetched one step ahead, pre-permuted so that every lane
// reads 16 contiguous bytes), matrix-core products, a cross-lane max for the
// power-of-two rescale and the per-sample diagonal of the next group.  The
// unary factors of a group are computed on the fly from the sample's
// width-set spins (staged once per wave in LDS) and the W-neighbour lists.
//
// The adjoint walks the chain backwards from checkpoints of A (every
// kRegSeg steps, in HBM), replaying each segment in registers.  With
// R_t = d(ln Z)/d(out_t) in R-layout:
//   Lambda_t = T_t R_t                 (matrix core, R-layout over x)
//   p_t      = A_t * Lambda_t          (marginal of the group's states)
//   R_{t-1}  = d_t * Lambda_t / 2^e_{t-1}
//   H_t      = sum_s g_s A_t[s] R_t[s]^T   (matrix core over the 16 samples,
//                                       operands transposed through LDS)
//   Q_t      = S_x^T (H_t o T_t) S_o  (two more matrix-core products)
// where the columns of S_x are the group's spins and the products of the
// spins of each edge inside the group, and the columns of S_o the output
// spins and a column of ones.  Q_t holds, weighted by g and summed over the
// samples, every edge correlation of the step and the group magnetisations;
// the W-R correlations come from p_t and the spins directly.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "wave.h"

namespace tnvan {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

constexpr int CW = 16;       // samples per 16-sample group
constexpr int kWaves = 4;    // waves per workgroup
constexpr int kGr = 6;       // largest group (4 tiles of 16 states)

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

// row stride (floats) of the adjoint's LDS transposes: a multiple of 16
// plus 16 or 32, so that the four row groups of a read land in different banks
__host__ __device__ constexpr int ldt_of(int tiles) { return 16 * tiles + ((tiles & 1) ? 32 : 16); }

struct RL {
  size_t sp, ex, ga, rs, qs, end;
};
__host__ __device__ inline RL rlayout(const ChainLim &L, bool bwd, int sg) {
  RL r{};
  size_t o = 0;
  r.sp = o; o = al16(o + (size_t)CW * sg * L.nw);
  if (bwd) {
    const int ldt = ldt_of(kRegBwdTiles);
    r.ex = o; o = al16(o + (size_t)L.max_steps * CW * 4);
    r.ga = o; o = al16(o + (size_t)CW * ldt * 4);
    r.rs = o; o = al16(o + (size_t)CW * ldt * 4);
    r.qs = o; o = al16(o + (size_t)CW * 17 * 4);
  }
  r.end = al16(o);
  return r;
}

// spins of 16 * sg samples into the wave's LDS (zero rows past the batch)
__device__ inline void stage_spins(const int8_t *src, int8_t *dst, int nw, int nvalid, int n,
                                   int lane) {
  for (int i = lane; i < n * nw; i += 64) dst[i] = i < nvalid * nw ? src[i] : (int8_t)0;
  wsync();
}

// Unary factors (normalised to max 1) of the group of g positions starting at
// order position gpos, for the sample whose spins are sp; adds sum beta |f|.
__device__ inline void group_unary(const ChainArgs &a, const InstDesc &D, int gpos, int g,
                                   const int8_t *sp, float beta, float (&p0)[kGr],
                                   float (&p1)[kGr], double &fab) {
#pragma unroll
  for (int j = 0; j < kGr; ++j) {
    p0[j] = 1.f;
    p1[j] = 1.f;
    if (j < g) {
      const int pos = gpos + j;
      float f = a.hR[D.hr_off + pos];
      const int k0 = a.fld_ptr[D.fld_off + pos], k1 = a.fld_ptr[D.fld_off + pos + 1];
      for (int k = k0; k < k1; ++k)
        f += a.fld_J[D.fld_nnz_off + k] * (float)sp[a.fld_w[D.fld_nnz_off + k]];
      const float af = beta * fabsf(f);
      const float sm = __expf(-2.f * af);
      p0[j] = f >= 0.f ? 1.f : sm;
      p1[j] = f >= 0.f ? sm : 1.f;
      fab += (double)af;
    }
  }
}

// d[t][r] = prod_j phi_j(bit j of x) for x = 16 t + 4 lg + r < K, else 0
template <int NTM>
__device__ inline void make_diag(const float (&p0)[kGr], const float (&p1)[kGr], int K, int lg,
                                 float (&d)[NTM][4]) {
  const float fl = ((lg & 1) ? p1[2] : p0[2]) * ((lg & 2) ? p1[3] : p0[3]);
  float fr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) fr[r] = ((r & 1) ? p1[0] : p0[0]) * ((r & 2) ? p1[1] : p0[1]) * fl;
#pragma unroll
  for (int t = 0; t < NTM; ++t) {
    const float ft = ((t & 1) ? p1[4] : p0[4]) * ((t & 2) ? p1[5] : p0[5]);
#pragma unroll
    for (int r = 0; r < 4; ++r) d[t][r] = (16 * t + 4 * lg + r < K) ? fr[r] * ft : 0.f;
  }
}

template <int NTM>
__device__ inline void load_t(const float *tab, int n_out, int n_in, int lane, f4 (&tc)[NTM][NTM]) {
  const f4 *p = reinterpret_cast<const f4 *>(tab) + lane;
#pragma unroll
  for (int i = 0; i < NTM; ++i)
#pragma unroll
    for (int j = 0; j < NTM; ++j)
      tc[i][j] = (i < n_out && j < n_in) ? p[(i * n_in + j) * 64] : f4{0.f, 0.f, 0.f, 0.f};
}

template <int NTM>
__device__ inline void load_tb(const uint16_t *tab, int n_out, int n_c, int lane,
                               u4v (&tb)[NTM][(NTM + 1) / 2]) {
  const u4v *p = reinterpret_cast<const u4v *>(tab) + lane;
#pragma unroll
  for (int i = 0; i < NTM; ++i)
#pragma unroll
    for (int c = 0; c < (NTM + 1) / 2; ++c)
      tb[i][c] = (i < n_out && c < n_c) ? p[(i * n_c + c) * 64] : u4v{0u, 0u, 0u, 0u};
}

// out^T = T^T A^T: tc[nt][xt] from the Tr table, x in R-layout
template <int NTM>
__device__ inline void mm_fwd(const f4 (&tc)[NTM][NTM], const float (&x)[NTM][4], int KT, int NT,
                              f4 (&acc)[NTM]) {
#pragma unroll
  for (int nt = 0; nt < NTM; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int xt = 0; xt < NTM; ++xt)
    if (xt < KT)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int nt = 0; nt < NTM; ++nt)
          if (nt < NT)
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(tc[nt][xt][r], x[xt][r], acc[nt], 0, 0, 0);
}

template <int NTM>
__device__ inline void mm_fwd_bf(const u4v (&tb)[NTM][(NTM + 1) / 2], const float (&x)[NTM][4],
                                 int KC, int NT, f4 (&acc)[NTM]) {
#pragma unroll
  for (int nt = 0; nt < NTM; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < (NTM + 1) / 2; ++c)
    if (c < KC) {
      bf8 bv;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int t = 2 * c + (i >> 2);
        bv[i] = (__bf16)(t < NTM ? x[t < NTM ? t : 0][i & 3] : 0.f);
      }
#pragma unroll
      for (int nt = 0; nt < NTM; ++nt)
        if (nt < NT)
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, tb[nt][c]), bv,
                                                            acc[nt], 0, 0, 0);
    }
}

__device__ inline float xlane_max(float v) {
  v = fmaxf(v, __shfl_xor(v, 16, 64));
  v = fmaxf(v, __shfl_xor(v, 32, 64));
  return v;
}
__device__ inline float xlane_sum(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// power-of-two rescale of the step output and the next diagonal:
// x = out * 2^-e * d; returns e of the lane's sample
template <int NTM>
__device__ inline int rescale_next(const f4 (&acc)[NTM], int NT, const float (&d)[NTM][4],
                                   float (&x)[NTM][4]) {
  float m = 0.f;
#pragma unroll
  for (int nt = 0; nt < NTM; ++nt)
    if (nt < NT)
#pragma unroll
      for (int r = 0; r < 4; ++r) m = fmaxf(m, acc[nt][r]);
  const int e = expo32(xlane_max(m));
  const float sc = pow2neg(e);
#pragma unroll
  for (int t = 0; t < NTM; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) x[t][r] = t < NT ? acc[t][r] * sc * d[t][r] : 0.f;
  return e;
}

struct Task {
  int q, c;
  int64_t b0, Bq;
};

__device__ inline Task wave_task(const ChainArgs &a, int wave) {
  Task k;
  const int i = blockIdx.x * kWaves + wave;
  k.q = -1;
  if (i >= a.n_tasks) return k;
  k.q = a.task_inst[i];
  k.c = a.task_chain[i];
  k.b0 = a.task_start[i];
  k.Bq = a.inst_B[k.q];
  return k;
}

template <bool kBF, int NTM, int SG>
__global__ __launch_bounds__(256) void rchain_fwd_kernel(ChainArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, ls = lane & 15, lg = lane >> 4;
  const Task tk = wave_task(a, wave);
  if (tk.q < 0) return;
  const InstDesc D = a.inst[tk.q];
  const ChainInst C = a.cinst[tk.q];
  const ChainDesc cd = a.chains[C.chain_off + tk.c];
  const ChainStep *cs = a.csteps + cd.cs_off;
  const RL L = rlayout(a.lim, false, SG);
  int8_t *spl = reinterpret_cast<int8_t *>(smem + (size_t)wave * L.end + L.sp);
  const int64_t left = tk.Bq - tk.b0;
  const int nvalid = (int)(left < CW * SG ? left : CW * SG);
  stage_spins(a.spins + a.inst_spin_off[tk.q] + tk.b0 * D.nw, spl, D.nw, nvalid, CW * SG, lane);
  const float beta = (float)D.beta;

  double fab[SG];
  int esum[SG];
  float x[SG][NTM][4], raw[SG];
  {
    const ChainStep s0 = cs[0];
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) {
      fab[gi] = 0.0;
      esum[gi] = 0;
      float p0[kGr], p1[kGr];
      group_unary(a, D, s0.gpos, s0.g, spl + (gi * CW + ls) * D.nw, beta, p0, p1, fab[gi]);
      make_diag<NTM>(p0, p1, 1 << s0.g, lg, x[gi]);
    }
  }
  constexpr int NC2 = (NTM + 1) / 2;
  f4 tc[NTM][NTM], tn[NTM][NTM];
  u4v bc[NTM][NC2], bn[NTM][NC2];
  {
    const ChainStep s0 = cs[0];
    if (kBF) load_tb<NTM>(a.Trb + s0.trb_off, s0.nt16, ((s0.kp >> 4) + 1) >> 1, lane, bc);
    else load_t<NTM>(a.Tr + s0.tr_off, s0.nt16, s0.kp >> 4, lane, tc);
  }
  for (int t = 0;; ++t) {
    const ChainStep st = cs[t];
    const int KT = st.kp >> 4, NT = st.nt16;
    const bool last = st.w == 0;
    ChainStep nx = st;
    if (!last) {
      nx = cs[t + 1];
      if (kBF) load_tb<NTM>(a.Trb + nx.trb_off, nx.nt16, ((nx.kp >> 4) + 1) >> 1, lane, bn);
      else load_t<NTM>(a.Tr + nx.tr_off, nx.nt16, nx.kp >> 4, lane, tn);
    }
    float d[SG][NTM][4];
    if (!last) {
#pragma unroll
      for (int gi = 0; gi < SG; ++gi) {
        float p0[kGr], p1[kGr];
        group_unary(a, D, nx.gpos, nx.g, spl + (gi * CW + ls) * D.nw, beta, p0, p1, fab[gi]);
        make_diag<NTM>(p0, p1, 1 << nx.g, lg, d[gi]);
      }
    }
    f4 acc[SG][NTM];
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) {
      if (kBF) mm_fwd_bf<NTM>(bc, x[gi], (KT + 1) >> 1, NT, acc[gi]);
      else mm_fwd<NTM>(tc, x[gi], KT, NT, acc[gi]);
    }
    if (last) {
#pragma unroll
      for (int gi = 0; gi < SG; ++gi) raw[gi] = __shfl(acc[gi][0][0], ls, 64);
      break;
    }
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) esum[gi] += rescale_next<NTM>(acc[gi], NT, d[gi], x[gi]);
#pragma unroll
    for (int i = 0; i < NTM; ++i) {
#pragma unroll
      for (int j = 0; j < NTM; ++j) tc[i][j] = tn[i][j];
#pragma unroll
      for (int c = 0; c < NC2; ++c) bc[i][c] = bn[i][c];
    }
  }
  if (lg == 0) {
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) {
      const int64_t b = tk.b0 + gi * CW + ls;
      if (b < tk.Bq)
        a.cpart[a.cpart_off[tk.q] + (int64_t)tk.c * tk.Bq + b] =
            fab[gi] + (double)esum[gi] * 0.69314718055994530942 + log((double)raw[gi]);
    }
  }
}

// spin sign of bit j of the state index x
__device__ inline float sgn(int x, int j) { return ((x >> j) & 1) ? -1.f : 1.f; }

template <int NTM>
__global__ __launch_bounds__(256) void rchain_bwd_kernel(ChainArgs a) {
  extern __shared__ __align__(16) char smem[];
  constexpr int KS = kRegSeg;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63, ls = lane & 15, lg = lane >> 4;
  const Task tk = wave_task(a, wave);
  if (tk.q < 0) return;
  const InstDesc D = a.inst[tk.q];
  const ChainInst C = a.cinst[tk.q];
  const ChainDesc cd = a.chains[C.chain_off + tk.c];
  const ChainStep *cs = a.csteps + cd.cs_off;
  const RL L = rlayout(a.lim, true, 1);
  char *base = smem + (size_t)wave * L.end;
  int8_t *spl = reinterpret_cast<int8_t *>(base + L.sp);
  int *ex = reinterpret_cast<int *>(base + L.ex);
  float *ga = reinterpret_cast<float *>(base + L.ga);
  float *rs = reinterpret_cast<float *>(base + L.rs);
  float *qs = reinterpret_cast<float *>(base + L.qs);
  constexpr int LDT = ldt_of(NTM);
  const int64_t left = tk.Bq - tk.b0;
  const int nvalid = (int)(left < CW ? left : CW);
  stage_spins(a.spins + a.inst_spin_off[tk.q] + tk.b0 * D.nw, spl, D.nw, nvalid, CW, lane);
  const int8_t *sp = spl + ls * D.nw;
  const float beta = (float)D.beta;
  const float gs = ls < nvalid ? (float)a.grad[a.inst_sample_off[tk.q] + tk.b0 + ls] : 0.f;
  float *prow = a.partial + a.inst_partial_off[tk.q] + (tk.b0 / CW) * (int64_t)D.n_partial;
  const int T = cd.n_steps;
  const int ncmax = (a.lim.max_steps + KS - 1) / KS;
  f4 *ck = reinterpret_cast<f4 *>(a.ckpt) + (int64_t)(blockIdx.x * kWaves + wave) * ncmax * NTM * 64 + lane;
  const EdgeDesc *ce = a.cedges + cd.e_src;

  // forward: checkpoints every KS steps, exponents in LDS, root value
  float x[NTM][4];
  double fab = 0.0;
  {
    const ChainStep s0 = cs[0];
    float p0[kGr], p1[kGr];
    group_unary(a, D, s0.gpos, s0.g, sp, beta, p0, p1, fab);
    make_diag<NTM>(p0, p1, 1 << s0.g, lg, x);
  }
  float raw = 1.f;
  {
    f4 tc[NTM][NTM], tn[NTM][NTM];
    load_t<NTM>(a.Tr + cs[0].tr_off, cs[0].nt16, cs[0].kp >> 4, lane, tc);
    for (int t = 0;; ++t) {
      const ChainStep st = cs[t];
      if (t % KS == 0) {
#pragma unroll
        for (int i = 0; i < NTM; ++i)
          ck[((t / KS) * NTM + i) * 64] = f4{x[i][0], x[i][1], x[i][2], x[i][3]};
      }
      const bool last = st.w == 0;
      ChainStep nx = st;
      float d[NTM][4];
      if (!last) {
        nx = cs[t + 1];
        load_t<NTM>(a.Tr + nx.tr_off, nx.nt16, nx.kp >> 4, lane, tn);
        float p0[kGr], p1[kGr];
        double dummy = 0.0;
        group_unary(a, D, nx.gpos, nx.g, sp, beta, p0, p1, dummy);
        make_diag<NTM>(p0, p1, 1 << nx.g, lg, d);
      }
      f4 acc[NTM];
      mm_fwd<NTM>(tc, x, st.kp >> 4, st.nt16, acc);
      if (last) {
        raw = __shfl(acc[0][0], ls, 64);
        break;
      }
      const int e = rescale_next<NTM>(acc, st.nt16, d, x);
      if (lg == 0) ex[t * CW + ls] = e;
#pragma unroll
      for (int i = 0; i < NTM; ++i)
#pragma unroll
        for (int j = 0; j < NTM; ++j) tc[i][j] = tn[i][j];
    }
  }
  wsync();

  // R of the closing step: d ln(raw) / d out = 1 / raw on its single entry
  float R[NTM][4];
#pragma unroll
  for (int i = 0; i < NTM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) R[i][r] = 0.f;
  if (lg == 0) R[0][0] = raw > 0.f ? 1.f / raw : 0.f;

  const int NC = (T + KS - 1) / KS;
  for (int seg = NC - 1; seg >= 0; --seg) {
    const int t0 = seg * KS;
    float As[KS][NTM][4];
#pragma unroll
    for (int i = 0; i < NTM; ++i) {
      const f4 v = ck[(seg * NTM + i) * 64];
#pragma unroll
      for (int r = 0; r < 4; ++r) As[0][i][r] = v[r];
    }
    // replay the segment
#pragma unroll
    for (int u = 1; u < KS; ++u) {
      if (t0 + u < T) {
        const ChainStep st = cs[t0 + u - 1], nx = cs[t0 + u];
        f4 tc[NTM][NTM];
        load_t<NTM>(a.Tr + st.tr_off, st.nt16, st.kp >> 4, lane, tc);
        float p0[kGr], p1[kGr], d[NTM][4];
        double dummy = 0.0;
        group_unary(a, D, nx.gpos, nx.g, sp, beta, p0, p1, dummy);
        make_diag<NTM>(p0, p1, 1 << nx.g, lg, d);
        f4 acc[NTM];
        mm_fwd<NTM>(tc, As[u - 1], st.kp >> 4, st.nt16, acc);
        rescale_next<NTM>(acc, st.nt16, d, As[u]);
      }
    }
    // walk the segment backwards
#pragma unroll
    for (int u = KS - 1; u >= 0; --u) {
      const int t = t0 + u;
      if (t >= T) continue;
      const ChainStep st = cs[t];
      const int KT = st.kp >> 4, OT = st.nt16, g = st.g, w = st.w;
      f4 tq[NTM][NTM], tr[NTM][NTM];
      load_t<NTM>(a.Tq + st.tq_off, KT, OT, lane, tq);
      load_t<NTM>(a.Tr + st.tr_off, OT, KT, lane, tr);
      // Lambda = T R (R-layout over the group states)
      f4 lam[NTM];
#pragma unroll
      for (int xt = 0; xt < NTM; ++xt) lam[xt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ot = 0; ot < NTM; ++ot)
        if (ot < OT)
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int xt = 0; xt < NTM; ++xt)
              if (xt < KT)
                lam[xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(tq[xt][ot][r], R[ot][r], lam[xt], 0, 0, 0);
      // W-R correlations: per-sample magnetisation of a group spin times the
      // neighbouring width-set spin, weighted and summed over the samples
      for (int j = 0; j < g; ++j) {
        const int pos = st.gpos + j;
        const int k0 = a.fld_ptr[D.fld_off + pos], k1 = a.fld_ptr[D.fld_off + pos + 1];
        if (k1 <= k0) continue;
        float m = 0.f;
#pragma unroll
        for (int xt = 0; xt < NTM; ++xt)
#pragma unroll
          for (int r = 0; r < 4; ++r) m += sgn(16 * xt + 4 * lg + r, j) * As[u][xt][r] * lam[xt][r];
        m = xlane_sum(m) * gs;
        for (int k = k0; k < k1; ++k) {
          const float v = row16_sum(m * (float)sp[a.fld_w[D.fld_nnz_off + k]]);
          if (lane == 0) prow[D.nr + a.fld_wr[D.fld_nnz_off + k]] = v;
        }
      }
      // R of the previous step
      float Rn[NTM][4];
      if (t > 0) {
        float p0[kGr], p1[kGr], d[NTM][4];
        double dummy = 0.0;
        group_unary(a, D, st.gpos, g, sp, beta, p0, p1, dummy);
        make_diag<NTM>(p0, p1, 1 << g, lg, d);
        const float sc = pow2neg(ex[(t - 1) * CW + ls]);
#pragma unroll
        for (int xt = 0; xt < NTM; ++xt)
#pragma unroll
          for (int r = 0; r < 4; ++r) Rn[xt][r] = xt < KT ? d[xt][r] * lam[xt][r] * sc : 0.f;
      }
      // H = sum_s (g A)[s] R[s]^T through an LDS transpose
#pragma unroll
      for (int xt = 0; xt < NTM; ++xt)
        if (xt < KT)
          *reinterpret_cast<f4 *>(ga + ls * LDT + 16 * xt + 4 * lg) =
              f4{gs * As[u][xt][0], gs * As[u][xt][1], gs * As[u][xt][2], gs * As[u][xt][3]};
#pragma unroll
      for (int ot = 0; ot < NTM; ++ot)
        if (ot < OT)
          *reinterpret_cast<f4 *>(rs + ls * LDT + 16 * ot + 4 * lg) =
              f4{R[ot][0], R[ot][1], R[ot][2], R[ot][3]};
      wsync();
      f4 hg[NTM][NTM];
#pragma unroll
      for (int xt = 0; xt < NTM; ++xt)
#pragma unroll
        for (int ot = 0; ot < NTM; ++ot) {
          hg[xt][ot] = f4{0.f, 0.f, 0.f, 0.f};
          if (xt < KT && ot < OT)
#pragma unroll
            for (int kc = 0; kc < 4; ++kc)
              hg[xt][ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  ga[(4 * kc + lg) * LDT + 16 * xt + ls], rs[(4 * kc + lg) * LDT + 16 * ot + ls],
                  hg[xt][ot], 0, 0, 0);
        }
      wsync();
      // G = H o T, then Q'^T = G^T S_x and Q = S_o^T Q'^T
      const int code = a.xcol[st.xc_off + ls];
      const int cu = code & 0xff, cv = (code >> 8) & 0xff;
      f4 qt[NTM];
#pragma unroll
      for (int ot = 0; ot < NTM; ++ot) {
        qt[ot] = f4{0.f, 0.f, 0.f, 0.f};
        if (ot < OT)
#pragma unroll
          for (int xt = 0; xt < NTM; ++xt)
            if (xt < KT)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int xs = 16 * xt + 4 * lg + r;
                const float sx = code < 0 ? 0.f : ((((xs >> cu) ^ (xs >> cv)) & 1) ? -1.f : 1.f);
                qt[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(hg[xt][ot][r] * tr[ot][xt][r], sx,
                                                              qt[ot], 0, 0, 0);
              }
      }
      f4 qq = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ot = 0; ot < NTM; ++ot)
        if (ot < OT)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int o = 16 * ot + 4 * lg + r;
            const float so = ls < w ? sgn(o, ls) : (ls == w ? 1.f : 0.f);
            qq = __builtin_amdgcn_mfma_f32_16x16x4f32(so, qt[ot][r], qq, 0, 0, 0);
          }
#pragma unroll
      for (int r = 0; r < 4; ++r) qs[ls * 17 + 4 * lg + r] = qq[r];
      wsync();
      for (int k = lane; k < st.n_edge; k += 64) {
        const EdgeDesc ed = ce[st.ce_off + k];
        prow[D.nr + D.n_wr + ed.rr] = qs[(ed.pad >> 4) * 17 + (ed.pad & 15)];
      }
      if (lane < g) prow[st.gpos + lane] = qs[lane * 17 + w];
      wsync();
#pragma unroll
      for (int i = 0; i < NTM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) R[i][r] = Rn[i][r];
    }
  }
}

template <int NTM>
void pick_rchain(bool bwd, bool bf, int sg, void (**k)(ChainArgs)) {
  if (bwd) {
    if constexpr (NTM <= kRegBwdTiles) *k = rchain_bwd_kernel<NTM>;
    return;
  }
  if (bf) *k = sg >= 2 ? rchain_fwd_kernel<true, NTM, 2> : rchain_fwd_kernel<true, NTM, 1>;
  else *k = sg >= 2 ? rchain_fwd_kernel<false, NTM, 2> : rchain_fwd_kernel<false, NTM, 1>;
}

}  // namespace

size_t rchain_wave_lds(const ChainLim &L, bool bwd, int sg) { return rlayout(L, bwd, sg).end; }

int64_t rchain_ckpt_floats(const ChainLim &L) {
  return (int64_t)((L.max_steps + kRegSeg - 1) / kRegSeg) * kRegBwdTiles * 64 * 4;
}

hipError_t launch_rchain(const ChainArgs &a, bool bwd, hipStream_t st) {
  if (a.n_tasks <= 0) return hipSuccess;
  const int sg = bwd ? 1 : (a.sg >= 2 ? 2 : 1);
  void (*k)(ChainArgs) = nullptr;
  if (bwd) pick_rchain<kRegBwdTiles>(true, false, 1, &k);
  else if (a.ntm <= 2) pick_rchain<2>(false, a.bf16 != 0, sg, &k);
  else if (a.ntm <= 4) pick_rchain<4>(false, a.bf16 != 0, sg, &k);
  if (!k || (bwd && a.ntm > kRegBwdTiles)) return hipErrorInvalidValue;
  const size_t lds = (size_t)kWaves * rlayout(a.lim, bwd, sg).end;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, dim3((a.n_tasks + kWaves - 1) / kWaves), dim3(64 * kWaves), lds, st, a);
  return hipGetLastError();
}

}  // namespace tnvan
