// Transfer-matrix form of the conditional contraction on the matrix cores.
//
// A chain of dense steps (a lattice strip eliminated row by row, or the two
// blocks of the SK remainder) is contracted as a product of per-sample
// diagonals and static transfer matrices (Sec. 2, Eqs. 2-4):
//
//   A_0 = d_0,  out_t = A_t . T_t,  A_{t+1} = d_{t+1} * (out_t / 2^e_t)
//
// where A_t is [16 samples x K] and T_t is [K x N].  A workgroup takes one
// chain and 16 samples per wave.  It first copies the chain's transfer
// tables, edge list and W-neighbour lists into LDS with coalesced loads (a
// chain walks its tables in order, so reading them step by step from HBM
// would expose one memory latency per step).  Each wave then runs its
// samples through the chain without waiting for the others: products on
// 16x16x4 FP32 (or 16x16x32 BF16, FP32 accumulate) MFMA tiles, the
// per-sample power-of-two rescale as a max over accumulator rows, and the
// next A written back to the wave's LDS slice in operand order.  The
// diagonal d of a group is a Kronecker product of its spins' two-entry unary
// factors; each lane builds the entries it needs once per step.
//
// The adjoint recomputes the chain from checkpoints (every k steps, kept in
// a per-wave HBM scratch area) and walks back with R_t = rho_t 2^-e_t
// (rho = marginal / scaled message, as in the generic kernel):
//   Lambda_t = R_t . T_t^T                       (MFMA, samples x K)
//   magnetisation of the group spins   sum_x sigma_j(x) A_t Lambda_t
//   R_{t-1} = d_t * Lambda_t / 2^e_{t-1}
//   H_t = (g A_t)^T . R_t                        (MFMA over the 16 samples)
//   edge correlations  sum_{x,o} T_t H_t sigma_u sigma_v
// and writes the gradient-weighted sums of one 16-sample group into one
// partial row (every entry of the row is owned by exactly one chain).  The
// adjoint uses FP32 products in both the FP32 and the BF16 precisions.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"
#include "wave.h"

namespace tnvan {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

constexpr int CW = 16;     // samples per wave
// NTM (template): largest number of 16-wide tiles of K or N in a launch
constexpr int kGM = 8;     // largest group

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

// Shared (per workgroup) LDS layout.
struct SL {
  size_t tl, ce, fp, fw, fwr, fj, end;
};
__host__ __device__ inline SL shared_layout(const ChainLim &L, bool bwd, bool bf16) {
  SL s{};
  size_t o = 0;
  s.tl = o;
  if (L.tlds) o = al16(o + ((bf16 && !bwd) ? (size_t)L.tbl_max * 2 : (size_t)L.tl_max * 4));
  s.ce = o;  o = al16(o + (size_t)L.ne_max * sizeof(EdgeDesc));
  s.fp = o;  o = al16(o + (size_t)(L.npos_max + 1) * 4);
  s.fw = o;  o = al16(o + (size_t)L.nf_max * 4);
  s.fwr = o; o = al16(o + (size_t)L.nf_max * 4);
  s.fj = o;  o = al16(o + (size_t)L.nf_max * 4);
  s.end = o;
  return s;
}

// Per-wave LDS layout.
struct WL {
  int lda;
  size_t sp, phi, dt, lz, es, A0, gs, raw, ex, M, pb, R0, R1, seg, buf, end;
};
__host__ __device__ inline WL wave_layout(const ChainLim &C, bool bwd) {
  WL L{};
  L.lda = C.kbuf + 4;
  L.buf = al16((size_t)CW * L.lda * 4);
  size_t o = 0;
  L.sp = o;  o = al16(o + (size_t)CW * C.nw);
  L.phi = o; o = al16(o + (size_t)C.npos_max * 2 * CW * 4);
  L.dt = o;  o += L.buf;
  L.lz = o;  o = al16(o + CW * 8);
  L.es = o;  o = al16(o + CW * 4);
  L.A0 = o;  o += L.buf;
  if (bwd) {
    L.gs = o;  o = al16(o + CW * 4);
    L.raw = o; o = al16(o + CW * 4);
    L.ex = o;  o = al16(o + (size_t)C.max_steps * CW * 4);
    L.M = o;   o = al16(o + (size_t)kGM * CW * 4);
    L.pb = o;  o = al16(o + (size_t)C.pmax * 4);
    L.R0 = o;  o += L.buf;
    L.R1 = o;  o += L.buf;
    L.seg = o; o += (size_t)(C.kseg > 1 ? C.kseg - 1 : 0) * L.buf;
  }
  L.end = al16(o);
  return L;
}

// transfer-table entry T[x][o] of a step: staged copy (rows padded by one)
// or the padded HBM table
template <bool kTL>
__device__ inline float tval(const ChainArgs &a, const float *tl, const ChainStep &cs, int x, int o) {
  return kTL ? tl[cs.tl_off + x * (cs.np + 1) + o] : a.Tp[cs.tp_off + x * cs.np + o];
}

// d[s][x] = prod_j phi_j(s, x_j) of a group of g spins starting at chain
// position po, into dst (row stride ld); entries x in [2^g, zero_to) are set
// to zero.  Lane (s = lane & 15) produces x = (lane >> 4) + 4m: the two low
// bits are fixed per lane, so each entry costs g - 2 multiplications.
__device__ inline void build_diag(int g, int po, const float *phi, float *dst, int ld,
                                  int zero_to, int lane) {
  const int s = lane & 15, lg = lane >> 4, K = 1 << g;
  float p0[kGM], p1[kGM];
#pragma unroll
  for (int j = 0; j < kGM; ++j) {
    p0[j] = j < g ? phi[((po + j) * 2) * CW + s] : 1.f;
    p1[j] = j < g ? phi[((po + j) * 2 + 1) * CW + s] : 1.f;
  }
  float lo = 1.f;
#pragma unroll
  for (int j = 0; j < 2; ++j)
    if (j < g) lo *= ((lg >> j) & 1) ? p1[j] : p0[j];
  const int top = K > zero_to ? K : zero_to;
  for (int m = 0; 4 * m + lg < top; ++m) {
    const int x = 4 * m + lg;
    float v = 0.f;
    if (x < K) {
      v = lo;
#pragma unroll
      for (int j = 2; j < kGM; ++j)
        if (j < g) v *= ((m >> (j - 2)) & 1) ? p1[j] : p0[j];
    }
    dst[s * ld + x] = v;
  }
}

// One forward step of a chain for the wave's 16 samples: Aout <- scaled
// product times the next step's diagonal (dtab, built here).  Returns the
// per-row exponents.
template <bool kBF, bool kTL, int NTM>
__device__ inline void chain_step(const ChainArgs &a, const void *tsh, const ChainStep &cs,
                                  const ChainStep &nx, const float *Ain, float *Aout, float *dtab,
                                  int lda, int kbuf, const float *phi, int pos_lo, int lane,
                                  int e[4]) {
  const int ls = lane & 15, lg = lane >> 4;
  const int NT = cs.np >> 4;
  build_diag(nx.g, nx.gpos - pos_lo, phi, dtab, lda, 0, lane);
  f4 acc[NTM];
#pragma unroll
  for (int nt = 0; nt < NTM; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
  if (!kBF) {
    const float *tl = static_cast<const float *>(tsh);
    const float *ap = Ain + ls * lda + lg;
    const int KC = cs.kp >> 2;        // a multiple of 4
    for (int k0 = 0; k0 < KC; k0 += 4) {
      float av[4], bv[4][NTM];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = ap[4 * (k0 + u)];
#pragma unroll
        for (int nt = 0; nt < NTM; ++nt)
          if (nt < NT) bv[u][nt] = tval<kTL>(a, tl, cs, 4 * (k0 + u) + lg, 16 * nt + ls);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int nt = 0; nt < NTM; ++nt)
          if (nt < NT) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[u][nt], acc[nt], 0, 0, 0);
    }
  } else {
    const int KC = cs.kb >> 5;
    const u4v *tb = kTL ? reinterpret_cast<const u4v *>(static_cast<const uint16_t *>(tsh) + cs.tbl_off)
                        : reinterpret_cast<const u4v *>(a.Tb + cs.tb_off);
    tb += lane;
    for (int kc = 0; kc < KC; ++kc) {
      bf8 av;
      const float *ap = Ain + ls * lda + 32 * kc + 8 * lg;
#pragma unroll
      for (int i = 0; i < 8; ++i) av[i] = (__bf16)ap[i];
#pragma unroll
      for (int nt = 0; nt < NTM; ++nt)
        if (nt < NT) {
          const u4v raw = tb[(nt * KC + kc) * 64];
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
  float sc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    e[r] = expo32(row16_max(m[r]));
    sc[r] = pow2neg(e[r]);
  }
  wsync();   // every read of Ain precedes the writes (Aout may alias Ain)
  const int N = 1 << cs.w;
#pragma unroll
  for (int nt = 0; nt < NTM; ++nt)
    if (nt < NT)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * nt + ls, s = 4 * lg + r;
        Aout[s * lda + o] = o < N ? acc[nt][r] * sc[r] * dtab[s * lda + o] : 0.f;
      }
  for (int i = lane; i < CW * (kbuf - cs.np); i += 64) Aout[(i & 15) * lda + cs.np + (i >> 4)] = 0.f;
  wsync();
}

// raw root value sum_x A[s][x] T[x] of sample (lane & 15), on every lane
template <bool kTL>
__device__ inline float chain_root(const ChainArgs &a, const float *tl, const ChainStep &cs,
                                   const float *A, int lda, int lane) {
  const int ls = lane & 15, lg = lane >> 4;
  const int K = 1 << cs.g;
  float part = 0.f;
  for (int x = lg; x < K; x += 4) part += A[ls * lda + x] * tval<kTL>(a, tl, cs, x, 0);
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part;
}

// the wave's 16 samples' width-set spins into LDS (zero for padding rows)
__device__ inline void stage_spins(const int8_t *src, int8_t *dst, int nw, int nb, int lane) {
  for (int i = lane; i < CW * nw; i += 64) dst[i] = i < nb * nw ? src[i] : (int8_t)0;
  wsync();
}

// Copy the chain's tables, edges and W-neighbour lists into the workgroup's
// shared LDS part (all threads, one barrier).
template <bool kBFT>
__device__ inline void stage_chain(const ChainArgs &a, const InstDesc &D, const ChainDesc &cd,
                                   char *sh, const SL &S) {
  if (a.lim.tlds) {
    if (kBFT) {
      const u4v *src = reinterpret_cast<const u4v *>(a.Tbl + cd.tbl_src);
      u4v *dst = reinterpret_cast<u4v *>(sh + S.tl);
      for (int i = threadIdx.x; i < cd.tbl_size / 8; i += blockDim.x) dst[i] = src[i];
    } else {
      const float *src = a.Tl + cd.tl_src;
      float *dst = reinterpret_cast<float *>(sh + S.tl);
      for (int i = threadIdx.x; i < cd.tl_size; i += blockDim.x) dst[i] = src[i];
    }
  }
  EdgeDesc *ce = reinterpret_cast<EdgeDesc *>(sh + S.ce);
  for (int i = threadIdx.x; i < cd.n_e; i += blockDim.x) ce[i] = a.cedges[cd.e_src + i];
  int32_t *fp = reinterpret_cast<int32_t *>(sh + S.fp);
  const int npos = cd.pos_hi - cd.pos_lo;
  for (int i = threadIdx.x; i <= npos; i += blockDim.x)
    fp[i] = a.fld_ptr[D.fld_off + cd.pos_lo + i] - cd.f_lo;
  int32_t *fw = reinterpret_cast<int32_t *>(sh + S.fw);
  int32_t *fwr = reinterpret_cast<int32_t *>(sh + S.fwr);
  float *fj = reinterpret_cast<float *>(sh + S.fj);
  for (int i = threadIdx.x; i < cd.f_hi - cd.f_lo; i += blockDim.x) {
    fw[i] = a.fld_w[D.fld_nnz_off + cd.f_lo + i];
    fwr[i] = a.fld_wr[D.fld_nnz_off + cd.f_lo + i];
    fj[i] = a.fld_J[D.fld_nnz_off + cd.f_lo + i];
  }
  __syncthreads();
}

// unary factors of the chain's positions, normalised to max 1; returns the
// sum of beta |f| of sample (lane & 15)
__device__ inline double chain_phi(const ChainArgs &a, const InstDesc &D, const ChainDesc &cd,
                                   const char *sh, const SL &S, const int8_t *spl, float *phi,
                                   int nb, int lane) {
  const int32_t *fp = reinterpret_cast<const int32_t *>(sh + S.fp);
  const int32_t *fw = reinterpret_cast<const int32_t *>(sh + S.fw);
  const float *fj = reinterpret_cast<const float *>(sh + S.fj);
  double fab = 0.0;
  const int npos = cd.pos_hi - cd.pos_lo;
  const float beta = (float)D.beta;
  for (int i = lane; i < npos * CW; i += 64) {
    const int pl = i >> 4, s = i & 15;
    float f = a.hR[D.hr_off + cd.pos_lo + pl];
    if (s < nb) {
      const int8_t *sp = spl + s * D.nw;
      for (int k = fp[pl]; k < fp[pl + 1]; ++k) f += fj[k] * (float)sp[fw[k]];
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

template <bool kBF, bool kTL, int NTM>
__global__ __launch_bounds__(256) void chain_fwd_kernel(ChainArgs a) {
  extern __shared__ __align__(16) char smem[];
  // the wave index is uniform inside a wave; saying so keeps every task and
  // step descriptor in scalar registers and the control flow uniform
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int q = a.task_inst[blockIdx.x], c = a.task_chain[blockIdx.x];
  const InstDesc D = a.inst[q];
  const ChainInst C = a.cinst[q];
  const ChainDesc cd = a.chains[C.chain_off + c];
  const ChainStep *cs = a.csteps + cd.cs_off;
  const SL S = shared_layout(a.lim, false, kBF);
  stage_chain<kBF>(a, D, cd, smem, S);
  const void *tsh = smem + S.tl;
  const int64_t Bq = a.inst_B[q];
  const int64_t b0 = a.task_start[blockIdx.x] + (int64_t)wave * CW;
  if (b0 >= Bq) return;
  const int nb = (int)((Bq - b0) < CW ? (Bq - b0) : CW);
  const WL L = wave_layout(a.lim, false);
  char *base = smem + S.end + (size_t)wave * L.end;
  float *phi = reinterpret_cast<float *>(base + L.phi);
  float *dtab = reinterpret_cast<float *>(base + L.dt);
  int *es = reinterpret_cast<int *>(base + L.es);
  float *A = reinterpret_cast<float *>(base + L.A0);
  int8_t *spl = reinterpret_cast<int8_t *>(base + L.sp);
  stage_spins(a.spins + a.inst_spin_off[q] + b0 * D.nw, spl, D.nw, nb, lane);
  const double fab = chain_phi(a, D, cd, smem, S, spl, phi, nb, lane);
  build_diag(cs[0].g, cs[0].gpos - cd.pos_lo, phi, A, L.lda, a.lim.kbuf, lane);
  wsync();
  int esum[4] = {0, 0, 0, 0};
  float raw = 1.f;
  for (int t = 0; t < cd.n_steps; ++t) {
    const ChainStep st = cs[t];
    if (st.w == 0) {
      raw = chain_root<kTL && !kBF>(a, static_cast<const float *>(tsh), st, A, L.lda, lane);
      break;
    }
    int e[4];
    chain_step<kBF, kTL, NTM>(a, tsh, st, cs[t + 1], A, A, dtab, L.lda, a.lim.kbuf, phi,
                              cd.pos_lo, lane, e);
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

template <bool kTL, int NTM>
__global__ __launch_bounds__(256) void chain_bwd_kernel(ChainArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int ls = lane & 15, lg = lane >> 4;
  const int q = a.task_inst[blockIdx.x], c = a.task_chain[blockIdx.x];
  const InstDesc D = a.inst[q];
  const ChainInst C = a.cinst[q];
  const ChainDesc cd = a.chains[C.chain_off + c];
  const ChainStep *cs = a.csteps + cd.cs_off;
  const SL S = shared_layout(a.lim, true, false);
  stage_chain<false>(a, D, cd, smem, S);
  const float *tl = reinterpret_cast<const float *>(smem + S.tl);
  const EdgeDesc *ce = reinterpret_cast<const EdgeDesc *>(smem + S.ce);
  const int32_t *fp = reinterpret_cast<const int32_t *>(smem + S.fp);
  const int32_t *fw = reinterpret_cast<const int32_t *>(smem + S.fw);
  const int32_t *fwr = reinterpret_cast<const int32_t *>(smem + S.fwr);
  const int64_t Bq = a.inst_B[q];
  const int64_t b0 = a.task_start[blockIdx.x] + (int64_t)wave * CW;
  if (b0 >= Bq) return;
  const int nb = (int)((Bq - b0) < CW ? (Bq - b0) : CW);
  const int kseg = a.lim.kseg;
  const WL L = wave_layout(a.lim, true);
  const int lda = L.lda, kbuf = a.lim.kbuf;
  char *base = smem + S.end + (size_t)wave * L.end;
  float *phi = reinterpret_cast<float *>(base + L.phi);
  float *dtab = reinterpret_cast<float *>(base + L.dt);
  float *A0 = reinterpret_cast<float *>(base + L.A0);
  float *gs = reinterpret_cast<float *>(base + L.gs);
  float *rawb = reinterpret_cast<float *>(base + L.raw);
  int *ex = reinterpret_cast<int *>(base + L.ex);
  float *Ms = reinterpret_cast<float *>(base + L.M);
  float *pb = reinterpret_cast<float *>(base + L.pb);
  float *Rc = reinterpret_cast<float *>(base + L.R0);
  float *Rn = reinterpret_cast<float *>(base + L.R1);
  int8_t *spl = reinterpret_cast<int8_t *>(base + L.sp);
  const int T = cd.n_steps;
  const int NC = (T + kseg - 1) / kseg;
  // checkpoints of this wave: NC buffers of [16][kbuf] in HBM
  float *ckw = a.ckpt + ((int64_t)blockIdx.x * a.lim.wpb + wave) *
                            (int64_t)((a.lim.max_steps + kseg - 1) / kseg) * CW * kbuf;
  stage_spins(a.spins + a.inst_spin_off[q] + b0 * D.nw, spl, D.nw, nb, lane);
  chain_phi(a, D, cd, smem, S, spl, phi, nb, lane);
  if (lane < CW) gs[lane] = lane < nb ? (float)a.grad[a.inst_sample_off[q] + b0 + lane] : 0.f;
  const int64_t row = a.inst_partial_off[q] + (b0 / CW) * (int64_t)D.n_partial;
  float *prow = a.partial + row;
  auto save_ck = [&](int i, const float *A) {
    float *dst = ckw + (int64_t)i * CW * kbuf;
    for (int k = lane; k < CW * kbuf; k += 64) dst[k] = A[(k / kbuf) * lda + k % kbuf];
  };
  auto load_ck = [&](int i, float *A) {
    const float *src = ckw + (int64_t)i * CW * kbuf;
    for (int k = lane; k < CW * kbuf; k += 64) A[(k / kbuf) * lda + k % kbuf] = src[k];
    wsync();
  };

  // forward, saving A every kseg steps
  build_diag(cs[0].g, cs[0].gpos - cd.pos_lo, phi, A0, lda, kbuf, lane);
  wsync();
  for (int t = 0; t < T; ++t) {
    const ChainStep st = cs[t];
    if (t % kseg == 0) save_ck(t / kseg, A0);
    if (st.w == 0) {
      const float raw = chain_root<kTL>(a, tl, st, A0, lda, lane);
      if (lane < CW) rawb[lane] = raw;
      wsync();
      break;
    }
    int e[4];
    chain_step<false, kTL, NTM>(a, tl, st, cs[t + 1], A0, A0, dtab, lda, kbuf, phi, cd.pos_lo,
                                lane, e);
    if (ls == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) ex[t * CW + 4 * lg + r] = e[r];
    }
    wsync();
  }

  for (int seg = NC - 1; seg >= 0; --seg) {
    const int t0 = seg * kseg;
    const int t1 = (t0 + kseg) < T ? (t0 + kseg) : T;
    auto sbuf = [&](int j) {
      return j == 0 ? A0 : reinterpret_cast<float *>(base + L.seg + (size_t)(j - 1) * L.buf);
    };
    load_ck(seg, A0);
    for (int t = t0; t < t1 - 1; ++t) {
      int e[4];
      chain_step<false, kTL, NTM>(a, tl, cs[t], cs[t + 1], sbuf(t - t0), sbuf(t + 1 - t0), dtab,
                                  lda, kbuf, phi, cd.pos_lo, lane, e);
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const ChainStep st = cs[t];
      const float *A = sbuf(t - t0);
      const int g = st.g, w = st.w, K = 1 << g;
      const int po = st.gpos - cd.pos_lo;
      const bool has_prev = t > 0;
      if (has_prev) {
        build_diag(g, po, phi, dtab, lda, 0, lane);
        wsync();
      }
      if (w == 0) {
        // closing step: R = 1 / raw, Lambda[s][x] = T[x] R[s]
        const float rinv = rawb[ls] > 0.f ? 1.f / rawb[ls] : 0.f;
        const float sc = has_prev ? pow2neg(ex[(t - 1) * CW + ls]) : 1.f;
        float mloc[kGM];
#pragma unroll
        for (int j = 0; j < kGM; ++j) mloc[j] = 0.f;
        for (int x = lg; x < st.kp; x += 4) {
          const float lam = x < K ? tval<kTL>(a, tl, st, x, 0) * rinv : 0.f;
          const float cval = A[ls * lda + x] * lam;
#pragma unroll
          for (int j = 0; j < kGM; ++j)
            if (j < g) mloc[j] += ((x >> j) & 1) ? -cval : cval;
          if (has_prev) Rn[ls * lda + x] = x < K ? dtab[ls * lda + x] * lam * sc : 0.f;
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
          for (int s = 0; s < CW; ++s)
            acc += gs[s] * A[s * lda + x] * (rawb[s] > 0.f ? 1.f / rawb[s] : 0.f);
          pb[x] = acc * tval<kTL>(a, tl, st, x, 0);
        }
        wsync();
      } else {
        const int NT = st.np >> 4, KT = st.kp >> 4;
        // Lambda = R . T^T  (samples x K)
        f4 lam[NTM];
#pragma unroll
        for (int xt = 0; xt < NTM; ++xt) lam[xt] = f4{0.f, 0.f, 0.f, 0.f};
        const float *rp = Rc + ls * lda + lg;
        const int OC = st.np >> 2;     // a multiple of 4
        for (int k0 = 0; k0 < OC; k0 += 4) {
          float av[4], bv[4][NTM];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            av[u] = rp[4 * (k0 + u)];
            const int o = 4 * (k0 + u) + lg;
#pragma unroll
            for (int xt = 0; xt < NTM; ++xt)
              if (xt < KT)
                bv[u][xt] = kTL ? tl[st.tl_off + (16 * xt + ls) * (st.np + 1) + o]
                                : a.Tt[st.tt_off + o * st.kp + 16 * xt + ls];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int xt = 0; xt < NTM; ++xt)
              if (xt < KT) lam[xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[u][xt], lam[xt], 0, 0, 0);
        }
        // magnetisations and R of the previous step
        float scp[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) scp[r] = has_prev ? pow2neg(ex[(t - 1) * CW + 4 * lg + r]) : 1.f;
        float Macc[4][kGM];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int j = 0; j < kGM; ++j) Macc[r][j] = 0.f;
#pragma unroll
        for (int xt = 0; xt < NTM; ++xt)
          if (xt < KT)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int x = 16 * xt + ls, s = 4 * lg + r;
              float cval = 0.f, rn = 0.f;
              if (x < K) {
                cval = A[s * lda + x] * lam[xt][r];
                if (has_prev) rn = dtab[s * lda + x] * lam[xt][r] * scp[r];
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
            if (j < g) Macc[r][j] = row16_sum(Macc[r][j]);
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
              const int o = 16 * nt + ls;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int x = 16 * mt + 4 * lg + r;
                const float G = (x < K && o < N) ? h[r] * tval<kTL>(a, tl, st, x, o) : 0.f;
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
                if (j < w || j == kGM) P[r][j] = row16_sum(P[r][j]);
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
      // edges folded into this step: lanes split the group states
      for (int k = 0; k < st.n_edge; ++k) {
        const EdgeDesc ed = ce[st.ce_off + k];
        const int ju = ed.bu - w;
        const bool vin = ed.bv >= w;
        const int jv = vin ? ed.bv - w : ed.bv;
        float acc = 0.f;
        for (int x = lane; x < K; x += 64) {
          const float v = vin ? (((x >> jv) & 1) ? -pb[x * (w + 1) + w] : pb[x * (w + 1) + w])
                              : pb[x * (w + 1) + jv];
          acc += ((x >> ju) & 1) ? -v : v;
        }
        acc = row16_sum(acc);
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        if (lane == 0) prow[D.nr + D.n_wr + ed.rr] = acc;
      }
      // gradient-weighted magnetisations and W-R correlations of the group:
      // lane (j, s) terms, reduced over the 16 samples of a row
      for (int j = 0; j < g; j += 4) {
        const int jj = j + lg;
        float acc = jj < g ? gs[ls] * Ms[jj * CW + ls] : 0.f;
        acc = row16_sum(acc);
        if (ls == 0 && jj < g) prow[st.gpos + jj] = acc;
      }
      for (int j = 0; j < g; ++j) {
        const int pl = po + j;
        const int k0 = fp[pl], k1 = fp[pl + 1];
        // four W-neighbours per pass, lane (neighbour, sample)
        for (int k = k0; k < k1; k += 4) {
          const int kk = k + lg;
          float acc = 0.f;
          if (kk < k1) acc = gs[ls] * (float)spl[ls * D.nw + fw[kk]] * Ms[j * CW + ls];
          acc = row16_sum(acc);
          if (ls == 0 && kk < k1) prow[D.nr + fwr[kk]] = acc;
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
                                 const double *cpart, const int64_t *f_off, const double *fabp,
                                 double *logz) {
  const int q = cis[blockIdx.y];
  const int64_t B = inst_B[q];
  const int nc = cinst[q].n_chains;
  const int nf = (inst[q].nr + kUnaryChunk - 1) / kUnaryChunk;
  const double lc = inst[q].log_const;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B;
       b += (int64_t)gridDim.x * blockDim.x) {
    double acc = lc;
    for (int c = 0; c < nc; ++c) acc += cpart[cpart_off[q] + (int64_t)c * B + b];
    if (fabp) {
      // loads in batches of 8 (independent), additions in chunk order
      const double *fp = fabp + f_off[q] + b;
      int c = 0;
      for (; c + 8 <= nf; c += 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = fp[(int64_t)(c + k) * B];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += v[k];
      }
      for (; c < nf; ++c) acc += fp[(int64_t)c * B];
    }
    logz[inst_sample_off[q] + b] = acc;
  }
}

// One thread per (sample, run of kUnaryChunk positions); grid.z picks the
// instance.  The field on R position p of sample s_W is h_p plus the W-R
// couplings times the neighbouring width-set spins (Sec. 2).  Positions
// with at most four W-neighbours read the dense slots (all loads of a
// position at once); others walk the neighbour list.
__global__ __launch_bounds__(256) void unary_kernel(ChainArgs a, const int32_t *cis,
                                                    const int64_t *f_off, float *U,
                                                    double *fabp) {
  typedef const __attribute__((address_space(4))) int32_t *ci32;
  typedef const __attribute__((address_space(4))) float *cf32;
  const int q = cis[blockIdx.z];
  const InstDesc D = a.inst[q];
  const int64_t B = a.inst_B[q];
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int p0 = blockIdx.y * kUnaryChunk;
  if (p0 >= D.nr) return;
  const int p1 = p0 + kUnaryChunk < D.nr ? p0 + kUnaryChunk : D.nr;
  // the chunk's descriptors (field, four W-neighbour records, neighbour
  // count) staged in LDS by one load per thread, then read with uniform
  // addresses: no scalar round trip per position
  __shared__ float s_h[kUnaryChunk], s_j[kUnaryChunk][4];
  __shared__ int32_t s_w[kUnaryChunk][4], s_r[kUnaryChunk][4], s_n[kUnaryChunk];
  {
    const int t = threadIdx.x, np = p1 - p0;
    if (t < 4 * np) {
      const int64_t e = 4 * ((int64_t)D.hr_off + p0) + t;
      s_w[t >> 2][t & 3] = a.cf_w[e];
      s_r[t >> 2][t & 3] = a.cf_r[e];
      s_j[t >> 2][t & 3] = a.cf_J[e];
    } else if (t >= 64 && t < 64 + np) {
      const int p = p0 + t - 64;
      s_h[t - 64] = a.hR[D.hr_off + p];
      s_n[t - 64] = a.fld_ptr[D.fld_off + p + 1] - a.fld_ptr[D.fld_off + p];
    }
  }
  __syncthreads();
  if (b >= B) return;
  // the sample's width-set spins as a bit mask, read with uniform indices;
  // width sets beyond the mask's 128 bits read the spin bytes instead
  const int8_t *srow = a.spins + a.inst_spin_off[q] + b * D.nw;
  const bool bits = D.nw <= 128;
  const SpinBits sb = bits ? load_bits_row(srow, D.nw) : SpinBits{{0u, 0u, 0u, 0u}};
  auto sigma = [&](int w) { return bits ? sb.sigma(w) : (float)srow[w]; };
  const float beta = (float)D.beta;
  float *Uq = U + a.u_off[q];
  double fab = 0.0;
  for (int p = p0; p < p1; ++p) {
    const int i = p - p0;
    // a position with no W-neighbour and no field has the factor +1, which
    // the table holds from its set-up: nothing to store (unless u_all)
    if (!a.u_all && s_n[i] == 0 && s_h[i] == 0.f) continue;
    float f = s_h[i];
    if (s_n[i] <= 4) {
      float t[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) t[k] = s_r[i][k] >= 0 ? s_j[i][k] * sigma(s_w[i][k]) : 0.f;
      f += (t[0] + t[1]) + (t[2] + t[3]);
    } else {
      const ci32 fptr = (ci32)(a.fld_ptr + D.fld_off);
      const ci32 fw = (ci32)(a.fld_w + D.fld_nnz_off);
      const cf32 fj = (cf32)(a.fld_J + D.fld_nnz_off);
      for (int k = fptr[p]; k < fptr[p + 1]; ++k) f += fj[k] * sigma(fw[k]);
    }
    const float af = beta * fabsf(f);
    const float sm = __expf(-2.f * af);
    Uq[(int64_t)p * B + b] = f >= 0.f ? sm : -sm;
    fab += (double)af;
  }
  fabp[f_off[q] + (int64_t)blockIdx.y * B + b] = fab;
}

__global__ __launch_bounds__(256) void layout_kernel(LayoutArgs a) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (tid < a.n_inst) {
    const int q = (int)tid;
    a.d_B[q] = a.B[q];
    a.d_sample_off[q] = a.sample_off[q];
    a.d_spin_off[q] = a.spin_off[q];
    a.d_cpart_off[q] = a.cpart_off[q];
    a.d_u_off[q] = a.u_off[q];
    a.d_f_off[q] = a.f_off[q];
    a.d_clist[q] = q;
  }
  for (int64_t t = tid; t < a.n_tasks; t += (int64_t)gridDim.x * blockDim.x) {
    // the (width group, instance) segment holding task t
    int gi = 0, q = 0;
    for (int g = 0; g < 3; ++g)
      for (int k = 0; k < a.n_inst; ++k)
        if (t >= a.seg_off[g][k] && t < a.seg_off[g][k + 1]) { gi = g; q = k; }
    const ChainInst C = a.cinst[q];
    const int rt = 1 << gi;
    int nm = 0;
    for (int c = 0; c < C.n_chains; ++c) {
      const int crt = a.chains[C.chain_off + c].rt;
      nm += (crt > 4 ? 4 : crt) == rt;
    }
    const int64_t li = t - a.seg_off[gi][q];
    const int64_t bi = li / nm;
    int ci = (int)(li - bi * nm), c = 0;
    for (; c < C.n_chains; ++c) {
      const int crt = a.chains[C.chain_off + c].rt;
      if ((crt > 4 ? 4 : crt) == rt && ci-- == 0) break;
    }
    a.d_ti[t] = q;
    a.d_tc[t] = c;
    a.d_ts[t] = (int32_t)(bi * a.per[gi]);
  }
}

template <int NTM>
void pick_chain_kernel(bool bwd, bool bf, bool tl, void (**k)(ChainArgs)) {
  if (bwd) *k = tl ? chain_bwd_kernel<true, NTM> : chain_bwd_kernel<false, NTM>;
  else if (bf) *k = tl ? chain_fwd_kernel<true, true, NTM> : chain_fwd_kernel<true, false, NTM>;
  else *k = tl ? chain_fwd_kernel<false, true, NTM> : chain_fwd_kernel<false, false, NTM>;
}

}  // namespace

int chain_kseg(const ChainInst &C) {
  int k = 1;
  while ((k + 1) * (k + 1) <= C.max_steps) ++k;
  return k;
}

size_t chain_shared_lds(const ChainLim &L, bool bwd, bool bf16) {
  return shared_layout(L, bwd, bf16).end;
}

size_t chain_wave_lds(const ChainLim &L, bool bwd) { return wave_layout(L, bwd).end; }

hipError_t launch_chain(const ChainArgs &a, bool bwd, hipStream_t st) {
  if (a.n_tasks <= 0) return hipSuccess;
  const size_t lds = chain_shared_lds(a.lim, bwd, a.bf16 != 0) +
                     (size_t)a.lim.wpb * chain_wave_lds(a.lim, bwd);
  void (*k)(ChainArgs) = nullptr;
  const bool tl = a.lim.tlds != 0;
  if (a.ntm <= 2) pick_chain_kernel<2>(bwd, a.bf16, tl, &k);
  else if (a.ntm <= 4) pick_chain_kernel<4>(bwd, a.bf16, tl, &k);
  else if (a.ntm <= 16) pick_chain_kernel<16>(bwd, a.bf16, tl, &k);
  else return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(a.n_tasks), dim3(64 * a.lim.wpb), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_chain_sum(const InstDesc *inst, const ChainInst *cinst,
                            const int32_t *chain_insts, int n_chain_insts,
                            const int64_t *inst_B, const int64_t *inst_sample_off,
                            const int64_t *cpart_off, const double *cpart, const int64_t *f_off,
                            const double *fabp, double *logz, hipStream_t st) {
  if (n_chain_insts <= 0) return hipSuccess;
  hipLaunchKernelGGL(chain_sum_kernel, dim3(32, n_chain_insts), dim3(256), 0, st, inst, cinst,
                     chain_insts, n_chain_insts, inst_B, inst_sample_off, cpart_off, cpart, f_off,
                     fabp, logz);
  return hipGetLastError();
}

hipError_t launch_layout(const LayoutArgs &a, hipStream_t st) {
  const int64_t n = std::max<int64_t>(a.n_inst, a.n_tasks);
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(layout_kernel, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_unary(const ChainArgs &a, const int32_t *cis, int n_cis, int max_chunks,
                        int64_t max_B, const int64_t *f_off, float *U, double *fabp,
                        hipStream_t st) {
  if (n_cis <= 0 || max_B <= 0 || max_chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(unary_kernel, dim3((unsigned)((max_B + 255) / 256), max_chunks, n_cis),
                     dim3(256), 0, st, a, cis, f_off, U, fabp);
  return hipGetLastError();
}

}  // namespace tnvan
