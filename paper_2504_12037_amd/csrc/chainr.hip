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
// diagonal's unary factors (fields plus W-R couplings, Eq. 4) are read from
// the table unary_kernel fills once per (sample, position), one load per
// position, issued steps ahead of their use.
//
// The adjoint's forward pass is the forward kernel's arithmetic step for
// step, so it also writes the chain's log partial (logZ comes with the
// adjoint).  It walks the chain backwards from checkpoints of A (every step,
// in HBM; nothing is recomputed).  With
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
// samples, every edge correlation of the step and the group magnetisations,
// which each lane stores from its registers to the columns a per-step table
// names; the W-R correlations come from p_t and the spins directly.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.h"
#include "wave.h"

namespace tnvan {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef int i4v __attribute__((ext_vector_type(4)));

constexpr int CW = 16;       // samples per 16-sample group
constexpr int kWaves = 4;    // waves per workgroup

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

// row stride (floats) of the adjoint's LDS transposes: a multiple of 16
// plus 16 or 32, so that the four row groups of a read land in different banks
__host__ __device__ constexpr int ldt_of(int tiles) { return 16 * tiles + ((tiles & 1) ? 32 : 16); }
// row stride (BF16 values) of the split adjoint's transpose of R's hi and lo
// parts: 20 words, so that the four row groups of a read start 16 banks apart
constexpr int kLdtH = 40;
static_assert(2 * 16 * kLdtH * 2 <= 16 * ldt_of(2) * 4, "split R fits the FP32 transpose buffer");
static_assert(16 * 2 <= kLdtH, "a row holds the states of two tiles");

struct RL {
  size_t sp, ex, ga, rs, seg, fx, xa, xb, end;
};
__host__ __device__ inline int rk_of(const ChainLim &L) { return L.rk > 1 ? L.rk : 1; }
// LDS of one wave.  meet: also the split adjoint's exponents of the
// backward vectors and the two vectors exchanged at the meeting step
__host__ __device__ inline RL rlayout(const ChainLim &L, bool bwd, int sg, bool meet = false) {
  RL r{};
  size_t o = 0;
  r.sp = o;
  (void)sg;
  if (bwd) {
    const int ldt = ldt_of(kRegBwdTiles);
    r.ex = o; o = al16(o + (size_t)L.max_steps * CW * 4);
    r.ga = o; o = al16(o + (size_t)CW * ldt * 4);
    r.rs = o; o = al16(o + (size_t)CW * ldt * 4);
    // states A_t of one checkpoint segment replayed in the reverse walk
    r.seg = o; o = al16(o + (size_t)(rk_of(L) - 1) * kRegBwdTiles * 64 * 16);
    if (meet) {
      r.fx = o; o = al16(o + (size_t)L.max_steps * CW * 4);
      r.xa = o; o = al16(o + (size_t)kRegBwdTiles * 64 * 16);
      r.xb = o; o = al16(o + (size_t)kRegBwdTiles * 64 * 16);
    }
  }
  r.end = al16(o);
  return r;
}
// rows of 64 lanes x 16 bytes per adjoint task in the checkpoint buffer:
// the states kept at the checkpoint interval, or one per step (the split
// adjoint of one-tile chains keeps every step's vector)
__host__ __device__ inline int64_t ck_rows(const ChainLim &L) {
  const int64_t kept = (int64_t)((L.max_steps + rk_of(L) - 1) / rk_of(L)) * kRegBwdTiles;
  return kept > L.max_steps ? kept : (int64_t)L.max_steps;
}

// d[t][r] = prod_j phi_j(bit j of x) for x = 16 t + 4 lg + r < K, else 0
// (K is wave-uniform: a full group, K = 16 CT, takes no masking)
template <int CT, int GR>
__device__ inline void make_diag(const float (&p0)[GR], const float (&p1)[GR], int K, int lg,
                                 float (&d)[CT][4]) {
  auto ph = [&](int j, bool bit) { return j < GR ? (bit ? p1[j < GR ? j : 0] : p0[j < GR ? j : 0]) : 1.f; };
  const float fl = ph(2, lg & 1) * ph(3, lg & 2);
  float fr[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) fr[r] = ph(0, r & 1) * ph(1, r & 2) * fl;
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const float ft = ph(4, t & 1) * ph(5, t & 2);
#pragma unroll
    for (int r = 0; r < 4; ++r) d[t][r] = fr[r] * ft;
  }
  if (K < 16 * CT) {
#pragma unroll
    for (int t = 0; t < CT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (16 * t + 4 * lg + r >= K) d[t][r] = 0.f;
  }
}

// Unary factors of the group of g <= GR positions starting at order
// position gpos, as stored by unary_kernel: +-exp(-2 beta |f|), the sign
// that of f.  ub = phi_base(...) of the sample (computed once per chain).
__device__ inline const float *phi_base(const ChainArgs &a, int q, int64_t Bq, int64_t b) {
  return a.U + a.u_off[q] + (b < Bq ? b : Bq - 1);   // past the batch: clamped
}
template <int GR>
__device__ inline void load_phi(const float *ub, int64_t Bq, int gpos, int g, float (&u)[GR]) {
#pragma unroll
  for (int j = 0; j < GR; ++j) u[j] = ub[(int64_t)(gpos + (j < g ? j : 0)) * Bq];
}

// phi(+1) = 1, phi(-1) = exp(-2 beta f) for f >= 0 and the mirror image for
// f < 0 (normalised to max 1); then the diagonal over the group's states
template <int CT, int GR>
__device__ inline void diag_from_phi(const float (&u)[GR], int g, int lg, float (&d)[CT][4]) {
  float p0[GR], p1[GR];
#pragma unroll
  for (int j = 0; j < GR; ++j) {
    const bool in = j < g, neg = __builtin_signbit(u[j]);
    const float m = fabsf(u[j]);
    p0[j] = in && neg ? m : 1.f;
    p1[j] = in && !neg ? m : 1.f;
  }
  make_diag<CT, GR>(p0, p1, 1 << g, lg, d);
}

// the chain's group sizes are at most 4 + log2(tiles)
template <int CT> struct GroupMax { static constexpr int v = CT == 1 ? 4 : CT == 2 ? 5 : 6; };

template <int CT>
__device__ inline void load_t(const float *tab, int lane, f4 (&tc)[CT][CT]) {
  const f4 *p = reinterpret_cast<const f4 *>(tab) + lane;
#pragma unroll
  for (int i = 0; i < CT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) tc[i][j] = p[(i * CT + j) * 64];
}

template <int CT>
__device__ inline void load_tb(const uint16_t *tab, int lane, u4v (&tb)[CT][(CT + 1) / 2]) {
  const u4v *p = reinterpret_cast<const u4v *>(tab) + lane;
#pragma unroll
  for (int i = 0; i < CT; ++i)
#pragma unroll
    for (int c = 0; c < (CT + 1) / 2; ++c) tb[i][c] = p[(i * ((CT + 1) / 2) + c) * 64];
}

// out^T = T^T A^T: tc[nt][xt] from the Tr table, x in R-layout
template <int CT>
__device__ inline void mm_fwd(const f4 (&tc)[CT][CT], const float (&x)[CT][4], f4 (&acc)[CT]) {
#pragma unroll
  for (int nt = 0; nt < CT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int xt = 0; xt < CT; ++xt)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int nt = 0; nt < CT; ++nt)
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(tc[nt][xt][r], x[xt][r], acc[nt], 0, 0, 0);
}

template <int CT>
__device__ inline void mm_fwd_bf(const u4v (&tb)[CT][(CT + 1) / 2], const float (&x)[CT][4],
                                 f4 (&acc)[CT]) {
#pragma unroll
  for (int nt = 0; nt < CT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < (CT + 1) / 2; ++c) {
    bf8 bv;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int t = 2 * c + (i >> 2);
      bv[i] = (__bf16)(t < CT ? x[t < CT ? t : 0][i & 3] : 0.f);
    }
#pragma unroll
    for (int nt = 0; nt < CT; ++nt)
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, tb[nt][c]), bv,
                                                        acc[nt], 0, 0, 0);
  }
}


// Split-BF16 products (the FP32 path under TNVAN_FLAG_SPLIT_BF16): an FP32
// product a b is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi on the BF16
// 16x16x32 matrix cores (a_hi = a rounded to BF16, a_lo = the rest rounded
// to BF16), FP32 accumulation.  Element j of a lane's K chunk c is state
// 16 (2c + j/4) + 4 (lane >> 4) + j % 4, so the R-layout registers are the
// operand as they are, zero past the chain's tiles.
template <int CT>
__device__ inline void split_chunk(const float (&x)[CT][4], int c, bf8 &h, bf8 &l) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int t = 2 * c + (j >> 2);
    const float v = t < CT ? x[t < CT ? t : 0][j & 3] : 0.f;
    h[j] = (__bf16)v;
    l[j] = (__bf16)(v - (float)h[j]);
  }
}
__device__ inline bf8 as_bf8(u4v v) { return __builtin_bit_cast(bf8, v); }
__device__ inline f4 mfma_bf(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Forward operands of one step, per product mode (0: FP32, 1: BF16 tables,
// 2: split BF16), loaded from the step's tables and multiplied by the
// R-layout state: out^T = T^T A^T
template <int kM, int CT> struct FwdOps;
template <int CT> struct FwdOps<0, CT> {
  f4 t[CT][CT];
  __device__ void load(const ChainArgs &a, const ChainStep &s, int lane) { load_t<CT>(a.Tr + s.tr_off, lane, t); }
  __device__ void mm(const float (&x)[CT][4], f4 (&acc)[CT]) const { mm_fwd<CT>(t, x, acc); }
};
template <int CT> struct FwdOps<1, CT> {
  u4v b[CT][(CT + 1) / 2];
  __device__ void load(const ChainArgs &a, const ChainStep &s, int lane) { load_tb<CT>(a.Trb + s.trb_off, lane, b); }
  __device__ void mm(const float (&x)[CT][4], f4 (&acc)[CT]) const { mm_fwd_bf<CT>(b, x, acc); }
};
template <int CT> struct FwdOps<2, CT> {
  static constexpr int NC = (CT + 1) / 2;
  u4v h[CT][NC], l[CT][NC];
  __device__ void load(const ChainArgs &a, const ChainStep &s, int lane) {
    const u4v *p = reinterpret_cast<const u4v *>(a.Ts3 + s.s3_off) + lane;
#pragma unroll
    for (int i = 0; i < CT; ++i)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        h[i][c] = p[(i * NC + c) * 64];
        l[i][c] = p[((CT + i) * NC + c) * 64];
      }
  }
  __device__ void mm(const float (&x)[CT][4], f4 (&acc)[CT]) const {
#pragma unroll
    for (int nt = 0; nt < CT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bf8 xh, xl;
      split_chunk<CT>(x, c, xh, xl);
#pragma unroll
      for (int nt = 0; nt < CT; ++nt) acc[nt] = mfma_bf(as_bf8(h[nt][c]), xh, acc[nt]);
#pragma unroll
      for (int nt = 0; nt < CT; ++nt) acc[nt] = mfma_bf(as_bf8(h[nt][c]), xl, acc[nt]);
#pragma unroll
      for (int nt = 0; nt < CT; ++nt) acc[nt] = mfma_bf(as_bf8(l[nt][c]), xh, acc[nt]);
    }
  }
};

// power-of-two rescale of the step output and the next diagonal:
// x = out * 2^-e * d; returns e of the lane's sample
template <int CT>
__device__ inline int rescale_next(const f4 (&acc)[CT], const float (&d)[CT][4], float (&x)[CT][4]) {
  float m = 0.f;
#pragma unroll
  for (int nt = 0; nt < CT; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) m = fmaxf(m, acc[nt][r]);
  const int e = expo32(rows4_max(m));
  const float sc = pow2neg(e);
#pragma unroll
  for (int t = 0; t < CT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) x[t][r] = acc[t][r] * sc * d[t][r];
  return e;
}

// the wave-uniform step descriptor t (scalar loads, not vector loads whose
// wait would also wait for every operand load issued before it)
// (the descriptors are never written on the device, so they are read
// through the constant address space, which the compiler loads with scalar
// instructions even where the kernel stores to global memory)
typedef const __attribute__((address_space(4))) int32_t *const_i32_ptr;
__device__ inline ChainStep step_at(const ChainStep *cs, int t) {
  static_assert(sizeof(ChainStep) % 4 == 0, "descriptor of whole words");
  const_i32_ptr src = (const_i32_ptr)(cs + __builtin_amdgcn_readfirstlane(t));
  ChainStep r;
  int32_t *dst = reinterpret_cast<int32_t *>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(ChainStep) / 4); ++i) dst[i] = src[i];
  return r;
}

struct Task {
  int q, c;
  int64_t b0, Bq;
};

__device__ inline Task task_at(const ChainArgs &a, int i) {
  Task k;
  k.q = a.task_inst[i];
  k.c = a.task_chain[i];
  k.b0 = a.task_start[i];
  k.Bq = a.inst_B[k.q];
  return k;
}

// Persistent form: the next task of a wave from the device counter, widest
// chains first (false when none is left); gi = width index (1 << gi tiles)
__device__ inline bool pq_task(const ChainArgs &a, int lane, int &task, int &gi) {
  int v = 0;
  if (lane == 0) v = atomicAdd(a.pq, 1);
  v = __builtin_amdgcn_readfirstlane(__shfl(v, 0, 64));
  for (int g = 2; g >= 0; --g) {
    if (v < a.pq_n[g]) {
      task = a.pq_lo[g] + v;
      gi = g;
      return true;
    }
    v -= a.pq_n[g];
  }
  return false;
}
// the last wave to leave resets the counter and the exit count
__device__ inline void pq_exit(const ChainArgs &a, int lane) {
  if (lane == 0 && atomicAdd(a.pq + 1, 1) == (int)gridDim.x * kWaves - 1) {
    atomicExch(a.pq, 0);
    atomicExch(a.pq + 1, 0);
  }
}

__device__ inline Task wave_task(const ChainArgs &a, int wave) {
  Task k;
  const int i = a.task_base + blockIdx.x * kWaves + wave;
  k.q = -1;
  if (i >= a.task_base + a.n_tasks) return k;
  k.q = a.task_inst[i];
  k.c = a.task_chain[i];
  k.b0 = a.task_start[i];
  k.Bq = a.inst_B[k.q];
  return k;
}

// forward of one chain for SG groups of 16 samples: per sample the sum of
// the step exponents (ln 2) and ln of the root value; the unary
// normalisations are added from unary_kernel's sums
template <int kM, int CT, int SG>
__device__ inline void fwd_chain(const ChainArgs &a, const Task &tk, const ChainDesc &cd, int lane) {
  constexpr int GR = GroupMax<CT>::v;
  const int ls = lane & 15, lg = lane >> 4;
  const ChainStep *cs = a.csteps + cd.cs_off;
  const int T = cd.n_steps;
  int esum[SG];
  float x[SG][CT][4], raw[SG];
  const float *ub[SG];
#pragma unroll
  for (int gi = 0; gi < SG; ++gi) ub[gi] = phi_base(a, tk.q, tk.Bq, tk.b0 + gi * CW + ls);
  {
    const ChainStep s0 = cs[0];
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) {
      float u[GR];
      load_phi<GR>(ub[gi], tk.Bq, s0.gpos, s0.g, u);
      diag_from_phi<CT, GR>(u, s0.g, lg, x[gi]);
      esum[gi] = 0;
    }
  }
  // step t with the descriptor nx of step t + 1, the operands of step t and
  // the unary factors uc of step t + 1's group; loads step t + 1's operands
  // and step t + 2's unary factors into the other register set (two sets
  // used in turn: a loaded value is never copied, which would wait for the
  // load)
  auto fstep = [&](int t, const ChainStep &nx, const FwdOps<kM, CT> &oc, const float (&uc)[SG][GR],
                   ChainStep &nn, FwdOps<kM, CT> &on, float (&un)[SG][GR]) -> bool {
    const bool last = t == T - 1;
    nn = step_at(cs, t + 2 < T ? t + 2 : T - 1);
    on.load(a, nx, lane);
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) load_phi<GR>(ub[gi], tk.Bq, nn.gpos, nn.g, un[gi]);
    f4 acc[SG][CT];
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) oc.mm(x[gi], acc[gi]);
    if (last) {
#pragma unroll
      for (int gi = 0; gi < SG; ++gi) raw[gi] = __shfl(acc[gi][0][0], ls, 64);
      return true;
    }
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) {
      float d[CT][4];
      diag_from_phi<CT, GR>(uc[gi], nx.g, lg, d);
      esum[gi] += rescale_next<CT>(acc[gi], d, x[gi]);
    }
    return false;
  };
  ChainStep nA = step_at(cs, T > 1 ? 1 : 0), nB;
  FwdOps<kM, CT> oA, oB;
  float uA[SG][GR], uB[SG][GR];
  oA.load(a, cs[0], lane);
#pragma unroll
  for (int gi = 0; gi < SG; ++gi) load_phi<GR>(ub[gi], tk.Bq, nA.gpos, nA.g, uA[gi]);
  for (int t = 0;; t += 2) {
    if (fstep(t, nA, oA, uA, nB, oB, uB)) break;
    if (fstep(t + 1, nB, oB, uB, nA, oA, uA)) break;
  }
  if (lg == 0) {
#pragma unroll
    for (int gi = 0; gi < SG; ++gi) {
      const int64_t b = tk.b0 + gi * CW + ls;
      if (b < tk.Bq)
        a.cpart[a.cpart_off[tk.q] + (int64_t)tk.c * tk.Bq + b] =
            (double)esum[gi] * 0.69314718055994530942 + log((double)raw[gi]);
    }
  }
}

template <int kM, int CT, int SG>
__global__ __launch_bounds__(256) void rchain_fwd_kernel(ChainArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const Task tk = wave_task(a, wave);
  if (tk.q < 0) return;
  const InstDesc D = a.inst[tk.q];
  const ChainInst C = a.cinst[tk.q];
  const ChainDesc cd = a.chains[C.chain_off + tk.c];
  (void)smem;
  (void)D;
  fwd_chain<kM, CT, SG>(a, tk, cd, lane);
}


template <int CT, bool kS, bool kK>
__device__ inline void bwd_chain(const ChainArgs &a, const Task &tk, const InstDesc &D,
                                 const ChainDesc &cd, char *base, const RL &L, int lane,
                                 int task_id) {
  // checkpoint interval: A_t is kept for t = 0, k, 2k, ...; the reverse walk
  // replays each segment's other states from its checkpoint into LDS with
  // the forward pass's own operations (so they are the same values)
  const int kk = kK ? rk_of(a.lim) : 1;
  constexpr int GR = GroupMax<CT>::v;
  constexpr int NC = (CT + 1) / 2;
  constexpr int kM = kS ? 2 : 0;
  constexpr int LDT = ldt_of(CT);
  const int ls = lane & 15, lg = lane >> 4;
  const ChainStep *cs = a.csteps + cd.cs_off;
  int *ex = reinterpret_cast<int *>(base + L.ex);
  float *ga = reinterpret_cast<float *>(base + L.ga);
  float *rs = reinterpret_cast<float *>(base + L.rs);
  __bf16 *rsb = reinterpret_cast<__bf16 *>(base + L.rs);   // split R (split products)
  const int64_t left = tk.Bq - tk.b0;
  const int nvalid = (int)(left < CW ? left : CW);
  const SpinBits sp = load_bits(a.spins + a.inst_spin_off[tk.q] + (tk.b0 + (ls < nvalid ? ls : 0)) * D.nw,
                                D.nw, ls < nvalid);
  const float gs = ls < nvalid ? (float)a.grad[a.inst_sample_off[tk.q] + tk.b0 + ls] : 0.f;
  float *prow = a.partial + a.inst_partial_off[tk.q] + (tk.b0 / CW) * (int64_t)D.n_partial;
  const int T = cd.n_steps;
  f4 *ck = reinterpret_cast<f4 *>(a.ckpt) + (int64_t)task_id * ck_rows(a.lim) * 64 + lane;
  f4 *seg = reinterpret_cast<f4 *>(base + L.seg) + lane;
  const float *ub = phi_base(a, tk.q, tk.Bq, tk.b0 + ls);

  // Both passes load the operands of the next step while one step is
  // processed, into two register sets used in turn: a loaded value is never
  // copied (a copy would wait for the load at the end of the step).

  // forward: A_t checkpointed every step, exponents in LDS, root value, and
  // the chain's log partial (the forward kernel's exact arithmetic, so the
  // adjoint also yields logZ)
  float x[CT][4];
  int esum = 0;
  {
    float u[GR];
    load_phi<GR>(ub, tk.Bq, cs[0].gpos, cs[0].g, u);
    diag_from_phi<CT, GR>(u, cs[0].g, lg, x);
  }
  float raw = 1.f;
  {
    // step t with the descriptor nx of step t + 1, operands oc of step t and
    // unary factors uc of step t + 1's group; loads step t + 1's operands
    // and step t + 2's unary factors
    auto fstep = [&](int t, const ChainStep &nx, const FwdOps<kM, CT> &oc, const float (&uc)[GR],
                     ChainStep &nn, FwdOps<kM, CT> &on, float (&un)[GR]) -> bool {
      if (!kK || t % kk == 0) {
#pragma unroll
        for (int i = 0; i < CT; ++i)
          ck[((t / kk) * kRegBwdTiles + i) * 64] = f4{x[i][0], x[i][1], x[i][2], x[i][3]};
      }
      const bool last = t == T - 1;
      nn = step_at(cs, t + 2 < T ? t + 2 : T - 1);
      on.load(a, nx, lane);
      load_phi<GR>(ub, tk.Bq, nn.gpos, nn.g, un);
      f4 acc[CT];
      oc.mm(x, acc);
      if (last) {
        raw = __shfl(acc[0][0], ls, 64);
        return true;
      }
      float d[CT][4];
      diag_from_phi<CT, GR>(uc, nx.g, lg, d);
      const int e = rescale_next<CT>(acc, d, x);
      esum += e;
      if (lg == 0) ex[t * CW + ls] = e;
      return false;
    };
    ChainStep nA = step_at(cs, T > 1 ? 1 : 0), nB;
    FwdOps<kM, CT> oA, oB;
    float uA[GR], uB[GR];
    oA.load(a, cs[0], lane);
    load_phi<GR>(ub, tk.Bq, nA.gpos, nA.g, uA);
    for (int t = 0;; t += 2) {
      if (fstep(t, nA, oA, uA, nB, oB, uB)) break;
      if (fstep(t + 1, nB, oB, uB, nA, oA, uA)) break;
    }
  }
  wsync();
  if (lg == 0 && tk.b0 + ls < tk.Bq)
    a.cpart[a.cpart_off[tk.q] + (int64_t)tk.c * tk.Bq + tk.b0 + ls] =
        (double)esum * 0.69314718055994530942 + log((double)raw);

  // R of the closing step: d ln(raw) / d out = 1 / raw on its single entry
  float R[CT][4];
#pragma unroll
  for (int i = 0; i < CT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) R[i][r] = 0.f;
  if (lg == 0) R[0][0] = raw > 0.f ? 1.f / raw : 0.f;

  // the walk, step t with its checkpoint A_t, Lambda operands and unary
  // factors loaded during step t + 1
  // (Lambda operands: FP32 tq, or split-BF16 qh / ql)
  struct Pre {
    f4 a[CT];
    f4 tq[kS ? 1 : CT][kS ? 1 : CT];
    u4v qh[kS ? CT : 1][NC], ql[kS ? CT : 1][NC];
    float u[GR];
  };
  auto prefetch = [&](const ChainStep &s, int t, Pre &p) {
    if (!kK || t % kk == 0) {
#pragma unroll
      for (int i = 0; i < CT; ++i) p.a[i] = ck[((t / kk) * kRegBwdTiles + i) * 64];
    }
    if constexpr (kS) {
      const u4v *q3 = reinterpret_cast<const u4v *>(a.Ts3 + s.s3_off) + lane + 2 * CT * NC * 64;
#pragma unroll
      for (int i = 0; i < CT; ++i)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          p.qh[i][c] = q3[(i * NC + c) * 64];
          p.ql[i][c] = q3[((CT + i) * NC + c) * 64];
        }
    } else {
      load_t<CT>(a.Tq + s.tq_off, lane, p.tq);
    }
    load_phi<GR>(ub, tk.Bq, s.gpos, s.g, p.u);
  };
  // A_{t0+1} .. A_top of the segment from its checkpoint A_t0
  auto replay = [&](int t0, int top) {
    float xr[CT][4];
#pragma unroll
    for (int i = 0; i < CT; ++i) {
      const f4 v = ck[((t0 / kk) * kRegBwdTiles + i) * 64];
#pragma unroll
      for (int r = 0; r < 4; ++r) xr[i][r] = v[r];
    }
    for (int j = t0; j < top; ++j) {
      const ChainStep sj = step_at(cs, j), sn1 = step_at(cs, j + 1);
      FwdOps<kM, CT> o;
      o.load(a, sj, lane);
      float u[GR];
      load_phi<GR>(ub, tk.Bq, sn1.gpos, sn1.g, u);
      f4 acc[CT];
      o.mm(xr, acc);
      float d[CT][4];
      diag_from_phi<CT, GR>(u, sn1.g, lg, d);
      (void)rescale_next<CT>(acc, d, xr);
#pragma unroll
      for (int i = 0; i < CT; ++i)
        seg[((j - t0) * kRegBwdTiles + i) * 64] = f4{xr[i][0], xr[i][1], xr[i][2], xr[i][3]};
    }
  };
  auto walk = [&](int t, const ChainStep &st, const Pre &cur, ChainStep &sn, Pre &nxt) {
    const int g = st.g, w = st.w;
    float As[CT][4];
    if (kK && t % kk != 0) {
      // the top of a segment replays it; its other steps read the result
      if (t % kk == kk - 1 || t == T - 1) replay(t - t % kk, t);
#pragma unroll
      for (int i = 0; i < CT; ++i) {
        const f4 v = seg[((t % kk - 1) * kRegBwdTiles + i) * 64];
#pragma unroll
        for (int r = 0; r < 4; ++r) As[i][r] = v[r];
      }
    } else {
#pragma unroll
      for (int i = 0; i < CT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) As[i][r] = cur.a[i][r];
    }
    // operands used later in this step, issued now: T (for G = H o T) and
    // the S_x / S_o tables, in FP32 or split-BF16 form
    f4 tr[CT][CT], sx[kS ? 1 : CT], so[kS ? 1 : CT];
    u4v sxb[NC], sob[NC];
    load_t<CT>(a.Tr + st.tr_off, lane, tr);
    if constexpr (kS) {
      const u4v *q3 = reinterpret_cast<const u4v *>(a.Ts3 + st.s3_off) + lane + 4 * CT * NC * 64;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        sxb[c] = q3[c * 64];
        sob[c] = q3[(NC + c) * 64];
      }
    } else {
      const f4 *sxo = reinterpret_cast<const f4 *>(a.Tsx + st.sx_off) + lane;
#pragma unroll
      for (int i = 0; i < CT; ++i) {
        sx[i] = sxo[i * 64];
        so[i] = sxo[(CT + i) * 64];
      }
    }
    // where this lane's four cells of the step's correlations are stored
    const i4v dq = reinterpret_cast<const i4v *>(a.Tdq + st.dq_off)[lane];
    // the next step walked: descriptor and operands (step 0 reloads itself)
    sn = step_at(cs, t > 0 ? t - 1 : 0);
    prefetch(sn, t > 0 ? t - 1 : 0, nxt);
    // Lambda = T R (R-layout over the group states)
    f4 lam[CT];
#pragma unroll
    for (int xt = 0; xt < CT; ++xt) lam[xt] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (kS) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        bf8 rh, rl;
        split_chunk<CT>(R, c, rh, rl);
        // the split R also goes to LDS (hi in rows 0-15, lo in rows 16-31,
        // row = sample) for the H product below, which reads it transposed:
        // R is split once per step
        typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
        if (2 * c < CT) {
          *reinterpret_cast<bf4 *>(rsb + ls * kLdtH + 32 * c + 4 * lg) = rh.lo;
          *reinterpret_cast<bf4 *>(rsb + (16 + ls) * kLdtH + 32 * c + 4 * lg) = rl.lo;
        }
        if (2 * c + 1 < CT) {
          *reinterpret_cast<bf4 *>(rsb + ls * kLdtH + 32 * c + 16 + 4 * lg) = rh.hi;
          *reinterpret_cast<bf4 *>(rsb + (16 + ls) * kLdtH + 32 * c + 16 + 4 * lg) = rl.hi;
        }
#pragma unroll
        for (int xt = 0; xt < CT; ++xt) lam[xt] = mfma_bf(as_bf8(cur.qh[xt][c]), rh, lam[xt]);
#pragma unroll
        for (int xt = 0; xt < CT; ++xt) lam[xt] = mfma_bf(as_bf8(cur.qh[xt][c]), rl, lam[xt]);
#pragma unroll
        for (int xt = 0; xt < CT; ++xt) lam[xt] = mfma_bf(as_bf8(cur.ql[xt][c]), rh, lam[xt]);
      }
    } else {
#pragma unroll
      for (int ot = 0; ot < CT; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int xt = 0; xt < CT; ++xt)
            lam[xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur.tq[xt][ot][r], R[ot][r], lam[xt], 0, 0, 0);
    }
    // W-R correlations: per-sample magnetisation of a group spin times the
    // neighbouring width-set spin, weighted and summed over the samples.
    // Bit j of this lane's state 16 t + 4 lg + r is bit j of r (j < 2), of
    // lg (j = 2, 3) or of t (j >= 4): a branch on the wave-uniform j turns
    // the signs into constants, or into the lane's own sign
    if (st.n_wri > 0) {
      float pa[CT][4], pr[4], pt[CT];
#pragma unroll
      for (int xt = 0; xt < CT; ++xt)
#pragma unroll
        for (int r = 0; r < 4; ++r) pa[xt][r] = As[xt][r] * lam[xt][r];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        pr[r] = pa[0][r];
#pragma unroll
        for (int xt = 1; xt < CT; ++xt) pr[r] += pa[xt][r];
      }
#pragma unroll
      for (int xt = 0; xt < CT; ++xt) pt[xt] = (pa[xt][0] + pa[xt][1]) + (pa[xt][2] + pa[xt][3]);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < st.n_wri) {
          const int j = __builtin_amdgcn_readfirstlane(st.wri[k] & 0xff), wi = st.wri[k] >> 8;
          float m;
          if (j == 0) {
            m = (pr[0] - pr[1]) + (pr[2] - pr[3]);
          } else if (j == 1) {
            m = (pr[0] + pr[1]) - (pr[2] + pr[3]);
          } else if (j < 4) {
            const float tot = (pr[0] + pr[1]) + (pr[2] + pr[3]);
            m = ((lg >> (j - 2)) & 1) ? -tot : tot;
          } else {
            m = 0.f;
#pragma unroll
            for (int xt = 0; xt < CT; ++xt) m += ((xt >> (j - 4)) & 1) ? -pt[xt] : pt[xt];
          }
          m = rows4_sum(m) * gs;
          const float v = row16_sum(m * sp.sigma(wi));
          if (lane == 0) prow[D.nr + st.wre[k]] = v;
        }
    }
    // R of the previous step (unused after the first step)
    float Rn[CT][4];
    {
      float d[CT][4];
      diag_from_phi<CT, GR>(cur.u, g, lg, d);
      const float sc = pow2neg(ex[(t > 0 ? t - 1 : 0) * CW + ls]);
#pragma unroll
      for (int xt = 0; xt < CT; ++xt)
#pragma unroll
        for (int r = 0; r < 4; ++r) Rn[xt][r] = d[xt][r] * lam[xt][r] * sc;
    }
    // H = sum_s (g A)[s] R[s]^T through an LDS transpose
#pragma unroll
    for (int xt = 0; xt < CT; ++xt)
      *reinterpret_cast<f4 *>(ga + ls * LDT + 16 * xt + 4 * lg) =
          f4{gs * As[xt][0], gs * As[xt][1], gs * As[xt][2], gs * As[xt][3]};
    if constexpr (!kS) {
#pragma unroll
      for (int ot = 0; ot < CT; ++ot)
        *reinterpret_cast<f4 *>(rs + ls * LDT + 16 * ot + 4 * lg) =
            f4{R[ot][0], R[ot][1], R[ot][2], R[ot][3]};
    }
    wsync();
    // per output tile: H (samples contracted), G = H o T, Q'^T = G^T S_x
    f4 qt[CT];
    if constexpr (kS) {
      // H with the 16 samples in each half of the 32-long contraction: the
      // first product takes hi and lo of g A against hi of R, the second hi
      // of g A against lo of R; lane (lg, ls) supplies samples 4 lg + j
      bf8 ah1[CT], ah2[CT], rb1[CT], rb2[CT];
#pragma unroll
      for (int xt = 0; xt < CT; ++xt)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float va = ga[(4 * lg + j) * LDT + 16 * xt + ls];
          const __bf16 h = (__bf16)va, l = (__bf16)(va - (float)h);
          ah1[xt][j] = h; ah1[xt][4 + j] = l;
          ah2[xt][j] = h; ah2[xt][4 + j] = (__bf16)0.f;
          const __bf16 rh = rsb[(4 * lg + j) * kLdtH + 16 * xt + ls];
          const __bf16 rl = rsb[(16 + 4 * lg + j) * kLdtH + 16 * xt + ls];
          rb1[xt][j] = rh; rb1[xt][4 + j] = rh;
          rb2[xt][j] = rl; rb2[xt][4 + j] = (__bf16)0.f;
        }
#pragma unroll
      for (int ot = 0; ot < CT; ++ot) {
        f4 hg[CT];
#pragma unroll
        for (int xt = 0; xt < CT; ++xt) hg[xt] = mfma_bf(ah1[xt], rb1[ot], f4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int xt = 0; xt < CT; ++xt) hg[xt] = mfma_bf(ah2[xt], rb2[ot], hg[xt]);
        // G = H o T (the FP32 table, R-layout), then Q'^T = G^T S_x with the
        // lane's 8 G values as the operand (S_x is exact in BF16: two
        // products)
        float gv[CT][4];
#pragma unroll
        for (int xt = 0; xt < CT; ++xt)
#pragma unroll
          for (int r = 0; r < 4; ++r) gv[xt][r] = hg[xt][r] * tr[ot][xt][r];
        bf8 gh, gl;
        split_chunk<CT>(gv, 0, gh, gl);
        qt[ot] = mfma_bf(gh, as_bf8(sxb[0]), f4{0.f, 0.f, 0.f, 0.f});
        qt[ot] = mfma_bf(gl, as_bf8(sxb[0]), qt[ot]);
      }
    } else {
#pragma unroll
      for (int ot = 0; ot < CT; ++ot) {
        f4 hg[CT];
#pragma unroll
        for (int xt = 0; xt < CT; ++xt) {
          hg[xt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int kc = 0; kc < 4; ++kc)
            hg[xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                ga[(4 * kc + lg) * LDT + 16 * xt + ls], rs[(4 * kc + lg) * LDT + 16 * ot + ls],
                hg[xt], 0, 0, 0);
        }
        qt[ot] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int xt = 0; xt < CT; ++xt)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            qt[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(hg[xt][r] * tr[ot][xt][r], sx[xt][r],
                                                          qt[ot], 0, 0, 0);
      }
    }
    wsync();
    // Q = S_o^T Q'^T (operand tables)
    f4 qq = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (kS) {
      float qv[CT][4];
#pragma unroll
      for (int ot = 0; ot < CT; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r) qv[ot][r] = qt[ot][r];
      bf8 qh, ql;
      split_chunk<CT>(qv, 0, qh, ql);
      qq = mfma_bf(as_bf8(sob[0]), qh, qq);
      qq = mfma_bf(as_bf8(sob[0]), ql, qq);
    } else {
#pragma unroll
      for (int ot = 0; ot < CT; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          qq = __builtin_amdgcn_mfma_f32_16x16x4f32(so[ot][r], qt[ot][r], qq, 0, 0, 0);
    }
    // magnetisations and edge correlations straight from the registers
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (dq[r] >= 0) prow[dq[r]] = qq[r];
#pragma unroll
    for (int i = 0; i < CT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) R[i][r] = Rn[i][r];
  };
  ChainStep sA = step_at(cs, T - 1), sB;
  Pre pA, pB;
  prefetch(sA, T - 1, pA);
  for (int t = T - 1; t >= 0; t -= 2) {
    walk(t, sA, pA, sB, pB);
    if (t == 0) break;
    walk(t - 1, sB, pB, sA, pA);
  }
}

// ---------------------------------------------------------------------------
// Magnetisation moments of the remainder on a chain: the Taylor jets in
// eta = beta H of the general moments kernel, in the chain's register
// layout.  Each state carries the coefficients (c0, c1, c2) of its message;
// the transfer tables act on each coefficient alike (FP32 products), and a
// group's diagonal brings the jet d (1, m, m^2 / 2) of its states'
// magnetisation m.  The rescale is the forward pass's: the power of two of
// the largest c0, applied to all three coefficients.  The closing entry z
// gives the chain's log partial, <M> = z1 / z0 and Var(M) = 2 z2 / z0 -
// (z1 / z0)^2 per sample (the chains of an instance are independent given
// s_W, so their means and variances add).

// magnetisation of state 16 t + 4 lg + r of a group of g spins (bit set:
// spin -1); states past the group have d = 0
__device__ inline float state_mag(int g, int t, int lg, int r) {
  return (float)(g - 2 * (__builtin_popcount(r) + __builtin_popcount(lg) + __builtin_popcount(t)));
}

// x_k = jet product of the step output (a0, a1, a2), rescaled by the power
// of two of its largest c0, with the diagonal jet of the next group;
// returns that exponent
template <int CT>
__device__ inline int jet_next(const f4 (&a0)[CT], const f4 (&a1)[CT], const f4 (&a2)[CT],
                               const float (&d)[CT][4], int g, int lg, float (&x0)[CT][4],
                               float (&x1)[CT][4], float (&x2)[CT][4]) {
  float mx = 0.f;
#pragma unroll
  for (int t = 0; t < CT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) mx = fmaxf(mx, a0[t][r]);
  const int e = expo32(rows4_max(mx));
  const float sc = pow2neg(e);
#pragma unroll
  for (int t = 0; t < CT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float D = d[t][r] * sc, mg = state_mag(g, t, lg, r);
      x0[t][r] = a0[t][r] * D;
      x1[t][r] = (a1[t][r] + mg * a0[t][r]) * D;
      x2[t][r] = (a2[t][r] + mg * a1[t][r] + 0.5f * mg * mg * a0[t][r]) * D;
    }
  return e;
}

template <int CT>
__device__ inline void mom_chain(const ChainArgs &a, const Task &tk, const ChainDesc &cd, int lane) {
  constexpr int GR = GroupMax<CT>::v;
  const int ls = lane & 15, lg = lane >> 4;
  const ChainStep *cs = a.csteps + cd.cs_off;
  const int T = cd.n_steps;
  const float *ub = phi_base(a, tk.q, tk.Bq, tk.b0 + ls);
  float x0[CT][4], x1[CT][4], x2[CT][4];
  {
    float u[GR], d[CT][4];
    load_phi<GR>(ub, tk.Bq, cs[0].gpos, cs[0].g, u);
    diag_from_phi<CT, GR>(u, cs[0].g, lg, d);
#pragma unroll
    for (int t = 0; t < CT; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float mg = state_mag(cs[0].g, t, lg, r);
        x0[t][r] = d[t][r];
        x1[t][r] = d[t][r] * mg;
        x2[t][r] = d[t][r] * (0.5f * mg * mg);
      }
  }
  int esum = 0;
  float z0 = 1.f, z1 = 0.f, z2 = 0.f;
  // step t with the descriptor nx of step t + 1, the operands of step t and
  // the unary factors uc of step t + 1's group; loads step t + 1's operands
  // and step t + 2's unary factors into the other register set
  auto fstep = [&](int t, const ChainStep &nx, const FwdOps<0, CT> &oc, const float (&uc)[GR],
                   ChainStep &nn, FwdOps<0, CT> &on, float (&un)[GR]) -> bool {
    nn = step_at(cs, t + 2 < T ? t + 2 : T - 1);
    on.load(a, nx, lane);
    load_phi<GR>(ub, tk.Bq, nn.gpos, nn.g, un);
    f4 a0[CT], a1[CT], a2[CT];
    oc.mm(x0, a0);
    oc.mm(x1, a1);
    oc.mm(x2, a2);
    if (t == T - 1) {
      z0 = __shfl(a0[0][0], ls, 64);
      z1 = __shfl(a1[0][0], ls, 64);
      z2 = __shfl(a2[0][0], ls, 64);
      return true;
    }
    float d[CT][4];
    diag_from_phi<CT, GR>(uc, nx.g, lg, d);
    esum += jet_next<CT>(a0, a1, a2, d, nx.g, lg, x0, x1, x2);
    return false;
  };
  ChainStep nA = step_at(cs, T > 1 ? 1 : 0), nB;
  FwdOps<0, CT> oA, oB;
  float uA[GR], uB[GR];
  oA.load(a, cs[0], lane);
  load_phi<GR>(ub, tk.Bq, nA.gpos, nA.g, uA);
  for (int t = 0;; t += 2) {
    if (fstep(t, nA, oA, uA, nB, oB, uB)) break;
    if (fstep(t + 1, nB, oB, uB, nA, oA, uA)) break;
  }
  if (lg == 0 && tk.b0 + ls < tk.Bq) {
    const int64_t i = a.cpart_off[tk.q] + (int64_t)tk.c * tk.Bq + tk.b0 + ls;
    const double r1 = (double)z1 / (double)z0, r2 = (double)z2 / (double)z0;
    a.cpart[i] = (double)esum * 0.69314718055994530942 + log((double)z0);
    a.mpart[i] = r1;
    a.mpart[a.mtot + i] = 2.0 * r2 - r1 * r1;
  }
}

template <int CT>
__global__ __launch_bounds__(256) void rchain_mom_kernel(ChainArgs a) {
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const Task tk = wave_task(a, wave);
  if (tk.q < 0) return;
  const ChainInst C = a.cinst[tk.q];
  const ChainDesc cd = a.chains[C.chain_off + tk.c];
  mom_chain<CT>(a, tk, cd, lane);
}

__global__ void chain_mom_sum_kernel(const ChainInst *cinst, const int32_t *cis,
                                     const int64_t *inst_B, const int64_t *inst_sample_off,
                                     const int64_t *cpart_off, const double *mpart, int64_t mtot,
                                     double *mean, double *var) {
  const int q = cis[blockIdx.y];
  const int64_t B = inst_B[q];
  const int nc = cinst[q].n_chains;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < B;
       b += (int64_t)gridDim.x * blockDim.x) {
    double m = 0.0, v = 0.0;
    for (int c = 0; c < nc; ++c) {
      const int64_t i = cpart_off[q] + (int64_t)c * B + b;
      m += mpart[i];
      v += mpart[mtot + i];
    }
    mean[inst_sample_off[q] + b] = m;
    var[inst_sample_off[q] + b] = v;
  }
}

// ---------------------------------------------------------------------------
// Split adjoint of one-tile chains.  The backward vectors need not wait for
// the forward pass: beta_{T-1} is the unit vector of the closing entry and
// beta_{t-1} = d_t * (T_t beta_t), each rescaled by a power of two of its
// own, 2^-f_{t-1}.  With out_t = T_t^T A_t the step outputs of the forward
// pass, R_t = d ln Z / d out_t = K_t beta_t for a per-sample scalar K_t:
// out_t . R_t = 1 at every step fixes K at the meeting step m - 1
// (m = ceil(T/2)), and the two recursions give K_t = K_{t-1} 2^(e_{t-1} -
// f_{t-1}).  Role A runs the forward pass of steps < m (checkpoints and
// exponents as in the one-wave walk); role B runs the backward vectors of
// steps >= m and keeps them in the checkpoint slots of those steps.  After
// the meeting, A continues the forward pass through steps >= m and takes
// their gradient terms with R_t = K_t beta_t, while B walks steps < m from
// R_{m-1} = K_{m-1} beta_{m-1} as the one-wave walk does.  Each wave's path
// is about half the chain's.  Two waves of a workgroup take the two roles of
// a chain, with one barrier between the phases; the persistent kernel runs
// the four phases in turn on one wave (the same arithmetic, so the same
// results bit for bit).

// Lambda operands of one step: FP32 tq, or split-BF16 qh / ql
template <int CT, bool kS> struct LamOps {
  static constexpr int NC = (CT + 1) / 2;
  f4 tq[kS ? 1 : CT][kS ? 1 : CT];
  u4v qh[kS ? CT : 1][NC], ql[kS ? CT : 1][NC];
  __device__ void load(const ChainArgs &a, const ChainStep &s, int lane) {
    if constexpr (kS) {
      const u4v *q3 = reinterpret_cast<const u4v *>(a.Ts3 + s.s3_off) + lane + 2 * CT * NC * 64;
#pragma unroll
      for (int i = 0; i < CT; ++i)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          qh[i][c] = q3[(i * NC + c) * 64];
          ql[i][c] = q3[((CT + i) * NC + c) * 64];
        }
    } else {
      load_t<CT>(a.Tq + s.tq_off, lane, tq);
    }
  }
};

// Lambda = T R in R-layout over the group's states; with kW (split
// products) the split R also goes to LDS, sample-major, for the H product
template <int CT, bool kS, bool kW>
__device__ inline void lam_mm(const LamOps<CT, kS> &o, const float (&R)[CT][4], __bf16 *rsb, int ls,
                              int lg, f4 (&lam)[CT]) {
  constexpr int NC = (CT + 1) / 2;
#pragma unroll
  for (int xt = 0; xt < CT; ++xt) lam[xt] = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (kS) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bf8 rh, rl;
      split_chunk<CT>(R, c, rh, rl);
      if constexpr (kW) {
        typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
        if (2 * c < CT) {
          *reinterpret_cast<bf4 *>(rsb + ls * kLdtH + 32 * c + 4 * lg) = rh.lo;
          *reinterpret_cast<bf4 *>(rsb + (16 + ls) * kLdtH + 32 * c + 4 * lg) = rl.lo;
        }
        if (2 * c + 1 < CT) {
          *reinterpret_cast<bf4 *>(rsb + ls * kLdtH + 32 * c + 16 + 4 * lg) = rh.hi;
          *reinterpret_cast<bf4 *>(rsb + (16 + ls) * kLdtH + 32 * c + 16 + 4 * lg) = rl.hi;
        }
      }
#pragma unroll
      for (int xt = 0; xt < CT; ++xt) lam[xt] = mfma_bf(as_bf8(o.qh[xt][c]), rh, lam[xt]);
#pragma unroll
      for (int xt = 0; xt < CT; ++xt) lam[xt] = mfma_bf(as_bf8(o.qh[xt][c]), rl, lam[xt]);
#pragma unroll
      for (int xt = 0; xt < CT; ++xt) lam[xt] = mfma_bf(as_bf8(o.ql[xt][c]), rh, lam[xt]);
    }
  } else {
#pragma unroll
    for (int ot = 0; ot < CT; ++ot)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int xt = 0; xt < CT; ++xt)
          lam[xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.tq[xt][ot][r], R[ot][r], lam[xt], 0, 0, 0);
  }
}

// the other operands of a step's gradient terms: T (for G = H o T), the S_x
// and S_o tables and the columns this lane's correlations go to
template <int CT, bool kS> struct GradOps {
  static constexpr int NC = (CT + 1) / 2;
  f4 tr[CT][CT], sx[kS ? 1 : CT], so[kS ? 1 : CT];
  u4v sxb[NC], sob[NC];
  i4v dq;
  __device__ void load(const ChainArgs &a, const ChainStep &st, int lane) {
    load_t<CT>(a.Tr + st.tr_off, lane, tr);
    if constexpr (kS) {
      const u4v *q3 = reinterpret_cast<const u4v *>(a.Ts3 + st.s3_off) + lane + 4 * CT * NC * 64;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        sxb[c] = q3[c * 64];
        sob[c] = q3[(NC + c) * 64];
      }
    } else {
      const f4 *sxo = reinterpret_cast<const f4 *>(a.Tsx + st.sx_off) + lane;
#pragma unroll
      for (int i = 0; i < CT; ++i) {
        sx[i] = sxo[i * 64];
        so[i] = sxo[(CT + i) * 64];
      }
    }
    dq = reinterpret_cast<const i4v *>(a.Tdq + st.dq_off)[lane];
  }
};

// The gradient terms of step st from A_t, R_t and Lambda_t: the W-R
// correlations from p_t = A_t * Lambda_t, then H = sum_s g A R^T, G = H o T
// and Q = S_o^T G^T S_x (the same products as the one-wave walk), stored to
// the sample group's row of partial sums
template <int CT, bool kS>
__device__ inline void grad_terms(const ChainArgs &a, const InstDesc &D, const ChainStep &st,
                                  const GradOps<CT, kS> &go, const float (&As)[CT][4],
                                  const float (&R)[CT][4], const f4 (&lam)[CT], float gs,
                                  const SpinBits &sp, float *prow, float *ga, float *rs,
                                  const __bf16 *rsb, int lane) {
  constexpr int LDT = ldt_of(CT);
  const int ls = lane & 15, lg = lane >> 4;
  if (st.n_wri > 0) {
    float pa[CT][4], pr[4], pt[CT];
#pragma unroll
    for (int xt = 0; xt < CT; ++xt)
#pragma unroll
      for (int r = 0; r < 4; ++r) pa[xt][r] = As[xt][r] * lam[xt][r];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      pr[r] = pa[0][r];
#pragma unroll
      for (int xt = 1; xt < CT; ++xt) pr[r] += pa[xt][r];
    }
#pragma unroll
    for (int xt = 0; xt < CT; ++xt) pt[xt] = (pa[xt][0] + pa[xt][1]) + (pa[xt][2] + pa[xt][3]);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k < st.n_wri) {
        const int j = __builtin_amdgcn_readfirstlane(st.wri[k] & 0xff), wi = st.wri[k] >> 8;
        float m;
        if (j == 0) {
          m = (pr[0] - pr[1]) + (pr[2] - pr[3]);
        } else if (j == 1) {
          m = (pr[0] + pr[1]) - (pr[2] + pr[3]);
        } else if (j < 4) {
          const float tot = (pr[0] + pr[1]) + (pr[2] + pr[3]);
          m = ((lg >> (j - 2)) & 1) ? -tot : tot;
        } else {
          m = 0.f;
#pragma unroll
          for (int xt = 0; xt < CT; ++xt) m += ((xt >> (j - 4)) & 1) ? -pt[xt] : pt[xt];
        }
        m = rows4_sum(m) * gs;
        const float v = row16_sum(m * sp.sigma(wi));
        if (lane == 0) prow[D.nr + st.wre[k]] = v;
      }
  }
#pragma unroll
  for (int xt = 0; xt < CT; ++xt)
    *reinterpret_cast<f4 *>(ga + ls * LDT + 16 * xt + 4 * lg) =
        f4{gs * As[xt][0], gs * As[xt][1], gs * As[xt][2], gs * As[xt][3]};
  if constexpr (!kS) {
#pragma unroll
    for (int ot = 0; ot < CT; ++ot)
      *reinterpret_cast<f4 *>(rs + ls * LDT + 16 * ot + 4 * lg) = f4{R[ot][0], R[ot][1], R[ot][2], R[ot][3]};
  }
  wsync();
  f4 qt[CT];
  if constexpr (kS) {
    bf8 ah1[CT], ah2[CT], rb1[CT], rb2[CT];
#pragma unroll
    for (int xt = 0; xt < CT; ++xt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float va = ga[(4 * lg + j) * LDT + 16 * xt + ls];
        const __bf16 h = (__bf16)va, l = (__bf16)(va - (float)h);
        ah1[xt][j] = h; ah1[xt][4 + j] = l;
        ah2[xt][j] = h; ah2[xt][4 + j] = (__bf16)0.f;
        const __bf16 rh = rsb[(4 * lg + j) * kLdtH + 16 * xt + ls];
        const __bf16 rl = rsb[(16 + 4 * lg + j) * kLdtH + 16 * xt + ls];
        rb1[xt][j] = rh; rb1[xt][4 + j] = rh;
        rb2[xt][j] = rl; rb2[xt][4 + j] = (__bf16)0.f;
      }
#pragma unroll
    for (int ot = 0; ot < CT; ++ot) {
      f4 hg[CT];
#pragma unroll
      for (int xt = 0; xt < CT; ++xt) hg[xt] = mfma_bf(ah1[xt], rb1[ot], f4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int xt = 0; xt < CT; ++xt) hg[xt] = mfma_bf(ah2[xt], rb2[ot], hg[xt]);
      float gv[CT][4];
#pragma unroll
      for (int xt = 0; xt < CT; ++xt)
#pragma unroll
        for (int r = 0; r < 4; ++r) gv[xt][r] = hg[xt][r] * go.tr[ot][xt][r];
      bf8 gh, gl;
      split_chunk<CT>(gv, 0, gh, gl);
      qt[ot] = mfma_bf(gh, as_bf8(go.sxb[0]), f4{0.f, 0.f, 0.f, 0.f});
      qt[ot] = mfma_bf(gl, as_bf8(go.sxb[0]), qt[ot]);
    }
  } else {
#pragma unroll
    for (int ot = 0; ot < CT; ++ot) {
      f4 hg[CT];
#pragma unroll
      for (int xt = 0; xt < CT; ++xt) {
        hg[xt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
          hg[xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              ga[(4 * kc + lg) * LDT + 16 * xt + ls], rs[(4 * kc + lg) * LDT + 16 * ot + ls],
              hg[xt], 0, 0, 0);
      }
      qt[ot] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int xt = 0; xt < CT; ++xt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          qt[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(hg[xt][r] * go.tr[ot][xt][r], go.sx[xt][r],
                                                        qt[ot], 0, 0, 0);
    }
  }
  wsync();
  f4 qq = f4{0.f, 0.f, 0.f, 0.f};
  if constexpr (kS) {
    float qv[CT][4];
#pragma unroll
    for (int ot = 0; ot < CT; ++ot)
#pragma unroll
      for (int r = 0; r < 4; ++r) qv[ot][r] = qt[ot][r];
    bf8 qh, ql;
    split_chunk<CT>(qv, 0, qh, ql);
    qq = mfma_bf(as_bf8(go.sob[0]), qh, qq);
    qq = mfma_bf(as_bf8(go.sob[0]), ql, qq);
  } else {
#pragma unroll
    for (int ot = 0; ot < CT; ++ot)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        qq = __builtin_amdgcn_mfma_f32_16x16x4f32(go.so[ot][r], qt[ot][r], qq, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (go.dq[r] >= 0) prow[go.dq[r]] = qq[r];
}

// one chain task of the split adjoint, common to both roles
struct MeetTask {
  Task tk;
  InstDesc D;
  const ChainStep *cs;
  int T, m;
  f4 *ck;            // the task's checkpoint rows, this lane
  const float *ub;   // the sample's unary factors
  float gs;          // g of the lane's sample (0 past the batch)
  SpinBits sp;
  float *prow;
};
__device__ inline MeetTask meet_task(const ChainArgs &a, int task_id, int lane) {
  MeetTask M;
  const int ls = lane & 15;
  M.tk = task_at(a, task_id);
  M.D = a.inst[M.tk.q];
  const ChainInst C = a.cinst[M.tk.q];
  const ChainDesc cd = a.chains[C.chain_off + M.tk.c];
  M.cs = a.csteps + cd.cs_off;
  M.T = cd.n_steps;
  M.m = (M.T + 1) / 2;
  M.ck = reinterpret_cast<f4 *>(a.ckpt) + (int64_t)task_id * ck_rows(a.lim) * 64 + lane;
  M.ub = phi_base(a, M.tk.q, M.tk.Bq, M.tk.b0 + ls);
  const int64_t left = M.tk.Bq - M.tk.b0;
  const int nvalid = (int)(left < CW ? left : CW);
  M.sp = load_bits(a.spins + a.inst_spin_off[M.tk.q] + (M.tk.b0 + (ls < nvalid ? ls : 0)) * M.D.nw,
                   M.D.nw, ls < nvalid);
  M.gs = ls < nvalid ? (float)a.grad[a.inst_sample_off[M.tk.q] + M.tk.b0 + ls] : 0.f;
  M.prow = a.partial + a.inst_partial_off[M.tk.q] + (M.tk.b0 / CW) * (int64_t)M.D.n_partial;
  return M;
}

// what a role carries from its first phase to its second
template <int CT> struct MeetState {
  float v[CT][4];    // A: the forward state A_m; B: beta_{m-1}
  int esum, elast;   // A: exponent sum of steps < m, e_{m-1}
  float raw;         // A: the closing value when m = T
};

// role A, steps 0 .. m-1 of the forward pass: checkpoints A_t in slots
// t < m, exponents e_t in LDS, out_{m-1} to the exchange slot xa
template <int CT, bool kS>
__device__ inline void meet_fwd1(const ChainArgs &a, const MeetTask &M, int *ex, f4 *xa, int lane,
                                 MeetState<CT> &S) {
  constexpr int GR = GroupMax<CT>::v;
  constexpr int kM = kS ? 2 : 0;
  const int ls = lane & 15, lg = lane >> 4;
  const ChainStep *cs = M.cs;
  const int T = M.T, m = M.m;
  {
    float u[GR];
    load_phi<GR>(M.ub, M.tk.Bq, cs[0].gpos, cs[0].g, u);
    diag_from_phi<CT, GR>(u, cs[0].g, lg, S.v);
  }
  S.esum = 0;
  S.elast = 0;
  S.raw = 1.f;
  auto fstep = [&](int t, const ChainStep &nx, const FwdOps<kM, CT> &oc, const float (&uc)[GR],
                   ChainStep &nn, FwdOps<kM, CT> &on, float (&un)[GR]) -> bool {
#pragma unroll
    for (int i = 0; i < CT; ++i) M.ck[(t * CT + i) * 64] = f4{S.v[i][0], S.v[i][1], S.v[i][2], S.v[i][3]};
    nn = step_at(cs, t + 2 < T ? t + 2 : T - 1);
    on.load(a, nx, lane);
    load_phi<GR>(M.ub, M.tk.Bq, nn.gpos, nn.g, un);
    f4 acc[CT];
    oc.mm(S.v, acc);
    if (t == m - 1) {
#pragma unroll
      for (int i = 0; i < CT; ++i) xa[i * 64] = acc[i];
    }
    if (t == T - 1) {
      S.raw = __shfl(acc[0][0], ls, 64);
      return true;
    }
    float d[CT][4];
    diag_from_phi<CT, GR>(uc, nx.g, lg, d);
    const int e = rescale_next<CT>(acc, d, S.v);
    S.esum += e;
    S.elast = e;
    if (lg == 0) ex[t * CW + ls] = e;
    return t == m - 1;
  };
  ChainStep nA = step_at(cs, T > 1 ? 1 : 0), nB;
  FwdOps<kM, CT> oA, oB;
  float uA[GR], uB[GR];
  oA.load(a, cs[0], lane);
  load_phi<GR>(M.ub, M.tk.Bq, nA.gpos, nA.g, uA);
  for (int t = 0;; t += 2) {
    if (fstep(t, nA, oA, uA, nB, oB, uB)) break;
    if (fstep(t + 1, nB, oB, uB, nA, oA, uA)) break;
  }
}

// role B, the backward vectors of steps T-1 .. m: beta_t to the checkpoint
// slot t, f_{t-1} to LDS, beta_{m-1} kept and written to the exchange slot
template <int CT, bool kS>
__device__ inline void meet_bwd1(const ChainArgs &a, const MeetTask &M, int *fx, f4 *xb, int lane,
                                 MeetState<CT> &S) {
  constexpr int GR = GroupMax<CT>::v;
  const int ls = lane & 15, lg = lane >> 4;
  const ChainStep *cs = M.cs;
  const int T = M.T, m = M.m;
#pragma unroll
  for (int i = 0; i < CT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) S.v[i][r] = 0.f;
  if (lg == 0) S.v[0][0] = 1.f;
  struct Pre {
    LamOps<CT, kS> o;
    float u[GR];
  };
  auto pre = [&](const ChainStep &s, Pre &p) {
    p.o.load(a, s, lane);
    load_phi<GR>(M.ub, M.tk.Bq, s.gpos, s.g, p.u);
  };
  auto bstep = [&](int t, const ChainStep &st, const Pre &cur, ChainStep &sn, Pre &nxt) {
#pragma unroll
    for (int i = 0; i < CT; ++i) M.ck[(t * CT + i) * 64] = f4{S.v[i][0], S.v[i][1], S.v[i][2], S.v[i][3]};
    sn = step_at(cs, t - 1 > m ? t - 1 : m);
    pre(sn, nxt);
    f4 lam[CT];
    lam_mm<CT, kS, false>(cur.o, S.v, nullptr, ls, lg, lam);
    float d[CT][4];
    diag_from_phi<CT, GR>(cur.u, st.g, lg, d);
    float mx = 0.f;
#pragma unroll
    for (int xt = 0; xt < CT; ++xt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        lam[xt][r] *= d[xt][r];
        mx = fmaxf(mx, lam[xt][r]);
      }
    const int f = expo32(rows4_max(mx));
    const float sc = pow2neg(f);
#pragma unroll
    for (int xt = 0; xt < CT; ++xt)
#pragma unroll
      for (int r = 0; r < 4; ++r) S.v[xt][r] = lam[xt][r] * sc;
    if (lg == 0) fx[(t - 1) * CW + ls] = f;
  };
  if (T - 1 >= m) {
    ChainStep sA = step_at(cs, T - 1), sB;
    Pre pA, pB;
    pre(sA, pA);
    for (int t = T - 1;; t -= 2) {
      bstep(t, sA, pA, sB, pB);
      if (t - 1 < m) break;
      bstep(t - 1, sB, pB, sA, pA);
      if (t - 2 < m) break;
    }
  }
#pragma unroll
  for (int i = 0; i < CT; ++i) xb[i * 64] = f4{S.v[i][0], S.v[i][1], S.v[i][2], S.v[i][3]};
}

// K_{m-1} = 1 / (out_{m-1} . beta_{m-1}) from the two exchange slots (the
// same sum in the same order on both roles)
template <int CT>
__device__ inline float meet_k(const f4 *xa, const f4 *xb) {
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < CT; ++i) {
    const f4 p = xa[i * 64], q = xb[i * 64];
#pragma unroll
    for (int r = 0; r < 4; ++r) s += p[r] * q[r];
  }
  s = rows4_sum(s);
  return s > 0.f ? 1.f / s : 0.f;
}

// role A after the meeting: steps m .. T-1 of the forward pass with their
// gradient terms (R_t = K_t beta_t), then the chain's log partial
template <int CT, bool kS>
__device__ inline void meet_fwd2(const ChainArgs &a, const MeetTask &M, const int *fx, float K,
                                 float *ga, float *rs, __bf16 *rsb, int lane, MeetState<CT> &S) {
  constexpr int GR = GroupMax<CT>::v;
  constexpr int kM = kS ? 2 : 0;
  const int ls = lane & 15, lg = lane >> 4;
  const ChainStep *cs = M.cs;
  const int T = M.T, m = M.m;
  if (m < T) {
    K = ldexpf(K, S.elast - fx[(m - 1) * CW + ls]);
    struct Pre {
      FwdOps<kM, CT> f;
      LamOps<CT, kS> o;
      f4 b[CT];
      float u[GR];   // unary factors of step t + 1's group
    };
    auto pre = [&](int t, const ChainStep &s, const ChainStep &s1, Pre &p) {
      p.f.load(a, s, lane);
      p.o.load(a, s, lane);
#pragma unroll
      for (int i = 0; i < CT; ++i) p.b[i] = M.ck[(t * CT + i) * 64];
      load_phi<GR>(M.ub, M.tk.Bq, s1.gpos, s1.g, p.u);
    };
    // step t with its descriptor st, that of step t + 1 (s1) and step t's
    // operands cur; loads step t + 1's operands into nxt
    auto fstep = [&](int t, const ChainStep &st, const ChainStep &s1, const Pre &cur, ChainStep &sn1,
                     Pre &nxt) -> bool {
      const bool last = t == T - 1;
      GradOps<CT, kS> go;
      go.load(a, st, lane);
      sn1 = step_at(cs, t + 2 < T ? t + 2 : T - 1);
      pre(last ? t : t + 1, s1, sn1, nxt);
      f4 acc[CT];
      cur.f.mm(S.v, acc);
      float R[CT][4];
#pragma unroll
      for (int i = 0; i < CT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) R[i][r] = K * cur.b[i][r];
      f4 lam[CT];
      lam_mm<CT, kS, true>(cur.o, R, rsb, ls, lg, lam);
      grad_terms<CT, kS>(a, M.D, st, go, S.v, R, lam, M.gs, M.sp, M.prow, ga, rs, rsb, lane);
      if (last) {
        S.raw = __shfl(acc[0][0], ls, 64);
        return true;
      }
      float d[CT][4];
      diag_from_phi<CT, GR>(cur.u, s1.g, lg, d);
      const int e = rescale_next<CT>(acc, d, S.v);
      S.esum += e;
      K = ldexpf(K, e - fx[t * CW + ls]);
      return false;
    };
    ChainStep sA = step_at(cs, m), sA1 = step_at(cs, m + 1 < T ? m + 1 : T - 1), sB, sB1;
    Pre pA, pB;
    pre(m, sA, sA1, pA);
    for (int t = m;; t += 2) {
      if (fstep(t, sA, sA1, pA, sB1, pB)) break;
      sB = sA1;
      if (fstep(t + 1, sB, sB1, pB, sA1, pA)) break;
      sA = sB1;
    }
  }
  if (lg == 0 && M.tk.b0 + ls < M.tk.Bq)
    a.cpart[a.cpart_off[M.tk.q] + (int64_t)M.tk.c * M.tk.Bq + M.tk.b0 + ls] =
        (double)S.esum * 0.69314718055994530942 + log((double)S.raw);
}

// role B after the meeting: the walk of steps m-1 .. 0 from
// R_{m-1} = K beta_{m-1}, with A's checkpoints and exponents
template <int CT, bool kS>
__device__ inline void meet_bwd2(const ChainArgs &a, const MeetTask &M, const int *ex, float K,
                                 float *ga, float *rs, __bf16 *rsb, int lane, MeetState<CT> &S) {
  constexpr int GR = GroupMax<CT>::v;
  const int ls = lane & 15, lg = lane >> 4;
  const ChainStep *cs = M.cs;
  float R[CT][4];
#pragma unroll
  for (int i = 0; i < CT; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) R[i][r] = K * S.v[i][r];
  struct Pre {
    f4 a[CT];
    LamOps<CT, kS> o;
    float u[GR];
  };
  auto pre = [&](int t, const ChainStep &s, Pre &p) {
#pragma unroll
    for (int i = 0; i < CT; ++i) p.a[i] = M.ck[(t * CT + i) * 64];
    p.o.load(a, s, lane);
    load_phi<GR>(M.ub, M.tk.Bq, s.gpos, s.g, p.u);
  };
  auto walk = [&](int t, const ChainStep &st, const Pre &cur, ChainStep &sn, Pre &nxt) {
    GradOps<CT, kS> go;
    go.load(a, st, lane);
    sn = step_at(cs, t > 0 ? t - 1 : 0);
    pre(t > 0 ? t - 1 : 0, sn, nxt);
    float As[CT][4];
#pragma unroll
    for (int i = 0; i < CT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) As[i][r] = cur.a[i][r];
    f4 lam[CT];
    lam_mm<CT, kS, true>(cur.o, R, rsb, ls, lg, lam);
    grad_terms<CT, kS>(a, M.D, st, go, As, R, lam, M.gs, M.sp, M.prow, ga, rs, rsb, lane);
    float d[CT][4];
    diag_from_phi<CT, GR>(cur.u, st.g, lg, d);
    const float sc = pow2neg(ex[(t > 0 ? t - 1 : 0) * CW + ls]);
#pragma unroll
    for (int xt = 0; xt < CT; ++xt)
#pragma unroll
      for (int r = 0; r < 4; ++r) R[xt][r] = d[xt][r] * lam[xt][r] * sc;
  };
  const int m = M.m;
  ChainStep sA = step_at(cs, m - 1), sB;
  Pre pA, pB;
  pre(m - 1, sA, pA);
  for (int t = m - 1; t >= 0; t -= 2) {
    walk(t, sA, pA, sB, pB);
    if (t == 0) break;
    walk(t - 1, sB, pB, sA, pA);
  }
}

template <int CT, bool kS>
__device__ inline void meet_phase(const ChainArgs &a, const MeetTask &M, int role, int phase,
                                  const RL &L, char *bA, char *bB, int lane, MeetState<CT> &S) {
  int *ex = reinterpret_cast<int *>(bA + L.ex);
  int *fx = reinterpret_cast<int *>(bB + L.fx);
  f4 *xa = reinterpret_cast<f4 *>(bA + L.xa) + lane;
  f4 *xb = reinterpret_cast<f4 *>(bB + L.xb) + lane;
  char *own = role == 0 ? bA : bB;
  float *ga = reinterpret_cast<float *>(own + L.ga);
  float *rs = reinterpret_cast<float *>(own + L.rs);
  __bf16 *rsb = reinterpret_cast<__bf16 *>(own + L.rs);
  if (phase == 0) {
    if (role == 0) meet_fwd1<CT, kS>(a, M, ex, xa, lane, S);
    else meet_bwd1<CT, kS>(a, M, fx, xb, lane, S);
  } else {
    const float K = meet_k<CT>(xa, xb);
    if (role == 0) {
      meet_fwd2<CT, kS>(a, M, fx, K, ga, rs, rsb, lane, S);
    } else {
      // beta_{m-1} from its exchange slot (the value role B left there)
#pragma unroll
      for (int i = 0; i < CT; ++i) {
        const f4 v = xb[i * 64];
#pragma unroll
        for (int r = 0; r < 4; ++r) S.v[i][r] = v[r];
      }
      meet_bwd2<CT, kS>(a, M, ex, K, ga, rs, rsb, lane, S);
    }
  }
}

// the split adjoint of one-tile chains: two waves per task, roles A (even
// wave) and B (odd wave), one barrier between the phases (every wave of the
// workgroup reaches it, with a task or not)
template <bool kS>
__global__ __launch_bounds__(256, 3) void rchain_meet_kernel(ChainArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int pair = wave >> 1, role = wave & 1;
  const int task = a.task_base + blockIdx.x * 2 + pair;
  const bool has = task < a.task_base + a.n_tasks;
  const RL L = rlayout(a.lim, true, 1, true);
  char *bA = smem + (size_t)(2 * pair) * L.end, *bB = bA + L.end;
  MeetTask M;
  MeetState<1> S;
  if (has) {
    M = meet_task(a, task, lane);
    meet_phase<1, kS>(a, M, role, 0, L, bA, bB, lane, S);
  }
  __syncthreads();
  if (has) meet_phase<1, kS>(a, M, role, 1, L, bA, bB, lane, S);
}

template <int CT, bool kS, bool kK>
__global__ __launch_bounds__(256, 3) void rchain_bwd_kernel(ChainArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const Task tk = wave_task(a, wave);
  if (tk.q < 0) return;
  const InstDesc D = a.inst[tk.q];
  const ChainInst C = a.cinst[tk.q];
  const ChainDesc cd = a.chains[C.chain_off + tk.c];
  const RL L = rlayout(a.lim, true, 1);
  char *base = smem + (size_t)wave * L.end;
  bwd_chain<CT, kS, kK>(a, tk, D, cd, base, L, lane, a.task_base + blockIdx.x * kWaves + wave);
}

// Persistent forward over every chain width (SG groups per wave on 1-2
// tile chains, one on 4-tile chains)
template <int kM, int SG>
__global__ __launch_bounds__(256) void rchain_fwd_pq_kernel(ChainArgs a) {
  const int lane = threadIdx.x & 63;
  int task = 0, gi = 0;
  while (pq_task(a, lane, task, gi)) {
    const Task tk = task_at(a, task);
    const ChainInst C = a.cinst[tk.q];
    const ChainDesc cd = a.chains[C.chain_off + tk.c];
    if (gi == 0) fwd_chain<kM, 1, SG>(a, tk, cd, lane);
    else if (gi == 1) fwd_chain<kM, 2, SG>(a, tk, cd, lane);
    else fwd_chain<kM, 4, 1>(a, tk, cd, lane);
  }
  pq_exit(a, lane);
}

// Persistent adjoint over both chain widths
template <bool kS, bool kK>
__global__ __launch_bounds__(256, 3) void rchain_bwd_pq_kernel(ChainArgs a) {
  extern __shared__ __align__(16) char smem[];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const RL L = rlayout(a.lim, true, 1, true);
  char *base = smem + (size_t)wave * L.end;
  int task = 0, gi = 0;
  while (pq_task(a, lane, task, gi)) {
    if (gi == 0) {
      // the split adjoint's four phases in turn on this wave
      // (role B's state between its phases is beta_{m-1}, which its
      // exchange slot holds)
      const MeetTask M = meet_task(a, task, lane);
      MeetState<1> SA;
      meet_phase<1, kS>(a, M, 0, 0, L, base, base, lane, SA);
      wsync();
      {
        MeetState<1> SB;
        meet_phase<1, kS>(a, M, 1, 0, L, base, base, lane, SB);
      }
      wsync();
      meet_phase<1, kS>(a, M, 0, 1, L, base, base, lane, SA);
      wsync();
      {
        MeetState<1> SB;
        meet_phase<1, kS>(a, M, 1, 1, L, base, base, lane, SB);
      }
    } else {
      const Task tk = task_at(a, task);
      const InstDesc D = a.inst[tk.q];
      const ChainInst C = a.cinst[tk.q];
      const ChainDesc cd = a.chains[C.chain_off + tk.c];
      bwd_chain<2, kS, kK>(a, tk, D, cd, base, L, lane, task);
    }
    wsync();
  }
  pq_exit(a, lane);
}

}  // namespace

size_t rchain_wave_lds(const ChainLim &L, bool bwd, int sg) { return rlayout(L, bwd, sg, bwd).end; }

hipError_t launch_rchain_pq(const ChainArgs &a, bool bwd, hipStream_t st) {
  const int total = a.pq_n[0] + a.pq_n[1] + a.pq_n[2];
  if (total <= 0) return hipSuccess;
  const bool sp = a.split != 0 && !a.bf16;
  const int sg = bwd ? 1 : (a.sg >= 2 ? 2 : 1);
  void (*k)(ChainArgs) = nullptr;
  if (bwd) {
    if (a.pq_n[2] > 0) return hipErrorInvalidValue;   // the adjoint takes chains of <= 2 tiles
    const bool kk = rk_of(a.lim) > 1;
    k = sp ? (kk ? rchain_bwd_pq_kernel<true, true> : rchain_bwd_pq_kernel<true, false>)
           : (kk ? rchain_bwd_pq_kernel<false, true> : rchain_bwd_pq_kernel<false, false>);
  } else {
    const int m = a.bf16 ? 1 : sp ? 2 : 0;
    if (m == 0) k = sg >= 2 ? rchain_fwd_pq_kernel<0, 2> : rchain_fwd_pq_kernel<0, 1>;
    else if (m == 1) k = sg >= 2 ? rchain_fwd_pq_kernel<1, 2> : rchain_fwd_pq_kernel<1, 1>;
    else k = sg >= 2 ? rchain_fwd_pq_kernel<2, 2> : rchain_fwd_pq_kernel<2, 1>;
  }
  const size_t lds = (size_t)kWaves * rlayout(a.lim, bwd, sg, bwd).end;
  hipError_t e;
  if (lds > 65536 && (e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                              hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)lds)) != hipSuccess)
    return e;
  int dev = 0, cus = 0, per = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess ||
      (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
      (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(k),
                                                        64 * kWaves, lds)) != hipSuccess)
    return e;
  const int grid = std::max(1, std::min((total + kWaves - 1) / kWaves, cus * std::max(per, 1)));
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * kWaves), lds, st, a);
  return hipGetLastError();
}

int64_t rchain_ckpt_floats(const ChainLim &L) { return ck_rows(L) * 64 * 4; }

hipError_t launch_rchain_moments(const ChainArgs &a, hipStream_t st) {
  if (a.n_tasks <= 0) return hipSuccess;
  void (*k)(ChainArgs) = a.ntm == 1 ? rchain_mom_kernel<1> : a.ntm == 2 ? rchain_mom_kernel<2> : nullptr;
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3((a.n_tasks + kWaves - 1) / kWaves), dim3(64 * kWaves), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_chain_mom_sum(const ChainInst *cinst, const int32_t *chain_insts,
                                int n_chain_insts, const int64_t *inst_B,
                                const int64_t *inst_sample_off, const int64_t *cpart_off,
                                const double *mpart, int64_t mtot, double *mean, double *var,
                                hipStream_t st) {
  if (n_chain_insts <= 0) return hipSuccess;
  hipLaunchKernelGGL(chain_mom_sum_kernel, dim3(32, n_chain_insts), dim3(256), 0, st, cinst,
                     chain_insts, inst_B, inst_sample_off, cpart_off, mpart, mtot, mean, var);
  return hipGetLastError();
}

// one launch per chain width: tasks [task_base, task_base + n_tasks) all
// belong to chains of a.ntm tiles
hipError_t launch_rchain(const ChainArgs &a, bool bwd, hipStream_t st) {
  if (a.n_tasks <= 0) return hipSuccess;
  const int sg = bwd ? 1 : (a.sg >= 2 ? 2 : 1);
  void (*k)(ChainArgs) = nullptr;
  const int ct = a.ntm;
  const bool sp = a.split != 0 && !a.bf16;
  if (bwd && ct == 1) {
    // one-tile chains: the split adjoint, two waves per task (every step's
    // vector kept, whatever the checkpoint interval)
    k = sp ? rchain_meet_kernel<true> : rchain_meet_kernel<false>;
    const size_t lds = (size_t)kWaves * rlayout(a.lim, true, 1, true).end;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k, dim3((a.n_tasks + 1) / 2), dim3(64 * kWaves), lds, st, a);
    return hipGetLastError();
  }
  if (bwd) {
    const bool kk = rk_of(a.lim) > 1;
    if (ct == 2)
      k = sp ? (kk ? rchain_bwd_kernel<2, true, true> : rchain_bwd_kernel<2, true, false>)
             : (kk ? rchain_bwd_kernel<2, false, true> : rchain_bwd_kernel<2, false, false>);
  } else if (a.bf16) {
    if (ct == 1) k = sg >= 2 ? rchain_fwd_kernel<1, 1, 2> : rchain_fwd_kernel<1, 1, 1>;
    else if (ct == 2) k = sg >= 2 ? rchain_fwd_kernel<1, 2, 2> : rchain_fwd_kernel<1, 2, 1>;
    else if (ct == 4) k = rchain_fwd_kernel<1, 4, 1>;
  } else if (sp) {
    if (ct == 1) k = sg >= 2 ? rchain_fwd_kernel<2, 1, 2> : rchain_fwd_kernel<2, 1, 1>;
    else if (ct == 2) k = sg >= 2 ? rchain_fwd_kernel<2, 2, 2> : rchain_fwd_kernel<2, 2, 1>;
    else if (ct == 4) k = rchain_fwd_kernel<2, 4, 1>;
  } else {
    if (ct == 1) k = sg >= 2 ? rchain_fwd_kernel<0, 1, 2> : rchain_fwd_kernel<0, 1, 1>;
    else if (ct == 2) k = sg >= 2 ? rchain_fwd_kernel<0, 2, 2> : rchain_fwd_kernel<0, 2, 1>;
    else if (ct == 4) k = rchain_fwd_kernel<0, 4, 1>;
  }
  if (!k) return hipErrorInvalidValue;
  const int sgl = (!bwd && ct == 4) ? 1 : sg;
  if (sgl != sg) return hipErrorInvalidValue;   // the task list was cut for sg samples
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
