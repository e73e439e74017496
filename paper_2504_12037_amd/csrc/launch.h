// Internal launch interface between the C ABI (api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/tnvan.h"
#include "program.h"

namespace tnvan {

// Device copies of the compiled program (one set per precision of T).
template <typename real>
struct ContractArgs {
  const InstDesc *inst;
  const StepDesc *steps;
  const InputDesc *inputs;
  const uint16_t *gtab;             // gather tables of SINGLE steps' inputs
  const uint32_t *gtab2;            // split gather tables of wide steps' inputs
  const EdgeDesc *edges;
  const real *esmall;               // per edge: exp(-2 beta |J|), negated for J < 0
  const real *T;
  const int32_t *fld_ptr;
  const int32_t *fld_w;
  const real *fld_J;
  const real *hR;
  const int32_t *wr_pos;
  const int32_t *wr_w;
  // tiles of samples: tile -> instance and first local sample
  const int32_t *tile_inst;
  const int32_t *tile_start;
  const int32_t *inst_first_tile;
  const int64_t *inst_sample_off;   // first global sample of each instance
  const int64_t *inst_B;            // samples of each instance
  const int64_t *inst_spin_off;     // first spin of each instance
  const int64_t *inst_partial_off;  // first partial entry of each instance
  const int8_t *spins;
  double *logz;                     // forward output
  const double *grad;               // backward input (upstream gradient)
  real *partial;                    // backward per-tile partial sums
  real *garena;                     // arena in global memory (or null)
  int64_t garena_stride;            // entries per tile
  int32_t S, logS;                  // samples per tile (power of two <= 64)
  int32_t *pq;                      // persistent form: tile counter and exit count (zero between launches)
  int32_t arena_per_block;          // device arena per resident workgroup (persistent), not per tile
  int32_t wide;                     // some instance has wide steps (their kernel variant)
};

struct LdsPlan {
  size_t bytes;          // dynamic LDS per workgroup
  bool global_arena;     // arena and scratch live in global memory
};

// Bytes of LDS one tile of S samples of instance D needs.
size_t contract_lds_bytes(const InstDesc &D, int S, bool bwd, bool global_arena,
                          int real_size);
// Global arena entries per tile (per sample entries times S).
int64_t contract_garena_entries(const InstDesc &D, int S, bool bwd);

// persistent: one workgroup per resident slot, tiles taken from a.pq in
// order (else one workgroup per tile)
// persistent with max_grid > 0: at most that many workgroups (each with its
// own arena when a.arena_per_block)
template <typename real>
hipError_t launch_contract(const ContractArgs<real> &a, int n_tiles, size_t lds,
                           bool bwd, bool global_arena, hipStream_t st, bool persistent = false,
                           int max_grid = 0);

// Sum per-tile partials and scatter dh, dJ, dbeta (FP64).
struct VjpArgs {
  const InstDesc *inst;
  const int32_t *rr_edge;
  const double *rr_J;
  const int32_t *wr_edge;
  const double *wr_J;
  const double *hR;
  const int32_t *vr;
  const int32_t *inst_first_tile;
  const int32_t *inst_n_tiles;
  const int64_t *inst_partial_off;
  const int64_t *inst_spin_base;   // offset of instance i in dh (sum of n)
  const int64_t *inst_edge_base;   // offset of instance i in dJ
  const int64_t *inst_sum_off;     // offset of instance i in col_out
  double *dh, *dJ, *dbeta;
  // split column sums in output order [n_inst][vjp_split()][maxo]; an
  // output without a column keeps the zero the buffer starts with
  double *part2;
  int32_t maxo;                    // largest n_spins + n_edges
  const int32_t *col_out;          // partial column -> output (vertex, or n + edge)
  const double *pcoef_out;         // per output: dbeta coefficient of its column, or 0
};
int vjp_split();
template <typename real>
hipError_t launch_vjp_reduce(const VjpArgs &a, const real *partial, int n_inst, int max_partial,
                             hipStream_t st);

// ---------------------------------------------------------------- network
struct MadeInst {
  int32_t n, H;             // |W|, hidden width
  int32_t L;                // lanes per sample in the sampler
  int32_t D;                // hidden layers (1 when H = 0)
  int64_t param_off;        // offset of the instance's parameters
  int64_t pack_off;         // offset of its matrix-core sampler tables
  int64_t sample_off;       // first global sample
  int64_t B;                // samples
  int64_t spin_off;         // first spin
};

template <typename real>
struct SampleArgs {
  const MadeInst *mi;
  const float *params;
  const float *uniforms;        // null => Philox
  const int32_t *blk_inst;      // block -> instance
  const int32_t *blk_start;     // block -> first local sample
  int8_t *spins;
  real *logq;
  uint64_t seed;
  const int32_t *step_ctr;      // per instance (device), Philox counter word 2
  int32_t spb;                  // samples per round of a block (256 / L)
  int32_t reps;                 // rounds per block
  const float *w0t;             // one-layer sampler: columns of W0 (w0t_kernel)
  const int64_t *w0t_off;       // per instance, floats
  real *sig;                    // one-layer sampler: q(s_i = +1 | s_<i) in the
                                // spins' layout, or null
};
// stage_bytes: LDS for the parameters (0 or too large: read them from HBM)
template <typename real>
hipError_t launch_sample(const SampleArgs<real> &a, int n_blocks, size_t stage_bytes,
                         hipStream_t st);
// One-layer nets (every instance H = 0, |W| <= kH0MaxN): one wave per
// sample, W0's columns from w0t (written by launch_w0t from the parameters;
// w0t_off[q] is instance q's offset, n_q^2 floats each).
constexpr int kH0MaxN = 512;
hipError_t launch_w0t(const MadeInst *mi, int n_inst, int max_n, const float *params,
                      const int64_t *w0t_off, float *w0t, hipStream_t st);
template <typename real>
hipError_t launch_sample_h0(const SampleArgs<real> &a, int n_inst, int64_t max_B, int max_n,
                            hipStream_t st);
size_t made_param_bytes(int n, int H);
// the largest parameter set the general sampler stages in LDS
size_t made_stage_max();

// Deeper networks (some instance with D > 1 hidden layers): one wave per
// sample for every instance, a lane owning hidden units lane + 64 kk and
// positions lane + 64 jj; the completed tanh values of each layer in LDS.
// small (every instance |W| <= kDeep16MaxN and H <= kDeep16MaxH): 16 lanes
// per sample instead, four samples per wave.
constexpr int kDeepMaxN = 256, kDeepMaxH = 256, kDeepMaxD = 4;
constexpr int kDeep16MaxN = 128, kDeep16MaxH = 64;
template <typename real>
hipError_t launch_sample_deep(const SampleArgs<real> &a, int n_inst, int64_t max_B, bool small,
                              hipStream_t st);

// Matrix-core sampler (FP32): one wave per 16 samples of one instance.
// Needs n <= 64 and at most 15 hidden units per degree (H <= 15 (n - 1)).
struct MSampleArgs {
  const MadeInst *mi;
  const float *pack;            // repacked parameters (made_pack_kernel)
  const int32_t *task_inst;     // per wave
  const int32_t *task_start;    // first local sample of the wave
  int32_t n_tasks;
  const float *uniforms;        // null => Philox
  int8_t *spins;
  float *logq;
  uint64_t seed;
  const int32_t *step_ctr;
};
// Fused REINFORCE backward (FP32): one workgroup per 64 samples of one
// instance writes a masked partial gradient row; rows are then summed per
// instance in a fixed order into grad.  Needs n <= 64 and H <= 256.
struct MGradArgs {
  const MadeInst *mi;
  int32_t n_inst, hmax;
  const float *params;
  const int8_t *spins;          // all instances
  const double *f;              // f_b per global sample
  const double *fpart;          // free-energy block sums [n_inst][4][fnblk]
  int32_t fnblk;
  double *stats;                // out [n_inst][4] (free_stats), by the first workgroup
  const int32_t *task_inst;     // per workgroup
  const int32_t *task_start;    // first local sample (multiple of 64)
  int32_t n_tasks;
  float *part;                  // [n_tasks][pstride]
  int64_t pstride;
  const int32_t *first_row, *n_rows;   // per instance: its workgroup rows
  const float *pack;            // made_pack_kernel output (holds the masked W2^T)
  float *grad;                  // flat parameter gradient
  int32_t split;                // products as split-BF16 (mgrad3_kernel)
};
size_t mgrad_lds_bytes(int H, int npt, bool split);
int mgrad_task_samples(bool split);   // samples per workgroup of the fused backward
hipError_t launch_mgrad(const MGradArgs &a, int npt, hipStream_t st);
struct OptArgs;
// the REINFORCE gradient (the fixed-order sum of each instance's workgroup
// rows) and the Adam step in one launch (grad_adam_kernel)
hipError_t launch_grad_adam(const MGradArgs &g, const OptArgs &o, int64_t max_pc, hipStream_t st);
int64_t made_pack_floats(int n, int npt, int H);
hipError_t launch_made_pack(const MadeInst *mi, int n_inst, int64_t max_floats, const float *params,
                            float *pack, int npt, hipStream_t st);
hipError_t launch_msample(const MSampleArgs &a, int npt, hipStream_t st);

// Per-sample rows of the log-prob pass and the REINFORCE backward.
template <typename real>
struct RowArgs {
  MadeInst mi;
  const float *params;
  const int8_t *spins;     // the instance's spins [B, n]
  const double *f;         // f_b per sample (global index)
  const double *stats;     // the instance's F_q (stats[0])
  int64_t chunk;           // samples per block
  real *hid;               // [B, H]
  real *da;                // [B, H]
  real *dlogit;            // [B, n]
  real *sf;                // [B, n] spins as real
  const real *sig;         // one-layer nets: the sampler's conditionals [B, n]
};
// The rows of every instance in one launch: job j is one instance with its
// chunk (samples per block) and its slices of the row buffers, and owns the
// blocks [lo[j], lo[j + 1]).  `staged`: parameters staged in LDS; `threads`
// per block, a multiple of 64 up to 1024.
struct RowJob {
  int32_t q, chunk;
  int64_t hoff, doff;      // offsets into hid / da and into dlogit / sf
};
template <typename real>
struct RowBatch {
  const MadeInst *mi;      // device, per instance
  const float *params;
  const int8_t *spins;     // every instance's spins (instance q at mi[q].spin_off)
  const double *f;         // f_b per sample (global index)
  const double *stats;     // [n_inst][4], F_q at [4 q]
  const RowJob *jobs;
  const int32_t *lo;       // [n_jobs + 1]
  int32_t n_jobs, blocks;
  real *hid, *da, *dlogit, *sf;
};
template <typename real>
hipError_t launch_rows_batch(const RowBatch<real> &a, bool staged, size_t lds_bytes,
                             int threads, hipStream_t st);
// LDS bytes of one block of the batched rows for an (n, H) instance
size_t rows_lds_bytes(int n, int H, size_t real_bytes, bool staged);
// deeper networks: hid and da hold every layer, [B, D * H] (layer-major
// inside a row); rb samples per block round
template <typename real>
hipError_t launch_rows_deep(const RowArgs<real> &a, int rb, hipStream_t st);
// one-layer nets: the rows from the conditionals the sampler stored
template <typename real>
hipError_t launch_rows_h0(const RowArgs<real> &a, hipStream_t st);

// The batch sums of a whole REINFORCE backward, every instance and matrix in
// one launch per kind.  An AtbJob is out[M, N] = mask * X^T Y over the batch
// (X [B, ldx] and Y [B, ldy] at their column offsets), summed in ks batch
// slices whose partial sums sit at part + part_off, then added in slice
// order; a ColJob is the column sums of X the same way.  Mask kinds: 0 none,
// 1 W2, 2 W0, 3 W1, 4 the deeper layers (the autoregressive masks of Eq. 7).
// The lo / flo arrays: the jobs' first blocks in each kernel (prefix sums,
// one more entry than jobs).
template <typename real>
struct AtbJob {
  const real *X, *Y;
  float *out;
  int64_t part_off, B;
  int32_t ldx, ldy, M, N, ks, ldo, mask, nW;
};
template <typename real>
struct ColJob {
  const real *X;
  float *out;
  int64_t part_off, B;
  int32_t ldx, M, ks, pad;
};
template <typename real>
struct BatchSums {
  const AtbJob<real> *atb;
  const int32_t *atb_lo, *atb_flo;   // atb blocks, finish blocks
  int32_t n_atb;
  const ColJob<real> *col;
  const int32_t *col_lo, *col_flo;
  int32_t n_col;
  int32_t atb_blocks, atb_fblocks, col_blocks, col_fblocks;
  real *part;
};
template <typename real>
hipError_t launch_batch_sums(const BatchSums<real> &a, hipStream_t st);
// blocks of one job: (atb, atb finish, colsum, colsum finish)
void batch_sum_blocks(int M, int N, int ks, int32_t *atb, int32_t *fin);
void batch_col_blocks(int M, int ks, int32_t *col, int32_t *fin);

// Free energy statistics of every instance of the batch.
template <typename real>
struct FreeArgs {
  const InstDesc *inst;
  const MadeInst *mi;
  const int32_t *hw_off;     // per instance offset into hW
  const int8_t *spins;
  const double *logz;
  // logZ from the chain partials instead (when cpart is set): log_const plus
  // the instance's per-chain partials in chain order, then its unary sums,
  // as launch_chain_sum
  const ChainInst *cinst;
  const int64_t *cpart_off;
  const double *cpart;
  const int64_t *f_off;
  const double *fabp;
  const real *logq;
  const int32_t *ww_a, *ww_b;
  const double *ww_J;
  const double *hW;
  double *f;                 // out [sum B]
  double *part;              // block sums [n_inst][4][nblk]
  int32_t nblk;
  int32_t finish;            // form stats here (else the fused backward does)
  double *stats;             // out [n_inst][4]
  int32_t *done;             // [n_inst] completion tickets, zero between launches
  int32_t *step_ctr;         // advanced by one per instance, or null
  int32_t *nonfinite;        // [n_inst] set to 1 where some f_b is not finite, or null
};
template <typename real>
hipError_t launch_free(const FreeArgs<real> &a, int n_inst, hipStream_t st);

// E_1(s_W) per sample (Eq. 4: the couplings and fields inside the width set)
// in FP64, every instance in one launch (grid.y = instance); the W-W terms in
// edge order, then the fields in width-set order.
struct E1Args {
  const InstDesc *inst;
  const MadeInst *mi;          // per-call B, sample_off and spin_off
  const int32_t *hw_off;
  const int8_t *spins;
  const int32_t *ww_a, *ww_b;
  const double *ww_J;
  const double *hW;
  double *e1;                  // out [sum B]
};
hipError_t launch_e1(const E1Args &a, int n_inst, int64_t max_B, hipStream_t st);

// Conditional mean and variance of the remainder's magnetisation given s_W
// (moments.hip): a second-order Taylor (jet) contraction of every
// instance's general step program in a uniform field on R, one thread per
// sample.  Programs with wide steps are not supported.
template <typename real>
struct MomentArgs {
  const InstDesc *inst;
  const StepDesc *steps;
  const InputDesc *inputs;
  const uint16_t *gtab;
  const real *T;
  const int32_t *fld_ptr, *fld_w;
  const real *fld_J;
  const real *hR;
  const int64_t *inst_sample_off, *inst_B, *inst_spin_off;
  const int8_t *spins;
  real *jarena;               // per instance (arena_fwd + scr_fwd) * 3 * B jets
  int32_t *jexp;              // per instance n_steps * B step exponents
  const int64_t *jar_off, *jexp_off;
  double *logz;               // out [sum B] or null
  double *mean, *var;         // out [sum B]
  const int32_t *skip;        // per instance: 1 where the chain kernels wrote it, or null
};
template <typename real>
hipError_t launch_moments(const MomentArgs<real> &a, int n_inst, int64_t max_B, hipStream_t st);

// Importance-weighted magnetisation moments of p per instance (moments.hip):
// out[q] = (<M>/N, <M^2>/N^2, beta N (<M^2>/N^2 - (<M>/N)^2), ess)
struct SusArgs {
  const InstDesc *inst;
  const int64_t *inst_sample_off, *inst_B, *inst_spin_off;
  const int8_t *spins;
  const double *g;            // w_b / beta (obs_weights_kernel)
  const double *ess;          // [n_inst]
  const double *mean, *var;   // conditional moments of M_R per sample
  double *out;                // [n_inst][4]
};
hipError_t launch_sus_reduce(const SusArgs &a, int n_inst, hipStream_t st);

// Exact slicing over every configuration of one instance's width set
// (slice_*_kernel): the configurations of one pass as spins, the per-block
// log-sum-exp pairs of -beta E_1 + logZ_R, and their fixed-order merge.
constexpr int kSliceBlocks = 64;   // blocks (and pairs) per pass
struct SliceArgs {
  const InstDesc *inst;
  int32_t q;                 // the instance
  const int32_t *ww_a, *ww_b;
  const double *ww_J;
  const double *hW;
  const int32_t *hw_off;
  const double *logz;        // logZ_R of the pass's configurations
  int64_t c0, n;             // first configuration of the pass, configurations
  int64_t pass;
  double *part;              // [passes][kSliceBlocks][2] (max, scaled sum)
};
hipError_t launch_slice_spins(int8_t *spins, int nw, int64_t c0, int64_t n, hipStream_t st);
hipError_t launch_slice_lse(const SliceArgs &a, hipStream_t st);
hipError_t launch_slice_final(const double *part, int64_t count, double beta, double *out,
                              hipStream_t st);

// Moments of the Boltzmann distribution from samples of q (obs_*_kernel):
// self-normalised importance weights exp(-beta f_b) / sum per instance, and
// the width-set moments (W magnetisations, W-W correlations) they weight.
struct ObsArgs {
  const InstDesc *inst;
  const MadeInst *mi;        // sample_off, B, spin_off, n (= |W|)
  const double *f;           // f_b per global sample (free_f_kernel)
  double *g;                 // out: w_b / beta per global sample
  double *ess;               // out [n_inst]: effective sample size 1 / sum w^2
  const int8_t *spins;
  const int32_t *ww_a, *ww_b, *ww_e;
  const int32_t *wv, *hw_off;   // W index -> vertex, per instance offset
  const int64_t *spin_base, *edge_base;   // per instance offsets of mag / corr
  double *mag, *corr;
  int32_t max_out;           // largest |W| + W-W edge count
};
hipError_t launch_obs_weights(const ObsArgs &a, int n_inst, hipStream_t st);
hipError_t launch_obs_w(const ObsArgs &a, int n_inst, hipStream_t st);

// One optimiser step of every instance (see adam_step_kernel).
struct OptArgs {
  const MadeInst *mi;
  float *params, *grad, *m, *v;
  float *pack;               // packed operand tables kept current, or null
  int32_t npt;               // position tiles of the packed tables
  float lr;
  const int32_t *step_ctr;   // already counting this step
};
hipError_t launch_adam_step(const OptArgs &a, int n_inst, int64_t max_pc, hipStream_t st);

// The net's signature for the autotuner's cache (precision, product form,
// kernels, widest message scope, instance count), its instance count, and
// the thread-local error message of the C ABI.
tnvan_status net_signature(const tnvan_net *net, std::string &out);
int net_instances(const tnvan_net *net);
void set_last_error(const char *msg);

}  // namespace tnvan

namespace tnvan {

// Transfer-matrix (chain) kernels: a workgroup takes one chain of one
// instance and wpb groups of 16 samples (one per wave).
struct ChainLim {             // launch-wide maxima that size the LDS layout
  int32_t kbuf, npos_max, max_steps, pmax, nw;
  int32_t tl_max, tbl_max, ne_max, nf_max;
  int32_t kseg;               // checkpoint interval of the adjoint
  int32_t wpb;                // waves per workgroup
  int32_t tlds;               // transfer tables staged in LDS
  int32_t rk;                 // register-resident adjoint: checkpoint every rk steps (1, 2, 4, 8)
};
struct ChainArgs {
  const InstDesc *inst;
  const ChainInst *cinst;
  const ChainDesc *chains;
  const ChainStep *csteps;
  const float *Tp, *Tt;       // per-step padded tables (HBM)
  const uint16_t *Tb;
  const float *Tl;            // per-chain staged blocks (HBM source)
  const uint16_t *Tbl;
  const EdgeDesc *cedges;
  const int32_t *fld_ptr, *fld_w, *fld_wr;
  const float *fld_J, *hR;
  const int32_t *task_inst, *task_chain, *task_start;   // per workgroup
  int32_t n_tasks;
  ChainLim lim;
  const int64_t *inst_B, *inst_sample_off, *inst_spin_off;
  const int64_t *cpart_off;         // per instance: chain-partial logZ offset
  const int8_t *spins;
  double *cpart;                    // [chain][B] per instance
  const double *grad;
  float *partial;                   // adjoint partial rows
  const int64_t *inst_partial_off;
  float *ckpt;                      // adjoint checkpoints, per wave
  int32_t bf16;
  int32_t ntm;                      // largest K or N of the launch in 16-wide tiles
  // register-resident kernels: per-wave tasks, permuted tables
  const float *Tr, *Tq;
  const uint16_t *Trb;
  const int32_t *xcol;
  const float *Tsx;                 // adjoint S_x / S_o operand tables
  const int32_t *Tdq;               // adjoint destinations (ChainStep::dq_off)
  const uint16_t *Ts3;              // split-BF16 operand tables (ChainStep::s3_off)
  int32_t split;                    // FP32 path with split-BF16 products
  int32_t sg;                       // 16-sample groups per wave (forward)
  int32_t task_base;                // first task of the launch
  // dense W-neighbour slots of every R position (index hr_off + position)
  const int32_t *cf_w, *cf_r;       // [4] per position: W index, W-R edge (-1: unused)
  const float *cf_J;                // [4] per position
  // unary factors of every (R position, sample), position-major per
  // instance: +-exp(-2 beta |f|), negative when f < 0 (unary_kernel)
  const float *U;
  const int64_t *u_off;             // per instance
  // unary_kernel writes every factor, also the +1 of positions with no
  // W-neighbour and no field (else those keep the +1 the table was filled
  // with when its layout was set)
  int32_t u_all;
  // persistent form of the register-resident kernels: task counter and exit
  // count (zero between launches), and the task range of each width (1, 2,
  // 4 tiles), taken widest first
  int32_t *pq;
  int32_t pq_lo[3], pq_n[3];
  // magnetisation moments launch: per chain and sample, the remainder's
  // conditional mean of M at the chain-partial index and its variance at
  // mtot plus that index
  double *mpart;
  int64_t mtot;
};
// U and the per-sample sums of beta |f| over each run of kUnaryChunk
// positions (fabp[f_off[q] + chunk * B + b]) of the instances in cis.
constexpr int kUnaryChunk = 16;
hipError_t launch_unary(const ChainArgs &a, const int32_t *cis, int n_cis, int max_chunks,
                        int64_t max_B, const int64_t *f_off, float *U, double *fabp,
                        hipStream_t st);
// LDS bytes: shared part of a workgroup and per-wave part
size_t chain_shared_lds(const ChainLim &L, bool bwd, bool bf16);
size_t chain_wave_lds(const ChainLim &L, bool bwd);
int chain_kseg(const ChainInst &C);
hipError_t launch_chain(const ChainArgs &a, bool bwd, hipStream_t st);
// Register-resident chain kernels: one task (instance, chain, 16 * sg
// samples; sg = 1 for the adjoint) per wave, four waves per workgroup.
// Forward: steps of at most 4 tiles (K, N <= 64); adjoint: at most 2 tiles.
constexpr int kRegFwdTiles = 4;
constexpr int kRegBwdTiles = 2;
size_t rchain_wave_lds(const ChainLim &L, bool bwd, int sg);
int64_t rchain_ckpt_floats(const ChainLim &L);   // per adjoint task
hipError_t launch_rchain(const ChainArgs &a, bool bwd, hipStream_t st);
// Magnetisation moments on the register-resident chains (the adjoint's task
// list: 16 samples per wave, chains of a.ntm <= 2 tiles): cpart and mpart
// of every task's chain and samples
hipError_t launch_rchain_moments(const ChainArgs &a, hipStream_t st);
// per sample of the chain instances: mean and var, the sums over the
// instance's chains of mpart (chain order)
hipError_t launch_chain_mom_sum(const ChainInst *cinst, const int32_t *chain_insts,
                                int n_chain_insts, const int64_t *inst_B,
                                const int64_t *inst_sample_off, const int64_t *cpart_off,
                                const double *mpart, int64_t mtot, double *mean, double *var,
                                hipStream_t st);
// every width of a.pq_lo / a.pq_n in one persistent launch
hipError_t launch_rchain_pq(const ChainArgs &a, bool bwd, hipStream_t st);
// logz[b] = log_const + sum over chains of the per-chain partials
// (plus the unary sums fabp of launch_unary when fabp is not null)
hipError_t launch_chain_sum(const InstDesc *inst, const ChainInst *cinst,
                            const int32_t *chain_insts, int n_chain_insts,
                            const int64_t *inst_B, const int64_t *inst_sample_off,
                            const int64_t *cpart_off, const double *cpart, const int64_t *f_off,
                            const double *fabp, double *logz, hipStream_t st);

// Per-call tables of the register-resident forward written on the device
// (no host copy): the per-instance offsets the host computed, the list of
// chain instances and the forward task list, (instance, chain, first sample)
// in the order width group, instance, sample group, chain.  Everything comes
// by value, so the launch allocates nothing and can be recorded in a graph.
constexpr int kLayoutMaxInst = 32;
struct LayoutArgs {
  int32_t n_inst;
  int32_t n_tasks;                           // total forward tasks
  int64_t B[kLayoutMaxInst], sample_off[kLayoutMaxInst], spin_off[kLayoutMaxInst];
  int64_t cpart_off[kLayoutMaxInst], u_off[kLayoutMaxInst], f_off[kLayoutMaxInst];
  int32_t seg_off[3][kLayoutMaxInst + 1];    // first task of (width group, instance)
  int32_t per[3];                            // samples per task of each width group
  const ChainInst *cinst;
  const ChainDesc *chains;
  // destinations
  int64_t *d_B, *d_sample_off, *d_spin_off, *d_cpart_off, *d_u_off, *d_f_off;
  int32_t *d_clist, *d_ti, *d_tc, *d_ts;
};
hipError_t launch_layout(const LayoutArgs &a, hipStream_t st);

}  // namespace tnvan
