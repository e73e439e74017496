/* tnvan.h - C ABI of the TNVAN hot path on MI355X (gfx950).
 *
 * Tensor-network-based variational autoregressive networks (arXiv 2504.12037):
 * a spin system E(s) = -sum_<ij> J_ij s_i s_j - sum_i h_i s_i (Sec. 2, Eq. 1;
 * the field term is this library's extension) is split into a width set W and
 * a remainder R.  For every width-set configuration s_W drawn from a masked
 * autoregressive network q (Sec. 3, Eqs. 6-8) the library contracts
 *
 *     logZ_R(s_W) = ln sum_r exp(-beta E_2(s_W, r))          (Eqs. 3-4)
 *
 * exactly along a fixed elimination order of R, differentiates it with a
 * hand-written adjoint, and trains q by the REINFORCE gradient of the
 * variational free energy (Eqs. 9-10, Algorithm 1).
 *
 * Conventions for every entry point
 *  - Host arrays are read during the call and copied; the caller keeps
 *    ownership.  Device pointers ("dev") are caller-owned device memory that
 *    must stay valid until the work queued on `stream` has completed.  A
 *    "dev" argument that is plain host memory (not device, managed or
 *    device-mapped pinned memory) is rejected with TNVAN_E_INVALID before
 *    any work is queued.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work of a call is queued on it; calls return without waiting
 *    unless stated otherwise.
 *  - Several instances (disorder realisations) can live in one net.  Their
 *    sample batches are concatenated in instance order ("instance-major"):
 *    instance i owns n_samples[i] consecutive samples.
 *  - Spins are int8 holding +1 or -1.  The spins of a sample are its width-set
 *    spins in the order of `width_set`.
 *  - Every function returns a tnvan_status and never aborts or throws.  On
 *    failure tnvan_last_error() returns a message (thread-local).  HIP errors
 *    map to TNVAN_E_HIP; an asynchronous device fault surfaces at the next
 *    synchronising call.
 *  - One net must not be used from two host threads or two streams at once:
 *    it owns workspaces that every call reuses.
 */
#ifndef TNVAN_H
#define TNVAN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tnvan_net tnvan_net;   /* opaque, library-owned */

typedef enum {
  TNVAN_OK = 0,
  TNVAN_E_INVALID = 1,    /* malformed instance or argument */
  TNVAN_E_WIDTH = 2,      /* a message scope exceeds the width limit */
  TNVAN_E_NOMEM = 3,      /* device or host allocation failed */
  TNVAN_E_HIP = 4,        /* a HIP runtime call failed */
  TNVAN_E_STATE = 5,      /* call out of order (e.g. missing build) */
  TNVAN_E_NONFINITE = 6   /* non-finite value detected */
} tnvan_status;

typedef enum {
  TNVAN_FP64 = 0,         /* plain FP64 path */
  TNVAN_FP32 = 1,         /* FP32 contraction, FP64 log-norm and reductions */
  TNVAN_BF16 = 2          /* as FP32 with BF16 inputs to the dense products */
} tnvan_precision;

/* One disorder instance (Sec. 2): couplings, fields, inverse temperature,
 * width set W and the elimination order of R = V \ W (Alg. 1, step 1). */
typedef struct {
  int32_t n_spins;
  int32_t n_edges;
  const int32_t *edge_i;      /* [n_edges], 0-based, edge_i < edge_j */
  const int32_t *edge_j;      /* [n_edges], no duplicate edges */
  const double *J;            /* [n_edges] couplings J_ij */
  const double *h;            /* [n_spins] fields, or NULL for h = 0 */
  double beta;                /* inverse temperature, >= 0 */
  int32_t n_width;
  const int32_t *width_set;   /* [n_width]; also the sampling order of q */
  int32_t n_order;
  const int32_t *order;       /* [n_order], a permutation of V \ W */
  int32_t n_groups;           /* 0 => one vertex per elimination step */
  const int32_t *group_ptr;   /* [n_groups+1] CSR over `order`, or NULL */
  int32_t hidden;             /* hidden width H of q (0: Eq. 7 exactly) */
  /* hidden layers of q (0 or 1: one; 2..4: D - 1 more tanh layers of width
   * H after the first, a unit seeing the units below of no larger degree;
   * their parameters follow W0, see tnvan_param_count).  Ignored when
   * H = 0.  Nets with a deeper instance run every instance through the
   * general sampler and REINFORCE kernels and need |W| <= 256, H <= 256. */
  int32_t depth;
} tnvan_instance;

typedef struct {
  int32_t precision;          /* tnvan_precision */
  int32_t max_width;          /* largest message scope allowed (<= 20; scopes of 15-20
                               * only for single-spin steps, whose transfer factors
                               * are formed on the fly) */
  int32_t deterministic;      /* reserved: every reduction is ordered */
  int32_t flags;              /* TNVAN_FLAG_* bits, 0 for the defaults */
  uint64_t seed;              /* key of the Philox4x32-10 stream of q */
  /* adjoint checkpoint interval k of the register-resident chain kernels:
   * the chain state is stored every k steps and the others are recomputed
   * from the checkpoint in the reverse walk (0 or 1: every step; 2, 4, 8).
   * Same results bit for bit; fewer HBM bytes, more work. */
  int32_t checkpoint_every;
} tnvan_options;

/* Run chains of narrow dense steps in the LDS-staged transfer-matrix kernels
 * instead of the register-resident ones (same results up to rounding; for
 * comparisons and timing). */
#define TNVAN_FLAG_LDS_CHAIN 1
/* Record HIP events on the launch stream around the kernels listed below;
 * tnvan_kernel_time reads them back. */
#define TNVAN_FLAG_PROFILE 2
/* tnvan_free_energy_step replays the whole training step from a captured HIP
 * graph.  A call whose batch shape, stats / spins_out pointers or lr differ
 * from the recorded ones, or that follows a change of the net's device
 * buffers or tables (another batch shape in any call), runs eagerly and
 * records a new graph for the next calls. */
#define TNVAN_FLAG_GRAPH 4
/* FP32 nets: the register-resident chain kernels form every FP32 product
 * as three BF16 matrix-core products of split operands (a = a_hi + a_lo,
 * each part rounded to BF16: a_hi b_hi + a_hi b_lo + a_lo b_hi, FP32
 * accumulation; about 16 bits of each operand, the a_lo b_lo term dropped),
 * at 16x the multiply rate of the FP32 products.  Spin-sign operands are
 * exact in BF16 and take two products.  Ignored by FP64 and BF16 nets. */
#define TNVAN_FLAG_SPLIT_BF16 8
/* tnvan_free_energy_step(_adjoint) waits for its step (eager or replayed),
 * and returns TNVAN_E_NONFINITE when any sample's free energy f_b (Eq. 9)
 * was not finite (a NaN or infinite parameter, log-probability or logZ);
 * the step's work has run, and the flags are cleared for the next call.
 * Without the flag the step does not wait and reports nothing. */
#define TNVAN_FLAG_CHECK_FINITE 16
/* roctx ranges around the phases of every call (tnvan/sample, tnvan/logz,
 * tnvan/boundary, tnvan/steps, tnvan/adjoint, tnvan/step,
 * tnvan/free_energy, tnvan/reinforce, tnvan/adam), for traces taken with
 * rocprofv3 --marker-trace; host-side ranges around the launches, nothing
 * waits.  Without the flag no roctx call is made. */
#define TNVAN_FLAG_MARKERS 32

/* Launch shapes of a net (tnvan_get_tuning, tnvan_set_tuning,
 * tnvan_autotune).  They change how the work is tiled, not what is computed:
 * every choice gives the same results up to the summation order of the
 * kernels involved (within each path's tolerance).  A field set to 0 takes
 * the library's default rule. */
#define TNVAN_TUNE_GENERAL 1     /* kinds: the general-step kernel runs */
#define TNVAN_TUNE_REG_CHAIN 2   /* the register-resident chain kernels run */
#define TNVAN_TUNE_LDS_CHAIN 4   /* the LDS-staged chain kernels run */
typedef struct {
  /* samples per workgroup tile of the general-step kernel (dense and
   * single-spin steps of non-chain programs), forward and adjoint: 0 or a
   * power of two 1..64 (the arena stays in LDS when the tile fits it, else
   * it moves to device memory) */
  int32_t general_tile_fwd;
  int32_t general_tile_bwd;
  /* 16-sample groups per wave of the register-resident chain forward on
   * chains of 1-2 tiles: 0, 1 or 2 */
  int32_t chain_groups;
  /* tnvan_get_tuning only: TNVAN_TUNE_* bits of the kernels the net runs */
  int32_t kinds;
  /* adjoint checkpoint interval of the register-resident chain kernels
   * (0: the tnvan_options value; 1, 2, 4, 8) */
  int32_t checkpoint_every;
  /* how the uneven batch is launched: 1 one workgroup per tile of the
   * general kernel and one launch per chain width; 2 persistent launches:
   * the general kernel's workgroups, and the chain kernels' waves over every
   * width, take (instance, tile or chain, sample group) items from a device
   * work queue, the costliest first (0: the default, 1) */
  int32_t launch_mode;
  /* upper bound in MiB on the general kernel's device arenas of one call
   * (0: the default budget, half of the device memory that is free or held
   * by the arena, at most 96 GiB); a batch whose arenas exceed it runs in
   * chunks of resident workgroups.  Not timed by the autotuner, which keeps
   * the value in effect. */
  int32_t arena_limit_mib;
  int32_t reserved[1];
} tnvan_tuning;

/* The launch shapes in effect (defaults resolved; chain_groups 0 until a
 * batch has been laid out). */
tnvan_status tnvan_get_tuning(const tnvan_net *net, tnvan_tuning *out);
/* Request launch shapes (0 = default rule per field).  The next call lays
 * its tables out again.  Errors: a field out of range or a general tile
 * whose LDS part does not fit even with the arena in device memory
 * (TNVAN_E_INVALID; the previous shapes stay). */
tnvan_status tnvan_set_tuning(tnvan_net *net, const tnvan_tuning *in);

/* Autotuner: on the given batch (the net's own sample counts and spins),
 * times tnvan_logz_batch for every candidate forward shape and
 * tnvan_logz_backward for every candidate adjoint shape of the kernels the
 * net runs (general tiles 1..64 samples, chain groups 1 or 2, adjoint
 * checkpoint intervals 1, 2, 4, launch modes 1 and 2), one field at
 * a time with the others at their best so far, each candidate as the mean
 * of 5 calls after one that lays the tables out (HIP events on `stream`).
 * A field keeps its default rule unless a candidate is at least 2% faster.
 * The choice is applied (tnvan_set_tuning) and written to *out.
 *   spins, grad_logz  dev inputs as tnvan_logz_backward
 *   logz, dh, dJ, dbeta  dev workspaces the timed calls write (as there)
 *   cache_path  host path of a JSON cache, or NULL: a key (GPU
 *               architecture | precision and product form | kernels |
 *               widest message scope | instances | batch size bucket)
 *               found there is applied without timing; a new choice is
 *               added to the file (rewritten through a temporary file)
 * Synchronises the stream.  Errors: those of the timed calls; an
 * unwritable cache (TNVAN_E_INVALID, the choice is still applied). */
tnvan_status tnvan_autotune(tnvan_net *net, const int64_t *n_samples, const int8_t *spins,
                            const double *grad_logz, double *logz, double *dh, double *dJ,
                            double *dbeta, const char *cache_path, tnvan_tuning *out,
                            void *stream);

/* Kernels timed under TNVAN_FLAG_PROFILE. */
typedef enum {
  TNVAN_KERNEL_CHAIN_FWD_1 = 0,   /* register-resident forward, chains of 1 tile (K, N <= 16) */
  TNVAN_KERNEL_CHAIN_FWD_2 = 1,   /* ... 2 tiles (K, N <= 32) */
  TNVAN_KERNEL_CHAIN_FWD_4 = 2,   /* ... 4 tiles (K, N <= 64) */
  TNVAN_KERNEL_CHAIN_BWD_1 = 3,   /* register-resident adjoint, chains of 1 tile */
  TNVAN_KERNEL_CHAIN_BWD_2 = 4,   /* ... 2 tiles */
  TNVAN_KERNEL_SAMPLE = 5,        /* matrix-core sampler */
  TNVAN_KERNEL_MADE_GRAD = 6,     /* fused REINFORCE backward (without its row reduction) */
  TNVAN_KERNEL_CHAIN_FWD_ALL = 7, /* register-resident forward, every width in one persistent launch */
  TNVAN_KERNEL_CHAIN_BWD_ALL = 8, /* register-resident adjoint, every width in one persistent launch */
  TNVAN_KERNEL_COUNT = 9
} tnvan_kernel;

/* Compile n_inst instances into one net (host work plus device uploads,
 * synchronous).  Validates every instance: W and order disjoint and covering
 * all spins, edges unique with i < j, finite J, h and beta >= 0, group sizes
 * <= 8 and a grouped step whose input message is not exactly its group
 * (TNVAN_E_INVALID); a message scope above max_width (TNVAN_E_WIDTH).
 * The initial parameters of q are zero; set them with tnvan_set_params.
 * On success *out owns all device state; free it with tnvan_free_network. */
tnvan_status tnvan_build_network(const tnvan_instance *inst, int32_t n_inst,
                                 const tnvan_options *opt, tnvan_net **out);

void tnvan_free_network(tnvan_net *net);

const char *tnvan_last_error(void);

/* Number of float32 parameters of q for instance i (flat layout
 * W1 [H,n], b1 [H], W2 [n,H], b2 [n], W0 [n,n], n = |W|, row-major; for
 * depth D > 1 followed by (W^l [H,H], b^l [H]) for l = 2..D). */
tnvan_status tnvan_param_count(const tnvan_net *net, int32_t inst, int64_t *count);

/* Copy the parameters of instance i from / to device memory (float32 in
 * every precision; stream-ordered).  set_params also clears the optimiser
 * state and the step counter of that instance. */
tnvan_status tnvan_set_params(tnvan_net *net, int32_t inst, const float *src_dev,
                              void *stream);
tnvan_status tnvan_get_params(tnvan_net *net, int32_t inst, float *dst_dev,
                              void *stream);

/* New couplings J, fields h and inverse temperature beta for instance i of
 * a built net (Sec. 2: E of Eq. 1 plus fields, and with it E_1, E_2 and the
 * static transfer factors exp(beta J s s') of the contraction, Eqs. 2-4).
 * The instance is compiled again from its build-time edges, width set,
 * order and grouping with the new values, and every device table is
 * rewritten in place; the parameters of q, the Adam moments, the step
 * counter and the launch shapes stay.  Synchronous: waits for all work the
 * net has queued (on any stream) before the tables change; the next call
 * lays its per-call tables out again, and a recorded training-step graph is
 * recorded anew.
 *   J     host double [n_edges], in the edge order of the build
 *   h     host double [n_spins], or NULL for h = 0
 *   beta  finite, >= 0
 * Errors: instance index out of range, J NULL with edges, non-finite J or h,
 * beta < 0 or not finite (TNVAN_E_INVALID; nothing changes); called while a
 * graph is recorded (TNVAN_E_STATE). */
tnvan_status tnvan_set_couplings(tnvan_net *net, int32_t inst, const double *J, const double *h,
                                 double beta);

/* Copy one state vector of instance i into device memory (float32,
 * param_count entries, stream-ordered): which = 0 parameters, 1 gradient of
 * the last free_energy_step, 2 Adam first moment, 3 Adam second moment.
 * Used for checkpoints and for checking the REINFORCE gradient. */
tnvan_status tnvan_get_state(tnvan_net *net, int32_t inst, int32_t which,
                             float *dst_dev, void *stream);

/* Restore one state vector of instance i from device memory (float32,
 * param_count entries, stream-ordered): which = 0 parameters (unlike
 * tnvan_set_params, the Adam moments and the step counter stay), 2 Adam
 * first moment, 3 Adam second moment.  With tnvan_set_step this resumes
 * Algorithm 1 from a checkpoint taken with tnvan_get_state and
 * tnvan_get_step: the continued run equals the uninterrupted one bit for bit.
 * Errors: which 1 (the gradient is recomputed every step) or out of range
 * (TNVAN_E_INVALID). */
tnvan_status tnvan_set_state(tnvan_net *net, int32_t inst, int32_t which, const float *src_dev,
                             void *stream);

/* The step counter of instance i: the number of training steps taken with
 * samples (Adam's t, and the step word of the Philox counter of q's
 * uniforms).  get waits for the stream; set is stream-ordered (step >= 0). */
tnvan_status tnvan_get_step(tnvan_net *net, int32_t inst, int32_t *step, void *stream);
tnvan_status tnvan_set_step(tnvan_net *net, int32_t inst, int32_t step, void *stream);

/* Ancestral sampling from q (Sec. 3, Eq. 8): for each position i in the
 * order of width_set, p_i = sigmoid(logit_i(s_<i)) and s_i = +1 iff
 * u_i < p_i; logq accumulates ln q(s) = sum_i log sigmoid(s_i logit_i).
 *   n_samples [n_inst] host: samples per instance
 *   uniforms  dev float32 [sum_i n_samples[i] * |W_i|], instance-major,
 *             sample-major inside; NULL => the net's Philox stream at the
 *             current step counter (the counter is not advanced)
 *   spins     dev int8 out, same layout as uniforms
 *   logq      dev out, [sum n_samples]: double for TNVAN_FP64, else float */
tnvan_status tnvan_sample(tnvan_net *net, const int64_t *n_samples,
                          const float *uniforms, int8_t *spins, void *logq,
                          void *stream);

/* Batched conditional log-partition function (Eqs. 3-4): for every sample,
 * logz[b] = ln sum_r exp(-beta E_2(s_W(b), r)), by exact contraction along
 * the compiled order with per-step power-of-two rescaling; the log-norm and
 * the result are FP64 in every precision.  Optionally also the width-set
 * energy of Eq. 4, E_1(s_W) = -sum_{W-W edges} J_ij s_i s_j - sum_{i in W}
 * h_i s_i, so that Etilde = E_1 - logz / beta (Eq. 3) needs nothing more.
 *   spins  dev int8 [sum n_samples * |W|] (layout as tnvan_sample)
 *   logz   dev double out [sum n_samples]
 *   e1     dev double out [sum n_samples], or NULL (not computed); FP64 in
 *          every precision, the W-W terms in edge order, then the fields */
tnvan_status tnvan_logz_batch(tnvan_net *net, const int64_t *n_samples,
                              const int8_t *spins, double *logz, double *e1, void *stream);

/* Adjoint of tnvan_logz_batch: writes the vector-Jacobian product
 *   dh[i]    = sum_b g_b dlogZ_R(b)/dh_i     = beta sum_b g_b <r_i>_b
 *   dJ[e]    = sum_b g_b dlogZ_R(b)/dJ_e     = beta sum_b g_b <x_i x_j>_b
 *   dbeta[k] = sum_b g_b dlogZ_R(b)/dbeta    = -sum_b g_b <E_2>_b
 * (magnetisations, edge correlations and internal energy of the remainder;
 * zero on W vertices and W-W edges).  The forward is recomputed inside.
 *   grad_logz dev double [sum n_samples] (g_b)
 *   dh        dev double out [sum_i n_spins_i], instance-major
 *   dJ        dev double out [sum_i n_edges_i]
 *   dbeta     dev double out [n_inst] */
tnvan_status tnvan_logz_backward(tnvan_net *net, const int64_t *n_samples,
                                 const int8_t *spins, const double *grad_logz,
                                 double *dh, double *dJ, double *dbeta,
                                 void *stream);

/* Allocation-free variant of tnvan_logz_batch, for callers that cannot
 * allocate device memory: code recorded into a HIP graph, serving loops and
 * harnesses that forbid hipMalloc.  The arguments of tnvan_logz_batch
 * without e1, and the same logz (bit for bit: the same kernels and
 * arithmetic), but every
 * per-call table and workspace lives in one file-scope device array of
 * TNVAN_NOALLOC_SCRATCH_BYTES (32 MiB) per GPU, which the library keeps
 * until the process ends; the call makes no allocation, no host-to-device
 * copy and no synchronisation, and its tables are written by a kernel from
 * the sample counts passed by value.
 *  - Needs a net whose every instance runs the register-resident chain
 *    kernels (FP32 or BF16 nets of dense chains of at most 64 states, e.g.
 *    lattice strips; TNVAN_E_STATE otherwise) and at most
 *    TNVAN_NOALLOC_MAX_INST instances (TNVAN_E_INVALID).
 *  - A batch whose workspace exceeds the array is rejected with
 *    TNVAN_E_INVALID before any work is queued.  It needs about
 *    (4 |R| + 8 ceil(|R| / 16) + 8 chains) bytes per sample: the 16x16
 *    lattice with two width-set columns fits 3 x 8192 samples.
 *  - Every call on a GPU shares that GPU's array and overwrites it: two
 *    calls whose work overlaps on one GPU (on different streams, or from
 *    different host threads, on any nets) race and give wrong results.
 *    Calls queued on one stream are ordered and safe.
 *  - The net must be used on the device it was built on (TNVAN_E_STATE). */
#define TNVAN_NOALLOC_SCRATCH_BYTES (32u << 20)
#define TNVAN_NOALLOC_MAX_INST 32
tnvan_status tnvan_logz_batch_noalloc(tnvan_net *net, const int64_t *n_samples,
                                      const int8_t *spins, double *logz, void *stream);

/* tnvan_logz_batch and tnvan_logz_backward of the same spins in one call,
 * with the same arguments and results (logz as tnvan_logz_batch writes it).
 * On FP32 nets whose every instance runs the register-resident chain
 * kernels, logZ is the adjoint's own forward contraction (the forward
 * kernel's arithmetic, step for step), so the contraction runs once;
 * otherwise the two calls are made in turn.
 *   logz dev double out [sum n_samples]; the other arguments as above */
tnvan_status tnvan_logz_and_backward(tnvan_net *net, const int64_t *n_samples,
                                     const int8_t *spins, const double *grad_logz,
                                     double *logz, double *dh, double *dJ,
                                     double *dbeta, void *stream);

/* One training iteration of Algorithm 1 for every instance: sample with the
 * Philox stream at the current step counter, contract, form
 * f_b = E_1 - logZ_R/beta + ln q/beta, F_q = mean f (Eq. 9), REINFORCE
 * weights (f_b - F_q)/B (Eq. 10, batch-mean baseline, FP64), the gradient of
 * q and one Adam step (lr; beta1 0.9, beta2 0.999, eps 1e-8); then the step
 * counter advances.  Needs beta > 0 (TNVAN_E_INVALID otherwise).
 *   stats     dev double out [n_inst, 4]: F_q, its standard error,
 *             mean Etilde, mean ln q / beta
 *   spins_out dev int8 out (optional, may be NULL): the sampled spins */
tnvan_status tnvan_free_energy_step(tnvan_net *net, const int64_t *n_samples,
                                    float lr, double *stats, int8_t *spins_out,
                                    void *stream);

/* tnvan_free_energy_step followed by tnvan_logz_backward of the spins it
 * sampled, with per-sample weights grad_logz, in one call (one recorded
 * graph under TNVAN_FLAG_GRAPH).  Where tnvan_logz_and_backward contracts
 * once, the step's logZ is taken from the adjoint's forward pass.  The
 * adjoint outputs (dh, dJ, dbeta) are those of tnvan_logz_backward; the
 * step's results are those of tnvan_free_energy_step.
 *   grad_logz dev double [sum n_samples] (g_b, set before the call) */
tnvan_status tnvan_free_energy_step_adjoint(tnvan_net *net, const int64_t *n_samples,
                                            float lr, double *stats, int8_t *spins_out,
                                            const double *grad_logz, double *dh,
                                            double *dJ, double *dbeta, void *stream);

/* Exact free energy of one instance by slicing (Sec. 2, Eqs. 3-4): every
 * configuration s of its width set W is contracted as one sample, and
 *   logZ = ln sum_s exp(-beta E_1(s) + logZ_R(s)),   F = -logZ / beta,
 * with the sum taken as a log-sum-exp in FP64 in a fixed order (bit-for-bit
 * repeatable).  Spin i of configuration x (0 <= x < 2^|W|, W in width_set
 * order) is -1 where bit i of x is set.  The configurations run in passes of
 * at most 65,536 through the net's logZ path (its precision and kernels);
 * the call sets the net's batch to one pass of this instance, so other
 * entry points re-lay their tables at their next call.
 *   inst  instance index
 *   out   dev double out [2]: logZ, F
 * Errors: |W| > 28 (TNVAN_E_WIDTH); beta <= 0 (TNVAN_E_INVALID). */
tnvan_status tnvan_exact_free_energy(tnvan_net *net, int32_t inst, double *out, void *stream);

/* Moments of the Boltzmann distribution p (Eq. 1) from samples of q: the
 * magnetisations <sigma_i>_p of every vertex and correlations
 * <sigma_i sigma_j>_p of every edge, by self-normalised importance weights.
 * The W-marginal of p is exp(-beta E_1) Z_R / Z, so the weight of sample b
 * is w_b = exp(-beta f_b) / sum_c exp(-beta f_c) with f_b of Eq. 9
 * (per instance).  Each moment is sum_b w_b times its expectation given s_W:
 * s_i on W, s_i s_j on W-W edges, and on the remainder the conditional
 * magnetisations and correlations, which the adjoint gives with grad_logz
 * = w_b / beta (as tnvan_logz_backward: dh = beta sum g <r>, dJ = beta sum
 * g <x x>).  All sums FP64, fixed order.  The step counter is not advanced.
 *   n_samples, spins  as tnvan_logz_batch (e.g. from tnvan_sample)
 *   logq  dev ln q(s_b) as tnvan_sample writes it: double for TNVAN_FP64,
 *         else float
 *   mag   dev double out [sum_i n_spins_i]; corr dev double out
 *         [sum_i n_edges_i]; ess dev double out [n_inst], the effective
 *         sample size (sum w)^2 / sum w^2
 * Errors: beta <= 0 on any instance; a buffer that is plain host memory
 * (not device, managed or device-mapped pinned memory) (TNVAN_E_INVALID). */
tnvan_status tnvan_observables(tnvan_net *net, const int64_t *n_samples, const int8_t *spins,
                               const void *logq, double *mag, double *corr, double *ess,
                               void *stream);

/* Conditional moments of the remainder's magnetisation M_R = sum_{r in R} r
 * given each sample's width-set spins, under p(r | s_W) proportional to
 * exp(-beta E_2(s_W, r)) (Eqs. 3-4): the ingredients of the susceptibility
 * (Sec. 3: magnetisation and susceptibility from the trained network).
 * With eta = beta H for a uniform field H on R, the mean is d ln Z_R / d eta
 * and the variance d^2 ln Z_R / d eta^2; both come exactly from one
 * contraction of second-order Taylor coefficients in eta (jets) along the
 * compiled order, in the net's precision (FP64 for TNVAN_FP64, else FP32
 * jets with the dense products in FP32), cumulants formed in FP64.
 *   spins  dev int8 as tnvan_logz_batch
 *   logz   dev double out [sum n_samples], or NULL: ln Z_R of the same pass
 *   mean   dev double out [sum n_samples]: <M_R | s_W>
 *   var    dev double out [sum n_samples]: Var(M_R | s_W)
 * Device workspace: (arena + scratch entries of the program) x 3 jets per
 * sample.  Errors: a message scope above 14 (TNVAN_E_WIDTH). */
tnvan_status tnvan_remainder_moments(tnvan_net *net, const int64_t *n_samples,
                                     const int8_t *spins, double *logz, double *mean, double *var,
                                     void *stream);

/* Magnetisation moments and susceptibility of the Boltzmann distribution p
 * (Eq. 1) from samples of q (Sec. 3), per instance with M = sum_i s_i over
 * all N spins:
 *   out[4 i + 0] = <M>_p / N
 *   out[4 i + 1] = <M^2>_p / N^2
 *   out[4 i + 2] = chi = beta N (out[1] - out[0]^2)  (beta (<M^2> - <M>^2) / N)
 *   out[4 i + 3] = effective sample size (sum w)^2 / sum w^2
 * Importance weights as tnvan_observables (w_b proportional to
 * exp(-beta f_b), f_b of Eq. 9); given s_W, M = M_W + M_R, so each sample
 * contributes M_W + <M_R> to <M> and (M_W + <M_R>)^2 + Var(M_R) to <M^2>
 * (tnvan_remainder_moments).  FP64 sums in a fixed order.  The step counter
 * is not advanced.
 *   n_samples, spins, logq  as tnvan_observables
 *   out   dev double out [n_inst * 4]
 * Errors: beta <= 0 on any instance; a plain host buffer (TNVAN_E_INVALID);
 * a message scope above 14 (TNVAN_E_WIDTH). */
tnvan_status tnvan_susceptibility(tnvan_net *net, const int64_t *n_samples, const int8_t *spins,
                                  const void *logq, double *out, void *stream);

/* Per-instance program statistics of the compiled order (host values):
 *   info[0] steps, [1] largest message scope, [2] arena entries per sample,
 *   [3] flops per sample of the forward contraction (2 per multiply-add,
 *   counting the dense step form as executed), [4] |W|, [5] |R| */
tnvan_status tnvan_program_info(const tnvan_net *net, int32_t inst, int64_t info[6]);

/* Total device time (milliseconds, from the recorded HIP events) and number
 * of launches of one kernel since the previous call for that kernel (waits
 * for the recorded launches to finish).  Needs TNVAN_FLAG_PROFILE at build,
 * else TNVAN_E_STATE. */
tnvan_status tnvan_kernel_time(tnvan_net *net, int32_t kernel, double *total_ms,
                               int64_t *launches);

/* Which kernels TNVAN_FLAG_PROFILE times: bit k set times tnvan_kernel k
 * (all of them after the build).  Each timed launch adds two event records
 * to the stream, so timing only the kernels of interest keeps the rest of
 * the stream's launches back to back.  Needs TNVAN_FLAG_PROFILE, else
 * TNVAN_E_STATE. */
tnvan_status tnvan_profile_mask(tnvan_net *net, uint32_t mask);

/* Host-only planning: validate and compile one instance without touching a
 * device and report the same statistics as tnvan_program_info. */
tnvan_status tnvan_plan(const tnvan_instance *inst, int32_t max_width, int64_t info[6]);

/* Width set W and elimination order of R = V \ W for a bound w_u on the
 * contraction width, by the recipe of Sec. 2 (finding the width set): a
 * greedy order pi of the whole interaction graph, then dynamic slicing, then
 * indices put back from W.  Host only; touches no device.
 *  - The width of an elimination order is its largest scope, the neighbours
 *    (fill edges included) of a vertex not yet eliminated when it is; the
 *    message it leaves has 2^scope entries.  Fixing W removes W and its
 *    edges; the order of R is always pi with the W vertices skipped.
 *  - pi is min-fill: the vertex whose current neighbours miss the fewest
 *    edges among themselves first (ties: fewest current neighbours, then
 *    smallest key).
 *  - Slicing: while the width exceeds w_u, the vertex lying in the most
 *    scopes of the maximum size moves to W (ties: larger degree, then
 *    smallest key).
 *  - Then each W vertex, in ascending key order, goes back to R if the
 *    width stays <= w_u.  At w_u = 1, R is a forest: W is a feedback vertex
 *    set.
 *  - With TNVAN_PLAN_REGREEDY in flags the tree is rebuilt instead of kept:
 *    after every pick and for every re-adding test, the min-fill order of
 *    the graph induced on R replaces pi restricted to R (slower; smaller W
 *    at small w_u).
 *   n_spins        1..16384
 *   edge_i, edge_j host int32 [n_edges], 0-based, i != j (duplicates ignored)
 *   w_u            width bound, >= 1
 *   key            host int32 [n_spins], a permutation of 0..n_spins-1
 *                  (random draws of the caller), or NULL for key = id
 *   flags          0 or TNVAN_PLAN_REGREEDY
 *   width_set      host int32 out [n_spins]: W ascending in the first
 *                  *n_width entries
 *   order          host int32 out [n_spins]: the order of R in the first
 *                  n_spins - *n_width entries
 *   greedy         host int32 out [n_spins]: pi, or NULL
 *   width          host out: the width of `order` (<= w_u)
 * Errors: any size, bound, endpoint, loop, key or flag out of range
 * (TNVAN_E_INVALID). */
#define TNVAN_PLAN_REGREEDY 1
tnvan_status tnvan_plan_width_set(int32_t n_spins, int32_t n_edges, const int32_t *edge_i,
                                  const int32_t *edge_j, int32_t w_u, const int32_t *key,
                                  int32_t flags, int32_t *width_set, int32_t *n_width,
                                  int32_t *order, int32_t *greedy, int32_t *width);

#ifdef __cplusplus
}
#endif
#endif /* TNVAN_H */
