// C ABI of the TNVAN hot path: build, sample, logz_batch, logz_backward,
// free_energy_step (Algorithm 1) and accessors.  Host orchestration only;
// every step of the path runs in the kernels of contract.hip and made.hip.
#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/tnvan.h"
#include "compile.h"
#include "launch.h"
#include "plan.h"

namespace tnvan {
}

using namespace tnvan;

namespace {

thread_local std::string g_err;

tnvan_status set_err(tnvan_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return set_err(TNVAN_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

// Generation of every device buffer's address and of every uploaded table:
// bumped on each reallocation and upload, so that a captured graph (whose
// kernel arguments hold addresses and whose task tables hold one batch
// shape) is known to be stale.
std::atomic<uint64_t> g_buf_gen{1};

// Device buffer that grows on demand (contents are not preserved).
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need) {
    if (need <= bytes) return hipSuccess;
    if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
    g_buf_gen.fetch_add(1);
    hipError_t e = hipMalloc(&p, need);
    if (e == hipSuccess) bytes = need;
    return e;
  }
  void release() { if (p) (void)hipFree(p); p = nullptr; bytes = 0; }
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

template <typename T>
hipError_t upload(DBuf &b, const std::vector<T> &v) {
  size_t n = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = b.ensure(n);
  if (e != hipSuccess) return e;
  g_buf_gen.fetch_add(1);
  if (!v.empty()) e = hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

// Scratch of the allocation-free entry point (tnvan_logz_batch_noalloc): a
// file-scope device array, one copy on every GPU the library runs on, held
// until the process ends.  On the host its name only stands in for the
// symbol; kernels get each device's own address, taken from
// hipGetSymbolAddress once per device (scratch_setup) and kept in
// g_scratch_dev.
}  // namespace

static __device__ __align__(256) unsigned char scratch[TNVAN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];
std::string g_scratch_err[kMaxDevices];

// Called with device `dev` current: its scratch address, once.
void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[dev]) return;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    g_scratch_err[dev] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    (void)hipGetLastError();
    return;
  }
  g_scratch_dev[dev] = p;
}

struct TileCache {
  std::vector<int64_t> key;       // n_samples it was built for
  int S = 0;
  int n_tiles = 0;
  DBuf tile_inst, tile_start, first_tile, n_tiles_i, partial_off;
  std::vector<int32_t> h_first, h_count;
  int64_t partial_total = 0;
};

}  // namespace

struct tnvan_net {
  int precision = TNVAN_FP32;
  int device = 0;             // the device current at build
  uint64_t seed = 0;
  HostProgram P;
  int n_inst = 0;
  // program on the device
  DBuf inst, steps, inputs, gtab, gtab2, esmall, edges, T, fld_ptr, fld_w, fld_J, hR, wr_pos, wr_w;
  DBuf rr_edge, rr_J, wr_edge, wr_J, hR64, vr, ww_a, ww_b, ww_J, hW;
  // network
  std::vector<MadeInst> mi;
  std::vector<int64_t> param_count;
  int64_t param_total = 0;
  DBuf d_mi, params, adam_m, adam_v, grad, step_ctr;
  DBuf nonfinite;             // [n_inst] flags of the free-energy kernel
  DBuf pq;                    // work-queue counters of the persistent launches [8]
  bool check_finite = false;  // TNVAN_FLAG_CHECK_FINITE
  // per-call tables
  std::vector<int64_t> nkey;
  std::vector<int64_t> sample_off, spin_off;
  int64_t B_total = 0, spin_total = 0;
  DBuf d_sample_off, d_B, d_spin_off, d_spin_base, d_edge_base;
  TileCache tc_fwd, tc_bwd;
  int S_fwd = 1, S_bwd = 1;
  bool glob_fwd = false, glob_bwd = false;
  size_t lds_fwd = 0, lds_bwd = 0;
  std::vector<int32_t> h_blk_inst, h_blk_start;
  DBuf blk_inst, blk_start;
  int n_sblocks = 0;
  std::vector<int64_t> skey;
  // workspaces
  DBuf w_xspins, w_xlogz, w_xpart;   // exact slicing
  DBuf ww_e, d_wv, w_og, w_ostats, w_odb;   // observables
  // magnetisation moments: jets and step exponents of the Taylor contraction,
  // their per-instance offsets (for the batch key mkey), and the
  // susceptibility's per-sample moments and effective sample sizes
  DBuf w_jar, w_jexp, d_jar_off, d_jexp_off, w_mmean, w_mvar, w_oess;
  std::vector<int64_t> mkey;
  // moments on the chain kernels: per (chain, sample) mean and variance,
  // and the per-instance flags that send the general kernel past them
  DBuf w_mpart, d_mskip;
  bool mskip_set = false;
  // jobs of the REINFORCE backward's batch sums (ensure_batch_sums) and
  // their key: batch shape, row-buffer addresses, precision
  DBuf bs_atb, bs_col, bs_alo, bs_aflo, bs_clo, bs_cflo;
  std::vector<int64_t> bkey;
  int32_t bs_counts[6] = {0, 0, 0, 0, 0, 0};
  // jobs of the batched REINFORCE rows of one-layer nets, one launch per
  // class of LDS need (ensure_batch_sums): jobs, first blocks, counts, LDS
  // bytes
  DBuf rw_jobs[4], rw_lo[4];
  int32_t rw_njobs[4] = {0, 0, 0, 0}, rw_blocks[4] = {0, 0, 0, 0};
  size_t rw_lds[4] = {0, 0, 0, 0};
  DBuf garena, partial, w_logz, w_logq, w_spins, w_f, w_fpart, w_hid, w_da, w_dlogit, w_sf,
      w_part, d_hw_off, d_sum_off;
  int max_partial = 0, max_out = 1;
  int sample_reps = 1;
  // transfer-matrix form (chain kernels, FP32 / BF16 precisions)
  std::vector<int32_t> use_chain;
  DBuf cinst, chains, csteps, Tp, Tt, Tb, fld_wr, fld_J32, hR32;
  ChainLim lim_fwd{}, lim_bwd{};
  DBuf Tl, Tbl, cedges, ckpt;
  // register-resident chain kernels (per-wave tasks)
  DBuf Tr, Tq, Trb, xcol, cf_w, cf_r, cf_J, Tsx, Ts3, Tdq;
  bool split = false;   // TNVAN_FLAG_SPLIT_BF16 on an FP32 net
  DBuf Ubuf, fabp, u_off, f_off, vjp_part, tickets, col_out, pcoef_out;
  // training step replayed from a captured graph (TNVAN_FLAG_GRAPH)
  bool use_graph = false, capturing = false;
  hipStream_t cap_stream = nullptr;
  struct StepGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<int64_t> key;
    double *stats = nullptr;
    int8_t *spins = nullptr;
    float lr = 0.f;
    bool adj = false;
    const double *grad = nullptr;
    double *dh = nullptr, *dJ = nullptr, *dbeta = nullptr;
    uint64_t gen = 0;
  } step_graph;
  // kernel timing (TNVAN_FLAG_PROFILE): event pairs recorded since the last read
  bool profile = false;
  bool markers = false;       // TNVAN_FLAG_MARKERS: roctx phase ranges
  uint32_t prof_mask = ~0u;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_used[TNVAN_KERNEL_COUNT], prof_pool;
  int u_chunks = 0;
  int64_t u_maxB = 0;
  bool rfwd = false, rbwd = false;
  int rtiles = 1, sg = 2;
  int rg_lo[3] = {0, 0, 0}, rg_n[3] = {0, 0, 0}, brg_lo[3] = {0, 0, 0}, brg_n[3] = {0, 0, 0};
  int sg_of(int rt) const { return rt >= 4 ? 1 : sg; }
  // one-layer sampler (every instance H = 0, the general path): W0's
  // columns, n_q^2 floats per instance
  bool h0 = false;
  // some instance has a deeper network: the deep sampler and rows kernels
  bool deep = false;
  int h0_nmax = 0;
  DBuf w0t, d_w0t_off, w_sig;
  // matrix-core sampler
  bool msample = false;
  int mpt = 1;
  int64_t mpack_total = 0, mpack_max = 0;
  DBuf mpack, mtask_inst, mtask_start;
  // the packed tables hold the current parameters: set by a full pack, kept
  // by the optimiser (which writes them as it updates), cleared by an upload
  bool pack_valid = false;
  int n_mtasks = 0;
  // fused REINFORCE backward
  bool mgrad = false;
  int mg_hmax = 0;
  int64_t mg_pstride = 0;
  DBuf mg_task_inst, mg_task_start, mg_first, mg_count;
  int n_mgtasks = 0;
  DBuf task_inst, task_chain, task_start, btask_inst, btask_chain, btask_start, cpart_off,
      chain_list, cpart;
  int n_tasks = 0, n_btasks = 0, n_chain_insts = 0;
  std::vector<int64_t> ckey;
  // streams this net's calls have queued work on since the last wait; the
  // per-call tables are re-uploaded with synchronous copies on the null
  // stream, which does not order with non-blocking streams, so an upload
  // first waits for these
  std::vector<hipStream_t> call_streams;
  // the instances as built (host copies): tnvan_set_couplings recompiles
  // them with new couplings, fields and inverse temperatures
  struct SrcInst {
    int32_t n_spins = 0, n_edges = 0, hidden = 0, depth = 0;
    std::vector<int32_t> ei, ej, W, order, gp;
    std::vector<double> J, h;
    double beta = 0.0;
  };
  std::vector<SrcInst> src;
  int max_width = 0;
  tnvan_tuning tune{};        // requested launch shapes (0: default rule)
  int rk_build = 1;           // adjoint checkpoint interval from the options
  bool wide = false;          // some general-kernel instance has a step wider than kTabW
  int rs() const { return precision == TNVAN_FP64 ? 8 : 4; }
};

namespace {

int ilog2(int x) { int r = 0; while ((1 << r) < x) ++r; return r; }

// Entry of a device call on `stream`: remember the stream, so that a later
// table upload waits for the work queued on it.
void note_stream(tnvan_net *net, void *stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (std::find(net->call_streams.begin(), net->call_streams.end(), st) ==
      net->call_streams.end())
    net->call_streams.push_back(st);
}

// Before overwriting a per-call table that kernels queued earlier (in this
// call or in earlier ones) may still read: wait for every stream the net has
// used.  Not while recording a graph (nothing is uploaded then: the eager
// step before the recording made every table current).
tnvan_status quiesce(tnvan_net *net) {
  if (net->capturing) return TNVAN_OK;
  for (hipStream_t st : net->call_streams) HIPCHK(hipStreamSynchronize(st));
  if (net->call_streams.size() > 1) net->call_streams.erase(net->call_streams.begin(),
                                                            net->call_streams.end() - 1);
  return TNVAN_OK;
}

// A roctx range around one phase of a call (sample, boundary, steps,
// adjoint, free energy, REINFORCE, Adam), under TNVAN_FLAG_MARKERS only.
struct Phase {
  bool on;
  Phase(const tnvan_net *n, const char *name, bool when = true) : on(n->markers && when) {
    if (on) roctxRangePushA(name);
  }
  ~Phase() {
    if (on) roctxRangePop();
  }
};

// Events around one launch of a profiled kernel (no-op unless profiling).
struct ProfScope {
  tnvan_net *net;
  int kind;
  hipStream_t st;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  ProfScope(tnvan_net *n, int k, hipStream_t s) : net(n), kind(k), st(s) {
    if (!net->profile || net->capturing || kind < 0 || kind >= TNVAN_KERNEL_COUNT ||
        !((net->prof_mask >> kind) & 1u))
      return;
    // device-scope release: the events only time, and a system-scope one
    // would write back caches and slow the launches around the timed one
    if (!net->prof_pool.empty()) {
      ev = net->prof_pool.back();
      net->prof_pool.pop_back();
    } else if (hipEventCreateWithFlags(&ev.first, hipEventReleaseToDevice) != hipSuccess ||
               hipEventCreateWithFlags(&ev.second, hipEventReleaseToDevice) != hipSuccess) {
      ev = {nullptr, nullptr};
      return;
    }
    (void)hipEventRecord(ev.first, st);
  }
  ~ProfScope() {
    if (!ev.first) return;
    (void)hipEventRecord(ev.second, st);
    net->prof_used[kind].push_back(ev);
  }
};

// Samples per tile S of the general-step kernel (a power of two <= 64).
// Default rule: the largest S whose tile, arena included, fits the LDS
// budget (80 KB, two workgroups per CU).  Below 4 samples for the adjoint,
// or 8 for the forward pass, the arena moves to global memory, with S the
// largest that fits up to 8 for the adjoint (more, smaller workgroups hide
// the arena's latency better: the 64-instance batch's adjoint step took
// 15.7 ms at 8, 19.1 ms at 16) and up to 16 (FP32) or 8 (FP64) for the
// forward pass (its logZ took 2.4 ms at 16 in device memory against 4.8 ms
// at 4 in LDS).  A requested S (tuning) is
// taken with the arena in LDS when it fits the whole LDS, else in global
// memory; false when even that does not fit.
bool choose_tiles(tnvan_net *net, bool bwd, int req = 0) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  int maxlds = 65536;
  (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  const size_t budget = std::min<size_t>((size_t)maxlds, 80 * 1024);
  // instances in transfer-matrix form run in the chain kernels instead
  auto worst_of = [&](int S, bool glob) {
    size_t worst = 0;
    for (size_t q = 0; q < net->P.insts.size(); ++q)
      if (!net->use_chain[q])
        worst = std::max(worst, contract_lds_bytes(net->P.insts[q], S, bwd, glob, net->rs()));
    return worst;
  };
  int S = 64;
  bool glob = false;
  if (net->wide) {
    // wide steps: the arena is in device memory and S = 1 (or the requested
    // one).  Each sample's step has 2^15 or more entries, enough for a
    // workgroup, and the samples the arena budget holds at once make the most
    // waves one sample per workgroup.
    glob = true;
    S = req > 0 ? req : 1;
    if (worst_of(S, true) > (size_t)maxlds) return false;
    const size_t worst = worst_of(S, true);
    if (bwd) { net->S_bwd = S; net->glob_bwd = true; net->lds_bwd = worst; }
    else { net->S_fwd = S; net->glob_fwd = true; net->lds_fwd = worst; }
    return true;
  }
  if (req > 0) {
    S = req;
    glob = worst_of(S, false) > (size_t)maxlds;
    if (glob && worst_of(S, true) > (size_t)maxlds) return false;
  } else {
    for (; S >= 1; S >>= 1)
      if (worst_of(S, false) <= budget) break;
    const int min_lds = bwd ? 4 : 8;
    const int max_glob = bwd ? 8 : (net->rs() == 4 ? 16 : 8);
    if (S < min_lds) {
      glob = true;
      for (S = 64; S >= 1; S >>= 1)
        if (worst_of(S, true) <= budget && S <= max_glob) break;
      if (S < 1) S = 1;
    }
  }
  const size_t worst = worst_of(S, glob);
  if (bwd) { net->S_bwd = S; net->glob_bwd = glob; net->lds_bwd = worst; }
  else { net->S_fwd = S; net->glob_fwd = glob; net->lds_fwd = worst; }
  return true;
}

bool persistent(const tnvan_net *net) { return net->tune.launch_mode == 2; }

// Device arenas of the general kernel above the arena budget are not laid
// out per tile: the launch goes persistent with one arena per workgroup, at
// most as many workgroups as fit (the batch then runs in chunks of that many
// tiles).  The budget is half of the device memory that is free or already
// held by the arena, at most 96 GiB (or the tuned limit).  Returns that workgroup count, or 0
// when one arena per tile fits.
constexpr int64_t kArenaMax = (int64_t)96 << 30;
int arena_cap(const tnvan_net *net, int64_t tile_bytes, int n_tiles) {
  size_t fr = 0, tot = 0;
  int64_t budget = kArenaMax;
  if (hipMemGetInfo(&fr, &tot) == hipSuccess)
    budget = std::min<int64_t>(budget, (int64_t)(fr + net->garena.bytes) / 2);
  if (net->tune.arena_limit_mib > 0)
    budget = std::min<int64_t>(budget, (int64_t)net->tune.arena_limit_mib << 20);
  if (tile_bytes <= 0 || tile_bytes * (int64_t)n_tiles <= budget) return 0;
  return (int)std::max<int64_t>(1, std::min<int64_t>(n_tiles, budget / tile_bytes));
}

// 16-sample groups per wave of the register-resident forward on chains of
// 1-2 tiles (the tuned value, else two when that still leaves a wave per
// SIMD for waves2 two-group waves, else one)
int chain_groups(const tnvan_net *net, int64_t waves2) {
  if (net->tune.chain_groups > 0) return net->tune.chain_groups;
  return waves2 >= 1024 ? 2 : 1;
}

// Every device table compiled from the instances (the program, the
// couplings and fields in their edge classes, the transfer tables of every
// kernel family): written at build, and rewritten in place by
// tnvan_set_couplings (same sizes).  *what names the table that failed.
hipError_t upload_tables(tnvan_net *net, const char **what) {
  HostProgram &P = net->P;
  hipError_t e;
#define UPT(buf, vec) if ((e = upload(net->buf, vec)) != hipSuccess) { *what = #buf; return e; }
  UPT(inst, P.insts) UPT(steps, P.steps) UPT(inputs, P.inputs) UPT(gtab, P.gtab)
  UPT(gtab2, P.gtab2) UPT(edges, P.edges)
  UPT(fld_ptr, P.fld_ptr) UPT(fld_w, P.fld_w) UPT(wr_pos, P.wr_pos) UPT(wr_w, P.wr_w)
  UPT(rr_edge, P.rr_edge) UPT(rr_J, P.rr_J) UPT(wr_edge, P.wr_edge) UPT(wr_J, P.wr_J)
  UPT(hR64, P.hR) UPT(vr, P.vr) UPT(ww_a, P.ww_a) UPT(ww_b, P.ww_b) UPT(ww_J, P.ww_J)
  UPT(hW, P.hW) UPT(d_hw_off, P.hw_off) UPT(ww_e, P.ww_e) UPT(d_wv, P.wv)
  if (net->precision == TNVAN_FP64) {
    UPT(T, P.T) UPT(fld_J, P.fld_J) UPT(hR, P.hR) UPT(esmall, P.esmall)
  } else {
    std::vector<float> t(P.T.begin(), P.T.end()), fj(P.fld_J.begin(), P.fld_J.end()),
        hr(P.hR.begin(), P.hR.end()), es(P.esmall.begin(), P.esmall.end());
    UPT(T, t) UPT(fld_J, fj) UPT(hR, hr) UPT(esmall, es)
  }
  {
    std::vector<float> fj(P.fld_J.begin(), P.fld_J.end()), hr(P.hR.begin(), P.hR.end());
    UPT(fld_J32, fj) UPT(hR32, hr) UPT(fld_wr, P.fld_wr) UPT(cinst, P.cinst)
    UPT(chains, P.chains) UPT(csteps, P.csteps) UPT(Tp, P.Tp) UPT(Tt, P.Tt) UPT(Tb, P.Tb)
  }
  UPT(Tl, P.Tl) UPT(Tbl, P.Tbl) UPT(cedges, P.cedges)
  UPT(Tr, P.Tr) UPT(Tq, P.Tq) UPT(Trb, P.Trb) UPT(xcol, P.xcol)
  UPT(col_out, P.col_out) UPT(pcoef_out, P.pcoef_out)
  UPT(cf_w, P.cf_w) UPT(cf_r, P.cf_r) UPT(cf_J, P.cf_J) UPT(Tsx, P.Tsx) UPT(Ts3, P.Ts3)
  UPT(Tdq, P.Tdq)
#undef UPT
  return hipSuccess;
}

// Whether two compiled programs have the same structure: every table of the
// same size, and the same integers everywhere (steps, edge classes, gather
// tables, chain layouts, output maps).  Values that follow from J, h and
// beta may differ.
template <typename T>
bool same_bytes(const std::vector<T> &a, const std::vector<T> &b) {
  return a.size() == b.size() && (a.empty() || !std::memcmp(a.data(), b.data(), a.size() * sizeof(T)));
}
bool same_structure(const HostProgram &a, const HostProgram &b) {
  if (a.insts.size() != b.insts.size()) return false;
  for (size_t q = 0; q < a.insts.size(); ++q) {
    InstDesc x = a.insts[q];
    x.beta = b.insts[q].beta;
    x.log_const = b.insts[q].log_const;
    if (std::memcmp(&x, &b.insts[q], sizeof(InstDesc))) return false;
  }
  return same_bytes(a.steps, b.steps) && same_bytes(a.inputs, b.inputs) &&
         same_bytes(a.gtab, b.gtab) && same_bytes(a.gtab2, b.gtab2) &&
         same_bytes(a.edges, b.edges) && same_bytes(a.fld_ptr, b.fld_ptr) &&
         same_bytes(a.fld_w, b.fld_w) && same_bytes(a.wr_pos, b.wr_pos) &&
         same_bytes(a.wr_w, b.wr_w) && same_bytes(a.wr_edge, b.wr_edge) &&
         same_bytes(a.rr_edge, b.rr_edge) && same_bytes(a.ww_a, b.ww_a) &&
         same_bytes(a.ww_b, b.ww_b) && same_bytes(a.ww_e, b.ww_e) && same_bytes(a.vr, b.vr) &&
         same_bytes(a.wv, b.wv) && same_bytes(a.hidden, b.hidden) &&
         same_bytes(a.hw_off, b.hw_off) && same_bytes(a.fld_wr, b.fld_wr) &&
         same_bytes(a.cinst, b.cinst) && same_bytes(a.chains, b.chains) &&
         same_bytes(a.csteps, b.csteps) && same_bytes(a.xcol, b.xcol) &&
         same_bytes(a.Tdq, b.Tdq) && same_bytes(a.col_out, b.col_out) &&
         same_bytes(a.cf_w, b.cf_w) && same_bytes(a.cf_r, b.cf_r) &&
         a.T.size() == b.T.size() && a.esmall.size() == b.esmall.size() &&
         a.fld_J.size() == b.fld_J.size() && a.hR.size() == b.hR.size() &&
         a.wr_J.size() == b.wr_J.size() && a.rr_J.size() == b.rr_J.size() &&
         a.ww_J.size() == b.ww_J.size() && a.hW.size() == b.hW.size() &&
         a.Tp.size() == b.Tp.size() && a.Tt.size() == b.Tt.size() && a.Tb.size() == b.Tb.size() &&
         a.Tl.size() == b.Tl.size() && a.Tbl.size() == b.Tbl.size() &&
         a.cedges.size() == b.cedges.size() && a.Tr.size() == b.Tr.size() &&
         a.Tq.size() == b.Tq.size() && a.Trb.size() == b.Trb.size() &&
         a.Tsx.size() == b.Tsx.size() && a.Ts3.size() == b.Ts3.size() &&
         a.pcoef_out.size() == b.pcoef_out.size() && a.cf_J.size() == b.cf_J.size() &&
         a.flops_fwd == b.flops_fwd;
}

tnvan_instance src_view(const tnvan_net::SrcInst &c) {
  tnvan_instance v{};
  v.n_spins = c.n_spins;
  v.n_edges = c.n_edges;
  v.edge_i = c.ei.data();
  v.edge_j = c.ej.data();
  v.J = c.J.data();
  v.h = c.h.data();
  v.beta = c.beta;
  v.n_width = (int32_t)c.W.size();
  v.width_set = c.W.data();
  v.n_order = (int32_t)c.order.size();
  v.order = c.order.data();
  v.n_groups = c.gp.empty() ? 0 : (int32_t)c.gp.size() - 1;
  v.group_ptr = c.gp.empty() ? nullptr : c.gp.data();
  v.hidden = c.hidden;
  v.depth = c.depth;
  return v;
}

tnvan_status set_batch(tnvan_net *net, const int64_t *n_samples) {
  if (!n_samples) return set_err(TNVAN_E_INVALID, "n_samples is NULL");
  std::vector<int64_t> key(n_samples, n_samples + net->n_inst);
  for (auto b : key)
    if (b < 0 || b > ((int64_t)1 << 31)) return set_err(TNVAN_E_INVALID, "bad sample count");
  if (key == net->nkey) return TNVAN_OK;
  if (tnvan_status s = quiesce(net)) return s;
  net->sample_off.assign(net->n_inst, 0);
  net->spin_off.assign(net->n_inst, 0);
  int64_t so = 0, sp = 0;
  for (int q = 0; q < net->n_inst; ++q) {
    net->sample_off[q] = so;
    net->spin_off[q] = sp;
    so += key[q];
    sp += key[q] * net->P.insts[q].nw;
  }
  net->B_total = so;
  net->spin_total = sp;
  HIPCHK(upload(net->d_sample_off, net->sample_off));
  HIPCHK(upload(net->d_B, key));
  HIPCHK(upload(net->d_spin_off, net->spin_off));
  for (int q = 0; q < net->n_inst; ++q) {
    net->mi[q].sample_off = net->sample_off[q];
    net->mi[q].B = key[q];
    net->mi[q].spin_off = net->spin_off[q];
  }
  HIPCHK(upload(net->d_mi, net->mi));
  net->nkey = key;
  net->tc_fwd.key.clear();
  net->tc_bwd.key.clear();
  net->skey.clear();
  net->ckey.clear();
  return TNVAN_OK;
}

tnvan_status ensure_tiles(tnvan_net *net, TileCache &tc, int S, bool bwd) {
  if (tc.key == net->nkey && tc.S == S) return TNVAN_OK;
  if (tnvan_status s = quiesce(net)) return s;
  std::vector<int32_t> ti, ts, first(net->n_inst), cnt(net->n_inst);
  std::vector<int64_t> poff(net->n_inst);
  int64_t ptot = 0;
  // tiles of the instances with the costliest samples first (each
  // instance's tiles stay contiguous): the long tiles start early and the
  // short ones fill the end of the launch
  std::vector<int> by_cost(net->n_inst);
  for (int q = 0; q < net->n_inst; ++q) by_cost[q] = q;
  std::stable_sort(by_cost.begin(), by_cost.end(), [&](int x, int y) {
    return net->P.flops_fwd[x] > net->P.flops_fwd[y];
  });
  for (int q : by_cost) {
    first[q] = (int32_t)ti.size();
    const int64_t B = net->nkey[q];
    if (net->use_chain[q]) {
      cnt[q] = (int32_t)((B + 15) / 16);        // one partial row per 16 samples
    } else {
      for (int64_t b = 0; b < B; b += S) { ti.push_back(q); ts.push_back((int32_t)b); }
      cnt[q] = (int32_t)ti.size() - first[q];
    }
  }
  for (int q = 0; q < net->n_inst; ++q) {
    poff[q] = ptot;
    if (bwd) ptot += (int64_t)cnt[q] * net->P.insts[q].n_partial;
  }
  HIPCHK(upload(tc.tile_inst, ti));
  HIPCHK(upload(tc.tile_start, ts));
  HIPCHK(upload(tc.first_tile, first));
  HIPCHK(upload(tc.n_tiles_i, cnt));
  HIPCHK(upload(tc.partial_off, poff));
  tc.h_first = first;
  tc.h_count = cnt;
  tc.n_tiles = (int)ti.size();
  tc.partial_total = ptot;
  tc.S = S;
  tc.key = net->nkey;
  return TNVAN_OK;
}

// Workgroup tasks of the chain kernels: (instance, chain, first sample) with
// 16 samples per wave; the forward and the adjoint use different waves per
// workgroup, hence two lists.
tnvan_status ensure_chain_tasks(tnvan_net *net) {
  if (net->ckey == net->nkey) return TNVAN_OK;
  if (tnvan_status s = quiesce(net)) return s;
  // two sample groups per forward wave on chains of 1-2 tiles (the groups
  // hide each other's latency) when that still leaves a wave per SIMD;
  // small batches take one group per wave and twice the waves
  {
    int64_t waves2 = 0;
    for (int q = 0; q < net->n_inst; ++q)
      if (net->use_chain[q]) waves2 += net->P.cinst[q].n_chains * ((net->nkey[q] + 31) / 32);
    net->sg = chain_groups(net, waves2);
  }
  std::vector<int32_t> clist;
  std::vector<int64_t> coff(net->n_inst, 0);
  int64_t ctot = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const bool reg = pass ? net->rbwd : net->rfwd;
    std::vector<int32_t> ti, tc, ts;
    for (int q = 0; q < net->n_inst; ++q) {
      if (!net->use_chain[q]) continue;
      const int64_t B = net->nkey[q];
      if (pass == 0) {
        clist.push_back(q);
        coff[q] = ctot;
        ctot += (int64_t)net->P.cinst[q].n_chains * B;
      }
    }
    // register-resident kernels: one task per wave, grouped by chain width
    // (one launch per width); LDS kernels: one task per workgroup
    for (int gi = 0; gi < (reg ? 3 : 1); ++gi) {
      const int rt = 1 << gi;
      int *lo = pass ? net->brg_lo : net->rg_lo, *cnt = pass ? net->brg_n : net->rg_n;
      lo[gi] = (int)ti.size();
      const int per = reg ? 16 * (pass ? 1 : net->sg_of(rt))
                          : 16 * (pass ? net->lim_bwd.wpb : net->lim_fwd.wpb);
      for (int q = 0; q < net->n_inst; ++q) {
        if (!net->use_chain[q]) continue;
        const ChainInst &C = net->P.cinst[q];
        const int64_t B = net->nkey[q];
        for (int64_t b = 0; b < B; b += per)
          for (int c = 0; c < C.n_chains; ++c) {
            const int crt = net->P.chains[C.chain_off + c].rt;
            if (reg && (crt > 4 ? 4 : crt) != rt) continue;
            ti.push_back(q); tc.push_back(c); ts.push_back((int32_t)b);
          }
      }
      cnt[gi] = (int)ti.size() - lo[gi];
    }
    if (pass == 0) {
      HIPCHK(upload(net->task_inst, ti));
      HIPCHK(upload(net->task_chain, tc));
      HIPCHK(upload(net->task_start, ts));
      net->n_tasks = (int)ti.size();
    } else {
      HIPCHK(upload(net->btask_inst, ti));
      HIPCHK(upload(net->btask_chain, tc));
      HIPCHK(upload(net->btask_start, ts));
      net->n_btasks = (int)ti.size();
    }
  }
  HIPCHK(upload(net->cpart_off, coff));
  HIPCHK(upload(net->chain_list, clist));
  {
    // unary factors of the register-resident kernels: [nr][B] floats and
    // [ceil(nr / kUnaryChunk)][B] partial sums per chain instance
    std::vector<int64_t> uo(net->n_inst, 0), fo(net->n_inst, 0);
    int64_t ut = 0, ft = 0;
    net->u_chunks = 0;
    net->u_maxB = 0;
    for (int q : clist) {
      const int64_t B = net->nkey[q];
      const int nr = net->P.insts[q].nr, nch = (nr + kUnaryChunk - 1) / kUnaryChunk;
      uo[q] = ut;
      fo[q] = ft;
      ut += (int64_t)nr * B;
      ft += (int64_t)nch * B;
      net->u_chunks = std::max(net->u_chunks, nch);
      net->u_maxB = std::max(net->u_maxB, B);
    }
    HIPCHK(upload(net->u_off, uo));
    HIPCHK(upload(net->f_off, fo));
    if (net->rfwd || net->rbwd) {
      HIPCHK(net->Ubuf.ensure(std::max<int64_t>(1, ut) * sizeof(float)));
      HIPCHK(net->fabp.ensure(std::max<int64_t>(1, ft) * sizeof(double)));
      // every factor +1 (float bits 0x3f800000): the unary kernel then only
      // writes the positions with a W-neighbour or a field (this runs in an
      // eager call when the batch shape changes, never inside a recording)
      // (complete before any later launch, on whatever stream it comes)
      if (ut > 0) {
        HIPCHK(hipMemsetD32(reinterpret_cast<hipDeviceptr_t>(net->Ubuf.p), 0x3f800000, (size_t)ut));
        HIPCHK(hipDeviceSynchronize());
      }
    }
  }
  HIPCHK(net->cpart.ensure(std::max<int64_t>(1, ctot) * sizeof(double)));
  const ChainLim &L = net->lim_bwd;
  int64_t ckf = 0;
  if (net->rbwd) {
    ckf = (int64_t)net->n_btasks * rchain_ckpt_floats(L);
  } else {
    const int64_t ncp = (L.max_steps + L.kseg - 1) / std::max(1, L.kseg);
    ckf = (int64_t)net->n_btasks * L.wpb * ncp * 16 * L.kbuf;
  }
  HIPCHK(net->ckpt.ensure(std::max<int64_t>(1, ckf) * sizeof(float)));
  net->n_chain_insts = (int)clist.size();
  net->ckey = net->nkey;
  return TNVAN_OK;
}

ChainArgs chain_args(tnvan_net *net, bool bwd) {
  ChainArgs a{};
  a.inst = net->inst.as<InstDesc>();
  a.cinst = net->cinst.as<ChainInst>();
  a.chains = net->chains.as<ChainDesc>();
  a.csteps = net->csteps.as<ChainStep>();
  a.Tp = net->Tp.as<float>();
  a.Tt = net->Tt.as<float>();
  a.Tb = net->Tb.as<uint16_t>();
  a.Tl = net->Tl.as<float>();
  a.Tbl = net->Tbl.as<uint16_t>();
  a.cedges = net->cedges.as<EdgeDesc>();
  a.fld_ptr = net->fld_ptr.as<int32_t>();
  a.fld_w = net->fld_w.as<int32_t>();
  a.fld_wr = net->fld_wr.as<int32_t>();
  a.fld_J = net->fld_J32.as<float>();
  a.hR = net->hR32.as<float>();
  if (bwd) {
    a.task_inst = net->btask_inst.as<int32_t>();
    a.task_chain = net->btask_chain.as<int32_t>();
    a.task_start = net->btask_start.as<int32_t>();
    a.n_tasks = net->n_btasks;
    a.lim = net->lim_bwd;
  } else {
    a.task_inst = net->task_inst.as<int32_t>();
    a.task_chain = net->task_chain.as<int32_t>();
    a.task_start = net->task_start.as<int32_t>();
    a.n_tasks = net->n_tasks;
    a.lim = net->lim_fwd;
  }
  a.inst_B = net->d_B.as<int64_t>();
  a.inst_sample_off = net->d_sample_off.as<int64_t>();
  a.inst_spin_off = net->d_spin_off.as<int64_t>();
  a.cpart_off = net->cpart_off.as<int64_t>();
  a.cpart = net->cpart.as<double>();
  a.ckpt = net->ckpt.as<float>();
  a.bf16 = (!bwd && net->precision == TNVAN_BF16) ? 1 : 0;
  a.ntm = std::max(16, (int)a.lim.kbuf) / 16;
  a.Tr = net->Tr.as<float>();
  a.Tq = net->Tq.as<float>();
  a.Trb = net->Trb.as<uint16_t>();
  a.xcol = net->xcol.as<int32_t>();
  a.Tsx = net->Tsx.as<float>();
  a.Ts3 = net->Ts3.as<uint16_t>();
  a.Tdq = net->Tdq.as<int32_t>();
  a.split = net->split ? 1 : 0;
  a.cf_w = net->cf_w.as<int32_t>();
  a.cf_r = net->cf_r.as<int32_t>();
  a.cf_J = net->cf_J.as<float>();
  a.U = net->Ubuf.as<float>();
  a.u_off = net->u_off.as<int64_t>();
  a.sg = net->sg;
  if (bwd ? net->rbwd : net->rfwd) a.ntm = net->rtiles;
  return a;
}

template <typename real>
ContractArgs<real> contract_args(tnvan_net *net, TileCache &tc, int S) {
  ContractArgs<real> a{};
  a.inst = net->inst.as<InstDesc>();
  a.steps = net->steps.as<StepDesc>();
  a.inputs = net->inputs.as<InputDesc>();
  a.gtab = net->gtab.as<uint16_t>();
  a.gtab2 = net->gtab2.as<uint32_t>();
  a.esmall = net->esmall.as<real>();
  a.edges = net->edges.as<EdgeDesc>();
  a.T = net->T.as<real>();
  a.fld_ptr = net->fld_ptr.as<int32_t>();
  a.fld_w = net->fld_w.as<int32_t>();
  a.fld_J = net->fld_J.as<real>();
  a.hR = net->hR.as<real>();
  a.wr_pos = net->wr_pos.as<int32_t>();
  a.wr_w = net->wr_w.as<int32_t>();
  a.tile_inst = tc.tile_inst.as<int32_t>();
  a.tile_start = tc.tile_start.as<int32_t>();
  a.inst_first_tile = tc.first_tile.as<int32_t>();
  a.inst_sample_off = net->d_sample_off.as<int64_t>();
  a.inst_B = net->d_B.as<int64_t>();
  a.inst_spin_off = net->d_spin_off.as<int64_t>();
  a.inst_partial_off = tc.partial_off.as<int64_t>();
  a.S = S;
  a.logS = ilog2(S);
  a.wide = net->wide ? 1 : 0;
  return a;
}

template <typename real>
tnvan_status run_logz(tnvan_net *net, const int8_t *spins, double *logz, hipStream_t st) {
  Phase ph0(net, "tnvan/logz");
  tnvan_status s = ensure_tiles(net, net->tc_fwd, net->S_fwd, false);
  if (s) return s;
  auto a = contract_args<real>(net, net->tc_fwd, net->S_fwd);
  a.spins = spins;
  a.logz = logz;
  int cap = 0;
  if (net->glob_fwd) {
    int64_t per = 0;
    for (auto &D : net->P.insts) per = std::max(per, contract_garena_entries(D, net->S_fwd, false));
    cap = arena_cap(net, per * (int64_t)sizeof(real), net->tc_fwd.n_tiles);
    HIPCHK(net->garena.ensure((size_t)per * (cap ? cap : net->tc_fwd.n_tiles) * sizeof(real)));
    a.garena = net->garena.as<real>();
    a.garena_stride = per;
    a.arena_per_block = cap > 0;
  }
  a.pq = net->pq.as<int32_t>();
  HIPCHK(launch_contract<real>(a, net->tc_fwd.n_tiles, net->lds_fwd, false, net->glob_fwd, st,
                               persistent(net) || cap > 0, cap));
  if (std::count(net->use_chain.begin(), net->use_chain.end(), 1)) {
    s = ensure_chain_tasks(net);
    if (s) return s;
    ChainArgs c = chain_args(net, false);
    c.spins = spins;
    if (net->rfwd) {
      {
        Phase ph(net, "tnvan/boundary");
        HIPCHK(launch_unary(c, net->chain_list.as<int32_t>(), net->n_chain_insts, net->u_chunks,
                            net->u_maxB, net->f_off.as<int64_t>(), net->Ubuf.as<float>(),
                            net->fabp.as<double>(), st));
      }
      Phase ph(net, "tnvan/steps");
      if (persistent(net)) {
        c.pq = net->pq.as<int32_t>() + 4;
        for (int gi = 0; gi < 3; ++gi) { c.pq_lo[gi] = net->rg_lo[gi]; c.pq_n[gi] = net->rg_n[gi]; }
        c.sg = net->sg;
        ProfScope ps(net, TNVAN_KERNEL_CHAIN_FWD_ALL, st);
        HIPCHK(launch_rchain_pq(c, false, st));
      } else {
        for (int gi = 0; gi < 3; ++gi) {
          c.task_base = net->rg_lo[gi];
          c.n_tasks = net->rg_n[gi];
          c.ntm = 1 << gi;
          c.sg = net->sg_of(1 << gi);
          if (c.n_tasks <= 0) continue;
          ProfScope ps(net, TNVAN_KERNEL_CHAIN_FWD_1 + gi, st);
          HIPCHK(launch_rchain(c, false, st));
        }
      }
    } else {
      HIPCHK(launch_chain(c, false, st));
    }
    HIPCHK(launch_chain_sum(net->inst.as<InstDesc>(), net->cinst.as<ChainInst>(),
                            net->chain_list.as<int32_t>(), net->n_chain_insts,
                            net->d_B.as<int64_t>(), net->d_sample_off.as<int64_t>(),
                            net->cpart_off.as<int64_t>(), net->cpart.as<double>(),
                            net->f_off.as<int64_t>(),
                            net->rfwd ? net->fabp.as<double>() : nullptr, logz, st));
  }
  return TNVAN_OK;
}

// logZ from the adjoint's own forward pass: FP32 nets whose every instance
// runs the register-resident chain kernels (their adjoint forward pass is the
// forward kernel's arithmetic, so logz is the same as tnvan_logz_batch's)
bool logz_with_adjoint(const tnvan_net *net) {
  // (BF16 nets: their forward rounds the step products to BF16, their
  // adjoint does not, so logZ keeps its own pass)
  if (net->precision == TNVAN_BF16) return false;
  // chain instances on the register-resident kernels, whose adjoint runs the
  // forward kernel's arithmetic first; the general kernel's adjoint sweeps
  // forward the same way as its forward pass
  for (int q = 0; q < net->n_inst; ++q)
    if (net->use_chain[q] && (!net->rfwd || !net->rbwd)) return false;
  return true;
}
bool all_chains(const tnvan_net *net) {
  for (int q = 0; q < net->n_inst; ++q)
    if (!net->use_chain[q]) return false;
  return true;
}

// the adjoint; with logz (only where logz_with_adjoint holds) also logZ
template <typename real>
tnvan_status run_backward(tnvan_net *net, const int8_t *spins, const double *grad,
                          double *dh, double *dJ, double *dbeta, hipStream_t st,
                          double *logz = nullptr) {
  Phase ph0(net, "tnvan/adjoint");
  tnvan_status s = ensure_tiles(net, net->tc_bwd, net->S_bwd, true);
  if (s) return s;
  TileCache &tc = net->tc_bwd;
  auto a = contract_args<real>(net, tc, net->S_bwd);
  a.spins = spins;
  a.grad = grad;
  HIPCHK(net->partial.ensure(std::max<int64_t>(1, tc.partial_total) * sizeof(real)));
  a.partial = net->partial.as<real>();
  int cap = 0;
  if (net->glob_bwd) {
    int64_t per = 0;
    for (auto &D : net->P.insts) per = std::max(per, contract_garena_entries(D, net->S_bwd, true));
    cap = arena_cap(net, per * (int64_t)sizeof(real), tc.n_tiles);
    HIPCHK(net->garena.ensure((size_t)per * (cap ? cap : tc.n_tiles) * sizeof(real)));
    a.garena = net->garena.as<real>();
    a.garena_stride = per;
    a.arena_per_block = cap > 0;
  }
  a.pq = net->pq.as<int32_t>() + 2;
  a.logz = logz;
  HIPCHK(launch_contract<real>(a, tc.n_tiles, net->lds_bwd, true, net->glob_bwd, st,
                               persistent(net) || cap > 0, cap));
  if (std::count(net->use_chain.begin(), net->use_chain.end(), 1)) {
    s = ensure_chain_tasks(net);
    if (s) return s;
    ChainArgs c = chain_args(net, true);
    c.spins = spins;
    c.grad = grad;
    c.partial = reinterpret_cast<float *>(net->partial.p);
    c.inst_partial_off = tc.partial_off.as<int64_t>();
    if (net->rbwd) {
      {
        Phase ph(net, "tnvan/boundary");
        HIPCHK(launch_unary(c, net->chain_list.as<int32_t>(), net->n_chain_insts, net->u_chunks,
                            net->u_maxB, net->f_off.as<int64_t>(), net->Ubuf.as<float>(),
                            net->fabp.as<double>(), st));
      }
      if (persistent(net)) {
        c.pq = net->pq.as<int32_t>() + 6;
        for (int gi = 0; gi < 3; ++gi) { c.pq_lo[gi] = net->brg_lo[gi]; c.pq_n[gi] = gi < 2 ? net->brg_n[gi] : 0; }
        ProfScope ps(net, TNVAN_KERNEL_CHAIN_BWD_ALL, st);
        HIPCHK(launch_rchain_pq(c, true, st));
      } else {
        for (int gi = 0; gi < 2; ++gi) {
          c.task_base = net->brg_lo[gi];
          c.n_tasks = net->brg_n[gi];
          c.ntm = 1 << gi;
          if (c.n_tasks <= 0) continue;
          ProfScope ps(net, TNVAN_KERNEL_CHAIN_BWD_1 + gi, st);
          HIPCHK(launch_rchain(c, true, st));
        }
      }
      if (logz)
        HIPCHK(launch_chain_sum(net->inst.as<InstDesc>(), net->cinst.as<ChainInst>(),
                                net->chain_list.as<int32_t>(), net->n_chain_insts,
                                net->d_B.as<int64_t>(), net->d_sample_off.as<int64_t>(),
                                net->cpart_off.as<int64_t>(), net->cpart.as<double>(),
                                net->f_off.as<int64_t>(), net->fabp.as<double>(), logz, st));
    } else {
      HIPCHK(launch_chain(c, true, st));
    }
  }
  VjpArgs v{};
  v.inst = net->inst.as<InstDesc>();
  v.rr_edge = net->rr_edge.as<int32_t>();
  v.rr_J = net->rr_J.as<double>();
  v.wr_edge = net->wr_edge.as<int32_t>();
  v.wr_J = net->wr_J.as<double>();
  v.hR = net->hR64.as<double>();
  v.vr = net->vr.as<int32_t>();
  v.inst_first_tile = tc.first_tile.as<int32_t>();
  v.inst_n_tiles = tc.n_tiles_i.as<int32_t>();
  v.inst_partial_off = tc.partial_off.as<int64_t>();
  v.inst_spin_base = net->d_spin_base.as<int64_t>();
  v.inst_edge_base = net->d_edge_base.as<int64_t>();
  v.dh = dh;
  v.dJ = dJ;
  v.dbeta = dbeta;
  v.inst_sum_off = net->d_sum_off.as<int64_t>();
  v.part2 = net->vjp_part.as<double>();
  v.maxo = net->max_out;
  v.col_out = net->col_out.as<int32_t>();
  v.pcoef_out = net->pcoef_out.as<double>();
  HIPCHK(launch_vjp_reduce<real>(v, net->partial.as<real>(), net->n_inst, net->max_partial, st));
  return TNVAN_OK;
}

tnvan_status ensure_sample_blocks(tnvan_net *net) {
  if (net->skey == net->nkey) return TNVAN_OK;
  if (tnvan_status s = quiesce(net)) return s;
  {
    // matrix-core sampler: one wave per 16 samples
    std::vector<int32_t> ti, ts;
    for (int q = 0; q < net->n_inst; ++q)
      for (int64_t b = 0; b < net->nkey[q]; b += 16) { ti.push_back(q); ts.push_back((int32_t)b); }
    HIPCHK(upload(net->mtask_inst, ti));
    HIPCHK(upload(net->mtask_start, ts));
    net->n_mtasks = (int)ti.size();
    // fused REINFORCE backward: one workgroup per mgrad_task_samples samples
    const int tsz = mgrad_task_samples(net->split && net->mpt <= 2);
    std::vector<int32_t> gi, gs, gf(net->n_inst), gc(net->n_inst);
    for (int q = 0; q < net->n_inst; ++q) {
      gf[q] = (int32_t)gi.size();
      for (int64_t b = 0; b < net->nkey[q]; b += tsz) { gi.push_back(q); gs.push_back((int32_t)b); }
      gc[q] = (int32_t)gi.size() - gf[q];
    }
    HIPCHK(upload(net->mg_task_inst, gi));
    HIPCHK(upload(net->mg_task_start, gs));
    HIPCHK(upload(net->mg_first, gf));
    HIPCHK(upload(net->mg_count, gc));
    net->n_mgtasks = (int)gi.size();
  }
  net->h_blk_inst.clear();
  net->h_blk_start.clear();
  const int spb = 256 / net->mi[0].L;
  int64_t groups = 0;
  for (int q = 0; q < net->n_inst; ++q) groups += (net->nkey[q] + spb - 1) / spb;
  // a few rounds per block so that each block stages its parameters once;
  // parameters too large to stage are read from global memory, and then
  // more, shorter blocks keep more waves in flight (the sampler is bound by
  // the latency of its position-by-position chain)
  size_t stage = 0;
  for (auto &m : net->mi) stage = std::max(stage, made_param_bytes(m.n, m.H));
  const int64_t target = stage <= made_stage_max() ? 512 : 8192;
  net->sample_reps = (int)std::max<int64_t>(1, (groups + target - 1) / target);
  const int64_t per_block = (int64_t)spb * net->sample_reps;
  for (int q = 0; q < net->n_inst; ++q) {
    for (int64_t b = 0; b < net->nkey[q]; b += per_block) {
      net->h_blk_inst.push_back(q);
      net->h_blk_start.push_back((int32_t)b);
    }
  }
  HIPCHK(upload(net->blk_inst, net->h_blk_inst));
  HIPCHK(upload(net->blk_start, net->h_blk_start));
  net->n_sblocks = (int)net->h_blk_inst.size();
  net->skey = net->nkey;
  return TNVAN_OK;
}

template <typename real>
tnvan_status run_sample(tnvan_net *net, const float *uniforms, int8_t *spins, void *logq,
                        hipStream_t st) {
  Phase ph0(net, "tnvan/sample");
  tnvan_status s = ensure_sample_blocks(net);
  if (s) return s;
  if ((net->msample || net->mgrad) && sizeof(real) == 4) {
    // parameters repacked for the matrix-core sampler and backward, unless
    // the tables already hold them
    const void *had = net->mpack.p;
    HIPCHK(net->mpack.ensure((std::max<int64_t>(1, net->mpack_total) + 16) * sizeof(float)));
    if (net->mpack.p != had) net->pack_valid = false;
    if (!net->pack_valid) {
      HIPCHK(launch_made_pack(net->d_mi.as<MadeInst>(), net->n_inst, net->mpack_max,
                              net->params.as<float>(), net->mpack.as<float>(), net->mpt, st));
      net->pack_valid = true;
    }
  }
  if (net->msample && sizeof(real) == 4) {
    MSampleArgs m{};
    m.mi = net->d_mi.as<MadeInst>();
    m.pack = net->mpack.as<float>();
    m.task_inst = net->mtask_inst.as<int32_t>();
    m.task_start = net->mtask_start.as<int32_t>();
    m.n_tasks = net->n_mtasks;
    m.uniforms = uniforms;
    m.spins = spins;
    m.logq = reinterpret_cast<float *>(logq);
    m.seed = net->seed;
    m.step_ctr = net->step_ctr.as<int32_t>();
    {
      ProfScope ps(net, TNVAN_KERNEL_SAMPLE, st);
      HIPCHK(launch_msample(m, net->mpt, st));
    }
    return TNVAN_OK;
  }
  SampleArgs<real> a{};
  a.mi = net->d_mi.as<MadeInst>();
  a.params = net->params.as<float>();
  a.uniforms = uniforms;
  if (net->deep) {
    // deeper networks: a wave per sample, every instance
    a.spins = spins;
    a.logq = static_cast<real *>(logq);
    a.seed = net->seed;
    a.step_ctr = net->step_ctr.as<int32_t>();
    int64_t maxB = 0;
    for (int q = 0; q < net->n_inst; ++q) maxB = std::max(maxB, net->nkey[q]);
    ProfScope ps(net, TNVAN_KERNEL_SAMPLE, st);
    // small networks: 16 lanes per sample
    bool small = true;
    for (auto &m : net->mi)
      if (m.n > kDeep16MaxN || m.H > kDeep16MaxH) small = false;
    HIPCHK(launch_sample_deep<real>(a, net->n_inst, maxB, small, st));
    return TNVAN_OK;
  }
  if (net->h0) {
    // the current parameters' columns of W0, then a wave per sample
    a.spins = spins;
    a.logq = static_cast<real *>(logq);
    a.seed = net->seed;
    a.step_ctr = net->step_ctr.as<int32_t>();
    a.w0t = net->w0t.as<float>();
    a.w0t_off = net->d_w0t_off.as<int64_t>();
    HIPCHK(net->w_sig.ensure((size_t)std::max<int64_t>(1, net->spin_total) * sizeof(real)));
    a.sig = net->w_sig.as<real>();
    int64_t maxB = 0;
    for (int q = 0; q < net->n_inst; ++q) maxB = std::max(maxB, net->nkey[q]);
    HIPCHK(launch_w0t(a.mi, net->n_inst, net->h0_nmax, a.params, a.w0t_off, net->w0t.as<float>(),
                      st));
    ProfScope ps(net, TNVAN_KERNEL_SAMPLE, st);
    HIPCHK(launch_sample_h0<real>(a, net->n_inst, maxB, net->h0_nmax, st));
    return TNVAN_OK;
  }
  a.blk_inst = net->blk_inst.as<int32_t>();
  a.blk_start = net->blk_start.as<int32_t>();
  a.spins = spins;
  a.logq = static_cast<real *>(logq);
  a.seed = net->seed;
  a.step_ctr = net->step_ctr.as<int32_t>();
  a.spb = 256 / net->mi[0].L;      // every instance uses the same lane count
  a.reps = net->sample_reps;
  size_t stage = 0;
  for (auto &m : net->mi) stage = std::max(stage, made_param_bytes(m.n, m.H));
  HIPCHK(launch_sample<real>(a, net->n_sblocks, stage, st));
  return TNVAN_OK;
}

// outputs of the adjoint of the sampled batch (tnvan_free_energy_step_adjoint)
struct StepAdjoint {
  const double *grad = nullptr;
  double *dh = nullptr, *dJ = nullptr, *dbeta = nullptr;
};

// The batch sums of the REINFORCE backward as jobs (one per instance and
// matrix, each with its own slices of the partial sums), laid out once per
// batch shape and row-buffer addresses
template <typename real>
tnvan_status ensure_batch_sums(tnvan_net *net, const std::vector<int64_t> &hoff,
                               const std::vector<int64_t> &doff, BatchSums<real> *out) {
  std::vector<int64_t> key(net->nkey);
  for (const void *p : {net->w_hid.p, net->w_da.p, net->w_dlogit.p, net->w_sf.p, net->grad.p})
    key.push_back((int64_t)reinterpret_cast<uintptr_t>(p));
  key.push_back((int64_t)sizeof(real));
  if (key != net->bkey) {
    std::vector<AtbJob<real>> aj;
    std::vector<ColJob<real>> cj;
    std::vector<int32_t> alo{0}, aflo{0}, clo{0}, cflo{0};
    int64_t ptot = 0;
    auto atb = [&](const real *X, int ldx, const real *Y, int ldy, int64_t B, int M, int N,
                   int ks, float *o, int ldo, int mask, int nW) {
      if (M <= 0 || N <= 0) return;
      AtbJob<real> j{X, Y, o, ptot, B, ldx, ldy, M, N, ks, ldo, mask, nW};
      ptot += (int64_t)ks * M * N;
      int32_t b = 0, f = 0;
      batch_sum_blocks(M, N, ks, &b, &f);
      aj.push_back(j);
      alo.push_back(alo.back() + b);
      aflo.push_back(aflo.back() + f);
    };
    auto col = [&](const real *X, int ldx, int64_t B, int M, int ks, float *o) {
      if (M <= 0) return;
      ColJob<real> j{X, o, ptot, B, ldx, M, ks, 0};
      ptot += (int64_t)ks * M;
      int32_t b = 0, f = 0;
      batch_col_blocks(M, ks, &b, &f);
      cj.push_back(j);
      clo.push_back(clo.back() + b);
      cflo.push_back(cflo.back() + f);
    };
    for (int q = 0; q < net->n_inst; ++q) {
      const MadeInst &m = net->mi[q];
      if (m.B <= 0) continue;
      const int n = m.n, H = m.H;
      const int D = (net->deep && n >= 2 && H > 0) ? m.D : 1;
      const real *hid = net->w_hid.as<real>() + hoff[q], *da = net->w_da.as<real>() + hoff[q];
      const real *dl = net->w_dlogit.as<real>() + doff[q], *sf = net->w_sf.as<real>() + doff[q];
      // batch slices of at least 64 rows, at most 64 slices
      const int ks = (int)std::max<int64_t>(1, std::min<int64_t>(64, m.B / 64));
      float *g = net->grad.as<float>() + m.param_off;
      float *gW1 = g, *gb1 = g + (int64_t)H * n, *gW2 = gb1 + H, *gb2 = gW2 + (int64_t)n * H,
            *gW0 = gb2 + n;
      if (H > 0) {
        // rows of D H: layer l at column (l - 1) H; the logits read layer D
        const int DH = D * H;
        atb(dl, n, hid + (int64_t)(D - 1) * H, DH, m.B, n, H, ks, gW2, H, 1, n);
        atb(da, DH, sf, n, m.B, H, n, ks, gW1, n, 3, n);
        col(da, DH, m.B, H, ks, gb1);
        // deeper layers l = 2..D after W0: W^l [H, H] (da^l against h^{l-1}), b^l
        float *gl = gW0 + (int64_t)n * n;
        for (int l = 2; l <= D; ++l, gl += (int64_t)H * H + H) {
          atb(da + (int64_t)(l - 1) * H, DH, hid + (int64_t)(l - 2) * H, DH, m.B, H, H, ks, gl, H,
              4, n);
          col(da + (int64_t)(l - 1) * H, DH, m.B, H, ks, gl + (int64_t)H * H);
        }
      }
      atb(dl, n, sf, n, m.B, n, n, ks, gW0, n, 2, n);
      col(dl, n, m.B, n, ks, gb2);
    }
    // one-layer nets: the per-sample rows, jobs in classes of LDS need
    // (staged parameters <= 40 KB, <= 80 KB, <= the device's block limit,
    // parameters read from global memory), one launch per class
    std::vector<RowJob> rj[4];
    std::vector<int32_t> rlo[4] = {{0}, {0}, {0}, {0}};
    size_t rlds[4] = {0, 0, 0, 0};
    if (!net->deep && !net->h0) {
      int dev = 0, maxlds = 65536;
      hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
      const size_t lim[3] = {40 * 1024, 80 * 1024, (size_t)maxlds};
      for (int q = 0; q < net->n_inst; ++q) {
        const MadeInst &m = net->mi[q];
        if (m.B <= 0) continue;
        const size_t need = rows_lds_bytes(m.n, m.H, sizeof(real), true);
        int c = 0;
        while (c < 3 && need > lim[c]) ++c;
        const size_t lds = rows_lds_bytes(m.n, m.H, sizeof(real), c < 3);
        if (lds > (size_t)maxlds)
          return set_err(TNVAN_E_INVALID, "instance %d: the REINFORCE rows of |W| = %d, H = %d "
                         "need %zu bytes of LDS per block, above the device's %d", q, m.n, m.H,
                         lds, maxlds);
        // samples per block: one round of 16 for small parameter sets, up
        // to four rounds per staging of the larger ones, and at most 256
        // blocks per instance
        const int64_t wb = (int64_t)(need - rows_lds_bytes(m.n, m.H, sizeof(real), false));
        int64_t chunk = 16 * std::min<int64_t>(4, std::max<int64_t>(1, (wb + 32767) / 32768));
        chunk = std::max<int64_t>(chunk, ((m.B + 255) / 256 + 15) / 16 * 16);
        const int64_t blocks = (m.B + chunk - 1) / chunk;
        if (rlo[c].back() + blocks > 0x7fffffff)
          return set_err(TNVAN_E_INVALID, "instance %d: %lld rows blocks", q, (long long)blocks);
        rj[c].push_back(RowJob{q, (int32_t)chunk, hoff[q], doff[q]});
        rlo[c].push_back(rlo[c].back() + (int32_t)blocks);
        rlds[c] = std::max(rlds[c], lds);
      }
    }
    if (tnvan_status s = quiesce(net)) return s;
    for (int c = 0; c < 4; ++c) {
      HIPCHK(upload(net->rw_jobs[c], rj[c]));
      HIPCHK(upload(net->rw_lo[c], rlo[c]));
      net->rw_njobs[c] = (int32_t)rj[c].size();
      net->rw_blocks[c] = rlo[c].back();
      net->rw_lds[c] = rlds[c];
    }
    HIPCHK(upload(net->bs_atb, aj));
    HIPCHK(upload(net->bs_col, cj));
    HIPCHK(upload(net->bs_alo, alo));
    HIPCHK(upload(net->bs_aflo, aflo));
    HIPCHK(upload(net->bs_clo, clo));
    HIPCHK(upload(net->bs_cflo, cflo));
    HIPCHK(net->w_part.ensure((size_t)std::max<int64_t>(1, ptot) * sizeof(real)));
    net->bs_counts[0] = (int)aj.size();
    net->bs_counts[1] = (int)cj.size();
    net->bs_counts[2] = alo.back();
    net->bs_counts[3] = aflo.back();
    net->bs_counts[4] = clo.back();
    net->bs_counts[5] = cflo.back();
    net->bkey = key;
  }
  BatchSums<real> &a = *out;
  a.atb = net->bs_atb.as<AtbJob<real>>();
  a.atb_lo = net->bs_alo.as<int32_t>();
  a.atb_flo = net->bs_aflo.as<int32_t>();
  a.n_atb = net->bs_counts[0];
  a.col = net->bs_col.as<ColJob<real>>();
  a.col_lo = net->bs_clo.as<int32_t>();
  a.col_flo = net->bs_cflo.as<int32_t>();
  a.n_col = net->bs_counts[1];
  a.atb_blocks = net->bs_counts[2];
  a.atb_fblocks = net->bs_counts[3];
  a.col_blocks = net->bs_counts[4];
  a.col_fblocks = net->bs_counts[5];
  a.part = net->w_part.as<real>();
  return TNVAN_OK;
}

template <typename real>
tnvan_status run_step(tnvan_net *net, float lr, double *stats, int8_t *spins_out,
                      hipStream_t st, const StepAdjoint *adj = nullptr) {
  Phase ph0(net, "tnvan/step");
  const int64_t B = net->B_total;
  HIPCHK(net->w_spins.ensure(std::max<int64_t>(1, net->spin_total)));
  HIPCHK(net->w_logz.ensure(std::max<int64_t>(1, B) * 8));
  HIPCHK(net->w_logq.ensure(std::max<int64_t>(1, B) * sizeof(real)));
  HIPCHK(net->w_f.ensure(std::max<int64_t>(1, B) * 8));
  int8_t *spins = spins_out ? spins_out : net->w_spins.as<int8_t>();
  tnvan_status s = run_sample<real>(net, nullptr, spins, net->w_logq.p, st);
  if (s) return s;
  // with the adjoint requested, logZ comes from its forward pass when the
  // net allows it (one contraction instead of two), else it follows the step
  // (the free-energy kernel then sums the chain partials itself)
  const bool adj_logz = adj && logz_with_adjoint(net);
  // (chain-only nets leave logZ as chain partials, which the free-energy
  // kernel sums itself; with general instances the adjoint writes it out)
  const bool cpart_logz = adj_logz && all_chains(net);
  if (adj_logz)
    s = run_backward<real>(net, spins, adj->grad, adj->dh, adj->dJ, adj->dbeta, st,
                           cpart_logz ? nullptr : net->w_logz.as<double>());
  else
    s = run_logz<real>(net, spins, net->w_logz.as<double>(), st);
  if (s) return s;
  // f_b and the batch statistics of every instance (Eq. 9)
  int64_t Bmax = 1;
  for (int q = 0; q < net->n_inst; ++q) Bmax = std::max(Bmax, net->nkey[q]);
  FreeArgs<real> f{};
  f.inst = net->inst.as<InstDesc>();
  f.mi = net->d_mi.as<MadeInst>();
  f.hw_off = net->d_hw_off.as<int32_t>();
  f.spins = spins;
  f.logz = net->w_logz.as<double>();
  if (cpart_logz) {
    f.cinst = net->cinst.as<ChainInst>();
    f.cpart_off = net->cpart_off.as<int64_t>();
    f.cpart = net->cpart.as<double>();
    f.f_off = net->f_off.as<int64_t>();
    f.fabp = net->fabp.as<double>();
  }
  f.logq = net->w_logq.as<real>();
  f.ww_a = net->ww_a.as<int32_t>();
  f.ww_b = net->ww_b.as<int32_t>();
  f.ww_J = net->ww_J.as<double>();
  f.hW = net->hW.as<double>();
  f.f = net->w_f.as<double>();
  f.nblk = (int)std::min<int64_t>(256, (4 * Bmax + 255) / 256);   // 4 lanes per sample
  HIPCHK(net->w_fpart.ensure((size_t)net->n_inst * f.nblk * 4 * sizeof(double)));
  f.part = net->w_fpart.as<double>();
  f.stats = stats;
  f.done = net->tickets.as<int32_t>();
  // with the fused backward, its workgroups sum the block sums themselves
  const bool fused = net->mgrad && sizeof(real) == 4;
  f.finish = !fused;
  f.step_ctr = net->step_ctr.as<int32_t>();
  f.nonfinite = net->nonfinite.as<int32_t>();
  {
    Phase ph(net, "tnvan/free_energy");
    HIPCHK(launch_free<real>(f, net->n_inst, st));
  }
  // Adam on every instance (one launch, after the REINFORCE gradient)
  OptArgs o{};
  o.mi = net->d_mi.as<MadeInst>();
  o.params = net->params.as<float>();
  o.grad = net->grad.as<float>();
  o.m = net->adam_m.as<float>();
  o.v = net->adam_v.as<float>();
  o.pack = (net->msample || net->mgrad) && sizeof(real) == 4 ? net->mpack.as<float>() : nullptr;
  o.npt = net->mpt;
  o.lr = lr;
  o.step_ctr = net->step_ctr.as<int32_t>();
  if (net->mgrad && sizeof(real) == 4) {
    // fused REINFORCE backward of every instance (Eq. 10)
    HIPCHK(net->w_part.ensure(std::max<int64_t>(1, (int64_t)net->n_mgtasks * net->mg_pstride) *
                              sizeof(float)));
    MGradArgs g{};
    g.mi = net->d_mi.as<MadeInst>();
    g.n_inst = net->n_inst;
    g.hmax = net->mg_hmax;
    g.params = net->params.as<float>();
    g.spins = spins;
    g.f = net->w_f.as<double>();
    g.stats = stats;
    g.fpart = f.part;
    g.fnblk = f.nblk;
    g.task_inst = net->mg_task_inst.as<int32_t>();
    g.task_start = net->mg_task_start.as<int32_t>();
    g.n_tasks = net->n_mgtasks;
    g.split = net->split && net->mpt <= 2 ? 1 : 0;
    g.part = net->w_part.as<float>();
    g.pstride = net->mg_pstride;
    g.first_row = net->mg_first.as<int32_t>();
    g.n_rows = net->mg_count.as<int32_t>();
    g.pack = net->mpack.as<float>();
    g.grad = net->grad.as<float>();
    {
      Phase ph(net, "tnvan/reinforce");
      ProfScope ps(net, TNVAN_KERNEL_MADE_GRAD, st);
      HIPCHK(launch_mgrad(g, net->mpt, st));
    }
    int64_t max_pc = 1;
    for (auto pc : net->param_count) max_pc = std::max(max_pc, pc);
    Phase ph(net, "tnvan/adam");
    HIPCHK(launch_grad_adam(g, o, max_pc, st));
  }
  {
  Phase ph_rf(net, "tnvan/reinforce", !fused);
  if (!fused) {
    // REINFORCE backward through q (Eq. 10): per-sample rows of every
    // instance into its own slice of the row buffers, then the batch sums of
    // every instance and matrix in one launch per kind
    std::vector<int64_t> hoff(net->n_inst, 0), doff(net->n_inst, 0);
    int64_t htot = 0, dtot = 0;
    for (int q = 0; q < net->n_inst; ++q) {
      const MadeInst &m = net->mi[q];
      const int D = (net->deep && m.n >= 2 && m.H > 0) ? m.D : 1;
      hoff[q] = htot;
      doff[q] = dtot;
      if (m.B <= 0) continue;
      htot += m.B * D * m.H;
      dtot += m.B * m.n;
    }
    HIPCHK(net->w_hid.ensure(std::max<int64_t>(1, htot) * sizeof(real)));
    HIPCHK(net->w_da.ensure(std::max<int64_t>(1, htot) * sizeof(real)));
    HIPCHK(net->w_dlogit.ensure(std::max<int64_t>(1, dtot) * sizeof(real)));
    HIPCHK(net->w_sf.ensure(std::max<int64_t>(1, dtot) * sizeof(real)));
    BatchSums<real> bs{};
    if (tnvan_status s2 = ensure_batch_sums<real>(net, hoff, doff, &bs)) return s2;
    for (int q = 0; q < net->n_inst; ++q) {
      const MadeInst &m = net->mi[q];
      if (m.B <= 0 || !(net->deep || net->h0)) continue;
      const int n = m.n, H = m.H;
      // hidden layers run (deeper networks hold every layer in a row)
      const int D = (net->deep && n >= 2 && H > 0) ? m.D : 1;
      RowArgs<real> r{};
      r.mi = m;
      r.params = net->params.as<float>();
      r.spins = spins + m.spin_off;
      r.f = net->w_f.as<double>();
      r.stats = stats + 4 * q;
      r.chunk = std::max<int64_t>(16, ((m.B + 255) / 256 + 15) / 16 * 16);
      r.hid = net->w_hid.as<real>() + hoff[q];
      r.da = net->w_da.as<real>() + hoff[q];
      r.dlogit = net->w_dlogit.as<real>() + doff[q];
      r.sf = net->w_sf.as<real>() + doff[q];
      if (net->deep) {
        // rows of at most 4096 / H samples and about 48 KB of LDS per round
        const size_t per = sizeof(real) * (2 * (size_t)n + (size_t)D * H + H);
        // (8 rows per block and one round each: every sample's rows are
        // independent, and the block count fills the CUs)
        const int rb = (int)std::max<int64_t>(1, std::min<int64_t>({8, 4096 / std::max(1, H),
                                                                    (int64_t)(49152 / per)}));
        r.chunk = rb;
        HIPCHK(launch_rows_deep<real>(r, rb, st));
      } else if (net->h0) {
        // the conditionals the sampler stored for these spins and parameters
        r.sig = net->w_sig.as<real>() + m.spin_off;
        HIPCHK(launch_rows_h0<real>(r, st));
      }
    }
    if (!net->deep && !net->h0) {
      RowBatch<real> rb{};
      rb.mi = net->d_mi.as<MadeInst>();
      rb.params = net->params.as<float>();
      rb.spins = spins;
      rb.f = net->w_f.as<double>();
      rb.stats = stats;
      rb.hid = net->w_hid.as<real>();
      rb.da = net->w_da.as<real>();
      rb.dlogit = net->w_dlogit.as<real>();
      rb.sf = net->w_sf.as<real>();
      // more waves per block where the LDS need leaves fewer blocks per CU
      const int threads[4] = {256, 512, 1024, 1024};
      for (int c = 0; c < 4; ++c) {
        rb.jobs = net->rw_jobs[c].as<RowJob>();
        rb.lo = net->rw_lo[c].as<int32_t>();
        rb.n_jobs = net->rw_njobs[c];
        rb.blocks = net->rw_blocks[c];
        HIPCHK(launch_rows_batch<real>(rb, c < 3, net->rw_lds[c], threads[c], st));
      }
    }
    HIPCHK(launch_batch_sums<real>(bs, st));
  }
  }
  if (!fused) {
    int64_t max_pc = 1;
    for (auto pc : net->param_count) max_pc = std::max(max_pc, pc);
    Phase ph(net, "tnvan/adam");
    HIPCHK(launch_adam_step(o, net->n_inst, max_pc, st));
  }
  if (adj && !adj_logz) return run_backward<real>(net, spins, adj->grad, adj->dh, adj->dJ, adj->dbeta, st);
  return TNVAN_OK;
}

// logZ, f_b (Eq. 9; the step counter is not advanced) and the
// self-normalised importance weights of the batch: w_og = w_b / beta, ess
// per instance.  *o is left set up for obs_w_kernel.
template <typename real>
tnvan_status obs_weights(tnvan_net *net, const int8_t *spins, const void *logq, double *ess,
                         ObsArgs *o, hipStream_t st) {
  const int64_t B = net->B_total;
  HIPCHK(net->w_logz.ensure(std::max<int64_t>(1, B) * 8));
  HIPCHK(net->w_f.ensure(std::max<int64_t>(1, B) * 8));
  HIPCHK(net->w_og.ensure(std::max<int64_t>(1, B) * 8));
  HIPCHK(net->w_ostats.ensure((size_t)net->n_inst * 4 * sizeof(double)));
  HIPCHK(net->w_odb.ensure((size_t)net->n_inst * sizeof(double)));
  if (tnvan_status s = run_logz<real>(net, spins, net->w_logz.as<double>(), st)) return s;
  // f_b (Eq. 9); the step counter is not advanced
  int64_t Bmax = 1;
  for (int q = 0; q < net->n_inst; ++q) Bmax = std::max(Bmax, net->nkey[q]);
  FreeArgs<real> f{};
  f.inst = net->inst.as<InstDesc>();
  f.mi = net->d_mi.as<MadeInst>();
  f.hw_off = net->d_hw_off.as<int32_t>();
  f.spins = spins;
  f.logz = net->w_logz.as<double>();
  f.logq = static_cast<const real *>(logq);
  f.ww_a = net->ww_a.as<int32_t>();
  f.ww_b = net->ww_b.as<int32_t>();
  f.ww_J = net->ww_J.as<double>();
  f.hW = net->hW.as<double>();
  f.f = net->w_f.as<double>();
  f.nblk = (int)std::min<int64_t>(256, (4 * Bmax + 255) / 256);
  HIPCHK(net->w_fpart.ensure((size_t)net->n_inst * f.nblk * 4 * sizeof(double)));
  f.part = net->w_fpart.as<double>();
  f.finish = 1;
  f.stats = net->w_ostats.as<double>();
  f.done = net->tickets.as<int32_t>();
  f.step_ctr = nullptr;
  HIPCHK(launch_free<real>(f, net->n_inst, st));
  *o = ObsArgs{};
  o->inst = net->inst.as<InstDesc>();
  o->mi = net->d_mi.as<MadeInst>();
  o->f = net->w_f.as<double>();
  o->g = net->w_og.as<double>();
  o->ess = ess;
  o->spins = spins;
  o->ww_a = net->ww_a.as<int32_t>();
  o->ww_b = net->ww_b.as<int32_t>();
  o->ww_e = net->ww_e.as<int32_t>();
  o->wv = net->d_wv.as<int32_t>();
  o->hw_off = net->d_hw_off.as<int32_t>();
  o->spin_base = net->d_spin_base.as<int64_t>();
  o->edge_base = net->d_edge_base.as<int64_t>();
  for (auto &D : net->P.insts) o->max_out = std::max(o->max_out, (int32_t)(D.nw + D.n_ww));
  HIPCHK(launch_obs_weights(*o, net->n_inst, st));
  return TNVAN_OK;
}

// moments of p from samples of q (tnvan_observables)
template <typename real>
tnvan_status run_observables(tnvan_net *net, const int8_t *spins, const void *logq, double *mag,
                             double *corr, double *ess, hipStream_t st) {
  ObsArgs o{};
  if (tnvan_status s = obs_weights<real>(net, spins, logq, ess, &o, st)) return s;
  o.mag = mag;
  o.corr = corr;
  // the remainder's moments: the adjoint with g_b = w_b / beta (dh = sum
  // w_b <r>, dJ = sum w_b <x x>; zero on W vertices and W-W edges) ...
  if (tnvan_status s = run_backward<real>(net, spins, net->w_og.as<double>(), mag, corr,
                                          net->w_odb.as<double>(), st))
    return s;
  // ... and the width set's, written over those zeros
  HIPCHK(launch_obs_w(o, net->n_inst, st));
  return TNVAN_OK;
}
// the conditional mean and variance of M_R per sample (tnvan_remainder_moments)
template <typename real>
tnvan_status run_moments(tnvan_net *net, const int8_t *spins, double *logz, double *mean,
                         double *var, hipStream_t st) {
  for (int q = 0; q < net->n_inst; ++q)
    if (net->P.insts[q].max_w > kTabW)
      return set_err(TNVAN_E_WIDTH, "instance %d: magnetisation moments need message scopes <= %d",
                     q, kTabW);
  // (every step of such programs has its transfer table)
  for (const StepDesc &sd : net->P.steps)
    if (sd.t_off < 0) return set_err(TNVAN_E_WIDTH, "magnetisation moments need every step's table");
  if (net->mkey != net->nkey) {
    std::vector<int64_t> jo(net->n_inst), eo(net->n_inst);
    int64_t jt = 0, et = 0;
    for (int q = 0; q < net->n_inst; ++q) {
      const InstDesc &D = net->P.insts[q];
      jo[q] = jt;
      eo[q] = et;
      jt += ((int64_t)D.arena_fwd + D.scr_fwd) * 3 * net->nkey[q];
      et += (int64_t)D.n_steps * net->nkey[q];
    }
    if (tnvan_status s = quiesce(net)) return s;
    HIPCHK(upload(net->d_jar_off, jo));
    HIPCHK(upload(net->d_jexp_off, eo));
    HIPCHK(net->w_jar.ensure((size_t)std::max<int64_t>(1, jt) * sizeof(real)));
    HIPCHK(net->w_jexp.ensure((size_t)std::max<int64_t>(1, et) * sizeof(int32_t)));
    net->mkey = net->nkey;
  }
  // instances whose program is a set of 1-2 tile chains take the jets on
  // the register-resident chain kernels (FP32 products; the adjoint's task
  // list), the others the general kernel
  const bool chains = sizeof(real) == 4 && net->rbwd &&
                      std::count(net->use_chain.begin(), net->use_chain.end(), 1) > 0;
  if (chains) {
    if (tnvan_status s = ensure_chain_tasks(net)) return s;
    if (!net->mskip_set) {
      std::vector<int32_t> fl(net->use_chain.begin(), net->use_chain.end());
      if (tnvan_status s = quiesce(net)) return s;
      HIPCHK(upload(net->d_mskip, fl));
      net->mskip_set = true;
    }
    int64_t mtot = 0;
    for (int q = 0; q < net->n_inst; ++q)
      if (net->use_chain[q]) mtot += (int64_t)net->P.cinst[q].n_chains * net->nkey[q];
    HIPCHK(net->w_mpart.ensure((size_t)std::max<int64_t>(1, 2 * mtot) * sizeof(double)));
    ChainArgs c = chain_args(net, true);
    c.spins = spins;
    c.mpart = net->w_mpart.as<double>();
    c.mtot = mtot;
    HIPCHK(launch_unary(c, net->chain_list.as<int32_t>(), net->n_chain_insts, net->u_chunks,
                        net->u_maxB, net->f_off.as<int64_t>(), net->Ubuf.as<float>(),
                        net->fabp.as<double>(), st));
    for (int gi = 0; gi < 2; ++gi) {
      c.task_base = net->brg_lo[gi];
      c.n_tasks = net->brg_n[gi];
      c.ntm = 1 << gi;
      HIPCHK(launch_rchain_moments(c, st));
    }
    if (logz)
      HIPCHK(launch_chain_sum(net->inst.as<InstDesc>(), net->cinst.as<ChainInst>(),
                              net->chain_list.as<int32_t>(), net->n_chain_insts,
                              net->d_B.as<int64_t>(), net->d_sample_off.as<int64_t>(),
                              net->cpart_off.as<int64_t>(), net->cpart.as<double>(),
                              net->f_off.as<int64_t>(), net->fabp.as<double>(), logz, st));
    HIPCHK(launch_chain_mom_sum(net->cinst.as<ChainInst>(), net->chain_list.as<int32_t>(),
                                net->n_chain_insts, net->d_B.as<int64_t>(),
                                net->d_sample_off.as<int64_t>(), net->cpart_off.as<int64_t>(),
                                net->w_mpart.as<double>(), mtot, mean, var, st));
    if (std::count(net->use_chain.begin(), net->use_chain.end(), 1) == net->n_inst)
      return TNVAN_OK;
  }
  MomentArgs<real> a{};
  a.skip = chains ? net->d_mskip.as<int32_t>() : nullptr;
  a.inst = net->inst.as<InstDesc>();
  a.steps = net->steps.as<StepDesc>();
  a.inputs = net->inputs.as<InputDesc>();
  a.gtab = net->gtab.as<uint16_t>();
  a.T = net->T.as<real>();
  a.fld_ptr = net->fld_ptr.as<int32_t>();
  a.fld_w = net->fld_w.as<int32_t>();
  a.fld_J = net->fld_J.as<real>();
  a.hR = net->hR.as<real>();
  a.inst_sample_off = net->d_sample_off.as<int64_t>();
  a.inst_B = net->d_B.as<int64_t>();
  a.inst_spin_off = net->d_spin_off.as<int64_t>();
  a.spins = spins;
  a.jarena = net->w_jar.as<real>();
  a.jexp = net->w_jexp.as<int32_t>();
  a.jar_off = net->d_jar_off.as<int64_t>();
  a.jexp_off = net->d_jexp_off.as<int64_t>();
  a.logz = logz;
  a.mean = mean;
  a.var = var;
  int64_t maxB = 0;
  for (auto b : net->nkey) maxB = std::max(maxB, b);
  HIPCHK(launch_moments<real>(a, net->n_inst, maxB, st));
  return TNVAN_OK;
}

// importance-weighted magnetisation moments and susceptibility of p
// (tnvan_susceptibility)
template <typename real>
tnvan_status run_susceptibility(tnvan_net *net, const int8_t *spins, const void *logq,
                                double *out, hipStream_t st) {
  const int64_t B = std::max<int64_t>(1, net->B_total);
  HIPCHK(net->w_oess.ensure((size_t)net->n_inst * sizeof(double)));
  HIPCHK(net->w_mmean.ensure((size_t)B * sizeof(double)));
  HIPCHK(net->w_mvar.ensure((size_t)B * sizeof(double)));
  ObsArgs o{};
  if (tnvan_status s = obs_weights<real>(net, spins, logq, net->w_oess.as<double>(), &o, st)) return s;
  if (tnvan_status s = run_moments<real>(net, spins, nullptr, net->w_mmean.as<double>(),
                                         net->w_mvar.as<double>(), st))
    return s;
  SusArgs a{};
  a.inst = net->inst.as<InstDesc>();
  a.inst_sample_off = net->d_sample_off.as<int64_t>();
  a.inst_B = net->d_B.as<int64_t>();
  a.inst_spin_off = net->d_spin_off.as<int64_t>();
  a.spins = spins;
  a.g = net->w_og.as<double>();
  a.ess = net->w_oess.as<double>();
  a.mean = net->w_mmean.as<double>();
  a.var = net->w_mvar.as<double>();
  a.out = out;
  HIPCHK(launch_sus_reduce(a, net->n_inst, st));
  return TNVAN_OK;
}

// a pointer the GPU can access (device or managed memory, or pinned host
// memory mapped for the device); plain host memory is rejected
bool is_device_ptr(const void *p) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();   // clear the sticky error of the query
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
         (at.type == hipMemoryTypeHost && at.devicePointer != nullptr);
}

// every non-null pointer of the list must be accessible by the device
tnvan_status check_device(std::initializer_list<const void *> ps) {
  for (const void *p : ps)
    if (p && !is_device_ptr(p)) return set_err(TNVAN_E_INVALID, "a buffer is not device memory");
  return TNVAN_OK;
}

tnvan_status check_net(const tnvan_net *net) {
  if (!net) return set_err(TNVAN_E_INVALID, "net is NULL");
  return TNVAN_OK;
}

}  // namespace

namespace tnvan {

tnvan_status net_signature(const tnvan_net *net, std::string &out) {
  if (tnvan_status s = check_net(net)) return s;
  tnvan_tuning t{};
  if (tnvan_status s = tnvan_get_tuning(net, &t)) return s;
  int maxw = 0;
  for (auto &D : net->P.insts) maxw = std::max(maxw, (int)D.max_w);
  static const char *prec[] = {"fp64", "fp32", "bf16"};
  out = std::string(prec[net->precision]) + (net->split ? "+split" : "") + "|k" +
        std::to_string(t.kinds) + "|w" + std::to_string(maxw) + "|n" + std::to_string(net->n_inst);
  return TNVAN_OK;
}

int net_instances(const tnvan_net *net) { return net ? net->n_inst : 0; }

void set_last_error(const char *msg) { g_err = msg; }

}  // namespace tnvan

extern "C" {

const char *tnvan_last_error(void) { return g_err.c_str(); }

tnvan_status tnvan_build_network(const tnvan_instance *inst, int32_t n_inst,
                                 const tnvan_options *opt, tnvan_net **out) {
  if (!out) return set_err(TNVAN_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!inst || n_inst <= 0 || n_inst > 65536) return set_err(TNVAN_E_INVALID, "bad instance list");
  if (!opt) return set_err(TNVAN_E_INVALID, "options are NULL");
  if (opt->precision < TNVAN_FP64 || opt->precision > TNVAN_BF16)
    return set_err(TNVAN_E_INVALID, "unknown precision %d", opt->precision);
  tnvan_net *net = new (std::nothrow) tnvan_net();
  if (!net) return set_err(TNVAN_E_NOMEM, "host allocation failed");
  net->precision = opt->precision;
  net->seed = opt->seed;
  net->profile = (opt->flags & TNVAN_FLAG_PROFILE) != 0;
  net->markers = (opt->flags & TNVAN_FLAG_MARKERS) != 0;
  net->use_graph = (opt->flags & TNVAN_FLAG_GRAPH) != 0;
  net->split = (opt->flags & TNVAN_FLAG_SPLIT_BF16) != 0 && net->precision == TNVAN_FP32;
  net->check_finite = (opt->flags & TNVAN_FLAG_CHECK_FINITE) != 0;
  {
    const int k = opt->checkpoint_every;
    if (k != 0 && k != 1 && k != 2 && k != 4 && k != 8) {
      delete net;
      return set_err(TNVAN_E_INVALID, "checkpoint_every must be 0, 1, 2, 4 or 8");
    }
    net->rk_build = k > 1 ? k : 1;
  }
  net->n_inst = n_inst;
  net->max_width = opt->max_width;
  for (int q = 0; q < n_inst; ++q) {
    std::string msg;
    tnvan_status s = compile_instance(inst[q], opt->max_width, net->P, msg);
    if (s != TNVAN_OK) {
      delete net;
      return set_err(s, "instance %d: %s", q, msg.c_str());
    }
    // the arrays were validated by the compiler
    const tnvan_instance &in = inst[q];
    tnvan_net::SrcInst c;
    c.n_spins = in.n_spins;
    c.n_edges = in.n_edges;
    c.hidden = in.hidden;
    c.depth = in.depth;
    c.beta = in.beta;
    c.ei.assign(in.edge_i, in.edge_i + in.n_edges);
    c.ej.assign(in.edge_j, in.edge_j + in.n_edges);
    c.J.assign(in.J, in.J + in.n_edges);
    c.h.assign(in.n_spins, 0.0);
    if (in.h) c.h.assign(in.h, in.h + in.n_spins);
    c.W.assign(in.width_set, in.width_set + in.n_width);
    c.order.assign(in.order, in.order + in.n_order);
    if (in.n_groups > 0 && in.group_ptr) c.gp.assign(in.group_ptr, in.group_ptr + in.n_groups + 1);
    net->src.push_back(std::move(c));
    const InstDesc &D = net->P.insts[q];
    if (D.nw > 2048) { delete net; return set_err(TNVAN_E_INVALID, "instance %d: |W| above 2048", q); }
  }
  // network layout
  int64_t poff = 0;
  for (int q = 0; q < n_inst; ++q) {
    MadeInst m{};
    m.n = net->P.insts[q].nw;
    m.H = net->P.hidden[q];
    m.D = net->P.depth[q];
    int L = 8;
    while (L < 64 && (m.H > 16 * L || m.n > 32 * L)) L <<= 1;
    if (m.H > 16 * L || m.n > 32 * L) { delete net; return set_err(TNVAN_E_INVALID, "instance %d: network too wide", q); }
    m.L = L;
    m.param_off = poff;
    const int64_t pc = (int64_t)m.H * m.n + m.H + (int64_t)m.n * m.H + m.n + (int64_t)m.n * m.n +
                       (int64_t)(m.D - 1) * ((int64_t)m.H * m.H + m.H);
    if (m.D > 1 && m.n >= 2) net->deep = true;
    net->param_count.push_back(pc);
    poff += pc;
    net->mi.push_back(m);
  }
  // deeper networks: every instance runs the general deep sampler and rows
  // kernels, whose per-lane tables hold |W| <= 256 and H <= 256
  if (net->deep)
    for (int q = 0; q < n_inst; ++q)
      if (net->mi[q].n > kDeepMaxN || net->mi[q].H > kDeepMaxH) {
        delete net;
        return set_err(TNVAN_E_INVALID, "instance %d: a net with a deeper network needs "
                       "|W| <= %d and H <= %d", q, kDeepMaxN, kDeepMaxH);
      }
  // one lane count for every instance keeps the sampler a single launch
  int Lmax = 8;
  for (auto &m : net->mi) Lmax = std::max(Lmax, (int)m.L);
  for (auto &m : net->mi) m.L = Lmax;
  net->param_total = poff;
  // matrix-core sampler: every instance with n <= 64 and at most 15 hidden
  // units per degree (FP32 / BF16 precisions)
  {
    int nmax = 1;
    bool fits = net->precision != TNVAN_FP64 && !net->deep;
    for (auto &m : net->mi) {
      nmax = std::max(nmax, (int)m.n);
      if (m.n > 64 || (m.n >= 2 && m.H > 15 * (m.n - 1))) fits = false;
    }
    net->mpt = nmax <= 16 ? 1 : nmax <= 32 ? 2 : 4;
    net->msample = fits;
    // one-layer nets outside the matrix-core sampler: a wave per sample
    bool h0 = !fits && nmax <= kH0MaxN && !net->deep;
    std::vector<int64_t> w0off;
    int64_t wo = 0;
    for (auto &m : net->mi) {
      if (m.H != 0 && m.n >= 2) h0 = false;
      w0off.push_back(wo);
      wo += (int64_t)m.n * m.n;
    }
    net->h0 = h0;
    net->h0_nmax = nmax;
    if (h0) {
      hipError_t e0 = upload(net->d_w0t_off, w0off);
      if (e0 == hipSuccess) e0 = net->w0t.ensure((size_t)std::max<int64_t>(1, wo) * sizeof(float));
      if (e0 != hipSuccess) {
        tnvan_free_network(net);
        return set_err(e0 == hipErrorOutOfMemory ? TNVAN_E_NOMEM : TNVAN_E_HIP, "w0t: %s",
                       hipGetErrorString(e0));
      }
    }
    int64_t po = 0;
    for (auto &m : net->mi) {
      m.pack_off = po;
      po += made_pack_floats(m.n, net->mpt, m.H);
      net->mpack_max = std::max(net->mpack_max, made_pack_floats(m.n, net->mpt, m.H));
    }
    net->mpack_total = po;
    // fused REINFORCE backward: n <= 64, H <= 256, rows of 64 samples in LDS
    int dev = 0, maxlds = 65536;
    hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    bool gfit = net->precision != TNVAN_FP64 && !net->deep;
    for (auto &m : net->mi) {
      net->mg_hmax = std::max(net->mg_hmax, (int)m.H);
      if (m.n > 64 || m.H > 256 || m.n % 4 || m.H % 4) gfit = false;
    }
    for (auto pc : net->param_count) net->mg_pstride = std::max(net->mg_pstride, pc);
    net->mg_pstride = (net->mg_pstride + 63) / 64 * 64;
    net->mgrad = gfit && mgrad_lds_bytes(net->mg_hmax, net->mpt, net->split && net->mpt <= 2) <=
                             (size_t)maxlds;
  }
  auto fail = [&](hipError_t e, const char *what) {
    tnvan_free_network(net);
    return set_err(e == hipErrorOutOfMemory ? TNVAN_E_NOMEM : TNVAN_E_HIP, "%s: %s", what,
                   hipGetErrorString(e));
  };
  hipError_t e;
  HostProgram &P = net->P;
#define UP(buf, vec) if ((e = upload(net->buf, vec)) != hipSuccess) return fail(e, #buf);
  {
    const char *what = "";
    if ((e = upload_tables(net, &what)) != hipSuccess) return fail(e, what);
  }
  {
    std::vector<int64_t> sb(n_inst), eb(n_inst);
    int64_t a = 0, b = 0;
    for (int q = 0; q < n_inst; ++q) { sb[q] = a; eb[q] = b; a += P.insts[q].n; b += P.insts[q].n_edges; }
    UP(d_spin_base, sb) UP(d_edge_base, eb)
    std::vector<int64_t> so(n_inst);
    int64_t tot = 0;
    for (int q = 0; q < n_inst; ++q) {
      so[q] = tot;
      tot += P.insts[q].n_partial;
      net->max_partial = std::max(net->max_partial, (int)P.insts[q].n_partial);
    }
    UP(d_sum_off, so)
  }
  UP(d_mi, net->mi)
  // 16 floats of padding: the kernels read parameter rows four floats at a
  // time, and the last row of an instance may end inside such a group
  const size_t pb = (std::max<int64_t>(1, net->param_total) + 16) * sizeof(float);
  if ((e = net->params.ensure(pb)) || (e = net->adam_m.ensure(pb)) || (e = net->adam_v.ensure(pb)) ||
      (e = net->grad.ensure(pb)) || (e = net->step_ctr.ensure(sizeof(int32_t) * n_inst)))
    return fail(e, "parameter buffers");
  if ((e = hipMemset(net->params.p, 0, pb)) || (e = hipMemset(net->adam_m.p, 0, pb)) ||
      (e = hipMemset(net->adam_v.p, 0, pb)) || (e = hipMemset(net->grad.p, 0, pb)) ||
      (e = hipMemset(net->step_ctr.p, 0, sizeof(int32_t) * n_inst)))
    return fail(e, "parameter init");
  // completion tickets of the free-energy kernel's last-block reduction:
  // zero between launches, each launch resets what it used
  if ((e = net->tickets.ensure(sizeof(int32_t) * n_inst)) ||
      (e = hipMemset(net->tickets.p, 0, sizeof(int32_t) * n_inst)))
    return fail(e, "tickets");
  if ((e = net->nonfinite.ensure(sizeof(int32_t) * n_inst)) ||
      (e = hipMemset(net->nonfinite.p, 0, sizeof(int32_t) * n_inst)))
    return fail(e, "non-finite flags");
  // counters of the persistent launches (each launch leaves them at zero):
  // [0,1] general forward, [2,3] general adjoint, [4,5] chain forward,
  // [6,7] chain adjoint
  if ((e = net->pq.ensure(sizeof(int32_t) * 8)) || (e = hipMemset(net->pq.p, 0, sizeof(int32_t) * 8)))
    return fail(e, "work-queue counters");
  // the adjoint's split column sums, in output order: the outputs without a
  // column are never written and keep these zeros
  for (auto &D : P.insts) net->max_out = std::max(net->max_out, (int)(D.n + D.n_edges));
  {
    const size_t vb = sizeof(double) * std::max(1, n_inst * vjp_split() * net->max_out);
    if ((e = net->vjp_part.ensure(vb)) || (e = hipMemset(net->vjp_part.p, 0, vb))) return fail(e, "adjoint sums");
  }
  // transfer-matrix form: instances whose program is a set of dense chains
  // (FP32 / BF16 only); the launch-wide maxima size the LDS layout
  net->use_chain.assign(n_inst, 0);
  {
    int dev = 0, maxlds = 65536;
    hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    ChainLim lim{};
    bool rq = true;
    lim.kbuf = 16;
    lim.kseg = 1;
    lim.rk = net->rk_build;
    for (int q = 0; q < n_inst; ++q) {
      const ChainInst &C = P.cinst[q];
      if (net->precision == TNVAN_FP64 || !C.ok) continue;
      net->use_chain[q] = 1;
      lim.kbuf = std::max(lim.kbuf, C.kbuf);
      lim.npos_max = std::max(lim.npos_max, C.npos_max);
      lim.max_steps = std::max(lim.max_steps, C.max_steps);
      lim.pmax = std::max(lim.pmax, C.pmax);
      lim.nw = std::max(lim.nw, C.nw);
      lim.tl_max = std::max(lim.tl_max, C.tl_max);
      lim.tbl_max = std::max(lim.tbl_max, C.tbl_max);
      lim.ne_max = std::max(lim.ne_max, C.ne_max);
      lim.nf_max = std::max(lim.nf_max, C.nf_max);
      lim.kseg = std::max(lim.kseg, chain_kseg(C));
      net->rtiles = std::max(net->rtiles, C.rtiles);
      rq = rq && C.rq_ok;
    }
    const bool any = std::count(net->use_chain.begin(), net->use_chain.end(), 1) > 0;
    // register-resident kernels when every chain step is narrow enough; the
    // adjoint's W-R sums hold the width-set spins as a 128-bit mask
    const bool reg = any && !(opt->flags & TNVAN_FLAG_LDS_CHAIN);
    net->rfwd = reg && rq && net->rtiles <= kRegFwdTiles &&
                4 * rchain_wave_lds(lim, false, net->sg) <= (size_t)maxlds;
    net->rbwd = reg && lim.nw <= 128 && rq && net->rtiles <= kRegBwdTiles &&
                4 * rchain_wave_lds(lim, true, 1) <= (size_t)maxlds;
    const bool bf = net->precision == TNVAN_BF16;
    bool ok = true;
    for (int pass = 0; pass < 2 && any; ++pass) {
      const bool bwd = pass == 1;
      ChainLim L = lim;
      L.wpb = 1;
      if (bwd ? net->rbwd : net->rfwd) {
        (bwd ? net->lim_bwd : net->lim_fwd) = L;
        continue;
      }
      L.tlds = 1;
      size_t sh = chain_shared_lds(L, bwd, bf && !bwd), per = chain_wave_lds(L, bwd);
      if (sh + per > (size_t)maxlds) {   // tables too large: read them from HBM
        L.tlds = 0;
        sh = chain_shared_lds(L, bwd, bf && !bwd);
      }
      if (sh + per > (size_t)maxlds) { ok = false; break; }
      L.wpb = (int)std::min<size_t>(4, ((size_t)maxlds - sh) / per);
      (bwd ? net->lim_bwd : net->lim_fwd) = L;
    }
    if (!ok) {
      net->use_chain.assign(n_inst, 0);
      net->rfwd = net->rbwd = false;
    }
  }
  for (int q = 0; q < n_inst; ++q)
    if (!net->use_chain[q] && net->P.insts[q].max_w > kTabW) net->wide = true;
  choose_tiles(net, false);
  choose_tiles(net, true);
#undef UP
  // the allocation-free entry point's scratch address on this device
  (void)hipGetDevice(&net->device);
  scratch_setup(net->device);
  *out = net;
  return TNVAN_OK;
}

void tnvan_free_network(tnvan_net *net) {
  if (!net) return;
  if (net->step_graph.exec) hipGraphExecDestroy(net->step_graph.exec);
  if (net->cap_stream) hipStreamDestroy(net->cap_stream);
  for (auto &v : net->prof_used)
    for (auto &e : v) net->prof_pool.push_back(e);
  for (auto &e : net->prof_pool) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  net->prof_pool.clear();
  DBuf *all[] = {&net->inst, &net->steps, &net->inputs, &net->gtab, &net->gtab2, &net->esmall,
                 &net->edges, &net->T, &net->fld_ptr,
                 &net->fld_w, &net->fld_J, &net->hR, &net->wr_pos, &net->wr_w, &net->rr_edge,
                 &net->rr_J, &net->wr_edge, &net->wr_J, &net->hR64, &net->vr, &net->ww_a,
                 &net->ww_b, &net->ww_J, &net->hW, &net->d_mi, &net->params, &net->adam_m,
                 &net->adam_v, &net->grad, &net->step_ctr, &net->d_sample_off, &net->d_B,
                 &net->d_spin_off, &net->d_spin_base, &net->d_edge_base, &net->blk_inst,
                 &net->blk_start, &net->garena, &net->partial, &net->w_logz, &net->w_logq,
                 &net->w_spins, &net->w_f, &net->w_fpart, &net->w_hid, &net->w_da, &net->d_hw_off,
                 &net->d_sum_off,
                 &net->w_dlogit, &net->w_sf, &net->w_part, &net->cinst, &net->chains,
                 &net->csteps, &net->Tp, &net->Tt, &net->Tb, &net->fld_wr, &net->fld_J32,
                 &net->hR32, &net->task_inst, &net->task_chain, &net->task_start,
                 &net->btask_inst, &net->btask_chain, &net->btask_start, &net->Tl, &net->Tbl,
                 &net->cedges, &net->ckpt, &net->Tr, &net->Tq, &net->Trb, &net->xcol,
                 &net->cf_w, &net->cf_r, &net->cf_J, &net->Tsx, &net->Ts3, &net->Tdq, &net->Ubuf, &net->vjp_part,
                 &net->tickets, &net->nonfinite, &net->pq, &net->col_out, &net->pcoef_out, &net->w_xspins, &net->w_xlogz, &net->w_xpart, &net->ww_e, &net->d_wv, &net->w_og,
                 &net->w_ostats, &net->w_odb, &net->fabp, &net->u_off,
                 &net->w_jar, &net->w_jexp, &net->d_jar_off, &net->d_jexp_off, &net->w_mmean,
                 &net->w_mvar, &net->w_oess, &net->w_mpart, &net->d_mskip,
                 &net->bs_atb, &net->bs_col, &net->bs_alo, &net->bs_aflo, &net->bs_clo,
                 &net->bs_cflo,
                 &net->f_off,
                 &net->mpack, &net->mtask_inst, &net->mtask_start, &net->mg_task_inst,
                 &net->mg_task_start, &net->mg_first, &net->mg_count,
                 &net->cpart_off, &net->chain_list, &net->cpart};
  for (DBuf *b : all) b->release();
  for (int c = 0; c < 4; ++c) {
    net->rw_jobs[c].release();
    net->rw_lo[c].release();
  }
  TileCache *tcs[] = {&net->tc_fwd, &net->tc_bwd};
  for (TileCache *tc : tcs) {
    tc->tile_inst.release(); tc->tile_start.release(); tc->first_tile.release();
    tc->n_tiles_i.release(); tc->partial_off.release();
  }
  delete net;
}

tnvan_status tnvan_param_count(const tnvan_net *net, int32_t inst, int64_t *count) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || !count) return set_err(TNVAN_E_INVALID, "bad instance index");
  *count = net->param_count[inst];
  return TNVAN_OK;
}

tnvan_status tnvan_set_params(tnvan_net *net, int32_t inst, const float *src, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || !src) return set_err(TNVAN_E_INVALID, "bad instance or source");
  if (tnvan_status s = check_device({src})) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t bytes = net->param_count[inst] * sizeof(float);
  const int64_t off = net->mi[inst].param_off;
  HIPCHK(hipMemcpyAsync(net->params.as<float>() + off, src, bytes, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemsetAsync(net->adam_m.as<float>() + off, 0, bytes, st));
  HIPCHK(hipMemsetAsync(net->adam_v.as<float>() + off, 0, bytes, st));
  HIPCHK(hipMemsetAsync(net->step_ctr.as<int32_t>() + inst, 0, sizeof(int32_t), st));
  // the packed tables are rebuilt from the new parameters at the next use,
  // and a recorded step (which does not repack) is recorded again
  net->pack_valid = false;
  g_buf_gen.fetch_add(1);
  return TNVAN_OK;
}

tnvan_status tnvan_get_params(tnvan_net *net, int32_t inst, float *dst, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || !dst) return set_err(TNVAN_E_INVALID, "bad instance or destination");
  if (tnvan_status s = check_device({dst})) return s;
  HIPCHK(hipMemcpyAsync(dst, net->params.as<float>() + net->mi[inst].param_off,
                        net->param_count[inst] * sizeof(float), hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  return TNVAN_OK;
}

tnvan_status tnvan_set_couplings(tnvan_net *net, int32_t inst, const double *J, const double *h,
                                 double beta) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst) return set_err(TNVAN_E_INVALID, "bad instance index");
  if (net->capturing) return set_err(TNVAN_E_STATE, "set_couplings while a graph is recorded");
  tnvan_net::SrcInst c = net->src[inst];
  if (c.n_edges > 0 && !J) return set_err(TNVAN_E_INVALID, "J is NULL");
  if (c.n_edges > 0) c.J.assign(J, J + c.n_edges);
  c.h.assign(c.n_spins, 0.0);
  if (h) c.h.assign(h, h + c.n_spins);
  c.beta = beta;
  // compile every instance again (the program's offsets run over all of
  // them); the compiler validates the new values
  HostProgram P2;
  for (int q = 0; q < net->n_inst; ++q) {
    std::string msg;
    const tnvan_instance v = src_view(q == inst ? c : net->src[q]);
    tnvan_status s = compile_instance(v, net->max_width, P2, msg);
    if (s != TNVAN_OK) return set_err(s, "instance %d: %s", q, msg.c_str());
  }
  if (!same_structure(net->P, P2))
    return set_err(TNVAN_E_STATE, "instance %d: the new values change the program's structure", inst);
  // kernels queued earlier may still read the tables
  if (tnvan_status s = quiesce(net)) return s;
  HIPCHK(hipDeviceSynchronize());
  std::swap(net->P, P2);
  const char *what = "";
  const hipError_t e = upload_tables(net, &what);
  if (e != hipSuccess) {
    // the device tables are now partly new: put the old program back
    // (same sizes, so nothing is reallocated)
    std::swap(net->P, P2);
    const char *w2 = "";
    (void)upload_tables(net, &w2);
    net->nkey.clear();
    return set_err(e == hipErrorOutOfMemory ? TNVAN_E_NOMEM : TNVAN_E_HIP, "%s: %s", what,
                   hipGetErrorString(e));
  }
  net->src[inst] = std::move(c);
  // the next call lays its per-call tables out again, which also refills
  // the unary-factor table (positions without a field or a W-neighbour keep
  // the +1 of that fill and are skipped by the unary kernel)
  net->nkey.clear();
  return TNVAN_OK;
}

tnvan_status tnvan_get_state(tnvan_net *net, int32_t inst, int32_t which, float *dst,
                             void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || !dst) return set_err(TNVAN_E_INVALID, "bad instance or destination");
  const DBuf *src = which == 0 ? &net->params : which == 1 ? &net->grad
                  : which == 2 ? &net->adam_m : which == 3 ? &net->adam_v : nullptr;
  if (!src) return set_err(TNVAN_E_INVALID, "unknown state %d", which);
  if (tnvan_status s = check_device({dst})) return s;
  HIPCHK(hipMemcpyAsync(dst, src->as<float>() + net->mi[inst].param_off,
                        net->param_count[inst] * sizeof(float), hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  return TNVAN_OK;
}

tnvan_status tnvan_set_state(tnvan_net *net, int32_t inst, int32_t which, const float *src,
                             void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || !src) return set_err(TNVAN_E_INVALID, "bad instance or source");
  DBuf *dst = which == 0 ? &net->params : which == 2 ? &net->adam_m : which == 3 ? &net->adam_v : nullptr;
  if (!dst) return set_err(TNVAN_E_INVALID, "state %d cannot be set (0, 2 or 3)", which);
  if (tnvan_status s = check_device({src})) return s;
  HIPCHK(hipMemcpyAsync(dst->as<float>() + net->mi[inst].param_off, src,
                        net->param_count[inst] * sizeof(float), hipMemcpyDeviceToDevice,
                        static_cast<hipStream_t>(stream)));
  if (which == 0) {
    // as tnvan_set_params: the packed tables follow at the next use
    net->pack_valid = false;
    g_buf_gen.fetch_add(1);
  }
  return TNVAN_OK;
}

tnvan_status tnvan_get_step(tnvan_net *net, int32_t inst, int32_t *step, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || !step) return set_err(TNVAN_E_INVALID, "bad instance or output");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t v = 0;
  HIPCHK(hipMemcpyAsync(&v, net->step_ctr.as<int32_t>() + inst, sizeof(int32_t),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *step = v;
  return TNVAN_OK;
}

tnvan_status tnvan_set_step(tnvan_net *net, int32_t inst, int32_t step, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || step < 0) return set_err(TNVAN_E_INVALID, "bad instance or step");
  HIPCHK(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(net->step_ctr.as<int32_t>() + inst),
                           step, 1, static_cast<hipStream_t>(stream)));
  return TNVAN_OK;
}

tnvan_status tnvan_sample(tnvan_net *net, const int64_t *n_samples, const float *uniforms,
                          int8_t *spins, void *logq, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, n_samples)) return s;
  if (net->B_total == 0) return TNVAN_OK;
  if (!spins || !logq) return set_err(TNVAN_E_INVALID, "spins and logq are required");
  if (tnvan_status s = check_device({uniforms, spins, logq})) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net->precision == TNVAN_FP64) return run_sample<double>(net, uniforms, spins, logq, st);
  return run_sample<float>(net, uniforms, spins, logq, st);
}

tnvan_status tnvan_logz_batch(tnvan_net *net, const int64_t *n_samples, const int8_t *spins,
                              double *logz, double *e1, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, n_samples)) return s;
  if (net->B_total == 0) return TNVAN_OK;
  if (!logz || (!spins && net->spin_total > 0)) return set_err(TNVAN_E_INVALID, "spins and logz are required");
  if (tnvan_status s = check_device({spins, logz})) return s;
  if (e1)
    if (tnvan_status s = check_device({e1})) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  tnvan_status s = net->precision == TNVAN_FP64 ? run_logz<double>(net, spins, logz, st)
                                                : run_logz<float>(net, spins, logz, st);
  if (s != TNVAN_OK || !e1) return s;
  E1Args a{};
  a.inst = net->inst.as<InstDesc>();
  a.mi = net->d_mi.as<MadeInst>();
  a.hw_off = net->d_hw_off.as<int32_t>();
  a.spins = spins;
  a.ww_a = net->ww_a.as<int32_t>();
  a.ww_b = net->ww_b.as<int32_t>();
  a.ww_J = net->ww_J.as<double>();
  a.hW = net->hW.as<double>();
  a.e1 = e1;
  int64_t maxB = 0;
  for (auto b : net->nkey) maxB = std::max(maxB, b);
  HIPCHK(launch_e1(a, net->n_inst, maxB, st));
  return TNVAN_OK;
}

namespace {
constexpr int kExactMaxW = 28;                  // |W| of exact slicing
constexpr int64_t kExactChunk = (int64_t)1 << 16;   // configurations per pass
}  // namespace

tnvan_status tnvan_exact_free_energy(tnvan_net *net, int32_t inst, double *out, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || !out) return set_err(TNVAN_E_INVALID, "bad instance or output");
  if (!is_device_ptr(out)) return set_err(TNVAN_E_INVALID, "out is not device memory");
  const InstDesc &D = net->P.insts[inst];
  if (D.nw > kExactMaxW)
    return set_err(TNVAN_E_WIDTH, "exact slicing takes |W| <= %d (here %d)", kExactMaxW, (int)D.nw);
  if (!(D.beta > 0)) return set_err(TNVAN_E_INVALID, "exact free energy needs beta > 0");
  const int64_t total = (int64_t)1 << D.nw, chunk = std::min(total, kExactChunk);
  const int64_t passes = total / chunk;
  std::vector<int64_t> key(net->n_inst, 0);
  key[inst] = chunk;
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, key.data())) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(net->w_xspins.ensure((size_t)std::max<int64_t>(1, chunk * D.nw)));
  HIPCHK(net->w_xlogz.ensure((size_t)chunk * sizeof(double)));
  HIPCHK(net->w_xpart.ensure((size_t)passes * kSliceBlocks * 2 * sizeof(double)));
  int8_t *sp = net->w_xspins.as<int8_t>();
  SliceArgs a{};
  a.inst = net->inst.as<InstDesc>();
  a.q = inst;
  a.ww_a = net->ww_a.as<int32_t>();
  a.ww_b = net->ww_b.as<int32_t>();
  a.ww_J = net->ww_J.as<double>();
  a.hW = net->hW.as<double>();
  a.hw_off = net->d_hw_off.as<int32_t>();
  a.logz = net->w_xlogz.as<double>();
  a.n = chunk;
  a.part = net->w_xpart.as<double>();
  for (int64_t p = 0; p < passes; ++p) {
    a.c0 = p * chunk;
    a.pass = p;
    HIPCHK(launch_slice_spins(sp, D.nw, a.c0, chunk, st));
    const tnvan_status s = net->precision == TNVAN_FP64
                               ? run_logz<double>(net, sp, net->w_xlogz.as<double>(), st)
                               : run_logz<float>(net, sp, net->w_xlogz.as<double>(), st);
    if (s) return s;
    HIPCHK(launch_slice_lse(a, st));
  }
  HIPCHK(launch_slice_final(a.part, passes * kSliceBlocks, D.beta, out, st));
  return TNVAN_OK;
}

tnvan_status tnvan_observables(tnvan_net *net, const int64_t *n_samples, const int8_t *spins,
                               const void *logq, double *mag, double *corr, double *ess,
                               void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (tnvan_status s = check_device({spins, logq, mag, corr, ess})) return s;
  for (auto &D : net->P.insts)
    if (!(D.beta > 0)) return set_err(TNVAN_E_INVALID, "observables need beta > 0");
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, n_samples)) return s;
  if (!mag || !corr || !ess) return set_err(TNVAN_E_INVALID, "mag, corr and ess are required");
  if (net->B_total > 0 && (!logq || (!spins && net->spin_total > 0)))
    return set_err(TNVAN_E_INVALID, "spins and logq are required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net->precision == TNVAN_FP64) return run_observables<double>(net, spins, logq, mag, corr, ess, st);
  return run_observables<float>(net, spins, logq, mag, corr, ess, st);
}

tnvan_status tnvan_remainder_moments(tnvan_net *net, const int64_t *n_samples,
                                     const int8_t *spins, double *logz, double *mean, double *var,
                                     void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, n_samples)) return s;
  if (net->B_total == 0) return TNVAN_OK;
  if (!mean || !var || (!spins && net->spin_total > 0))
    return set_err(TNVAN_E_INVALID, "spins, mean and var are required");
  if (tnvan_status s = check_device({spins, mean, var})) return s;
  if (logz)
    if (tnvan_status s = check_device({logz})) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net->precision == TNVAN_FP64) return run_moments<double>(net, spins, logz, mean, var, st);
  return run_moments<float>(net, spins, logz, mean, var, st);
}

tnvan_status tnvan_susceptibility(tnvan_net *net, const int64_t *n_samples, const int8_t *spins,
                                  const void *logq, double *out, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  for (const InstDesc &D : net->P.insts)
    if (!(D.beta > 0)) return set_err(TNVAN_E_INVALID, "the susceptibility needs beta > 0");
  if (tnvan_status s = check_device({spins, logq, out})) return s;
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, n_samples)) return s;
  if (!out) return set_err(TNVAN_E_INVALID, "out is required");
  if (net->B_total > 0 && (!logq || (!spins && net->spin_total > 0)))
    return set_err(TNVAN_E_INVALID, "spins and logq are required");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net->precision == TNVAN_FP64) return run_susceptibility<double>(net, spins, logq, out, st);
  return run_susceptibility<float>(net, spins, logq, out, st);
}

tnvan_status tnvan_logz_backward(tnvan_net *net, const int64_t *n_samples, const int8_t *spins,
                                 const double *grad, double *dh, double *dJ, double *dbeta,
                                 void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, n_samples)) return s;
  if (!dh || !dJ || !dbeta) return set_err(TNVAN_E_INVALID, "dh, dJ and dbeta are required");
  if (net->B_total > 0 && (!grad || (!spins && net->spin_total > 0)))
    return set_err(TNVAN_E_INVALID, "spins and grad_logz are required");
  if (tnvan_status s = check_device({spins, grad, dh, dJ, dbeta})) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (net->precision == TNVAN_FP64) return run_backward<double>(net, spins, grad, dh, dJ, dbeta, st);
  return run_backward<float>(net, spins, grad, dh, dJ, dbeta, st);
}

namespace {

// one training step, eagerly or (TNVAN_FLAG_GRAPH) replayed from the graph
// recorded for the same batch shape, outputs and adjoint buffers
tnvan_status step_entry(tnvan_net *net, const int64_t *n_samples, float lr, double *stats,
                        int8_t *spins_out, const StepAdjoint *adj, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (!stats) return set_err(TNVAN_E_INVALID, "stats is required");
  for (auto &D : net->P.insts)
    if (!(D.beta > 0)) return set_err(TNVAN_E_INVALID, "free_energy_step needs beta > 0");
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, n_samples)) return s;
  if (adj && (!adj->dh || !adj->dJ || !adj->dbeta || (net->B_total > 0 && !adj->grad)))
    return set_err(TNVAN_E_INVALID, "grad_logz, dh, dJ and dbeta are required");
  if (tnvan_status s = check_device({stats, spins_out})) return s;
  if (adj)
    if (tnvan_status s = check_device({adj->grad, adj->dh, adj->dJ, adj->dbeta})) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto eager = [&](hipStream_t s2) {
    return net->precision == TNVAN_FP64 ? run_step<double>(net, lr, stats, spins_out, s2, adj)
                                        : run_step<float>(net, lr, stats, spins_out, s2, adj);
  };
  if (!net->use_graph) return eager(st);
  auto &G = net->step_graph;
  const StepAdjoint none{};
  const StepAdjoint &A = adj ? *adj : none;
  if (G.exec && G.key == net->nkey && G.stats == stats && G.spins == spins_out && G.lr == lr &&
      G.adj == (adj != nullptr) && G.grad == A.grad && G.dh == A.dh && G.dJ == A.dJ &&
      G.dbeta == A.dbeta && G.gen == g_buf_gen.load()) {
    HIPCHK(hipGraphLaunch(G.exec, st));
    return TNVAN_OK;
  }
  // run this step eagerly (allocating and uploading what it needs), then
  // record the same step on a private stream for the next calls
  if (tnvan_status s = eager(st)) return s;
  if (G.exec) {
    hipGraphExecDestroy(G.exec);
    G.exec = nullptr;
  }
  if (!net->cap_stream) HIPCHK(hipStreamCreateWithFlags(&net->cap_stream, hipStreamNonBlocking));
  const uint64_t gen = g_buf_gen.load();
  HIPCHK(hipStreamBeginCapture(net->cap_stream, hipStreamCaptureModeThreadLocal));
  net->capturing = true;
  tnvan_status s = eager(net->cap_stream);
  net->capturing = false;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(net->cap_stream, &graph);
  if (s != TNVAN_OK || e != hipSuccess || g_buf_gen.load() != gen) {
    if (graph) hipGraphDestroy(graph);
    if (s != TNVAN_OK) return s;
    if (e != hipSuccess) return set_err(TNVAN_E_HIP, "graph capture: %s", hipGetErrorString(e));
    return TNVAN_OK;   // buffers moved while recording: stay eager this call
  }
  e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) {
    G.exec = nullptr;
    return set_err(TNVAN_E_HIP, "graph instantiate: %s", hipGetErrorString(e));
  }
  G.key = net->nkey;
  G.stats = stats;
  G.spins = spins_out;
  G.lr = lr;
  G.adj = adj != nullptr;
  G.grad = A.grad;
  G.dh = A.dh;
  G.dJ = A.dJ;
  G.dbeta = A.dbeta;
  G.gen = gen;
  return TNVAN_OK;
}

}  // namespace

namespace {

// TNVAN_FLAG_CHECK_FINITE: after the step (eager or replayed), wait for it,
// read the free-energy kernel's per-instance flags and clear them
tnvan_status finite_check(tnvan_net *net, void *stream) {
  if (!net->check_finite) return TNVAN_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int32_t> fl(net->n_inst, 0);
  HIPCHK(hipMemcpyAsync(fl.data(), net->nonfinite.p, sizeof(int32_t) * net->n_inst,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int q = 0; q < net->n_inst; ++q)
    if (fl[q]) {
      HIPCHK(hipMemsetAsync(net->nonfinite.p, 0, sizeof(int32_t) * net->n_inst, st));
      HIPCHK(hipStreamSynchronize(st));
      return set_err(TNVAN_E_NONFINITE, "instance %d: a non-finite free energy f_b (Eq. 9) in "
                                        "this step", q);
    }
  return TNVAN_OK;
}

}  // namespace

tnvan_status tnvan_free_energy_step(tnvan_net *net, const int64_t *n_samples, float lr,
                                    double *stats, int8_t *spins_out, void *stream) {
  if (tnvan_status s = step_entry(net, n_samples, lr, stats, spins_out, nullptr, stream)) return s;
  return finite_check(net, stream);
}

tnvan_status tnvan_free_energy_step_adjoint(tnvan_net *net, const int64_t *n_samples, float lr,
                                            double *stats, int8_t *spins_out,
                                            const double *grad_logz, double *dh, double *dJ,
                                            double *dbeta, void *stream) {
  StepAdjoint adj;
  adj.grad = grad_logz;
  adj.dh = dh;
  adj.dJ = dJ;
  adj.dbeta = dbeta;
  if (tnvan_status s = step_entry(net, n_samples, lr, stats, spins_out, &adj, stream)) return s;
  return finite_check(net, stream);
}

tnvan_status tnvan_logz_and_backward(tnvan_net *net, const int64_t *n_samples,
                                     const int8_t *spins, const double *grad, double *logz,
                                     double *dh, double *dJ, double *dbeta, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  note_stream(net, stream);
  if (tnvan_status s = set_batch(net, n_samples)) return s;
  if (!dh || !dJ || !dbeta) return set_err(TNVAN_E_INVALID, "dh, dJ and dbeta are required");
  if (net->B_total > 0 && (!grad || !logz || (!spins && net->spin_total > 0)))
    return set_err(TNVAN_E_INVALID, "spins, grad_logz and logz are required");
  if (tnvan_status s = check_device({spins, grad, logz, dh, dJ, dbeta})) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (logz_with_adjoint(net))
    return net->precision == TNVAN_FP64
               ? run_backward<double>(net, spins, grad, dh, dJ, dbeta, st, logz)
               : run_backward<float>(net, spins, grad, dh, dJ, dbeta, st, logz);
  if (net->precision == TNVAN_FP64) {
    if (tnvan_status s = run_logz<double>(net, spins, logz, st)) return s;
    return run_backward<double>(net, spins, grad, dh, dJ, dbeta, st);
  }
  if (tnvan_status s = run_logz<float>(net, spins, logz, st)) return s;
  return run_backward<float>(net, spins, grad, dh, dJ, dbeta, st);
}

tnvan_status tnvan_logz_batch_noalloc(tnvan_net *net, const int64_t *n_samples,
                                      const int8_t *spins, double *logz, void *stream) {
  if (tnvan_status s = check_net(net)) return s;
  if (!n_samples) return set_err(TNVAN_E_INVALID, "n_samples is NULL");
  if (net->n_inst > kLayoutMaxInst)
    return set_err(TNVAN_E_INVALID, "the allocation-free call takes at most %d instances",
                   kLayoutMaxInst);
  bool chains = net->rfwd;
  for (int q = 0; q < net->n_inst; ++q) chains = chains && net->use_chain[q];
  if (!chains)
    return set_err(TNVAN_E_STATE, "the allocation-free call needs every instance on the "
                                  "register-resident chain kernels");
  // the per-call layout, as ensure_chain_tasks lays it for the net's own calls
  LayoutArgs L{};
  L.n_inst = net->n_inst;
  int64_t so = 0, sp = 0, cp = 0, uo = 0, fo = 0, waves2 = 0, maxB = 0;
  int max_nch = 0;
  for (int q = 0; q < net->n_inst; ++q) {
    const int64_t B = n_samples[q];
    if (B < 0 || B > ((int64_t)1 << 31)) return set_err(TNVAN_E_INVALID, "bad sample count");
    const InstDesc &D = net->P.insts[q];
    const ChainInst &C = net->P.cinst[q];
    const int nch = (D.nr + kUnaryChunk - 1) / kUnaryChunk;
    L.B[q] = B;
    L.sample_off[q] = so;
    L.spin_off[q] = sp;
    L.cpart_off[q] = cp;
    L.u_off[q] = uo;
    L.f_off[q] = fo;
    so += B;
    sp += B * D.nw;
    cp += (int64_t)C.n_chains * B;
    uo += (int64_t)D.nr * B;
    fo += (int64_t)nch * B;
    waves2 += C.n_chains * ((B + 31) / 32);
    maxB = std::max(maxB, B);
    max_nch = std::max(max_nch, nch);
  }
  const int sg = chain_groups(net, waves2);
  int64_t nt = 0;
  for (int gi = 0; gi < 3; ++gi) {
    const int rt = 1 << gi;
    L.per[gi] = 16 * (rt >= 4 ? 1 : sg);
    for (int q = 0; q < net->n_inst; ++q) {
      L.seg_off[gi][q] = (int32_t)nt;
      const ChainInst &C = net->P.cinst[q];
      int nm = 0;
      for (int c = 0; c < C.n_chains; ++c) {
        const int crt = net->P.chains[C.chain_off + c].rt;
        nm += (crt > 4 ? 4 : crt) == rt;
      }
      nt += nm * ((L.B[q] + L.per[gi] - 1) / L.per[gi]);
      if (nt > (1 << 30)) return set_err(TNVAN_E_INVALID, "batch too large");
    }
    L.seg_off[gi][net->n_inst] = (int32_t)nt;
  }
  L.n_tasks = (int32_t)nt;
  // scratch: the small tables, then U, the unary sums and the chain partials
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t n8 = sizeof(int64_t) * net->n_inst;
  const size_t oB = take(n8), oS = take(n8), oSp = take(n8), oC = take(n8), oU = take(n8),
               oF = take(n8), oCl = take(sizeof(int32_t) * net->n_inst),
               oTi = take(sizeof(int32_t) * nt), oTc = take(sizeof(int32_t) * nt),
               oTs = take(sizeof(int32_t) * nt), oUb = take(sizeof(float) * uo),
               oFa = take(sizeof(double) * fo), oCp = take(sizeof(double) * cp);
  if (off > (size_t)TNVAN_NOALLOC_SCRATCH_BYTES)
    return set_err(TNVAN_E_INVALID, "the batch needs %zu bytes of scratch, above the %u of "
                                    "the allocation-free call", off,
                   (unsigned)TNVAN_NOALLOC_SCRATCH_BYTES);
  if (so == 0) return TNVAN_OK;
  if (!logz || (!spins && sp > 0)) return set_err(TNVAN_E_INVALID, "spins and logz are required");
  if (tnvan_status s = check_device({spins, logz})) return s;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != net->device)
    return set_err(TNVAN_E_STATE, "the net lives on device %d, device %d is current",
                   net->device, dev);
  char *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev >= 0 && dev < kMaxDevices) base = static_cast<char *>(g_scratch_dev[dev]);
    if (!base)
      return set_err(TNVAN_E_HIP, "no scratch address on device %d: %s", dev,
                     dev >= 0 && dev < kMaxDevices ? g_scratch_err[dev].c_str() : "");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  L.cinst = net->cinst.as<ChainInst>();
  L.chains = net->chains.as<ChainDesc>();
  L.d_B = reinterpret_cast<int64_t *>(base + oB);
  L.d_sample_off = reinterpret_cast<int64_t *>(base + oS);
  L.d_spin_off = reinterpret_cast<int64_t *>(base + oSp);
  L.d_cpart_off = reinterpret_cast<int64_t *>(base + oC);
  L.d_u_off = reinterpret_cast<int64_t *>(base + oU);
  L.d_f_off = reinterpret_cast<int64_t *>(base + oF);
  L.d_clist = reinterpret_cast<int32_t *>(base + oCl);
  L.d_ti = reinterpret_cast<int32_t *>(base + oTi);
  L.d_tc = reinterpret_cast<int32_t *>(base + oTc);
  L.d_ts = reinterpret_cast<int32_t *>(base + oTs);
  float *U = reinterpret_cast<float *>(base + oUb);
  double *fabp = reinterpret_cast<double *>(base + oFa), *cpart = reinterpret_cast<double *>(base + oCp);
  HIPCHK(launch_layout(L, st));
  ChainArgs c = chain_args(net, false);
  c.spins = spins;
  c.inst_B = L.d_B;
  c.inst_sample_off = L.d_sample_off;
  c.inst_spin_off = L.d_spin_off;
  c.cpart_off = L.d_cpart_off;
  c.cpart = cpart;
  c.U = U;
  c.u_off = L.d_u_off;
  c.u_all = 1;
  c.task_inst = L.d_ti;
  c.task_chain = L.d_tc;
  c.task_start = L.d_ts;
  HIPCHK(launch_unary(c, L.d_clist, net->n_inst, max_nch, maxB, L.d_f_off, U, fabp, st));
  for (int gi = 0; gi < 3; ++gi) {
    c.task_base = L.seg_off[gi][0];
    c.n_tasks = L.seg_off[gi][net->n_inst] - L.seg_off[gi][0];
    c.ntm = 1 << gi;
    c.sg = (1 << gi) >= 4 ? 1 : sg;
    if (c.n_tasks > 0) HIPCHK(launch_rchain(c, false, st));
  }
  HIPCHK(launch_chain_sum(net->inst.as<InstDesc>(), net->cinst.as<ChainInst>(), L.d_clist,
                          net->n_inst, L.d_B, L.d_sample_off, L.d_cpart_off, cpart, L.d_f_off,
                          fabp, logz, st));
  return TNVAN_OK;
}

tnvan_status tnvan_get_tuning(const tnvan_net *net, tnvan_tuning *out) {
  if (tnvan_status s = check_net(net)) return s;
  if (!out) return set_err(TNVAN_E_INVALID, "out is NULL");
  *out = tnvan_tuning{};
  bool gen = false, chain = false;
  for (int q = 0; q < net->n_inst; ++q) (net->use_chain[q] ? chain : gen) = true;
  out->kinds = (gen ? TNVAN_TUNE_GENERAL : 0) | (chain && net->rfwd ? TNVAN_TUNE_REG_CHAIN : 0) |
               (chain && !net->rfwd ? TNVAN_TUNE_LDS_CHAIN : 0);
  out->general_tile_fwd = gen ? net->S_fwd : 0;
  out->general_tile_bwd = gen ? net->S_bwd : 0;
  out->chain_groups = chain && net->rfwd ? (net->tune.chain_groups > 0 ? net->tune.chain_groups
                                                                       : net->ckey.empty() ? 0 : net->sg)
                                         : 0;
  out->checkpoint_every = chain && net->rbwd ? net->lim_bwd.rk : 0;
  out->launch_mode = net->tune.launch_mode > 0 ? net->tune.launch_mode : 1;
  out->arena_limit_mib = net->tune.arena_limit_mib;
  return TNVAN_OK;
}

tnvan_status tnvan_set_tuning(tnvan_net *net, const tnvan_tuning *in) {
  if (tnvan_status s = check_net(net)) return s;
  if (!in) return set_err(TNVAN_E_INVALID, "tuning is NULL");
  auto tile_ok = [](int v) { return v == 0 || (v >= 1 && v <= 64 && (v & (v - 1)) == 0); };
  if (!tile_ok(in->general_tile_fwd) || !tile_ok(in->general_tile_bwd))
    return set_err(TNVAN_E_INVALID, "general tiles must be 0 or a power of two up to 64");
  if (in->chain_groups < 0 || in->chain_groups > 2)
    return set_err(TNVAN_E_INVALID, "chain_groups must be 0, 1 or 2");
  const int k = in->checkpoint_every;
  if (k != 0 && k != 1 && k != 2 && k != 4 && k != 8)
    return set_err(TNVAN_E_INVALID, "checkpoint_every must be 0, 1, 2, 4 or 8");
  if (in->launch_mode < 0 || in->launch_mode > 2)
    return set_err(TNVAN_E_INVALID, "launch_mode must be 0, 1 or 2");
  if (in->arena_limit_mib < 0) return set_err(TNVAN_E_INVALID, "arena_limit_mib must be >= 0");
  if (net->rbwd) {
    // the replayed states of one segment live in LDS beside each wave's data
    ChainLim L = net->lim_bwd;
    L.rk = k > 0 ? k : net->rk_build;
    int dev = 0, maxlds = 65536;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (4 * rchain_wave_lds(L, true, 1) > (size_t)maxlds)
      return set_err(TNVAN_E_INVALID, "checkpoint_every %d does not fit the LDS", L.rk);
  }
  const tnvan_tuning old = net->tune;
  net->tune = tnvan_tuning{};
  net->tune.general_tile_fwd = in->general_tile_fwd;
  net->tune.general_tile_bwd = in->general_tile_bwd;
  net->tune.chain_groups = in->chain_groups;
  net->tune.checkpoint_every = k;
  net->tune.launch_mode = in->launch_mode;
  net->tune.arena_limit_mib = in->arena_limit_mib;
  net->lim_bwd.rk = k > 0 ? k : net->rk_build;
  if (!choose_tiles(net, false, in->general_tile_fwd) || !choose_tiles(net, true, in->general_tile_bwd)) {
    net->tune = old;
    net->lim_bwd.rk = old.checkpoint_every > 0 ? old.checkpoint_every : net->rk_build;
    choose_tiles(net, false, old.general_tile_fwd);
    choose_tiles(net, true, old.general_tile_bwd);
    return set_err(TNVAN_E_INVALID, "a requested general tile does not fit the LDS");
  }
  // every per-call table is laid out again at the next call (after a wait
  // for the work queued with the old layout), and a recorded step is stale
  net->tc_fwd.key.clear();
  net->tc_bwd.key.clear();
  net->ckey.clear();
  g_buf_gen.fetch_add(1);
  return TNVAN_OK;
}

tnvan_status tnvan_program_info(const tnvan_net *net, int32_t inst, int64_t info[6]) {
  if (tnvan_status s = check_net(net)) return s;
  if (inst < 0 || inst >= net->n_inst || !info) return set_err(TNVAN_E_INVALID, "bad instance index");
  const InstDesc &D = net->P.insts[inst];
  info[0] = D.n_steps; info[1] = D.max_w; info[2] = D.arena_all;
  info[3] = net->P.flops_fwd[inst]; info[4] = D.nw; info[5] = D.nr;
  return TNVAN_OK;
}

tnvan_status tnvan_profile_mask(tnvan_net *net, uint32_t mask) {
  if (tnvan_status s = check_net(net)) return s;
  if (!net->profile) return set_err(TNVAN_E_STATE, "net built without TNVAN_FLAG_PROFILE");
  net->prof_mask = mask;
  return TNVAN_OK;
}

tnvan_status tnvan_kernel_time(tnvan_net *net, int32_t kernel, double *total_ms,
                               int64_t *launches) {
  if (tnvan_status s = check_net(net)) return s;
  if (kernel < 0 || kernel >= TNVAN_KERNEL_COUNT || !total_ms || !launches)
    return set_err(TNVAN_E_INVALID, "bad kernel id or output pointer");
  if (!net->profile) return set_err(TNVAN_E_STATE, "net built without TNVAN_FLAG_PROFILE");
  double tot = 0.0;
  int64_t n = 0;
  auto &used = net->prof_used[kernel];
  for (auto &e : used) {
    hipError_t r = hipEventSynchronize(e.second);
    float ms = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e.first, e.second);
    if (r != hipSuccess) return set_err(TNVAN_E_HIP, "event timing: %s", hipGetErrorString(r));
    tot += ms;
    ++n;
    net->prof_pool.push_back(e);
  }
  used.clear();
  *total_ms = tot;
  *launches = n;
  return TNVAN_OK;
}

tnvan_status tnvan_plan(const tnvan_instance *inst, int32_t max_width, int64_t info[6]) {
  if (!inst || !info) return set_err(TNVAN_E_INVALID, "instance and info are required");
  HostProgram P;
  std::string msg;
  tnvan_status s = compile_instance(*inst, max_width, P, msg);
  if (s != TNVAN_OK) return set_err(s, "%s", msg.c_str());
  const InstDesc &D = P.insts[0];
  info[0] = D.n_steps; info[1] = D.max_w; info[2] = D.arena_all;
  info[3] = P.flops_fwd[0]; info[4] = D.nw; info[5] = D.nr;
  return TNVAN_OK;
}

tnvan_status tnvan_plan_width_set(int32_t n_spins, int32_t n_edges, const int32_t *edge_i,
                                  const int32_t *edge_j, int32_t w_u, const int32_t *key,
                                  int32_t flags, int32_t *width_set, int32_t *n_width,
                                  int32_t *order, int32_t *greedy, int32_t *width) {
  if (flags & ~TNVAN_PLAN_REGREEDY) return set_err(TNVAN_E_INVALID, "unknown plan flags %d", flags);
  if (!width_set || !n_width || !order || !width)
    return set_err(TNVAN_E_INVALID, "width_set, n_width, order and width are required");
  if (n_edges < 0 || (n_edges > 0 && (!edge_i || !edge_j)))
    return set_err(TNVAN_E_INVALID, "bad edge arrays");
  if (n_spins <= 0 || n_spins > kPlanMaxSpins)
    return set_err(TNVAN_E_INVALID, "n_spins %d out of range 1..%d", n_spins, kPlanMaxSpins);
  std::vector<int32_t> ei(edge_i, edge_i + n_edges), ej(edge_j, edge_j + n_edges), k;
  if (key) k.assign(key, key + n_spins);
  PlanResult R;
  std::string msg;
  if (tnvan_status s = plan_width_set(n_spins, ei, ej, w_u, k, (flags & TNVAN_PLAN_REGREEDY) != 0,
                                      R, msg))
    return set_err(s, "%s", msg.c_str());
  std::copy(R.W.begin(), R.W.end(), width_set);
  std::copy(R.order.begin(), R.order.end(), order);
  if (greedy) std::copy(R.pi.begin(), R.pi.end(), greedy);
  *n_width = (int32_t)R.W.size();
  *width = R.width;
  return TNVAN_OK;
}

}  // extern "C"
