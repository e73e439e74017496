// Instance compiler: validation, edge classification and the elimination
// program (Sec. 2: fixing W turns the W-R couplings into fields on R, and
// the remainder is contracted along the given order).
#include "compile.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <set>
#include <utility>

namespace tnvan {

namespace {

struct Msg {
  int32_t step;                 // local step index
  std::vector<int32_t> scope;   // ascending order positions
};

// First-fit allocator over a linear arena (entries), used for the
// liveness-reusing layout of the forward-only kernel.
struct Arena {
  std::map<int32_t, int32_t> free_;   // offset -> size
  int32_t top = 0;
  int32_t alloc(int32_t size) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= size) {
        int32_t off = it->first, rest = it->second - size;
        free_.erase(it);
        if (rest) free_[off + size] = rest;
        return off;
      }
    }
    int32_t off = top;
    top += size;
    return off;
  }
  void release(int32_t off, int32_t size) {
    auto it = free_.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

bool fail(std::string &msg, const char *fmt, long a = 0, long b = 0) {
  char buf[256];
  snprintf(buf, sizeof buf, fmt, a, b);
  msg = buf;
  return false;
}

}  // namespace

tnvan_status compile_instance(const tnvan_instance &in, int max_width,
                              HostProgram &P, std::string &msg) {
  const int n = in.n_spins;
  if (n <= 0 || n > (1 << 24)) { fail(msg, "n_spins %ld out of range", n); return TNVAN_E_INVALID; }
  if (in.n_edges < 0 || (in.n_edges > 0 && (!in.edge_i || !in.edge_j || !in.J))) {
    fail(msg, "bad edge arrays"); return TNVAN_E_INVALID;
  }
  if (!(std::isfinite(in.beta) && in.beta >= 0.0)) { fail(msg, "beta must be finite and >= 0"); return TNVAN_E_INVALID; }
  if (in.n_width < 0 || in.n_order < 0 || in.n_width + in.n_order != n ||
      (in.n_width > 0 && !in.width_set) || (in.n_order > 0 && !in.order)) {
    fail(msg, "width set (%ld) and order (%ld) must partition the spins", in.n_width, in.n_order);
    return TNVAN_E_INVALID;
  }
  if (in.hidden < 0 || in.hidden > 65536) { fail(msg, "hidden width %ld out of range", in.hidden); return TNVAN_E_INVALID; }
  if (max_width <= 0 || max_width > kMaxW) max_width = kMaxW;

  std::vector<int32_t> pos(n, -1), widx(n, -1);
  for (int k = 0; k < in.n_width; ++k) {
    int v = in.width_set[k];
    if (v < 0 || v >= n || widx[v] >= 0) { fail(msg, "width_set[%ld] = %ld invalid or repeated", k, v); return TNVAN_E_INVALID; }
    widx[v] = k;
  }
  for (int k = 0; k < in.n_order; ++k) {
    int v = in.order[k];
    if (v < 0 || v >= n || pos[v] >= 0 || widx[v] >= 0) { fail(msg, "order[%ld] = %ld invalid, repeated or in W", k, v); return TNVAN_E_INVALID; }
    pos[v] = k;
  }
  const int nr = in.n_order, nw = in.n_width;

  // groups
  std::vector<int32_t> gp;
  if (in.n_groups > 0) {
    if (!in.group_ptr) { fail(msg, "group_ptr missing"); return TNVAN_E_INVALID; }
    gp.assign(in.group_ptr, in.group_ptr + in.n_groups + 1);
    if (gp.front() != 0 || gp.back() != nr) { fail(msg, "group_ptr must run from 0 to n_order"); return TNVAN_E_INVALID; }
    for (int k = 0; k < in.n_groups; ++k) {
      int sz = gp[k + 1] - gp[k];
      if (sz <= 0 || sz > kMaxG) { fail(msg, "group %ld has size %ld (1..8 allowed)", k, sz); return TNVAN_E_INVALID; }
    }
  } else {
    gp.resize(nr + 1);
    for (int k = 0; k <= nr; ++k) gp[k] = k;
  }

  InstDesc D{};
  D.n = n; D.n_edges = in.n_edges; D.nw = nw; D.nr = nr;
  D.beta = in.beta;
  const double beta = in.beta;

  // fields and edge classes
  std::vector<double> h(n, 0.0);
  if (in.h) for (int v = 0; v < n; ++v) {
    if (!std::isfinite(in.h[v])) { fail(msg, "h[%ld] not finite", v); return TNVAN_E_INVALID; }
    h[v] = in.h[v];
  }
  std::set<std::pair<int, int>> seen;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> radj(nr);   // (nbr pos, rr idx)
  std::vector<std::vector<std::pair<int32_t, double>>> fld(nr);     // (w idx, J)
  D.ww_off = (int32_t)P.ww_a.size();
  D.wr_off = (int32_t)P.wr_pos.size();
  D.rr_off = (int32_t)P.rr_edge.size();
  int n_rr = 0;
  std::vector<double> rrJ;
  for (int e = 0; e < in.n_edges; ++e) {
    int a = in.edge_i[e], b = in.edge_j[e];
    if (a < 0 || b >= n || a >= b) { fail(msg, "edge %ld must satisfy 0 <= i < j < n", e); return TNVAN_E_INVALID; }
    if (!seen.insert({a, b}).second) { fail(msg, "edge %ld is a duplicate", e); return TNVAN_E_INVALID; }
    double J = in.J[e];
    if (!std::isfinite(J)) { fail(msg, "J[%ld] not finite", e); return TNVAN_E_INVALID; }
    bool wa = widx[a] >= 0, wb = widx[b] >= 0;
    if (wa && wb) {
      P.ww_a.push_back(widx[a]); P.ww_b.push_back(widx[b]); P.ww_J.push_back(J);
    } else if (wa || wb) {
      int w = wa ? a : b, r = wa ? b : a;
      P.wr_pos.push_back(pos[r]); P.wr_w.push_back(widx[w]);
      P.wr_edge.push_back(e); P.wr_J.push_back(J);
      fld[pos[r]].push_back({widx[w], J});
    } else {
      P.rr_edge.push_back(e); P.rr_J.push_back(J); rrJ.push_back(J);
      radj[pos[a]].push_back({pos[b], n_rr});
      radj[pos[b]].push_back({pos[a], n_rr});
      ++n_rr;
    }
  }
  D.n_ww = (int32_t)P.ww_a.size() - D.ww_off;
  D.n_wr = (int32_t)P.wr_pos.size() - D.wr_off;
  D.n_rr = n_rr;
  D.n_partial = nr + D.n_wr + D.n_rr;

  D.fld_off = (int32_t)P.fld_ptr.size();
  D.fld_nnz_off = (int32_t)P.fld_w.size();
  {
    int32_t c = 0;
    for (int p = 0; p < nr; ++p) {
      P.fld_ptr.push_back(c);
      for (auto &pr : fld[p]) { P.fld_w.push_back(pr.first); P.fld_J.push_back(pr.second); ++c; }
    }
    P.fld_ptr.push_back(c);
  }
  D.hr_off = (int32_t)P.hR.size();
  D.vr_off = (int32_t)P.vr.size();
  for (int p = 0; p < nr; ++p) { P.hR.push_back(h[in.order[p]]); P.vr.push_back(in.order[p]); }
  D.wv_off = (int32_t)P.wv.size();
  P.hw_off.push_back((int32_t)P.hW.size());
  for (int k = 0; k < nw; ++k) { P.wv.push_back(in.width_set[k]); P.hW.push_back(h[in.width_set[k]]); }

  // elimination program
  D.step_off = (int32_t)P.steps.size();
  std::vector<Msg> active;
  std::vector<int32_t> step_w;            // output size per local step
  std::vector<int32_t> consumer;          // consuming step per local step (-1 root)
  double log_const = 0.0;
  int64_t flops = 0;
  int max_w = 0, scr_fwd = 0, scr_bwd = 0, pbuf = 0;
  const int ngroups = (int)gp.size() - 1;
  for (int k = 0; k < ngroups; ++k) {
    const int gs = gp[k], ge = gp[k + 1], g = ge - gs;
    const int t = (int)step_w.size();
    std::vector<Msg> ins;
    std::vector<Msg> keep;
    for (auto &m : active) {
      bool hit = false;
      for (int p : m.scope) if (p >= gs && p < ge) { hit = true; break; }
      (hit ? ins : keep).push_back(m);
    }
    active.swap(keep);
    std::set<int32_t> out;
    for (auto &m : ins) for (int p : m.scope) if (p >= ge) out.insert(p);
    for (int p = gs; p < ge; ++p)
      for (auto &nb : radj[p]) if (nb.first >= ge) out.insert(nb.first);
    std::vector<int32_t> S(out.begin(), out.end());
    const int w = (int)S.size();
    if (w > max_width) {
      fail(msg, "step %ld creates a message over %ld spins (above the width limit)", t, w);
      return TNVAN_E_WIDTH;
    }
    if (g + w > 20) { fail(msg, "step %ld: group plus scope above 20 bits", t); return TNVAN_E_WIDTH; }
    if ((int)ins.size() > kMaxInputs) { fail(msg, "step %ld has too many input messages", t); return TNVAN_E_INVALID; }
    StepDesc sd{};
    sd.g = g; sd.gpos = gs; sd.w = w; sd.n_in = (int32_t)ins.size();
    bool dense = ins.empty();
    if (ins.size() == 1 && (int)ins[0].scope.size() == g) {
      dense = true;
      for (int j = 0; j < g; ++j) if (ins[0].scope[j] != gs + j) dense = false;
    }
    if (dense) sd.kind = STEP_DENSE;
    else if (g == 1) sd.kind = STEP_SINGLE;
    else {
      fail(msg, "grouped step %ld: its input messages must form exactly one message over the group", t);
      return TNVAN_E_INVALID;
    }
    // inputs
    sd.in_off = (int32_t)P.inputs.size();
    for (auto &m : ins) {
      InputDesc id{};
      id.step = m.step;
      id.nbits = (int32_t)m.scope.size();
      id.xbit = -1;
      for (int b = 0; b < id.nbits; ++b) {
        int p = m.scope[b];
        if (p >= gs && p < ge) { id.src[b] = -1; id.xbit = b; }
        else {
          int j = (int)(std::lower_bound(S.begin(), S.end(), p) - S.begin());
          id.src[b] = (int8_t)j;
        }
      }
      consumer[m.step] = t;
      P.inputs.push_back(id);
    }
    // edges folded into T: R-R edges from G to G (once) or to S_out
    sd.edge_off = (int32_t)P.edges.size();
    std::vector<std::pair<int, int>> tb;    // combined bits
    std::vector<double> tj;
    for (int p = gs; p < ge; ++p) {
      for (auto &nb : radj[p]) {
        int q = nb.first;
        if (q < ge && q <= p) continue;     // earlier step, or counted from the other end
        int bu = w + (p - gs), bv;
        if (q < ge) bv = w + (q - gs);
        else bv = (int)(std::lower_bound(S.begin(), S.end(), q) - S.begin());
        EdgeDesc ed{};
        ed.rr = nb.second; ed.bu = bu; ed.bv = bv;
        P.edges.push_back(ed);
        tb.push_back({bu, bv});
        tj.push_back(rrJ[nb.second]);
        log_const += beta * std::fabs(rrJ[nb.second]);
      }
    }
    sd.n_edge = (int32_t)P.edges.size() - sd.edge_off;
    // T[(x << w) | o] = prod_e exp(beta J s_u s_v - beta |J|), bit 1 <=> spin -1
    sd.t_off = (int64_t)P.T.size();
    const int64_t nT = (int64_t)1 << (g + w);
    for (int64_t c = 0; c < nT; ++c) {
      double lg = 0.0;
      for (size_t e = 0; e < tb.size(); ++e) {
        int su = ((c >> tb[e].first) & 1) ? -1 : 1;
        int sv = ((c >> tb[e].second) & 1) ? -1 : 1;
        lg += beta * (tj[e] * su * sv - std::fabs(tj[e]));
      }
      P.T.push_back(std::exp(lg));
    }
    if (w > 0) active.push_back({t, S});
    step_w.push_back(w);
    consumer.push_back(-1);
    max_w = std::max(max_w, w);
    if (sd.kind == STEP_DENSE) {
      scr_fwd = std::max(scr_fwd, 1 << g);
      scr_bwd = std::max(scr_bwd, (1 << g) * (w + 2));
      pbuf = std::max(pbuf, (1 << g) * (w + 1));
      flops += 2 * nT + (int64_t)(g + (sd.n_in ? 1 : 0)) * (1 << g);
    } else {
      scr_bwd = std::max(scr_bwd, 2 << w);
      flops += (int64_t)(2 << w) * (2 + sd.n_in);
    }
    P.steps.push_back(sd);
  }
  D.n_steps = (int32_t)step_w.size();
  D.log_const = log_const;
  D.max_w = max_w;
  D.scr_fwd = scr_fwd;
  D.scr_bwd = scr_bwd;
  D.pbuf = pbuf;
  // arenas
  {
    int32_t off = 0;
    Arena ar;
    std::vector<int32_t> fwd_off(D.n_steps);
    std::vector<std::vector<int32_t>> frees(D.n_steps);
    for (int t = 0; t < D.n_steps; ++t)
      if (consumer[t] >= 0) frees[consumer[t]].push_back(t);
    for (int t = 0; t < D.n_steps; ++t) {
      int32_t sz = 1 << step_w[t];
      StepDesc &sd = P.steps[D.step_off + t];
      sd.off_all = off;
      off += sz;
      fwd_off[t] = ar.alloc(sz);
      sd.off_fwd = fwd_off[t];
      for (int u : frees[t]) ar.release(fwd_off[u], 1 << step_w[u]);
    }
    D.arena_all = off;
    D.arena_fwd = ar.top;
  }
  P.insts.push_back(D);
  P.hidden.push_back(in.hidden);
  P.flops_fwd.push_back(flops);
  return TNVAN_OK;
}

}  // namespace tnvan
