// Instance compiler: validation, edge classification and the elimination
// program (Sec. 2: fixing W turns the W-R couplings into fields on R, and
// the remainder is contracted along the given order).
#include "compile.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
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

// Round-to-nearest-even float -> bfloat16 bits.
uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Recognise the transfer-matrix form (see program.h) and emit padded tables.
void build_chains(const InstDesc &D, const std::vector<int32_t> &consumer, HostProgram &P) {
  ChainInst ci{};
  ci.chain_off = (int32_t)P.chains.size();
  const StepDesc *st = P.steps.data() + D.step_off;
  bool ok = D.n_steps > 0;
  for (int t = 0; t < D.n_steps && ok; ++t) {
    if (st[t].kind != STEP_DENSE || st[t].g > 8 || st[t].w > 8) ok = false;
    if (st[t].w > 0 && consumer[t] < 0) ok = false;
  }
  std::vector<std::vector<int32_t>> chains;
  if (ok) {
    std::vector<int32_t> seen(D.n_steps, 0);
    for (int t0 = 0; t0 < D.n_steps && ok; ++t0) {
      if (st[t0].n_in != 0) continue;
      std::vector<int32_t> ch;
      int t = t0;
      while (true) {
        if (seen[t]) { ok = false; break; }
        seen[t] = 1;
        ch.push_back(t);
        if (st[t].w == 0) break;
        const int nx = consumer[t];
        const InputDesc &id = P.inputs[st[nx].in_off];
        if (st[nx].n_in != 1 || id.step != t || st[nx].g != st[t].w) { ok = false; break; }
        t = nx;
      }
      if (!ok) break;
      // the chain's positions must be one contiguous range
      int lo = st[ch[0]].gpos, hi = lo;
      for (int u : ch) {
        if (st[u].gpos != hi) ok = false;
        hi = st[u].gpos + st[u].g;
      }
      chains.push_back(ch);
    }
    for (int t = 0; t < D.n_steps; ++t) if (!seen[t]) ok = false;
  }
  if (!ok) {
    ci.ok = 0;
    P.cinst.push_back(ci);
    return;
  }
  ci.ok = 1;
  ci.nw = D.nw;
  bool ok_rq = true;
  for (int p = 0; p < D.nr; ++p)
    if (P.fld_ptr[D.fld_off + p + 1] - P.fld_ptr[D.fld_off + p] > 4) ok_rq = false;
  ci.n_chains = (int32_t)chains.size();
  for (auto &ch : chains) {
    ChainDesc cd{};
    cd.n_steps = (int32_t)ch.size();
    cd.cs_off = (int32_t)P.csteps.size();
    cd.pos_lo = st[ch.front()].gpos;
    cd.pos_hi = st[ch.back()].gpos + st[ch.back()].g;
    cd.tl_src = (int64_t)P.Tl.size();
    cd.tbl_src = (int64_t)P.Tbl.size();
    cd.e_src = (int32_t)P.cedges.size();
    cd.f_lo = P.fld_ptr[D.fld_off + cd.pos_lo];
    cd.f_hi = P.fld_ptr[D.fld_off + cd.pos_hi];
    ci.npos_max = std::max(ci.npos_max, cd.pos_hi - cd.pos_lo);
    ci.max_steps = std::max(ci.max_steps, cd.n_steps);
    // register-resident form: one tile count for every step of the chain
    int rt = 1;
    for (int t : ch) {
      const int K = 1 << st[t].g, N = st[t].w == 0 ? 1 : 1 << st[t].w;
      while (16 * rt < K || 16 * rt < N) rt <<= 1;
    }
    cd.rt = rt;
    ci.rtiles = std::max(ci.rtiles, rt);
    for (int t : ch) {
      const StepDesc &sd = st[t];
      ChainStep cs{};
      cs.step = t;
      cs.g = sd.g; cs.w = sd.w; cs.gpos = sd.gpos;
      const int K = 1 << sd.g, N = 1 << sd.w;
      cs.kp = std::max(16, K);
      cs.kb = std::max(32, K);
      cs.np = sd.w == 0 ? 1 : std::max(16, N);
      cs.n_edge = sd.n_edge;
      cs.edge_off = sd.edge_off;
      ci.kbuf = std::max({ci.kbuf, cs.kb, cs.np});
      ci.gmax = std::max(ci.gmax, sd.g);
      ci.pmax = std::max(ci.pmax, cs.kp * (sd.w + 1));
      const double *T = P.T.data() + sd.t_off;
      cs.tp_off = (int64_t)P.Tp.size();
      for (int x = 0; x < cs.kp; ++x)
        for (int o = 0; o < cs.np; ++o)
          P.Tp.push_back((x < K && o < N) ? (float)T[((int64_t)x << sd.w) | o] : 0.0f);
      cs.tt_off = (int64_t)P.Tt.size();
      for (int o = 0; o < cs.np; ++o)
        for (int x = 0; x < cs.kp; ++x)
          P.Tt.push_back((x < K && o < N) ? (float)T[((int64_t)x << sd.w) | o] : 0.0f);
      cs.tb_off = (int64_t)P.Tb.size();
      cs.tbl_off = (int32_t)(P.Tbl.size() - cd.tbl_src);
      if (sd.w > 0) {
        const int KC = cs.kb / 32, NT = cs.np / 16;
        for (int nt = 0; nt < NT; ++nt)
          for (int kc = 0; kc < KC; ++kc)
            for (int l = 0; l < 64; ++l)
              for (int i = 0; i < 8; ++i) {
                const int x = 32 * kc + 8 * (l / 16) + i, o = 16 * nt + l % 16;
                const float v = (x < K && o < N) ? (float)T[((int64_t)x << sd.w) | o] : 0.0f;
                P.Tb.push_back(to_bf16(v));
                P.Tbl.push_back(to_bf16(v));
              }
      }
      // rows padded by one word: lanes walking down a column hit distinct banks
      cs.tl_off = (int32_t)(P.Tl.size() - cd.tl_src);
      for (int x = 0; x < cs.kp; ++x) {
        for (int o = 0; o < cs.np; ++o)
          P.Tl.push_back((x < K && o < N) ? (float)T[((int64_t)x << sd.w) | o] : 0.0f);
        P.Tl.push_back(0.0f);
      }
      cs.ce_off = (int32_t)P.cedges.size() - cd.e_src;
      // register-resident operand tables (program.h: R-layout)
      auto tv = [&](int x, int o) {
        return (x < K && o < N) ? (float)T[((int64_t)x << sd.w) | o] : 0.0f;
      };
      const int CT = rt, KC2 = (CT + 1) / 2;
      cs.nt16 = sd.w == 0 ? 1 : cs.np / 16;
      cs.tr_off = (int64_t)P.Tr.size();
      for (int nt = 0; nt < CT; ++nt)
        for (int xt = 0; xt < CT; ++xt)
          for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) P.Tr.push_back(tv(16 * xt + 4 * (l >> 4) + r, 16 * nt + (l & 15)));
      cs.tq_off = (int64_t)P.Tq.size();
      for (int xt = 0; xt < CT; ++xt)
        for (int nt = 0; nt < CT; ++nt)
          for (int l = 0; l < 64; ++l)
            for (int r = 0; r < 4; ++r) P.Tq.push_back(tv(16 * xt + (l & 15), 16 * nt + 4 * (l >> 4) + r));
      cs.trb_off = (int64_t)P.Trb.size();
      for (int nt = 0; nt < CT; ++nt)
        for (int c = 0; c < KC2; ++c)
          for (int l = 0; l < 64; ++l)
            for (int i = 0; i < 8; ++i)
              P.Trb.push_back(to_bf16(tv(16 * (2 * c + (i >> 2)) + 4 * (l >> 4) + (i & 3), 16 * nt + (l & 15))));
      // adjoint columns: the group's spins, then the edges inside the group
      cs.xc_off = (int32_t)P.xcol.size();
      int32_t xc[16];
      for (int c = 0; c < 16; ++c) xc[c] = c < sd.g ? (c | (31 << 8)) : -1;
      int nxx = 0;
      for (int k = 0; k < sd.n_edge; ++k) {
        EdgeDesc e = P.edges[sd.edge_off + k];
        if (e.bu < sd.w) std::swap(e.bu, e.bv);
        if (e.bu < sd.w) { ok_rq = false; e.pad = 0; }
        else if (e.bv >= sd.w) {
          const int col = sd.g + nxx++;
          if (col < 16 && sd.w < 16) xc[col] = (e.bu - sd.w) | ((e.bv - sd.w) << 8);
          else ok_rq = false;
          e.pad = col * 16 + sd.w;
        } else {
          e.pad = (e.bu - sd.w) * 16 + e.bv;
        }
        P.cedges.push_back(e);
      }
      if (sd.w >= 16) ok_rq = false;
      for (int c = 0; c < 16; ++c) P.xcol.push_back(xc[c]);
      // adjoint destinations of the 256 cells, in the R-layout lane order
      {
        int32_t dq[256];
        for (int c = 0; c < 256; ++c) dq[c] = -1;
        if (sd.w < 16) {
          for (int j = 0; j < sd.g && j < 16; ++j) dq[j * 16 + sd.w] = sd.gpos + j;
          for (int k = cs.ce_off; k < (int)P.cedges.size() - cd.e_src; ++k) {
            const EdgeDesc &e = P.cedges[cd.e_src + k];
            if (e.pad >= 0 && e.pad < 256) dq[e.pad] = D.nr + D.n_wr + e.rr;
          }
        }
        cs.dq_off = (int32_t)P.Tdq.size();
        for (int l = 0; l < 64; ++l)
          for (int r = 0; r < 4; ++r) P.Tdq.push_back(dq[(l & 15) * 16 + 4 * (l >> 4) + r]);
      }
      // S_x operand of lane l: column l & 15 at state x = 16 xt + 4 (l >> 4) + r;
      // S_o operand: row j = l & 15 (output spin j < w, all-ones j = w) at
      // output state o = 16 ot + 4 (l >> 4) + r
      // W-R couplings of the group, in the step descriptor
      cs.n_wri = 0;
      for (int j = 0; j < sd.g; ++j) {
        const int pos = sd.gpos + j;
        for (int k = P.fld_ptr[D.fld_off + pos]; k < P.fld_ptr[D.fld_off + pos + 1]; ++k) {
          if (cs.n_wri >= 4) { ok_rq = false; break; }
          cs.wri[cs.n_wri] = j | (P.fld_w[D.fld_nnz_off + k] << 8);
          cs.wre[cs.n_wri] = P.fld_wr[D.fld_nnz_off + k];
          ++cs.n_wri;
        }
      }
      cs.sx_off = (int64_t)P.Tsx.size();
      auto par = [](int v) { return __builtin_popcount((unsigned)v) & 1; };
      for (int xt = 0; xt < CT; ++xt)
        for (int l = 0; l < 64; ++l)
          for (int r = 0; r < 4; ++r) {
            const int code = xc[l & 15], x = 16 * xt + 4 * (l >> 4) + r;
            float v = 0.f;
            if (code >= 0) {
              const int cu = code & 0xff, cv = (code >> 8) & 0xff;
              const int m = (1 << cu) | (cv < 31 ? (1 << cv) : 0);
              v = par(x & m) ? -1.f : 1.f;
            }
            P.Tsx.push_back(v);
          }
      auto so_val = [&](int o, int j) {
        return j < sd.w ? (((o >> j) & 1) ? -1.f : 1.f) : (j == sd.w ? 1.f : 0.f);
      };
      auto sx_val = [&](int x, int col) {
        const int code = xc[col];
        if (code < 0) return 0.f;
        const int cu = code & 0xff, cv = (code >> 8) & 0xff;
        const int m = (1 << cu) | (cv < 31 ? (1 << cv) : 0);
        return par(x & m) ? -1.f : 1.f;
      };
      for (int ot = 0; ot < CT; ++ot)
        for (int l = 0; l < 64; ++l)
          for (int r = 0; r < 4; ++r) P.Tsx.push_back(so_val(16 * ot + 4 * (l >> 4) + r, l & 15));
      // split-BF16 tables (program.h)
      {
        auto st3 = [&](int c, int l, int j) {   // state of element j, or -1
          const int t = 2 * c + (j >> 2);
          return t < CT ? 16 * t + 4 * (l >> 4) + (j & 3) : -1;
        };
        auto hi = [](float v) { return to_bf16(v); };
        auto lo = [](float v) {
          const uint16_t h = to_bf16(v);
          uint32_t u = (uint32_t)h << 16;
          float hv;
          std::memcpy(&hv, &u, 4);
          return to_bf16(v - hv);
        };
        cs.s3_off = (int64_t)P.Ts3.size();
        for (int part = 0; part < 2; ++part)
          for (int nt = 0; nt < CT; ++nt)
            for (int c = 0; c < KC2; ++c)
              for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 8; ++j) {
                  const int x = st3(c, l, j);
                  const float v = x < 0 ? 0.f : tv(x, 16 * nt + (l & 15));
                  P.Ts3.push_back(part ? lo(v) : hi(v));
                }
        for (int part = 0; part < 2; ++part)
          for (int xt = 0; xt < CT; ++xt)
            for (int c = 0; c < KC2; ++c)
              for (int l = 0; l < 64; ++l)
                for (int j = 0; j < 8; ++j) {
                  const int o = st3(c, l, j);
                  const float v = o < 0 ? 0.f : tv(16 * xt + (l & 15), o);
                  P.Ts3.push_back(part ? lo(v) : hi(v));
                }
        for (int c = 0; c < KC2; ++c)
          for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 8; ++j) {
              const int x = st3(c, l, j);
              P.Ts3.push_back(to_bf16(x < 0 ? 0.f : sx_val(x, l & 15)));
            }
        for (int c = 0; c < KC2; ++c)
          for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 8; ++j) {
              const int o = st3(c, l, j);
              P.Ts3.push_back(to_bf16(o < 0 ? 0.f : so_val(o, l & 15)));
            }
      }
      P.csteps.push_back(cs);
    }
    cd.tl_size = (int32_t)(P.Tl.size() - cd.tl_src);
    cd.tbl_size = (int32_t)(P.Tbl.size() - cd.tbl_src);
    cd.n_e = (int32_t)P.cedges.size() - cd.e_src;
    ci.tl_max = std::max(ci.tl_max, cd.tl_size);
    ci.tbl_max = std::max(ci.tbl_max, cd.tbl_size);
    ci.ne_max = std::max(ci.ne_max, cd.n_e);
    ci.nf_max = std::max(ci.nf_max, cd.f_hi - cd.f_lo);
    P.chains.push_back(cd);
  }
  ci.rq_ok = ok_rq ? 1 : 0;
  P.cinst.push_back(ci);
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
  if (in.depth < 0 || in.depth > 4) { fail(msg, "depth %ld out of range (0..4)", in.depth); return TNVAN_E_INVALID; }
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
  std::vector<std::vector<int32_t>> fldk(nr);                        // W-R edge index
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
      P.ww_e.push_back(e);
    } else if (wa || wb) {
      int w = wa ? a : b, r = wa ? b : a;
      P.wr_pos.push_back(pos[r]); P.wr_w.push_back(widx[w]);
      P.wr_edge.push_back(e); P.wr_J.push_back(J);
      fld[pos[r]].push_back({widx[w], J});
      fldk[pos[r]].push_back((int32_t)P.wr_pos.size() - 1 - D.wr_off);
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
      for (size_t k = 0; k < fld[p].size(); ++k) {
        P.fld_w.push_back(fld[p][k].first); P.fld_J.push_back(fld[p][k].second);
        P.fld_wr.push_back(fldk[p][k]); ++c;
      }
    }
    P.fld_ptr.push_back(c);
    // dense form: four (W index, J, W-R edge) slots per R position, unused
    // slots (0, 0, -1); positions with more W-neighbours keep only the CSR
    for (int p = 0; p < nr; ++p)
      for (int k = 0; k < 4; ++k) {
        const bool u = k < (int)fld[p].size();
        P.cf_w.push_back(u ? fld[p][k].first : 0);
        P.cf_J.push_back(u ? (float)fld[p][k].second : 0.0f);
        P.cf_r.push_back(u ? fldk[p][k] : -1);
      }
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
    // single-spin steps may reach kMaxW output bits (wide steps); grouped
    // steps keep their full tables, 2^(g + w) <= 2^20 entries
    if (g + w > 20 && !(g == 1 && w <= kMaxW)) { fail(msg, "step %ld: group plus scope above 20 bits", t); return TNVAN_E_WIDTH; }
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
    const bool wide = w > kTabW;
    if (wide && (dense || (int)ins.size() > kWideIn)) {
      fail(msg, "step %ld: a message over %ld spins from a grouped step or with too many inputs", t, w);
      return TNVAN_E_WIDTH;
    }
    // inputs
    sd.in_off = (int32_t)P.inputs.size();
    for (auto &m : ins) {
      InputDesc id{};
      id.step = m.step;
      id.nbits = (int32_t)m.scope.size();
      id.xbit = -1;
      id.omask = 0;
      for (int b = 0; b < id.nbits; ++b) {
        int p = m.scope[b];
        if (p >= gs && p < ge) { id.src[b] = -1; id.xbit = b; }
        else {
          int j = (int)(std::lower_bound(S.begin(), S.end(), p) - S.begin());
          id.src[b] = (int8_t)j;
          id.omask |= 1 << j;
        }
      }
      id.gb_off = -1;
      if (wide) {
        // split tables: the entry for o's low 10 bits and for its high bits
        id.gb_off = (int32_t)P.gtab2.size();
        for (int part = 0; part < 2; ++part)
          for (int j = 0; j < 1024; ++j) {
            const int o = part ? j << 10 : j;
            uint32_t idx = 0;
            for (int b = 0; b < id.nbits; ++b)
              if (id.src[b] >= 0 && o < (1 << w)) idx |= (uint32_t)((o >> id.src[b]) & 1) << b;
            P.gtab2.push_back(idx);
          }
      } else if (!dense) {
        // the input's entry for every output entry o (eliminated spin +1)
        if (P.gtab.size() + ((size_t)1 << w) > (size_t)INT32_MAX) {
          fail(msg, "gather tables above 2^31 entries");
          return TNVAN_E_INVALID;
        }
        id.gb_off = (int32_t)P.gtab.size();
        for (int o = 0; o < (1 << w); ++o) {
          int idx = 0;
          for (int b = 0; b < id.nbits; ++b)
            if (id.src[b] >= 0) idx |= ((o >> id.src[b]) & 1) << b;
          P.gtab.push_back((uint16_t)idx);
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
        {
          const double Jv = rrJ[nb.second];
          const double sm = std::exp(-2.0 * beta * std::fabs(Jv));
          P.esmall.push_back(Jv < 0.0 ? -sm : sm);
        }
        tb.push_back({bu, bv});
        tj.push_back(rrJ[nb.second]);
        log_const += beta * std::fabs(rrJ[nb.second]);
      }
    }
    sd.n_edge = (int32_t)P.edges.size() - sd.edge_off;
    if (wide && sd.n_edge > kWideEdges) {
      fail(msg, "step %ld: a message over %ld spins consuming too many edges", t, w);
      return TNVAN_E_WIDTH;
    }
    // T[(x << w) | o] = prod_e exp(beta J s_u s_v - beta |J|), bit 1 <=> spin -1
    // (a wide step forms it on the fly from its edges)
    sd.t_off = wide ? -1 : (int64_t)P.T.size();
    const int64_t nT = wide ? 0 : (int64_t)1 << (g + w);
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
  build_chains(D, consumer, P);
  {
    // the adjoint's outputs, vertices then edges: the output of every
    // partial column, and per output the dbeta coefficient of its column
    // (0 for W vertices and W-W edges, which have none)
    const size_t o0 = P.pcoef_out.size();
    P.pcoef_out.resize(o0 + n + in.n_edges, 0.0);
    for (int k = 0; k < nr; ++k) {
      const int o = P.vr[D.vr_off + k];
      P.col_out.push_back(o);
      P.pcoef_out[o0 + o] = P.hR[D.hr_off + k];
    }
    for (int j = 0; j < D.n_wr; ++j) {
      const int o = n + P.wr_edge[D.wr_off + j];
      P.col_out.push_back(o);
      P.pcoef_out[o0 + o] = P.wr_J[D.wr_off + j];
    }
    for (int j = 0; j < D.n_rr; ++j) {
      const int o = n + P.rr_edge[D.rr_off + j];
      P.col_out.push_back(o);
      P.pcoef_out[o0 + o] = P.rr_J[D.rr_off + j];
    }
  }
  P.insts.push_back(D);
  P.hidden.push_back(in.hidden);
  P.depth.push_back(in.hidden > 0 && in.depth > 1 ? in.depth : 1);
  P.flops_fwd.push_back(flops);
  return TNVAN_OK;
}

}  // namespace tnvan
