"""Oracle for the conditional partition function of the remainder R.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (Sec. 2, Eq. 1, with a field term added as the problem statement of
this library asks for it): E(s) = -sum_<ij> J_ij s_i s_j - sum_i h_i s_i,
spins s_i in {+1, -1}.  The width set W is fixed to a sample s_W; the rest R
is summed out (Eqs. 3-4):

  E_1(s_W)    = -sum_{<ij> in W x W} J s_i s_j - sum_{i in W} h_i s_i
  E_2(s_W, r) = -sum_{<ij> in R x R} J r_i r_j - sum_{<ij> in W x R} J s r
                - sum_{i in R} h_i r_i
  logZ_R(s_W) = ln sum_r exp(-beta E_2(s_W, r))
  Etilde(s_W) = E_1(s_W) - logZ_R(s_W) / beta           (Eq. 4)

Functions and what pins them (tests/test_oracle_ising.py):
  energy_split            pinned: E_1 + E_2 = E on random configurations,
                          E from a direct edge sum
  logz_r_bruteforce       the plain definition (enumeration of all r);
                          pinned by beta = 0 (|R| ln 2), the open-chain closed
                          form |R| ln 2 + sum ln cosh(beta J), 2x2 transfer
                          matrices, gauge and global-flip invariance and the
                          slice-sum identity of Eq. 3 against full enumeration
  logz_r_elimination      log-domain variable elimination along the given
                          order; pinned against brute force on random graphs
                          and by order independence
  marginals_bruteforce    <r_i>, <x_i x_j>, <E_2> by enumeration; pinned by
                          central finite differences of logz_r_bruteforce
  marginals_elimination   reverse (outside) pass over the elimination; pinned
                          against marginals_bruteforce, finite differences,
                          the Euler identity and beta = 0
  logz_r_vjp              batch vector-Jacobian product from the marginals
"""

from __future__ import annotations

import numpy as np


def _logsumexp(a: np.ndarray, axis):
    m = np.max(a, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    out = np.log(np.sum(np.exp(a - m), axis=axis, keepdims=True)) + m
    return np.squeeze(out, axis=axis)


class Split:
    """Edge classes and field wiring of an instance for a fixed width set."""

    def __init__(self, inst):
        n = int(inst.n)
        self.n = n
        self.beta = float(inst.beta)
        self.edges = np.asarray(inst.edges, np.int64).reshape(-1, 2)
        self.J = np.asarray(inst.J, np.float64)
        self.h = (np.zeros(n) if inst.h is None
                  else np.asarray(inst.h, np.float64))
        self.W = [int(v) for v in inst.width_set]
        self.order = [int(v) for v in inst.order]
        self.widx = {v: k for k, v in enumerate(self.W)}
        self.R = list(self.order)
        self.rset = set(self.R)
        assert len(self.widx) + len(self.rset) == n
        assert not (set(self.widx) & self.rset)
        ww, wr, rr = [], [], []
        for e, (a, b) in enumerate(self.edges):
            a, b = int(a), int(b)
            ina, inb = a in self.widx, b in self.widx
            if ina and inb:
                ww.append(e)
            elif ina or inb:
                wr.append(e)
            else:
                rr.append(e)
        self.ww, self.wr, self.rr = ww, wr, rr

    def fields_on_r(self, spins: np.ndarray) -> np.ndarray:
        """Effective field on each R vertex: h_r + sum_{w in W} J_rw s_w.

        Returns [B, n] with zeros on W vertices.
        """
        s = np.asarray(spins, np.float64)
        B = s.shape[0]
        f = np.tile(self.h, (B, 1))
        for v in self.W:
            f[:, v] = 0.0
        for e in self.wr:
            a, b = (int(x) for x in self.edges[e])
            w, r = (a, b) if a in self.widx else (b, a)
            f[:, r] += self.J[e] * s[:, self.widx[w]]
        return f


def energy(inst, full: np.ndarray) -> np.ndarray:
    """E(s) of full configurations [B, n] (Eq. 1 plus fields)."""
    s = np.asarray(full, np.float64)
    e = np.asarray(inst.edges, np.int64).reshape(-1, 2)
    h = np.zeros(inst.n) if inst.h is None else np.asarray(inst.h)
    return -(s[:, e[:, 0]] * s[:, e[:, 1]]) @ np.asarray(inst.J) - s @ h


def energy_split(inst, spins: np.ndarray, r: np.ndarray):
    """(E_1(s_W), E_2(s_W, r)) for spins [B, |W|] and r [B, |R|] (R in the
    order given by ``inst.order``)."""
    sp = Split(inst)
    s = np.asarray(spins, np.float64)
    rr = np.asarray(r, np.float64)
    B = s.shape[0]
    full = np.zeros((B, sp.n))
    for k, v in enumerate(sp.W):
        full[:, v] = s[:, k]
    for k, v in enumerate(sp.order):
        full[:, v] = rr[:, k]
    e1 = np.zeros(B)
    for e in sp.ww:
        a, b = sp.edges[e]
        e1 -= sp.J[e] * full[:, a] * full[:, b]
    for v in sp.W:
        e1 -= sp.h[v] * full[:, v]
    e2 = np.zeros(B)
    for e in sp.rr + sp.wr:
        a, b = sp.edges[e]
        e2 -= sp.J[e] * full[:, a] * full[:, b]
    for v in sp.R:
        e2 -= sp.h[v] * full[:, v]
    return e1, e2


def e1_energy(inst, spins: np.ndarray) -> np.ndarray:
    """E_1(s_W) only (interactions and fields inside the width set)."""
    sp = Split(inst)
    s = np.asarray(spins, np.float64)
    e1 = np.zeros(s.shape[0])
    for e in sp.ww:
        a, b = sp.edges[e]
        e1 -= sp.J[e] * s[:, sp.widx[int(a)]] * s[:, sp.widx[int(b)]]
    for v in sp.W:
        e1 -= sp.h[v] * s[:, sp.widx[v]]
    return e1


def _all_configs(m: int) -> np.ndarray:
    """All 2^m spin configurations, [2^m, m], row k has bit j -> spin j."""
    k = np.arange(2 ** m, dtype=np.int64)[:, None]
    bits = (k >> np.arange(m)[None, :]) & 1
    return (1 - 2 * bits).astype(np.float64)


def _r_quadratic(sp: Split):
    """Coupling matrix among R (in order positions) for brute force."""
    pos = {v: k for k, v in enumerate(sp.R)}
    nr = len(sp.R)
    Jrr = np.zeros((nr, nr))
    for e in sp.rr:
        a, b = sp.edges[e]
        Jrr[pos[int(a)], pos[int(b)]] += sp.J[e]
    return Jrr, pos


def logz_r_bruteforce(inst, spins: np.ndarray, chunk: int = 1 << 14) -> np.ndarray:
    """ln sum_r exp(-beta E_2(s_W, r)) by enumerating all r (|R| <= 22)."""
    sp = Split(inst)
    nr = len(sp.R)
    s = np.asarray(spins)
    B = s.shape[0]
    if nr == 0:
        return np.zeros(B)
    assert nr <= 22, "brute force limited to |R| <= 22"
    Jrr, pos = _r_quadratic(sp)
    f = sp.fields_on_r(s)[:, sp.R]                       # [B, nr]
    out = np.full(B, -np.inf)
    for c0 in range(0, 2 ** nr, chunk):
        k = np.arange(c0, min(2 ** nr, c0 + chunk), dtype=np.int64)[:, None]
        r = (1 - 2 * ((k >> np.arange(nr)[None, :]) & 1)).astype(np.float64)
        pair = np.einsum("ci,ij,cj->c", r, Jrr, r)     # sum_RR J r r
        expo = sp.beta * (pair[None, :] + f @ r.T)      # -beta E_2  [B, C]
        out = np.logaddexp(out, _logsumexp(expo, axis=1))
    return out


def marginals_bruteforce(inst, spins: np.ndarray):
    """Per-sample <r_v> (v in R), <x_i x_j> for every edge (x = s on W), and
    <E_2>, by enumerating all r.  Returns (mag [B, n], corr [B, E], e2 [B]);
    mag is zero on W, corr on W-W edges is s_i s_j."""
    sp = Split(inst)
    nr = len(sp.R)
    s = np.asarray(spins, np.float64)
    B = s.shape[0]
    r = _all_configs(nr)                                  # [C, nr]
    Jrr, pos = _r_quadratic(sp)
    f = sp.fields_on_r(s)[:, sp.R]
    pair = np.einsum("ci,ij,cj->c", r, Jrr, r)
    expo = sp.beta * (pair[None, :] + f @ r.T)
    lz = _logsumexp(expo, axis=1)
    p = np.exp(expo - lz[:, None])                        # [B, C] Boltzmann weights
    # <r_v> = sum_c p_c r_v(c); <r_a r_b> = sum_c p_c r_a(c) r_b(c); a W spin
    # is fixed, so its factor comes out of the sum
    magR = p @ r                                          # [B, nr]
    mag = np.zeros((B, sp.n))
    mag[:, sp.R] = magR
    corr = np.zeros((B, len(sp.edges)))
    for e in sp.rr:
        a, b = (pos[int(x)] for x in sp.edges[e])
        corr[:, e] = p @ (r[:, a] * r[:, b])
    for e in sp.wr:
        a, b = (int(x) for x in sp.edges[e])
        w, v = (a, b) if a in sp.widx else (b, a)
        corr[:, e] = s[:, sp.widx[w]] * magR[:, pos[v]]
    for e in sp.ww:
        a, b = (int(x) for x in sp.edges[e])
        corr[:, e] = s[:, sp.widx[a]] * s[:, sp.widx[b]]
    e2 = -(p @ pair) - np.sum(f * magR, axis=1)
    return mag, corr, e2


# ---------------------------------------------------------------------------
# log-domain variable elimination

def _align(tab: np.ndarray, scope, U):
    """Broadcast a [B]+[2]*len(scope) table to the axes of scope U."""
    present = [scope.index(u) for u in U if u in scope]
    t = np.transpose(tab, [0] + [1 + i for i in present])
    shape = [tab.shape[0]] + [2 if u in scope else 1 for u in U]
    return t.reshape(shape)


def _spin_axis(k: int, nd: int) -> np.ndarray:
    """+1/-1 values along axis k of an nd-dimensional scope table."""
    shape = [1] * (nd + 1)
    shape[k + 1] = 2
    return np.array([1.0, -1.0]).reshape(shape)


def _initial_factors(sp: Split, spins: np.ndarray):
    """Log-factors of the remainder: one unary per R vertex and one pairwise
    per R-R edge (index 0 of an axis is spin +1, index 1 is spin -1)."""
    f = sp.fields_on_r(spins)
    B = f.shape[0]
    fac = []
    for v in sp.R:
        tab = sp.beta * f[:, v][:, None] * np.array([1.0, -1.0])[None, :]
        fac.append(((v,), tab, ("unary", v)))
    for e in sp.rr:
        a, b = (int(x) for x in sp.edges[e])
        xy = np.array([[1.0, -1.0], [-1.0, 1.0]])
        tab = (sp.beta * sp.J[e] * xy)[None, :, :]
        fac.append(((a, b), np.broadcast_to(tab, (1, 2, 2)), ("edge", e)))
    return fac, B


def _eliminate(sp: Split, spins: np.ndarray, keep: bool):
    """Forward pass; returns (logZ_R [B], per-step records if keep)."""
    fac, B = _initial_factors(sp, spins)
    live = list(range(len(fac)))       # indices into `items`
    items = [(sc, tab, tag) for sc, tab, tag in fac]
    records = []
    logz = np.zeros(B)
    for v in sp.order:
        bucket = [k for k in live if v in items[k][0]]
        live = [k for k in live if k not in bucket]
        U = [v]
        for k in bucket:
            for u in items[k][0]:
                if u not in U:
                    U.append(u)
        comb = np.zeros([B] + [2] * len(U))
        for k in bucket:
            comb = comb + _align(items[k][1], list(items[k][0]), U)
        msg = _logsumexp(comb, axis=1)                    # sum out v
        scope = tuple(U[1:])
        if keep:
            records.append({"v": v, "U": U, "bucket": bucket, "comb": comb,
                            "msg_item": len(items)})
        if len(scope) == 0:
            logz = logz + msg
            if keep:
                items.append((scope, msg, ("root", v)))
        else:
            items.append((scope, msg, ("msg", v)))
            live.append(len(items) - 1)
    return logz, records, items


def logz_r_elimination(inst, spins: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """logZ_R by eliminating R one vertex at a time in ``inst.order``,
    every factor kept as a log-table (no grouping, no rescaling)."""
    sp = Split(inst)
    s = np.asarray(spins)
    out = []
    for c0 in range(0, s.shape[0], chunk):
        lz, _, _ = _eliminate(sp, s[c0:c0 + chunk], keep=False)
        out.append(lz)
    return np.concatenate(out) if out else np.zeros(0)


def marginals_elimination(inst, spins: np.ndarray, chunk: int = 1024):
    """Reverse (outside) pass over the elimination of ``logz_r_elimination``.

    For each eliminated vertex the joint log-probability of (v, its message
    scope) is comb + outside - logZ, where the outside term of a message is
    obtained from its consumer by summing the consumer's joint over the
    variables not in the message.  Returns (logz [B], mag [B, n],
    corr [B, E], e2 [B]) like ``marginals_bruteforce``.
    """
    sp = Split(inst)
    s_all = np.asarray(spins, np.float64)
    res = []
    for c0 in range(0, s_all.shape[0], chunk):
        s = s_all[c0:c0 + chunk]
        B = s.shape[0]
        logz, recs, items = _eliminate(sp, s, keep=True)
        outside = {}                                   # item index -> table
        consumer = {}
        for t, rec in enumerate(recs):
            for k in rec["bucket"]:
                consumer[k] = t
        mag = np.zeros((B, sp.n))
        corr = np.zeros((B, len(sp.edges)))
        for t in range(len(recs) - 1, -1, -1):
            rec = recs[t]
            U = rec["U"]
            mi = rec["msg_item"]
            scope = list(items[mi][0])
            if len(scope) == 0:
                out_t = (logz - items[mi][1]).reshape([B])
                out_al = out_t.reshape([B] + [1] * len(U))
            else:
                out_al = _align(outside[mi], scope, U)
            joint = rec["comb"] + out_al - logz.reshape([B] + [1] * len(U))
            P = np.exp(joint)                             # [B] + [2]*|U|
            for k in rec["bucket"]:
                sc, tab, tag = items[k]
                if tag[0] == "msg":
                    other = [a for a in range(len(U)) if U[a] not in sc]
                    lp = np.log(np.maximum(
                        np.sum(P, axis=tuple(1 + a for a in other)), 1e-300))
                    # lp axes are in U order restricted to sc; reorder to sc
                    ordU = [u for u in U if u in sc]
                    perm = [ordU.index(u) for u in sc]
                    lp = np.transpose(lp, [0] + [1 + p for p in perm])
                    outside[k] = lp - tab + logz.reshape([B] + [1] * len(sc))
                elif tag[0] == "unary":
                    v = tag[1]
                    ax = U.index(v)
                    mag[:, v] = np.sum(P * _spin_axis(ax, len(U)),
                                       axis=tuple(range(1, len(U) + 1)))
                elif tag[0] == "edge":
                    e = tag[1]
                    a, b = (int(x) for x in sp.edges[e])
                    corr[:, e] = np.sum(
                        P * _spin_axis(U.index(a), len(U))
                        * _spin_axis(U.index(b), len(U)),
                        axis=tuple(range(1, len(U) + 1)))
        for e in sp.ww:
            a, b = sp.edges[e]
            corr[:, e] = s[:, sp.widx[int(a)]] * s[:, sp.widx[int(b)]]
        for e in sp.wr:
            a, b = (int(x) for x in sp.edges[e])
            w, r = (a, b) if a in sp.widx else (b, a)
            corr[:, e] = s[:, sp.widx[w]] * mag[:, r]
        f = sp.fields_on_r(s)
        e2 = -(corr[:, sp.rr] @ sp.J[sp.rr]) if sp.rr else np.zeros(B)
        e2 = e2 - np.sum(f[:, sp.R] * mag[:, sp.R], axis=1)
        res.append((logz, mag, corr, e2))
    return tuple(np.concatenate([r[i] for r in res]) for i in range(4))


def logz_r_vjp(inst, spins: np.ndarray, g: np.ndarray, marg=None):
    """Batch VJP of logZ_R: sum_b g_b dlogZ_R(s_b)/d(h, J, beta).

    dlogZ_R/dh_v = beta <r_v> (v in R, else 0); dlogZ_R/dJ_e = beta <x_i x_j>
    for edges touching R (0 on W-W edges); dlogZ_R/dbeta = -<E_2>.
    """
    sp = Split(inst)
    if marg is None:
        _, mag, corr, e2 = marginals_elimination(inst, spins)
    else:
        mag, corr, e2 = marg
    g = np.asarray(g, np.float64)
    dh = sp.beta * (g @ mag)
    dJ = sp.beta * (g @ corr)
    dJ[sp.ww] = 0.0
    dbeta = float(g @ (-e2))
    return dh, dJ, dbeta


def logz_full_bruteforce(inst) -> float:
    """ln Z of the whole system by enumerating all 2^n states (n <= 22)."""
    n = int(inst.n)
    assert n <= 22
    c = _all_configs(n)
    out = -np.inf
    step = 1 << 14
    for c0 in range(0, c.shape[0], step):
        out = np.logaddexp(out, _logsumexp(-inst.beta * energy(inst, c[c0:c0 + step]), 0))
    return float(out)
