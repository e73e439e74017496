"""Oracle for the magnetisation moments and the susceptibility.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Once q is trained, its samples give physical quantities of the Boltzmann
distribution p of Eq. 1, among them the magnetisation and the susceptibility
(Sec. 3, after Eq. 10; the outlook of Sec. 5).  With M = sum_i s_i over all
N spins, the susceptibility per spin is read here as

  chi = beta (<M^2>_p - <M>_p^2) / N

(the fluctuation-dissipation form, d<M>/dH per spin for a uniform field H).
Given a width-set configuration s_W, M = M_W(s_W) + M_R with M_R the
remainder's magnetisation, whose conditional law p(r | s_W) is proportional
to exp(-beta E_2(s_W, r)) (Eqs. 3-4).  So

  <M>_p   = E_{s_W ~ p} [ M_W + mu_R(s_W) ]
  <M^2>_p = E_{s_W ~ p} [ (M_W + mu_R(s_W))^2 + v_R(s_W) ]

with mu_R and v_R the conditional mean and variance of M_R.  The W-marginal
of p is exp(-beta E_1) Z_R / Z, so from samples of q the expectation is the
self-normalised importance-weighted mean with w_b proportional to
exp(-beta f_b), f_b of Eq. 9.

Functions and what pins them (tests/test_oracle_magnetisation.py):
  remainder_magnetisation_bruteforce
                        the plain definition (enumeration of all r, |R| <= 22);
                        pinned by beta = 0 (mean 0, variance |R|), isolated
                        remainder spins (sum tanh, sum sech^2 of the effective
                        fields), the open chain's product of tanh(beta J)
                        correlations, the global flip, the sum of the
                        marginals of ising.marginals_bruteforce, and the
                        second difference of ising.logz_r_bruteforce in a
                        uniform field on R
  remainder_magnetisation_distribution
                        log P(M_R = |R| - 2k | s_W), k = 0..|R|, by
                        log-domain elimination along the order in which
                        every factor also carries the count k of -1 spins
                        summed into it; pinned against the brute-force
                        distribution and, at |R| beyond enumeration, by the
                        open chain's closed form, the marginals of
                        ising.marginals_elimination and the second
                        difference of ising.logz_r_elimination
  remainder_magnetisation
                        mean and variance from that distribution
  susceptibility        the importance-weighted estimator; pinned exact
                        under full enumeration of W with a uniform q against
                        brute-force moments of the whole system
"""

from __future__ import annotations

import numpy as np

from . import ising
from .objective import free_energy_terms


def remainder_magnetisation_bruteforce(inst, spins: np.ndarray):
    """(mean [B], var [B]) of M_R under p(r | s_W) by enumerating all r."""
    sp = ising.Split(inst)
    nr = len(sp.R)
    s = np.asarray(spins, np.float64)
    B = s.shape[0]
    if nr == 0:
        return np.zeros(B), np.zeros(B)
    assert nr <= 22, "brute force limited to |R| <= 22"
    Jrr, _ = ising._r_quadratic(sp)
    f = sp.fields_on_r(s)[:, sp.R]
    r = ising._all_configs(nr)                            # [C, nr]
    pair = np.einsum("ci,ij,cj->c", r, Jrr, r)
    expo = sp.beta * (pair[None, :] + f @ r.T)             # -beta E_2  [B, C]
    lz = ising._logsumexp(expo, axis=1)
    p = np.exp(expo - lz[:, None])
    m = r.sum(axis=1)                                      # M_R of every r
    mean = p @ m
    var = p @ (m * m) - mean * mean
    return mean, var


def _conv(f: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Log-domain convolution over the last axis: h[k] = LSE_{i+j=k} f[i] + g[j]
    (the other axes broadcast)."""
    K1, K2 = f.shape[-1], g.shape[-1]
    shape = np.broadcast_shapes(f.shape[:-1], g.shape[:-1]) + (K1 + K2 - 1,)
    h = np.full(shape, -np.inf)
    for i in range(K1):
        h[..., i:i + K2] = np.logaddexp(h[..., i:i + K2], f[..., i:i + 1] + g)
    return h


def _align_counted(tab: np.ndarray, scope, U):
    """Broadcast a [B] + [2]*len(scope) + [K] table to the axes of scope U
    (the count axis stays last)."""
    present = [scope.index(u) for u in U if u in scope]
    nd = len(scope)
    t = np.transpose(tab, [0] + [1 + i for i in present] + [nd + 1])
    shape = [tab.shape[0]] + [2 if u in scope else 1 for u in U] + [tab.shape[-1]]
    return t.reshape(shape)


def remainder_magnetisation_distribution(inst, spins: np.ndarray) -> np.ndarray:
    """log P(M_R = |R| - 2k | s_W) for k = 0..|R|, [B, |R| + 1].

    Variable elimination along ``inst.order`` as in ising.logz_r_elimination,
    where each log-factor has one more axis: the number k of -1 spins among
    the remainder spins already summed into it.  Multiplying factors adds
    their counts (a log-domain convolution over k); summing out a spin v
    keeps k for v = +1 and adds one for v = -1.  The roots (connected parts
    of R) are convolved, and the result is normalised."""
    sp = ising.Split(inst)
    s = np.asarray(spins, np.float64)
    B = s.shape[0]
    nr = len(sp.R)
    f = sp.fields_on_r(s)
    items = []
    for v in sp.R:
        tab = sp.beta * f[:, v][:, None] * np.array([1.0, -1.0])[None, :]
        items.append(((v,), tab[:, :, None]))
    for e in sp.rr:
        a, b = (int(x) for x in sp.edges[e])
        xy = np.array([[1.0, -1.0], [-1.0, 1.0]])
        items.append(((a, b), (sp.beta * sp.J[e] * xy)[None, :, :, None]))
    live = list(range(len(items)))
    total = np.zeros((B, 1))                               # count 0, log 1
    for v in sp.order:
        bucket = [k for k in live if v in items[k][0]]
        live = [k for k in live if k not in bucket]
        U = [v]
        for k in bucket:
            for u in items[k][0]:
                if u not in U:
                    U.append(u)
        comb = np.zeros([B] + [1] * len(U) + [1])
        for k in bucket:
            comb = _conv(comb, _align_counted(items[k][1], list(items[k][0]), U))
        comb = np.broadcast_to(comb, [B] + [2] * len(U) + [comb.shape[-1]])
        K = comb.shape[-1]
        msg = np.full(comb.shape[:1] + comb.shape[2:-1] + (K + 1,), -np.inf)
        msg[..., :K] = comb[:, 0]                          # v = +1: count kept
        msg[..., 1:] = np.logaddexp(msg[..., 1:], comb[:, 1])   # v = -1: one more
        scope = tuple(U[1:])
        if len(scope) == 0:
            total = _conv(total, msg)
        else:
            items.append((scope, msg))
            live.append(len(items) - 1)
    assert total.shape[1] == nr + 1
    m = total.max(axis=1, keepdims=True)
    return total - (np.log(np.exp(total - m).sum(axis=1, keepdims=True)) + m)


def remainder_magnetisation(inst, spins: np.ndarray):
    """(mean [B], var [B]) of M_R from remainder_magnetisation_distribution."""
    nr = len(inst.order)
    lp = remainder_magnetisation_distribution(inst, spins)
    p = np.exp(lp)
    m = nr - 2.0 * np.arange(nr + 1)
    mean = p @ m
    var = p @ (m * m) - mean * mean
    return mean, var


def susceptibility(inst, spins, logq, logz_r=None, moments=None):
    """Importance-weighted magnetisation moments of p from samples of q.

    Returns (m, m2, chi, ess): m = <M>_p / N, m2 = <M^2>_p / N^2,
    chi = beta N (m2 - m^2) and the effective sample size 1 / sum w_b^2.
    logz_r and moments = (mean, var) of M_R given s_W may be passed in
    (else computed by elimination)."""
    beta = float(inst.beta)
    n = int(inst.n)
    s = np.asarray(spins)
    if logz_r is None:
        logz_r = ising.logz_r_elimination(inst, s)
    if moments is None:
        moments = remainder_magnetisation(inst, s)
    mu, var = moments
    f, _ = free_energy_terms(inst, s, logq, logz_r)
    lw = -beta * f
    w = np.exp(lw - lw.max())
    w /= w.sum()
    mw = s.astype(np.float64).sum(axis=1)
    M = mw + mu
    m1 = float(w @ M)
    m2 = float(w @ (M * M + var))
    return m1 / n, m2 / (n * n), beta * (m2 - m1 * m1) / n, float(1.0 / np.sum(w * w))
