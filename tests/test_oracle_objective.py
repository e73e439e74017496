"""Pins of the oracle's objective, gradient estimator, optimiser and random
number generator (Sec. 3 Eqs. 5, 9, 10; Algorithm 1).

Every pin of the objective runs at beta != 1 as well: at beta = 1 the
entropy term ln q / beta of Eq. 9 cannot be told from ln q * beta."""

import os

import numpy as np
import pytest

import synthetic as S
from oracle import ising as I
from oracle import made as M
from oracle import objective as O
from oracle import philox as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = P.philox4x32_10(np.array(v[:4], np.uint64), np.array(v[4:6], np.uint64))
        assert [int(x) for x in out] == v[6:10]


def test_sampler_uniforms_range_and_counter_layout():
    u = P.sampler_uniforms(seed=12345, step=3, inst_index=1, B=5, n=7)
    assert u.dtype == np.float32 and u.shape == (5, 7)
    assert np.all(u >= 0) and np.all(u < 1)
    w = P.philox4x32_10(np.array([1, 4, 3, 1], np.uint64),
                        np.array([12345, 0], np.uint64))
    assert u[4, 5] == np.float32((int(w[1]) >> 8) * 2.0 ** -24)


def test_adam_first_steps_by_hand():
    th = np.array([1.0, -2.0, 0.5])
    g1 = np.array([0.1, -3.0, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    th1, m, v = O.adam_step(th, g1, m, v, 1, 0.01)
    # first step: m_hat = g, v_hat = g^2 => update lr * g / (|g| + eps)
    np.testing.assert_allclose(th1, th - 0.01 * g1 / (np.abs(g1) + 1e-8), atol=1e-15)
    g2 = np.array([0.2, 1.0, -1.0])
    th2, m, v = O.adam_step(th1, g2, m, v, 2, 0.01)
    m2 = 0.9 * 0.1 * g1 + 0.1 * g2
    v2 = 0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2
    want = th1 - 0.01 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(th2, want, atol=1e-14)


BETAS = (0.5, 1.0, 2.0)


def _c1(H=16, seed=0, noise=0.0, beta=1.0):
    inst = S.c1_small_lattice(hidden=H).with_beta(beta)
    th = S.made_init(4, H, seed).astype(np.float64)
    if noise:
        th = th + noise * np.random.default_rng(seed).standard_normal(th.shape)
    return inst, th


@pytest.mark.parametrize("beta", BETAS)
def test_variational_bound(beta):
    # Eq. 5: F_q >= F for every q; equality needs q = p
    for seed, noise in [(0, 0.0), (1, 1.0), (2, 3.0)]:
        inst, th = _c1(seed=seed, noise=noise, beta=beta)
        Fq, _ = O.exact_fq_and_grad(inst, th, 16)
        F = O.exact_free_energy(inst)
        assert Fq >= F - 1e-12


@pytest.mark.parametrize("beta", BETAS)
def test_exact_gradient_finite_differences(beta):
    inst, th = _c1(noise=0.5, beta=beta)
    _, g = O.exact_fq_and_grad(inst, th, 16)
    eps = 1e-6
    rng = np.random.default_rng(0)
    for k in rng.choice(th.shape[0], 25, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (O.exact_fq_and_grad(inst, tp, 16)[0]
              - O.exact_fq_and_grad(inst, tm, 16)[0]) / (2 * eps)
        assert abs(fd - g[k]) < 1e-7


@pytest.mark.parametrize("beta", BETAS)
def test_reinforce_estimator_is_unbiased(beta):
    inst, th = _c1(noise=0.7, beta=beta)
    _, gex = O.exact_fq_and_grad(inst, th, 16)
    reps, B = 400, 256
    acc = []
    for r in range(reps):
        u = P.sampler_uniforms(99, r, 0, B, 4)
        s, lq, _ = M.sample(th, u, 4, 16)
        lz = I.logz_r_elimination(inst, s)
        f, _ = O.free_energy_terms(inst, s, lq, lz)
        acc.append(M.logq_backward(th, s, O.reinforce_weights(f), 4, 16))
    acc = np.asarray(acc)
    mean = acc.mean(0)
    se = acc.std(0, ddof=1) / np.sqrt(reps)
    # the mean-baseline estimator has an O(1/B) bias: -cov/B; allow 4 sigma
    # plus a 2/B relative slack
    assert np.all(np.abs(mean - gex) <= 4 * se + 2.0 / B * np.abs(gex) + 1e-12)


@pytest.mark.parametrize("beta", (0.5, 2.0))
def test_training_reduces_exact_fq_and_respects_bound(beta):
    inst, th = _c1(beta=beta)
    F = O.exact_free_energy(inst)
    Fq0, _ = O.exact_fq_and_grad(inst, th, 16)
    th1, stats = O.train(inst, th, 16, steps=60, B=256, lr=1e-2, seed=1)
    Fq1, _ = O.exact_fq_and_grad(inst, th1, 16)
    assert F - 1e-12 <= Fq1 < Fq0
    assert stats.shape == (60, 4)


def test_observables_exact_under_full_enumeration_with_uniform_q():
    # every width-set configuration once, with a uniform q: the
    # self-normalised weights are the exact W-marginal of p, so the estimates
    # are the exact moments (brute force over all 2^16 states)
    inst = S.c1_small_lattice()
    nw = inst.n_width
    x = np.arange(1 << nw)[:, None]
    sw = (1 - 2 * ((x >> np.arange(nw)[None, :]) & 1)).astype(np.int8)
    m, c, ess = O.observables(inst, sw, np.zeros(sw.shape[0]))
    n = inst.n
    y = np.arange(1 << n)[:, None]
    full = (1 - 2 * ((y >> np.arange(n)[None, :]) & 1)).astype(np.float64)
    e = I.energy(inst, full)
    p = np.exp(-inst.beta * (e - e.min()))
    p /= p.sum()
    m_ex = p @ full
    ed = np.asarray(inst.edges).reshape(-1, 2)
    c_ex = p @ (full[:, ed[:, 0]] * full[:, ed[:, 1]])
    np.testing.assert_allclose(m, m_ex, atol=1e-12)
    np.testing.assert_allclose(c, c_ex, atol=1e-12)
    assert 1.0 <= ess <= sw.shape[0]


# --------------------------------------------------------------------------
# Eq. 5 written against the full Boltzmann distribution (Eq. 1), at beta != 1

def _w_marginal(inst):
    """ln p_W(s) of every width-set configuration (the order of
    objective.all_width_states: bit i of the index set <=> s_{W_i} = -1) and
    ln Z, by enumerating all 2^n states of Eq. 1 and summing out R."""
    n, nw = int(inst.n), int(inst.n_width)
    W = np.asarray(inst.width_set, np.int64)
    lw_parts, idx_parts = [], []
    step = 1 << 16
    for y0 in range(0, 1 << n, step):
        y = np.arange(y0, min(1 << n, y0 + step), dtype=np.int64)[:, None]
        full = (1 - 2 * ((y >> np.arange(n)[None, :]) & 1)).astype(np.float64)
        lw_parts.append(-inst.beta * I.energy(inst, full))
        idx_parts.append(((full[:, W] < 0).astype(np.int64) << np.arange(nw)).sum(1))
    lw = np.concatenate(lw_parts)
    idx = np.concatenate(idx_parts)
    m = lw.max()
    acc = np.zeros(1 << nw)
    np.add.at(acc, idx, np.exp(lw - m))
    lnZ = float(np.log(acc.sum()) + m)
    return np.log(acc) + m - lnZ, lnZ


def _eq5_cases():
    out = []
    for beta in (0.5, 2.0):
        out.append(("c1", S.c1_small_lattice(hidden=16).with_beta(beta)))
        # an N = 20 random 3-regular +-J graph with Gaussian fields
        out.append(("rrg20", S.c4_small_copies(limit=3)[1].with_beta(beta)))
    return out


@pytest.mark.parametrize("name,inst", _eq5_cases(), ids=lambda v: v if isinstance(v, str) else v.name)
def test_eq5_equality_when_q_is_the_exact_w_marginal(name, inst):
    # With q(s) = p_W(s) = exp(-beta Etilde(s)) / Z, Eq. 5 makes the KL
    # divergence zero, so every per-sample f_b of Eq. 9 equals F = -ln Z /
    # beta exactly (zero variance), and Etilde(s) = -(ln p_W(s) + ln Z)/beta
    # sample by sample; all of it from the full enumeration, none from the
    # E_1 / E_2 split or the elimination that free_energy_terms is fed
    ln_pw, lnZ = _w_marginal(inst)
    beta = float(inst.beta)
    s = O.all_width_states(inst.n_width)
    lz = I.logz_r_elimination(inst, s)
    f, st = O.free_energy_terms(inst, s, ln_pw, lz)
    F = -lnZ / beta
    tol = 1e-11 * max(1.0, abs(F))
    assert np.abs(f - F).max() <= tol
    assert abs(st[0] - F) <= tol
    assert abs(st[1]) <= tol
    et = -(ln_pw + lnZ) / beta
    assert abs(st[2] - et.mean()) <= tol
    assert abs(st[3] - ln_pw.mean() / beta) <= tol
    # and the slice sum (Eq. 3) reproduces ln Z from the same split
    assert abs(O.exact_free_energy(inst) - F) <= tol


@pytest.mark.parametrize("beta", (0.5, 2.0))
@pytest.mark.parametrize("which", ("c1", "rrg20"))
def test_eq5_kl_identity_for_a_network_q(beta, which):
    # Eq. 5 for any q: beta (F_q - F) = KL(q | p_W), with p_W from the full
    # enumeration; F_q both from exact_fq_and_grad and from the q-weighted
    # per-sample f of free_energy_terms over every width-set configuration
    if which == "c1":
        inst = S.c1_small_lattice(hidden=16).with_beta(beta)
        H = 16
    else:
        inst = S.c4_small_copies(limit=3)[1].with_beta(beta)
        H = 2 * inst.n_width
    nw = inst.n_width
    th = S.made_init(nw, H, 11).astype(np.float64)
    th += 0.8 * np.random.default_rng(11).standard_normal(th.shape)
    ln_pw, lnZ = _w_marginal(inst)
    s = O.all_width_states(nw)
    lq = M.logq(th, s, nw, H)
    q = np.exp(lq)
    kl = float(np.sum(q * (lq - ln_pw)))
    F = -lnZ / beta
    Fq, _ = O.exact_fq_and_grad(inst, th, H)
    assert kl > 1e-3
    assert abs(beta * (Fq - F) - kl) <= 1e-10 * max(1.0, abs(beta * F))
    f, _ = O.free_energy_terms(inst, s, lq, I.logz_r_elimination(inst, s))
    assert abs(float(q @ f) - Fq) <= 1e-10 * max(1.0, abs(F))


def test_stderr_matches_the_spread_of_batch_means():
    # the standard error free_energy_terms reports is the spread of F_q over
    # independent batches: 400 batches of 64 samples of a network q (C1 at
    # beta = 2); the root mean square of the reported standard errors and
    # the standard deviation of the 400 batch means agree within the
    # sampling error of a 400-point spread (about 3.5%, 4 sigma = 15%), and
    # the mean of the batch means is the exact F_q within 4 standard errors
    beta, B, reps = 2.0, 64, 400
    inst, th = _c1(noise=0.7, beta=beta)
    Fq_exact, _ = O.exact_fq_and_grad(inst, th, 16)
    s_all = O.all_width_states(4)
    lz_all = I.logz_r_elimination(inst, s_all)
    means, ses = [], []
    for r in range(reps):
        u = P.sampler_uniforms(314, r, 0, B, 4)
        s, lq, _ = M.sample(th, u, 4, 16)
        k = ((s < 0).astype(np.int64) << np.arange(4)).sum(1)
        _, st = O.free_energy_terms(inst, s, lq, lz_all[k])
        means.append(st[0])
        ses.append(st[1])
    means = np.asarray(means)
    spread = float(means.std(ddof=1))
    rms_se = float(np.sqrt(np.mean(np.square(ses))))
    assert 0.85 <= rms_se / spread <= 1.15
    assert abs(means.mean() - Fq_exact) <= 4 * spread / np.sqrt(reps)
