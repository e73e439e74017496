"""Pins of the oracle's objective, gradient estimator, optimiser and random
number generator (Sec. 3 Eqs. 5, 9, 10; Algorithm 1)."""

import os

import numpy as np

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


def _c1(H=16, seed=0, noise=0.0):
    inst = S.c1_small_lattice(hidden=H)
    th = S.made_init(4, H, seed).astype(np.float64)
    if noise:
        th = th + noise * np.random.default_rng(seed).standard_normal(th.shape)
    return inst, th


def test_variational_bound():
    # Eq. 5: F_q >= F for every q; equality needs q = p
    for seed, noise in [(0, 0.0), (1, 1.0), (2, 3.0)]:
        inst, th = _c1(seed=seed, noise=noise)
        Fq, _ = O.exact_fq_and_grad(inst, th, 16)
        F = O.exact_free_energy(inst)
        assert Fq >= F - 1e-12


def test_exact_gradient_finite_differences():
    inst, th = _c1(noise=0.5)
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


def test_reinforce_estimator_is_unbiased():
    inst, th = _c1(noise=0.7)
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


def test_training_reduces_exact_fq_and_respects_bound():
    inst, th = _c1()
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
