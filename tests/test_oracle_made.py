"""Pins of the oracle's masked autoregressive network (Sec. 3, Eqs. 6-8)."""

import numpy as np
import pytest

import synthetic as S
from oracle import made as M
from oracle.objective import all_width_states


@pytest.mark.parametrize("n,H", [(5, 8), (4, 16), (6, 0), (1, 4)])
def test_q_normalised(n, H):
    th = S.made_init(n, H, 3).astype(np.float64)
    th = th + 0.3 * np.random.default_rng(1).standard_normal(th.shape)
    s = all_width_states(n)
    assert abs(np.exp(M.logq(th, s, n, H)).sum() - 1.0) < 1e-12


def test_autoregressive_jacobian_pattern():
    n, H = 6, 12
    th = S.made_init(n, H, 0).astype(np.float64)
    th = th + 0.5 * np.random.default_rng(2).standard_normal(th.shape)
    x = np.random.default_rng(3).standard_normal((1, n))
    eps = 1e-6
    for j in range(n):
        xp, xm = x.copy(), x.copy()
        xp[0, j] += eps
        xm[0, j] -= eps
        d = (M.forward(th, xp, n, H)[2] - M.forward(th, xm, n, H)[2]) / (2 * eps)
        for i in range(n):
            if j >= i:
                assert abs(d[0, i]) < 1e-9
            else:
                assert abs(d[0, i]) > 1e-8


def test_no_hidden_layer_is_eq7():
    n = 7
    th = S.made_init(n, 0, 4).astype(np.float64)
    th = th + np.random.default_rng(0).standard_normal(th.shape)
    _, _, _, b2, W0 = M.unpack(th, n, 0)
    s = all_width_states(n)[:50].astype(np.float64)
    want = np.zeros((50, n))
    for b in range(50):
        for i in range(n):
            z = b2[i]
            for j in range(i):
                z += W0[i, j] * s[b, j]
            want[b, i] = z
    np.testing.assert_allclose(M.forward(th, s, n, 0)[2], want, atol=1e-12)


def test_sampling_inverse_cdf_and_frequencies():
    n, H = 4, 16
    th = S.made_init(n, H, 7).astype(np.float64)
    th = th + 0.8 * np.random.default_rng(5).standard_normal(th.shape)
    B = 200000
    u = S.uniforms(B, n, 9)
    s, lq, p = M.sample(th, u, n, H)
    # every drawn spin follows the strict rule s = +1 iff u < p
    assert np.all((s == 1) == (u < p))
    np.testing.assert_allclose(lq, M.logq(th, s, n, H), atol=1e-12)
    # chi-square of the 16 state frequencies against the exact q
    states = all_width_states(n)
    q = np.exp(M.logq(th, states, n, H))
    code = ((1 - s.astype(np.int64)) // 2) @ (1 << np.arange(n))
    cnt = np.bincount(code, minlength=2 ** n)
    chi2 = np.sum((cnt - B * q) ** 2 / (B * q))
    assert chi2 < 45.0        # 15 degrees of freedom, p ~ 1e-4


def test_logq_backward_finite_differences():
    n, H = 5, 6
    th = S.made_init(n, H, 1).astype(np.float64)
    th = th + 0.4 * np.random.default_rng(6).standard_normal(th.shape)
    s = S.uniform_spins(30, n, 2)
    w = np.random.default_rng(7).standard_normal(30)
    g = M.logq_backward(th, s, w, n, H)
    eps = 1e-6
    M1, M2, M0 = M.masks(n, H)
    mask = M.pack(M1, np.ones(H), M2, np.ones(n), M0)
    for k in range(th.shape[0]):
        tp, tm = th.copy(), th.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (w @ M.logq(tp, s, n, H) - w @ M.logq(tm, s, n, H)) / (2 * eps)
        assert abs(fd * mask[k] - g[k]) < 1e-7


# ---------------------------------------------------------------- depth > 1

@pytest.mark.parametrize("n,H,D", [(5, 8, 2), (4, 6, 3), (6, 5, 2)])
def test_deep_q_normalised(n, H, D):
    th = S.made_init(n, H, 3, depth=D).astype(np.float64)
    th = th + 0.4 * np.random.default_rng(1).standard_normal(th.shape)
    s = all_width_states(n)
    assert abs(np.exp(M.logq(th, s, n, H, depth=D)).sum() - 1.0) < 1e-12


def test_deep_autoregressive_jacobian_pattern():
    n, H, D = 6, 10, 3
    th = S.made_init(n, H, 0, depth=D).astype(np.float64)
    th = th + 0.5 * np.random.default_rng(2).standard_normal(th.shape)
    x = np.random.default_rng(3).standard_normal((1, n))
    eps = 1e-6
    for j in range(n):
        xp, xm = x.copy(), x.copy()
        xp[0, j] += eps
        xm[0, j] -= eps
        d = (M.forward(th, xp, n, H, D)[2] - M.forward(th, xm, n, H, D)[2]) / (2 * eps)
        for i in range(n):
            if j >= i:
                assert abs(d[0, i]) < 1e-9
            else:
                assert abs(d[0, i]) > 1e-8


def test_depth_one_is_the_one_layer_network():
    # the depth argument at 1 changes nothing, and a depth-2 draw starts
    # with the depth-1 draw of the same seed
    n, H = 5, 7
    th1 = S.made_init(n, H, 4)
    th2 = S.made_init(n, H, 4, depth=2)
    assert np.array_equal(th2[:th1.shape[0]], th1)
    s = all_width_states(n)
    th = th1.astype(np.float64)
    np.testing.assert_array_equal(M.logq(th, s, n, H, depth=1), M.logq(th, s, n, H))
    # a second layer that copies the first through tanh(W h) with W = c I
    # is the composition written out by hand
    c = 1.7
    W = c * np.eye(H)
    th2 = np.concatenate([th, W.ravel(), np.zeros(H)])
    W1, b1, W2, b2, W0 = M.unpack(th, n, H)
    M1, M2, M0 = M.masks(n, H)
    sf = s.astype(np.float64)
    h = np.tanh(c * np.tanh(sf @ (W1 * M1).T + b1))
    logit = h @ (W2 * M2).T + sf @ (W0 * M0).T + b2
    np.testing.assert_allclose(M.forward(th2, s, n, H, 2)[2], logit, atol=1e-13)


def test_deep_sampling_frequencies():
    n, H, D = 4, 9, 2
    th = S.made_init(n, H, 7, depth=D).astype(np.float64)
    th = th + 0.8 * np.random.default_rng(5).standard_normal(th.shape)
    B = 200000
    u = S.uniforms(B, n, 9)
    s, lq, p = M.sample(th, u, n, H, depth=D)
    assert np.all((s == 1) == (u < p))
    np.testing.assert_allclose(lq, M.logq(th, s, n, H, D), atol=1e-12)
    states = all_width_states(n)
    q = np.exp(M.logq(th, states, n, H, D))
    code = ((1 - s.astype(np.int64)) // 2) @ (1 << np.arange(n))
    cnt = np.bincount(code, minlength=2 ** n)
    chi2 = np.sum((cnt - B * q) ** 2 / (B * q))
    assert chi2 < 45.0


@pytest.mark.parametrize("D", [2, 3])
def test_deep_logq_backward_finite_differences(D):
    n, H = 5, 4
    th = S.made_init(n, H, 1, depth=D).astype(np.float64)
    th = th + 0.4 * np.random.default_rng(6).standard_normal(th.shape)
    s = S.uniform_spins(30, n, 2)
    w = np.random.default_rng(7).standard_normal(30)
    g = M.logq_backward(th, s, w, n, H, D)
    eps = 1e-6
    M1, M2, M0 = M.masks(n, H)
    MH = M.hidden_mask(n, H)
    mask = M.pack(M1, np.ones(H), M2, np.ones(n), M0, [(MH, np.ones(H))] * (D - 1))
    assert mask.shape == th.shape
    for k in range(th.shape[0]):
        tp, tm = th.copy(), th.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (w @ M.logq(tp, s, n, H, D) - w @ M.logq(tm, s, n, H, D)) / (2 * eps)
        assert abs(fd * mask[k] - g[k]) < 1e-7
