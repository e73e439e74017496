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
