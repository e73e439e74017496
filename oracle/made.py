"""Oracle for the masked autoregressive network.  TEST INFRASTRUCTURE ONLY.

The variational distribution factorises over the width set in its given
order (Sec. 3, Eq. 6).  Each conditional is a Bernoulli variable whose
probability of spin up is the sigmoid of a masked affine function of the
spins before it (Eqs. 7-8).  The network is the masked autoencoder (MADE,
Germain et al. 2015, the architecture Fig. 1(d) names) with one tanh hidden
layer of width H plus a direct input-to-output connection:

  positions i = 1..n (1-based), hidden units k = 0..H-1 with degree
  m(k) = 1 + (k mod (n - 1))   (n >= 2)
  a_k     = b1_k + sum_{j <= m(k)} W1[k, j] s_j,        h_k = tanh(a_k)
  logit_i = b2_i + sum_{k : m(k) < i} W2[i, k] h_k + sum_{j < i} W0[i, j] s_j
  q(s_i = +1 | s_<i) = sigmoid(logit_i)
  ln q(s) = sum_i log sigmoid(s_i * logit_i)

With H = 0 this is exactly Eq. 7.  Sampling draws s_i = +1 iff u_i < p_i for
given uniforms u in [0, 1), one position after the other (Eq. 8).

Functions and what pins them (tests/test_oracle_made.py):
  masks         pinned by the autoregressive Jacobian test: d logit_i / d s_j
                is zero for j >= i (finite differences), nonzero otherwise
  logits        pinned: sum over all 2^n configurations of q(s) is 1; H = 0
                reduces to Eq. 7 written out with a plain loop
  sample        pinned: sampled spins reproduce the Bernoulli frequencies of
                the exact q (chi-square on the 4-spin workload); spins equal
                the inverse-CDF rule applied to the exact conditionals
  logq_backward pinned against central finite differences of
                sum_b w_b ln q(s_b)
"""

from __future__ import annotations

import numpy as np


def degrees(n: int, H: int) -> np.ndarray:
    if n < 2:
        return np.zeros(H, np.int64)
    return 1 + (np.arange(H) % (n - 1))


def masks(n: int, H: int):
    """(M1 [H, n], M2 [n, H], M0 [n, n]) as float64 0/1 arrays."""
    m = degrees(n, H)
    j = np.arange(1, n + 1)
    M1 = (j[None, :] <= m[:, None]).astype(np.float64)
    M2 = (j[:, None] > m[None, :]).astype(np.float64)
    if n < 2:
        M2[:] = 0.0
        M1[:] = 0.0
    M0 = (j[None, :] < j[:, None]).astype(np.float64)
    return M1, M2, M0


def unpack(theta: np.ndarray, n: int, H: int):
    """Flat layout W1 [H, n], b1 [H], W2 [n, H], b2 [n], W0 [n, n]."""
    t = np.asarray(theta, np.float64)
    o = 0
    W1 = t[o:o + H * n].reshape(H, n); o += H * n
    b1 = t[o:o + H]; o += H
    W2 = t[o:o + n * H].reshape(n, H); o += n * H
    b2 = t[o:o + n]; o += n
    W0 = t[o:o + n * n].reshape(n, n); o += n * n
    assert o == t.shape[0]
    return W1, b1, W2, b2, W0


def pack(W1, b1, W2, b2, W0) -> np.ndarray:
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2),
                           np.ravel(b2), np.ravel(W0)])


def forward(theta, s: np.ndarray, n: int, H: int):
    """Hidden activations and logits for spins s [B, n]."""
    W1, b1, W2, b2, W0 = unpack(theta, n, H)
    M1, M2, M0 = masks(n, H)
    s = np.asarray(s, np.float64)
    a = s @ (W1 * M1).T + b1[None, :]
    hid = np.tanh(a)
    logit = hid @ (W2 * M2).T + s @ (W0 * M0).T + b2[None, :]
    return a, hid, logit


def log_sigmoid(z):
    return -np.logaddexp(0.0, -z)


def logq(theta, s, n: int, H: int) -> np.ndarray:
    _, _, logit = forward(theta, s, n, H)
    return np.sum(log_sigmoid(np.asarray(s, np.float64) * logit), axis=1)


def sample(theta, u: np.ndarray, n: int, H: int, force=None):
    """Ancestral sampling with uniforms u [B, n].  Returns (spins int8 [B, n],
    ln q [B], p [B, n] the conditional probabilities used).

    ``force`` (optional [B, n] int8, 0 = free) overrides the drawn spin at a
    position, for comparing against another sampler at near-ties.
    """
    u = np.asarray(u, np.float64)
    B = u.shape[0]
    s = np.zeros((B, n))
    p_all = np.zeros((B, n))
    for i in range(n):
        _, _, logit = forward(theta, s, n, H)
        p = 1.0 / (1.0 + np.exp(-logit[:, i]))
        p_all[:, i] = p
        si = np.where(u[:, i] < p, 1.0, -1.0)
        if force is not None:
            fi = np.asarray(force)[:, i]
            si = np.where(fi != 0, fi.astype(np.float64), si)
        s[:, i] = si
    return s.astype(np.int8), logq(theta, s, n, H), p_all


def logq_backward(theta, s, wts, n: int, H: int) -> np.ndarray:
    """Gradient of L = sum_b wts_b ln q(s_b) with respect to the flat
    parameters (masked entries get zero)."""
    W1, b1, W2, b2, W0 = unpack(theta, n, H)
    M1, M2, M0 = masks(n, H)
    s = np.asarray(s, np.float64)
    w = np.asarray(wts, np.float64)
    a, hid, logit = forward(theta, s, n, H)
    sig = 1.0 / (1.0 + np.exp(-logit))
    dlogit = w[:, None] * ((1.0 + s) / 2.0 - sig)           # [B, n]
    dW2 = (dlogit.T @ hid) * M2
    db2 = dlogit.sum(0)
    dW0 = (dlogit.T @ s) * M0
    dhid = dlogit @ (W2 * M2)
    da = dhid * (1.0 - hid ** 2)
    dW1 = (da.T @ s) * M1
    db1 = da.sum(0)
    return pack(dW1, db1, dW2, db2, dW0)
