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

Deeper networks (depth D > 1, Table 1's depth as a parameter): D - 1 more
tanh layers of width H between the first hidden layer and the output,
  a^l_k' = b^l_k' + sum_{k : m(k) <= m(k')} W^l[k', k] h^{l-1}_k,  h^l = tanh(a^l)
(the MADE rule: a unit sees the units of the layer below whose degree does
not exceed its own, every layer with the same degrees m), and the logits
read the last layer.  Their parameters follow W0 in the flat vector as
(W^l [H, H], b^l [H]) for l = 2..D.

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
  every function at depth 2 and 3: the same normalisation, Jacobian,
  frequency and finite-difference pins; depth 1 is the one-layer network
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


def hidden_mask(n: int, H: int) -> np.ndarray:
    """MH [H, H]: unit k' of a later hidden layer sees unit k of the layer
    below iff m(k) <= m(k')."""
    m = degrees(n, H)
    if n < 2:
        return np.zeros((H, H))
    return (m[None, :] <= m[:, None]).astype(np.float64)


def param_count(n: int, H: int, depth: int = 1) -> int:
    extra = (depth - 1) * (H * H + H) if H > 0 else 0
    return H * n + H + n * H + n + n * n + extra


def unpack(theta: np.ndarray, n: int, H: int, depth: int = 1):
    """Flat layout W1 [H, n], b1 [H], W2 [n, H], b2 [n], W0 [n, n] (then the
    deeper layers, see unpack_hidden)."""
    t = np.asarray(theta, np.float64)
    o = 0
    W1 = t[o:o + H * n].reshape(H, n); o += H * n
    b1 = t[o:o + H]; o += H
    W2 = t[o:o + n * H].reshape(n, H); o += n * H
    b2 = t[o:o + n]; o += n
    W0 = t[o:o + n * n].reshape(n, n); o += n * n
    assert t.shape[0] == param_count(n, H, depth)
    return W1, b1, W2, b2, W0


def unpack_hidden(theta: np.ndarray, n: int, H: int, depth: int):
    """[(W^l [H, H], b^l [H]) for l = 2..depth] after W0."""
    t = np.asarray(theta, np.float64)
    o = param_count(n, H, 1)
    out = []
    for _ in range(depth - 1 if H > 0 else 0):
        W = t[o:o + H * H].reshape(H, H); o += H * H
        b = t[o:o + H]; o += H
        out.append((W, b))
    assert o == t.shape[0]
    return out


def pack(W1, b1, W2, b2, W0, hidden=()) -> np.ndarray:
    parts = [np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(W0)]
    for W, b in hidden:
        parts += [np.ravel(W), np.ravel(b)]
    return np.concatenate(parts)


def _layers(theta, s, n, H, depth):
    """Activations a^l, h^l of every hidden layer and the logits."""
    W1, b1, W2, b2, W0 = unpack(theta, n, H, depth)
    M1, M2, M0 = masks(n, H)
    MH = hidden_mask(n, H)
    s = np.asarray(s, np.float64)
    a = s @ (W1 * M1).T + b1[None, :]
    acts, hids = [a], [np.tanh(a)]
    for W, b in unpack_hidden(theta, n, H, depth):
        a = hids[-1] @ (W * MH).T + b[None, :]
        acts.append(a)
        hids.append(np.tanh(a))
    logit = hids[-1] @ (W2 * M2).T + s @ (W0 * M0).T + b2[None, :]
    return acts, hids, logit


def forward(theta, s: np.ndarray, n: int, H: int, depth: int = 1):
    """Last hidden layer's activations, its tanh values and the logits for
    spins s [B, n]."""
    acts, hids, logit = _layers(theta, s, n, H, depth)
    return acts[-1], hids[-1], logit


def log_sigmoid(z):
    return -np.logaddexp(0.0, -z)


def logq(theta, s, n: int, H: int, depth: int = 1) -> np.ndarray:
    _, _, logit = forward(theta, s, n, H, depth)
    return np.sum(log_sigmoid(np.asarray(s, np.float64) * logit), axis=1)


def sample(theta, u: np.ndarray, n: int, H: int, force=None, depth: int = 1):
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
        _, _, logit = forward(theta, s, n, H, depth)
        p = 1.0 / (1.0 + np.exp(-logit[:, i]))
        p_all[:, i] = p
        si = np.where(u[:, i] < p, 1.0, -1.0)
        if force is not None:
            fi = np.asarray(force)[:, i]
            si = np.where(fi != 0, fi.astype(np.float64), si)
        s[:, i] = si
    return s.astype(np.int8), logq(theta, s, n, H, depth), p_all


def logq_backward(theta, s, wts, n: int, H: int, depth: int = 1) -> np.ndarray:
    """Gradient of L = sum_b wts_b ln q(s_b) with respect to the flat
    parameters (masked entries get zero)."""
    W1, b1, W2, b2, W0 = unpack(theta, n, H, depth)
    M1, M2, M0 = masks(n, H)
    MH = hidden_mask(n, H)
    deep = unpack_hidden(theta, n, H, depth)
    s = np.asarray(s, np.float64)
    w = np.asarray(wts, np.float64)
    _, hids, logit = _layers(theta, s, n, H, depth)
    sig = 1.0 / (1.0 + np.exp(-logit))
    dlogit = w[:, None] * ((1.0 + s) / 2.0 - sig)           # [B, n]
    dW2 = (dlogit.T @ hids[-1]) * M2
    db2 = dlogit.sum(0)
    dW0 = (dlogit.T @ s) * M0
    dhid = dlogit @ (W2 * M2)
    grads = []
    for l in range(len(hids) - 1, 0, -1):          # layers D..2
        da = dhid * (1.0 - hids[l] ** 2)
        W, _ = deep[l - 1]
        grads.append(((da.T @ hids[l - 1]) * MH, da.sum(0)))
        dhid = da @ (W * MH)
    da = dhid * (1.0 - hids[0] ** 2)
    dW1 = (da.T @ s) * M1
    db1 = da.sum(0)
    return pack(dW1, db1, dW2, db2, dW0, grads[::-1])
