"""Seeded random draws that feed both implementations as inputs.

* ``uniform_spins``: i.i.d. +-1 spins of the width set, int8 [B, |W|];
* ``uniforms``: FP32 uniforms in [0, 1) for ancestral sampling, [B, |W|];
* ``made_init``: initial parameters of the masked-dense network.

The parameter draw is dense: every weight gets a value, including the ones
the autoregressive masks switch off.  Each implementation applies the masks
itself, so no mask pattern lives here.  Layout of the flat vector:
W1 [H, n], b1 [H], W2 [n, H], b2 [n], W0 [n, n] (row-major, float32),
with weights ~ U(-1/sqrt(fan), 1/sqrt(fan)) where fan is the full input
count of the layer (n for W1, H + n for W2 and W0) and zero biases.  A
network of depth D > 1 (and H > 0) continues with D - 1 hidden-to-hidden
layers (W [H, H] with fan H, b [H] zero), drawn after the others, so the
first part equals the depth-1 draw of the same seed.
"""

from __future__ import annotations

import numpy as np


def uniform_spins(B: int, nw: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (2 * rng.integers(0, 2, size=(B, nw)) - 1).astype(np.int8)


def uniforms(B: int, nw: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((B, nw), dtype=np.float32)


def made_param_count(nw: int, H: int, depth: int = 1) -> int:
    extra = (depth - 1) * (H * H + H) if H > 0 else 0
    return H * nw + H + nw * H + nw + nw * nw + extra


def made_init(nw: int, H: int, seed: int, depth: int = 1) -> np.ndarray:
    """Flat float32 parameter vector (layout in the module docstring)."""
    rng = np.random.default_rng(seed)
    parts = []
    if H > 0:
        a1 = 1.0 / np.sqrt(max(nw, 1))
        parts.append(rng.uniform(-a1, a1, (H, nw)).ravel())
        parts.append(np.zeros(H))
        a2 = 1.0 / np.sqrt(max(H + nw, 1))
        parts.append(rng.uniform(-a2, a2, (nw, H)).ravel())
    else:
        a2 = 1.0 / np.sqrt(max(nw, 1))
    parts.append(np.zeros(nw))
    parts.append(rng.uniform(-a2, a2, (nw, nw)).ravel())
    for _ in range(depth - 1 if H > 0 else 0):
        ah = 1.0 / np.sqrt(H)
        parts.append(rng.uniform(-ah, ah, (H, H)).ravel())
        parts.append(np.zeros(H))
    out = np.concatenate(parts).astype(np.float32)
    assert out.shape[0] == made_param_count(nw, H, depth)
    return out


def split_params(theta: np.ndarray, nw: int, H: int):
    """Views (W1, b1, W2, b2, W0) of a flat parameter vector."""
    o = 0
    W1 = theta[o:o + H * nw].reshape(H, nw); o += H * nw
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + nw * H].reshape(nw, H); o += nw * H
    b2 = theta[o:o + nw]; o += nw
    W0 = theta[o:o + nw * nw].reshape(nw, nw); o += nw * nw
    return W1, b1, W2, b2, W0
