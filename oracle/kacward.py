"""Exact ln Z of a zero-field Ising model on a planar graph drawn with
straight edges: the Kac-Ward determinant (Sec. 4 uses it for the exact free
energy of the open-boundary 2D lattices).

Test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use this module.

The high-temperature expansion writes
    Z = 2^N prod_e cosh(beta J_e) * sum over even subgraphs of prod x_e,
    x_e = tanh(beta J_e),
and for a planar drawing the even-subgraph sum is sqrt(det(I - T)) with T
indexed by directed edges: T[(a->b), (b->c)] = x_bc exp(i theta / 2), where
theta is the turning angle from the direction a->b to the direction b->c
(in (-pi, pi)), and T is zero when c = a (no backtracking) or the edges do
not meet head to tail (Kac and Ward 1952; the planar case proven by
Cimasoni 2010).  The determinant is real and positive; it is taken with
numpy's LU-based slogdet in complex128.

Pinned in tests/test_oracle_kacward.py against brute-force ln Z on small
lattices with couplings of both signs.
"""

from __future__ import annotations

import numpy as np


def logz_planar(n: int, edges, J, beta: float, xy) -> float:
    """ln Z for couplings J on the edges of a planar straight-line drawing
    with vertex coordinates ``xy`` [n, 2]; no fields."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    J = np.asarray(J, dtype=np.float64)
    xy = np.asarray(xy, dtype=np.float64)
    E = edges.shape[0]
    x = np.tanh(beta * J)
    # directed edge d = 2e (i -> j) and 2e + 1 (j -> i)
    tail = np.concatenate([edges[:, 0], edges[:, 1]])
    head = np.concatenate([edges[:, 1], edges[:, 0]])
    idx = np.concatenate([2 * np.arange(E), 2 * np.arange(E) + 1])
    t_of = np.empty(2 * E, np.int64)
    h_of = np.empty(2 * E, np.int64)
    t_of[idx] = tail
    h_of[idx] = head
    w_of = np.repeat(x, 2)
    ang = np.arctan2(xy[h_of, 1] - xy[t_of, 1], xy[h_of, 0] - xy[t_of, 0])
    out_of = [[] for _ in range(n)]
    for d in range(2 * E):
        out_of[t_of[d]].append(d)
    T = np.zeros((2 * E, 2 * E), np.complex128)
    for d in range(2 * E):
        b = h_of[d]
        for d2 in out_of[b]:
            if h_of[d2] == t_of[d]:
                continue   # backtracking
            th = ang[d2] - ang[d]
            th = (th + np.pi) % (2 * np.pi) - np.pi
            T[d, d2] = w_of[d2] * np.exp(0.5j * th)
    sign, logdet = np.linalg.slogdet(np.eye(2 * E) - T)
    # det(I - T) is real and positive
    assert abs(sign - 1.0) < 1e-6, sign
    return float(n * np.log(2.0) + np.sum(np.log(np.cosh(beta * J))) + 0.5 * logdet)


def lattice_xy(L: int) -> np.ndarray:
    """Coordinates of the L x L lattice with vertex r * L + c at (c, r)."""
    r, c = np.divmod(np.arange(L * L), L)
    return np.stack([c, r], 1).astype(np.float64)
