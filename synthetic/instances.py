"""Seeded spin-glass instances and their width-set / order inputs.

The paper's workloads are synthetic random spin models (Sec. 4): ferromagnetic
and Gaussian 2D lattices with open boundaries, +-J spin glasses on random
regular graphs, and the fully connected Sherrington-Kirkpatrick model.  This
module draws such instances from a seed and attaches the inputs the method
needs besides the couplings: the width set W (sampling order of the network),
the elimination order of the remainder R and its optional grouping.

Conventions (all host-side numpy, FP64):
  * vertices are 0-based; an edge is stored once as (i, j) with i < j;
  * lattice vertex id = r * L + c (row-major); horizontal edges first
    (row-major), then vertical edges (row-major); J drawn in that order;
  * lattice column numbers given to ``lattice_column_split`` are 1-based;
  * SK couplings J_ij ~ N(0, 1/n) for i < j in lexicographic order;
  * random regular graphs: configuration-model pairing with rejection,
    J_ij = +-1 uniform, h_i ~ N(0, variance h_var).
Nothing here evaluates Boltzmann weights, partition functions or networks.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Instance:
    """One disorder instance plus its decomposition inputs."""

    n: int
    edges: np.ndarray            # int32 [E, 2], i < j
    J: np.ndarray                # float64 [E]
    h: np.ndarray                # float64 [n]
    beta: float
    width_set: np.ndarray        # int32 [|W|], sampling order of W
    order: np.ndarray            # int32 [|R|], elimination order of R
    group_ptr: Optional[np.ndarray] = None   # int32 CSR over `order`, or None
    hidden: int = 0              # hidden width of the masked-dense network
    name: str = ""
    meta: dict = field(default_factory=dict)
    depth: int = 1               # hidden layers of the masked-dense network

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    @property
    def n_width(self) -> int:
        return int(self.width_set.shape[0])

    def with_beta(self, beta: float) -> "Instance":
        return Instance(self.n, self.edges, self.J, self.h, float(beta),
                        self.width_set, self.order, self.group_ptr,
                        self.hidden, f"{self.name.split('@')[0]}@b{beta:g}",
                        dict(self.meta), self.depth)

    def groups(self) -> List[np.ndarray]:
        """The elimination groups as lists of vertices (singletons if no CSR)."""
        if self.group_ptr is None:
            return [self.order[i:i + 1] for i in range(len(self.order))]
        gp = self.group_ptr
        return [self.order[gp[k]:gp[k + 1]] for k in range(len(gp) - 1)]


# --------------------------------------------------------------------------
# graphs

def lattice_edges(L: int) -> np.ndarray:
    """Open-boundary L x L square lattice, horizontal then vertical bonds."""
    e = []
    for r in range(L):
        for c in range(L - 1):
            e.append((r * L + c, r * L + c + 1))
    for r in range(L - 1):
        for c in range(L):
            e.append((r * L + c, (r + 1) * L + c))
    return np.asarray(e, dtype=np.int32).reshape(-1, 2)


def lattice_2d(L: int, seed: int, beta: float = 1.0, ferro: bool = False,
               h_var: float = 0.0) -> Instance:
    """L x L open-boundary lattice; J ~ N(0,1) (or J = 1 if ``ferro``)."""
    rng = np.random.default_rng(seed)
    edges = lattice_edges(L)
    E = edges.shape[0]
    J = np.ones(E) if ferro else rng.standard_normal(E)
    h = rng.normal(0.0, np.sqrt(h_var), L * L) if h_var > 0 else np.zeros(L * L)
    n = L * L
    return Instance(n, edges, J.astype(np.float64), h.astype(np.float64),
                    float(beta), np.zeros(0, np.int32),
                    np.arange(n, dtype=np.int32), None, 0,
                    f"lattice{L}x{L}_s{seed}", {"L": L, "kind": "lattice"})


def lattice_column_split(inst: Instance, width_cols_1based, hidden: int = 0,
                         row_groups: bool = True) -> Instance:
    """Width set = whole lattice columns; R = the strips between them.

    The residual strips are eliminated one after the other, each row by row
    (top to bottom, left to right inside a row).  With ``row_groups`` every
    strip row is one elimination group (a transfer-matrix step); otherwise
    every spin is its own group.
    """
    L = inst.meta["L"]
    wc = sorted(int(c) - 1 for c in width_cols_1based)
    W = [r * L + c for r in range(L) for c in wc]          # ascending id
    W = sorted(W)
    strips, cur = [], []
    for c in range(L):
        if c in wc:
            if cur:
                strips.append(cur)
            cur = []
        else:
            cur.append(c)
    if cur:
        strips.append(cur)
    order, gp = [], [0]
    for cols in strips:
        for r in range(L):
            if row_groups:
                order.extend(r * L + c for c in cols)
                gp.append(len(order))
            else:
                for c in cols:
                    order.append(r * L + c)
                    gp.append(len(order))
    out = Instance(inst.n, inst.edges, inst.J, inst.h, inst.beta,
                   np.asarray(W, np.int32), np.asarray(order, np.int32),
                   np.asarray(gp, np.int32), hidden,
                   inst.name + f"_W{'-'.join(str(c + 1) for c in wc)}",
                   dict(inst.meta, strips=[len(s) for s in strips]))
    return out


def lattice_auto_split(L: int) -> List[int]:
    """1-based width-set columns for an L x L lattice.

    k = max(0, ceil((L - 5) / 6)) whole columns go to W; the L - k residual
    columns form k + 1 strips as even as possible, wider strips outermost.
    For L = 16 this gives W = {6, 11} (strips 5, 4, 5).
    """
    k = max(0, -(-(L - 5) // 6))
    if k == 0:
        return []
    rest = L - k
    base, extra = divmod(rest, k + 1)
    widths = [base] * (k + 1)
    # hand the extra columns to the outermost strips first
    idx = []
    lo, hi = 0, k
    while lo <= hi:
        idx.append(lo)
        if hi != lo:
            idx.append(hi)
        lo += 1
        hi -= 1
    for t in range(extra):
        widths[idx[t]] += 1
    cols, c = [], 0
    for s in range(k):
        c += widths[s]
        cols.append(c + 1)        # next column (1-based) is a W column
        c += 1
    return cols


def sherrington_kirkpatrick(n: int, seed: int, beta: float = 1.0,
                            n_width: int = 48, group_size: int = 8,
                            hidden: int = 0) -> Instance:
    """Fully connected SK model, J_ij ~ N(0, 1/n), h = 0.

    W = vertices 0..n_width-1; R = the rest, eliminated in groups of
    ``group_size`` consecutive vertices.
    """
    rng = np.random.default_rng(seed)
    ii, jj = np.triu_indices(n, k=1)
    edges = np.stack([ii, jj], 1).astype(np.int32)
    J = rng.normal(0.0, np.sqrt(1.0 / n), edges.shape[0])
    W = np.arange(n_width, dtype=np.int32)
    order = np.arange(n_width, n, dtype=np.int32)
    nr = n - n_width
    gp = np.arange(0, nr + 1, group_size, dtype=np.int32)
    if gp[-1] != nr:
        gp = np.append(gp, nr).astype(np.int32)
    return Instance(n, edges, J, np.zeros(n), float(beta), W, order, gp,
                    hidden, f"sk{n}_s{seed}", {"kind": "sk"})


def random_regular_edges(n: int, d: int, rng: np.random.Generator) -> np.ndarray:
    """Configuration-model pairing of n*d stubs; redraw on loops/multi-edges."""
    assert (n * d) % 2 == 0
    stubs = np.repeat(np.arange(n), d)
    for _ in range(10000):
        p = stubs[rng.permutation(stubs.shape[0])].reshape(-1, 2)
        a, b = np.minimum(p[:, 0], p[:, 1]), np.maximum(p[:, 0], p[:, 1])
        if np.any(a == b):
            continue
        key = a.astype(np.int64) * n + b
        if np.unique(key).shape[0] != key.shape[0]:
            continue
        o = np.argsort(key)
        return np.stack([a[o], b[o]], 1).astype(np.int32)
    raise RuntimeError("could not draw a simple regular graph")


def random_regular(n: int, d: int, seed: int, beta: float = 1.0,
                   h_var: float = 0.1, width_limit: int = 10,
                   hidden: int = 0) -> Instance:
    """+-J spin glass on a random d-regular graph with Gaussian fields.

    W and the order come from the greedy planner at ``width_limit``.
    """
    from .planner import greedy_width_set
    rng = np.random.default_rng(seed)
    edges = random_regular_edges(n, d, rng)
    J = rng.choice(np.array([-1.0, 1.0]), edges.shape[0])
    h = rng.normal(0.0, np.sqrt(h_var), n) if h_var > 0 else np.zeros(n)
    W, order = greedy_width_set(n, edges, width_limit, seed=seed)
    return Instance(n, edges, J.astype(np.float64), h.astype(np.float64),
                    float(beta), W, order, None, hidden,
                    f"rrg{n}d{d}_s{seed}_w{width_limit}",
                    {"kind": "rrg", "d": d, "width_limit": width_limit})


# --------------------------------------------------------------------------
# the benchmark workloads

def c1_small_lattice(hidden: int = 16) -> Instance:
    """4x4 Gaussian lattice, seed 1, beta 1, W = column 2, row groups."""
    base = lattice_2d(4, seed=1, beta=1.0)
    return lattice_column_split(base, [2], hidden=hidden)


def c2_lattice(beta: float = 1.0, hidden: int = 256) -> Instance:
    """16x16 Gaussian lattice, seed 2, W = columns 6 and 11, row groups."""
    base = lattice_2d(16, seed=2, beta=beta)
    return lattice_column_split(base, [6, 11], hidden=hidden)


def c3_sk(beta: float = 1.0, hidden: int = 128) -> Instance:
    """SK N=64, seed 3, |W| = 48, R split into two groups of 8."""
    return sherrington_kirkpatrick(64, seed=3, beta=beta, n_width=48,
                                   group_size=8, hidden=hidden)


def c4_rrg(hidden: int = 0) -> Instance:
    """Random 3-regular +-J graph N=256, seed 4, greedy width limit 10."""
    return random_regular(256, 3, seed=4, beta=1.0, h_var=0.1,
                          width_limit=10, hidden=hidden)


def c4_small_copies(limit: int = 3) -> List[Instance]:
    """Five N=20 random 3-regular copies (seeds 40-44) for brute force."""
    return [random_regular(20, 3, seed=s, beta=1.0, h_var=0.1,
                           width_limit=limit) for s in range(40, 45)]


def mixed_batch_instances(count: int = 64, hidden: int = 128,
                          base_seed: int = 5000) -> List[Instance]:
    """Uneven multi-instance batch: lattices L in {8,12,16,24}, RRG N in
    {64,128,256}, type chosen by i mod 7, seed base_seed + i."""
    kinds = [("lat", 8), ("lat", 12), ("lat", 16), ("lat", 24),
             ("rrg", 64), ("rrg", 128), ("rrg", 256)]
    out = []
    for i in range(count):
        kind, size = kinds[i % 7]
        seed = base_seed + i
        if kind == "lat":
            base = lattice_2d(size, seed=seed, beta=1.0)
            inst = lattice_column_split(base, lattice_auto_split(size),
                                        hidden=hidden)
        else:
            inst = random_regular(size, 3, seed=seed, beta=1.0, h_var=0.1,
                                  width_limit=10, hidden=hidden)
        inst.meta["samples"] = 512 * (2 ** (i % 4))
        out.append(inst)
    return out


def mixed_batch_sizes(insts: List[Instance]) -> List[int]:
    return [int(i.meta.get("samples", 512)) for i in insts]


def paper_configs():
    """Name -> list of instances for the five benchmark workloads."""
    return {
        "c1": [c1_small_lattice()],
        "c2": [c2_lattice(b) for b in (0.5, 1.0, 2.0)],
        "c3": [c3_sk(b) for b in (0.5, 1.0, 1.5)],
        "c4": [c4_rrg()],
        "c5": mixed_batch_instances(),
    }
