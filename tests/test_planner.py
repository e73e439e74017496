"""The native width-set planner (tnvan_plan_width_set, Sec. 2 dynamic
slicing) against the oracle's: identical width sets, orders, widths and
greedy orders on lattices, random regular graphs, complete graphs, trees,
cycles and k-trees over several bounds and seeded keys; error handling; and
at the paper's graph sizes (a 40x40 lattice, random regular graphs with
n = 300, d = 4 and n = 1000, d = 3) outputs that satisfy the bound, with
the width recomputed by the oracle.  Host only: no GPU needed."""

import numpy as np
import pytest

from synthetic import instances as SI
from oracle import planner as OP

L = pytest.importorskip("paper_2504_12037_amd._lib")


def _grid(Lr, M):
    e = []
    for i in range(Lr):
        for j in range(M):
            v = i * M + j
            if j + 1 < M:
                e.append((v, v + 1))
            if i + 1 < Lr:
                e.append((v, v + M))
    return e


def _rrg(n, d, seed):
    return [tuple(map(int, x)) for x in SI.random_regular_edges(n, d, np.random.default_rng(seed))]


def _graphs():
    rng = np.random.default_rng(5)
    tree = [(int(rng.integers(0, i)), i) for i in range(1, 25)]
    cyc = [(i, i + 1) for i in range(13)] + [(0, 13)]
    kt = set((i, j) for i in range(4) for j in range(i + 1, 4))
    cl = [(0, 1, 2)]
    for v in range(4, 22):
        base = cl[int(rng.integers(0, len(cl)))]
        kt |= {(u, v) for u in base}
        cl += [tuple(sorted((base[a], base[b], v))) for a in range(3) for b in range(a + 1, 3)]
    return [("grid6", 36, _grid(6, 6)), ("grid5x8", 40, _grid(5, 8)),
            ("rrg40d3", 40, _rrg(40, 3, 1)), ("rrg60d3", 60, _rrg(60, 3, 2)),
            ("rrg30d4", 30, _rrg(30, 4, 3)), ("sk12", 12, [(i, j) for i in range(12)
                                                            for j in range(i + 1, 12)]),
            ("tree", 25, tree), ("cycle", 14, cyc), ("3tree", 22, sorted(kt))]


@pytest.mark.parametrize("name,n,edges", _graphs(), ids=[g[0] for g in _graphs()])
def test_native_planner_equals_the_oracle(name, n, edges):
    for w_u in (1, 2, 3, 4, 6):
        for seed in (None, 0, 1):
            key = None if seed is None else np.random.default_rng(100 + seed).permutation(n)
            W, order, w, pi = L.plan_width_set(n, edges, w_u, key)
            oW, oorder, ow, opi = OP.plan(n, edges, w_u, None if key is None else list(key))
            assert list(pi) == opi, (name, w_u, seed)
            assert list(W) == oW, (name, w_u, seed)
            assert list(order) == oorder, (name, w_u, seed)
            assert w == ow <= w_u


@pytest.mark.parametrize("name,n,edges", _graphs()[:6], ids=[g[0] for g in _graphs()[:6]])
def test_native_regreedy_planner_equals_the_oracle(name, n, edges):
    # the tree rebuilt by min-fill on R after every pick
    for w_u in (1, 3, 5):
        key = np.random.default_rng(200 + w_u).permutation(n)
        W, order, w, pi = L.plan_width_set(n, edges, w_u, key, regreedy=True)
        oW, oorder, ow, opi = OP.plan(n, edges, w_u, list(key), regreedy=True)
        assert list(pi) == opi and list(W) == oW and list(order) == oorder, (name, w_u)
        assert w == ow <= w_u


def test_native_planner_rejects_bad_input():
    e = [(0, 1), (1, 2)]
    for args in [(3, e, 0), (0, [], 1), (3, [(0, 3)], 1), (3, [(1, 1)], 1),
                 (3, [(0, -1)], 1), (20000, [], 1)]:
        with pytest.raises(L.TnvanError):
            L.plan_width_set(*args)
    with pytest.raises(L.TnvanError):
        L.plan_width_set(3, e, 1, key=[0, 0, 1])
    with pytest.raises(L.TnvanError):
        L.plan_width_set(3, e, 1, key=[0, 1, 3])
    # no edges: nothing to slice
    W, order, w, _ = L.plan_width_set(4, [], 1)
    assert len(W) == 0 and sorted(order) == [0, 1, 2, 3] and w == 0


def _valid(n, edges, w_u, out):
    W, order, w, pi = out
    assert sorted(list(W) + list(order)) == list(range(n))
    assert list(order) == [v for v in pi if v not in set(W.tolist())]
    assert w == OP.width(edges, order.tolist(), order.tolist()) <= w_u


@pytest.mark.parametrize("w_u", [1, 3, 8, 13, 17, 20])
def test_paper_sized_random_regular_degree_four(w_u):
    # the n = 300, d = 4 sweep of the paper's random-graph experiment, both
    # modes; rebuilding the tree never needs more width-set vertices at the
    # smallest bound here
    n, e = 300, _rrg(300, 4, 7)
    key = np.random.default_rng(8).permutation(n)
    out = L.plan_width_set(n, e, w_u, key)
    _valid(n, e, w_u, out)
    out2 = L.plan_width_set(n, e, w_u, key, regreedy=True)
    W2, order2, w2, _ = out2
    assert sorted(list(W2) + list(order2)) == list(range(n))
    assert w2 == OP.width(e, order2.tolist(), order2.tolist()) <= w_u
    if w_u == 1:
        assert len(W2) <= len(out[0])


def test_paper_sized_sweeps_shrink_the_width_set():
    # |W| against w_u on the 40x40 lattice and an n = 1000, d = 3 random
    # regular graph: every plan within its bound, and larger bounds leave
    # smaller width sets (loosely: the heuristic is not monotone step by step)
    n, e = 1600, _grid(40, 40)
    sizes = []
    for w_u in (2, 4, 10, 20):
        out = L.plan_width_set(n, e, w_u)
        _valid(n, e, w_u, out)
        sizes.append(len(out[0]))
    assert sizes[0] > sizes[1] > sizes[2] > sizes[3] > 0
    n, e = 1000, _rrg(1000, 3, 9)
    sizes = []
    for w_u in (1, 10, 20, 30):
        out = L.plan_width_set(n, e, w_u)
        _valid(n, e, w_u, out)
        sizes.append(len(out[0]))
    assert sizes[0] > sizes[1] > sizes[2] > sizes[3] > 0
