"""Pins of the oracle's width-set planner (Sec. 2, the dynamic-slicing recipe)
against closed forms and brute force, independent of its own code:

  * elimination width of trees (1), cycles (2), complete graphs (n - 1) and
    grids eliminated row by row (the row length) for any vertex labels;
  * min-fill on a k-tree (a chordal graph of treewidth k) finds a perfect
    elimination order, so its width is exactly k;
  * the planner's output covers V, has width <= w_u, and at w_u = 1 leaves a
    forest (union-find) whose complement is at least a minimum feedback
    vertex set (brute force over subsets);
  * exact sizes where they are forced: one vertex per disjoint cycle,
    n - w_u - 1 vertices of a complete graph, none when w_u is at least the
    greedy order's width.
"""

import itertools

import numpy as np
import pytest

from oracle import planner as P


def _relabel(n, edges, rng):
    p = rng.permutation(n)
    return [(int(min(p[a], p[b])), int(max(p[a], p[b]))) for a, b in edges], p


def _random_tree(n, rng):
    return [(int(rng.integers(0, i)), i) for i in range(1, n)]


def _cycle(n, start=0):
    return [(start + i, start + (i + 1) % n) if i + 1 < n else (start, start + n - 1)
            for i in range(n)]


def _complete(n):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def _grid(L, M):
    e = []
    for i in range(L):
        for j in range(M):
            v = i * M + j
            if j + 1 < M:
                e.append((v, v + 1))
            if i + 1 < L:
                e.append((v, v + M))
    return e


def _k_tree(n, k, rng):
    edges = set(_complete(k + 1))
    kcl = [c for c in itertools.combinations(range(k + 1), k)]
    for v in range(k + 1, n):
        base = kcl[int(rng.integers(0, len(kcl)))]
        for u in base:
            edges.add((u, v))
        for drop in range(k):
            kcl.append(tuple(sorted(base[:drop] + base[drop + 1:] + (v,))))
    return sorted(edges)


def _is_forest(vertices, edges):
    parent = {v: v for v in vertices}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x
    for a, b in edges:
        if a in parent and b in parent:
            ra, rb = find(a), find(b)
            if ra == rb:
                return False
            parent[ra] = rb
    return True


def _min_fvs(n, edges):
    for k in range(n + 1):
        for W in itertools.combinations(range(n), k):
            R = set(range(n)) - set(W)
            if _is_forest(R, edges):
                return k
    return n


def _rrg(n, d, rng):
    while True:
        stubs = rng.permutation(np.repeat(np.arange(n), d)).reshape(-1, 2)
        e = {(int(min(a, b)), int(max(a, b))) for a, b in stubs}
        if len(e) == n * d // 2 and all(a != b for a, b in e):
            return sorted(e)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_elimination_width_closed_forms(seed):
    rng = np.random.default_rng(seed)
    # a tree eliminated leaves first (reverse of attachment order): width 1
    n = 30
    t = _random_tree(n, rng)
    assert P.width(t, range(n), list(range(n - 1, -1, -1))) == 1
    # a cycle, any order: width 2
    c = _cycle(12)
    assert P.width(c, range(12), list(rng.permutation(12))) == 2
    # a complete graph, any order: width n - 1
    assert P.width(_complete(9), range(9), list(rng.permutation(9))) == 8
    # an L x M grid eliminated row by row: width M, whatever the labels
    g, p = _relabel(5 * 7, _grid(5, 7), rng)
    assert P.width(g, range(35), [int(p[v]) for v in range(35)]) == 7
    # no edges: width 0; no vertices: 0
    assert P.width([], range(5), list(range(5))) == 0
    assert P.width([], [], []) == 0


@pytest.mark.parametrize("k,seed", [(1, 3), (2, 4), (3, 5), (5, 6)])
def test_min_fill_is_a_perfect_elimination_on_k_trees(k, seed):
    rng = np.random.default_rng(seed)
    n = 24
    e, _ = _relabel(n, _k_tree(n, k, rng), rng)
    o = P.min_fill_order(n, e, key=list(rng.permutation(n)))
    assert sorted(o) == list(range(n))
    assert P.width(e, range(n), o) == k


def test_min_fill_on_forests_and_cycles():
    rng = np.random.default_rng(7)
    t = _random_tree(20, rng) + [(20 + a, 20 + b) for a, b in _random_tree(10, rng)]
    assert P.width(t, range(30), P.min_fill_order(30, t)) == 1
    c = _cycle(15)
    assert P.width(c, range(15), P.min_fill_order(15, c)) == 2


def _check_plan(n, edges, w_u, key=None, regreedy=False):
    W, order, w, pi = P.plan(n, edges, w_u, key, regreedy)
    assert sorted(W + order) == list(range(n))
    if regreedy:
        R = [v for v in range(n) if v not in set(W)]
        assert order == P.min_fill_order(n, edges, key, R)
    else:
        assert order == [v for v in pi if v not in set(W)]
    assert w == P.width(edges, order, order) <= w_u
    if w_u == 1:
        assert _is_forest(set(order), edges)
    return W, order, w, pi


@pytest.mark.parametrize("regreedy", [False, True])
@pytest.mark.parametrize("w_u", [1, 2, 3, 5])
def test_plan_outputs_are_valid(w_u, regreedy):
    rng = np.random.default_rng(10 + w_u)
    graphs = [(36, _grid(6, 6)), (40, _rrg(40, 3, rng)), (30, _rrg(30, 4, rng)),
              (10, _complete(10))]
    for n, e in graphs:
        _check_plan(n, e, w_u, key=list(rng.permutation(n)), regreedy=regreedy)


@pytest.mark.parametrize("regreedy", [False, True])
@pytest.mark.parametrize("seed", range(4))
def test_plan_at_width_one_is_a_feedback_vertex_set(seed, regreedy):
    rng = np.random.default_rng(20 + seed)
    n = 11
    e = _rrg(n - 1, 3, rng) + [(int(rng.integers(0, n - 1)), n - 1)]
    e = sorted({(min(a, b), max(a, b)) for a, b in e})
    W, _, _, _ = _check_plan(n, e, 1, key=list(rng.permutation(n)), regreedy=regreedy)
    assert len(W) >= _min_fvs(n, e)


@pytest.mark.parametrize("regreedy", [False, True])
def test_plan_forced_sizes(regreedy):
    # one vertex per disjoint cycle
    e = _cycle(7) + _cycle(5, start=7) + _cycle(4, start=12)
    W, _, _, _ = _check_plan(16, e, 1, regreedy=regreedy)
    assert len(W) == 3
    assert len(set(W) & set(range(7))) == 1 and len(set(W) & set(range(7, 12))) == 1
    # complete graph: n - w_u - 1 vertices, whatever the key
    rng = np.random.default_rng(30)
    for w_u in (1, 3, 6):
        W, _, _, _ = _check_plan(12, _complete(12), w_u, key=list(rng.permutation(12)),
                                 regreedy=regreedy)
        assert len(W) == 12 - w_u - 1
    # a forest needs no width set at w_u = 1 once the order is rebuilt on it
    if regreedy:
        t = [(int(rng.integers(0, i)), i) for i in range(1, 20)]
        W, _, w, _ = _check_plan(20, t, 1, key=list(rng.permutation(20)), regreedy=True)
        assert W == [] and w == 1
    # a bound at or above the greedy order's width slices nothing
    n, e = 36, _grid(6, 6)
    pi = P.min_fill_order(n, e)
    W, order, _, _ = _check_plan(n, e, P.width(e, range(n), pi))
    assert W == [] and order == pi


def test_plan_rejects_a_zero_bound():
    with pytest.raises(ValueError):
        P.plan(3, [(0, 1)], 0)
