"""Oracle of the width-set planner: greedy order, dynamic slicing, re-adding.

Test infrastructure: only tests/, the smoke check and the benchmark's CPU
baseline use this module.  Plain Python sets, no speed tricks.

Sec. 2 (the paragraph on finding the width set) describes the recipe: take a
heuristic contraction order pi of the whole network, build the contraction
tree from it, then repeatedly remove the index of largest width (moving that
spin into W) and update the tree until its width is within the bound w_u;
finally take indices out of W again in random order wherever the tree stays
within the bound.  The readings taken here:

  * the network is the interaction graph with spins as hyper-indices and one
    Boltzmann matrix per edge; fields and couplings do not enter;
  * a contraction order is an elimination order of vertices.  Eliminating v
    sums its index and leaves a tensor over its scope S(v), the neighbours
    of v not yet eliminated (fill edges included), so the width of an order
    is max |S(v)| (log2 of the largest intermediate), 0 for no vertices;
  * fixing the spins of W removes W and its edges from the graph (their
    couplings become fields on R), and "updating the tree" keeps pi: the
    order of R is pi with the W vertices skipped;
  * the greedy order is min-fill: repeatedly eliminate the vertex whose
    current neighbours miss the fewest edges among themselves; ties go to
    the fewest current neighbours, then the smallest key;
  * "the index of largest width" is the vertex that lies in the most scopes
    of the maximum size; ties go to the larger degree in the original
    graph, then the smallest key;
  * the bound holds when the width is <= w_u (w_u = 1 then makes R a
    forest, so W is a feedback vertex set, as the paper states for w_u = 1);
  * the random order of the re-adding phase is ascending key, with the key
    a permutation of the vertex ids passed in by the caller (the identity
    when none is given).

With ``regreedy`` the tree is rebuilt instead of kept: after every slicing
pick, and for every re-adding test, the min-fill order of the graph induced
on R replaces pi restricted to R (the greedy heuristic run again on the
network left after fixing W).

Pinned in tests/test_oracle_planner.py against closed forms (trees, cycles,
complete graphs, grids in row-major order, k-trees), a union-find forest
check, and brute-force minimum feedback vertex sets on tiny graphs.
"""

from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Set, Tuple


def _graph(vertices: Sequence[int], edges) -> Dict[int, Set[int]]:
    """Adjacency sets of the graph induced on ``vertices``."""
    keep = set(int(v) for v in vertices)
    adj = {v: set() for v in keep}
    for a, b in edges:
        a, b = int(a), int(b)
        if a in keep and b in keep:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def _eliminate(adj: Dict[int, Set[int]], v: int) -> List[int]:
    """Remove v, join its neighbours into a clique, return its scope."""
    nb = adj.pop(v)
    for a in nb:
        adj[a].discard(v)
    for a in nb:
        adj[a] |= nb - {a}
    return sorted(nb)


def scopes(edges, vertices: Sequence[int], order: Sequence[int]) -> List[Tuple[int, List[int]]]:
    """(v, S(v)) of every step of eliminating ``order`` on the graph induced
    on ``vertices`` (``order`` must be a permutation of ``vertices``)."""
    adj = _graph(vertices, edges)
    assert sorted(adj) == sorted(int(v) for v in order)
    return [(int(v), _eliminate(adj, int(v))) for v in order]


def width(edges, vertices: Sequence[int], order: Sequence[int]) -> int:
    """Largest scope of the elimination order; 0 for an empty order."""
    return max((len(s) for _, s in scopes(edges, vertices, order)), default=0)


def min_fill_order(n: int, edges, key: Optional[Sequence[int]] = None,
                   vertices: Optional[Sequence[int]] = None) -> List[int]:
    """Greedy min-fill elimination order of the graph induced on
    ``vertices`` (all n vertices when None)."""
    key = list(range(n)) if key is None else [int(k) for k in key]
    adj = _graph(range(n) if vertices is None else vertices, edges)
    order = []
    while adj:
        def fill(v):
            nb = sorted(adj[v])
            return sum(1 for i in range(len(nb)) for j in range(i + 1, len(nb))
                       if nb[j] not in adj[nb[i]])
        v = min(adj, key=lambda u: (fill(u), len(adj[u]), key[u]))
        _eliminate(adj, v)
        order.append(v)
    return order


def restrict(order: Sequence[int], W: Set[int]) -> List[int]:
    return [int(v) for v in order if int(v) not in W]


def plan(n: int, edges, w_u: int, key: Optional[Sequence[int]] = None,
         regreedy: bool = False):
    """Width set W (ascending id), order of R and its width.

    Returns (W, order, width, pi)."""
    if w_u < 1:
        raise ValueError("w_u must be at least 1")
    key = list(range(n)) if key is None else [int(k) for k in key]
    assert sorted(key) == list(range(n))
    deg = [0] * n
    for a, b in edges:
        deg[int(a)] += 1
        deg[int(b)] += 1
    pi = min_fill_order(n, edges, key)
    W: Set[int] = set()

    def order_of(Wset):
        if not regreedy:
            return restrict(pi, Wset)
        return min_fill_order(n, edges, key, [v for v in range(n) if v not in Wset])

    # dynamic slicing
    while True:
        R = order_of(W)
        sc = scopes(edges, R, R)
        w = max((len(s) for _, s in sc), default=0)
        if w <= w_u:
            break
        count: Dict[int, int] = {}
        for _, s in sc:
            if len(s) == w:
                for u in s:
                    count[u] = count.get(u, 0) + 1
        pick = min(count, key=lambda u: (-count[u], -deg[u], key[u]))
        W.add(pick)
    # re-adding in ascending key order
    for v in sorted(W, key=lambda u: key[u]):
        R2 = order_of(W - {v})
        if width(edges, R2, R2) <= w_u:
            W.discard(v)
    order = order_of(W)
    return sorted(W), order, width(edges, order, order), pi
