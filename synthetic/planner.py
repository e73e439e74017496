"""Graph-structure helpers that choose the width set W and the order of R.

The paper takes W and the contraction order as given by an external planner
(Sec. 2: an order from a heuristic such as greedy, then dynamic slicing that
moves the index of largest width into W until the width is below w_u, then
tries to put removed indices back).  This is a small deterministic version of
that recipe working on the interaction graph only:

  * width of an order = the largest number of not-yet-eliminated neighbours
    a vertex has when it is eliminated (log2 of the entry count of the
    largest message the elimination creates);
  * order = min-fill (ties: min degree, then lowest id);
  * while the width exceeds the limit, the vertex that appears in the most
    maximum-size elimination scopes (ties: larger degree, then lowest id)
    moves to W;
  * then, in a seeded random order, each W vertex goes back to R if the
    width stays within the limit.

No Boltzmann weight or partition function is computed here.
"""

from __future__ import annotations

from typing import Dict, List, Sequence, Set, Tuple

import numpy as np


def _adjacency(n: int, edges: np.ndarray, keep: Set[int]) -> Dict[int, Set[int]]:
    adj = {v: set() for v in keep}
    for a, b in edges:
        a, b = int(a), int(b)
        if a in keep and b in keep:
            adj[a].add(b)
            adj[b].add(a)
    return adj


def _fill(adj: Dict[int, Set[int]], v: int) -> int:
    nb = list(adj[v])
    f = 0
    for i in range(len(nb)):
        ai = adj[nb[i]]
        for j in range(i + 1, len(nb)):
            if nb[j] not in ai:
                f += 1
    return f


def min_fill_order(n: int, edges: np.ndarray, R: Sequence[int]) -> List[int]:
    """Min-fill elimination order of the graph induced on R."""
    adj = _adjacency(n, edges, set(int(v) for v in R))
    fill = {v: _fill(adj, v) for v in adj}
    order = []
    while adj:
        v = min(adj, key=lambda u: (fill[u], len(adj[u]), u))
        nb = adj.pop(v)
        order.append(v)
        touched = set(nb)
        for a in nb:
            adj[a].discard(v)
        nbl = list(nb)
        for i in range(len(nbl)):
            for j in range(i + 1, len(nbl)):
                a, b = nbl[i], nbl[j]
                if b not in adj[a]:
                    adj[a].add(b)
                    adj[b].add(a)
        for a in nb:
            touched |= adj[a]
        del fill[v]
        for u in touched:
            if u in adj:
                fill[u] = _fill(adj, u)
    return order


def elimination_scopes(n: int, edges: np.ndarray, R: Sequence[int],
                       order: Sequence[int]) -> List[Tuple[int, List[int]]]:
    """(v, neighbours at elimination) for each v of ``order`` (one per step)."""
    adj = _adjacency(n, edges, set(int(v) for v in R))
    out = []
    for v in order:
        v = int(v)
        nb = adj.pop(v)
        for a in nb:
            adj[a].discard(v)
        nbl = sorted(nb)
        for i in range(len(nbl)):
            for j in range(i + 1, len(nbl)):
                adj[nbl[i]].add(nbl[j])
                adj[nbl[j]].add(nbl[i])
        out.append((v, nbl))
    return out


def order_width(n: int, edges: np.ndarray, R: Sequence[int],
                order: Sequence[int]) -> int:
    sc = elimination_scopes(n, edges, R, order)
    return max((len(s) for _, s in sc), default=0)


def greedy_width_set(n: int, edges: np.ndarray, limit: int,
                     seed: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Width set W (ascending id) and min-fill order of R with width <= limit."""
    deg = np.zeros(n, np.int64)
    for a, b in edges:
        deg[a] += 1
        deg[b] += 1
    W: Set[int] = set()
    R = [v for v in range(n)]
    order = min_fill_order(n, edges, R)
    while True:
        sc = elimination_scopes(n, edges, R, order)
        width = max((len(s) for _, s in sc), default=0)
        if width <= limit:
            break
        count = {}
        for v, s in sc:
            if len(s) == width:
                for u in [v] + s:
                    count[u] = count.get(u, 0) + 1
        pick = min(count, key=lambda u: (-count[u], -int(deg[u]), u))
        W.add(pick)
        R = [v for v in range(n) if v not in W]
        order = min_fill_order(n, edges, R)
    rng = np.random.default_rng(seed)
    for v in [int(x) for x in rng.permutation(sorted(W))]:
        R2 = sorted(set(R) | {v})
        o2 = min_fill_order(n, edges, R2)
        if order_width(n, edges, R2, o2) <= limit:
            W.discard(v)
            R, order = R2, o2
    return (np.asarray(sorted(W), np.int32), np.asarray(order, np.int32))
