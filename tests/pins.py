"""Independent computations that pin the oracle (none shares code with it).

* brute_force_mvc -- the definition of MVC written out: the smallest subset
  (bitmask) that touches every edge, by exhaustive enumeration (n <= 24).
* mis_bitset -- maximum independent set by a plain bitmask branch and bound,
  summed over connected components;
  MVC = n - alpha(G) because the complement of a vertex cover is an
  independent set and vice versa (Gallai).
* koenig_mvc -- for bipartite graphs MVC equals the maximum matching size
  (Koenig's theorem); the matching comes from scipy's bipartite matcher.
* tree_mvc -- linear-time dynamic program on forests.
"""
from __future__ import annotations

import numpy as np

_POP8 = np.array([bin(i).count("1") for i in range(256)], dtype=np.uint8)


def _popcount(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint32)
    return (_POP8[x & 0xFF].astype(np.int32) + _POP8[(x >> 8) & 0xFF]
            + _POP8[(x >> 16) & 0xFF] + _POP8[(x >> 24) & 0xFF])


def brute_force_mvc(g) -> int:
    """min |C| over all subsets C of V that cover every edge (n <= 24)."""
    n = g.n
    assert n <= 24
    u, v = g.edges()
    if u.size == 0:
        return 0
    best = n
    chunk = 1 << 20
    for start in range(0, 1 << n, chunk):
        masks = np.arange(start, min(start + chunk, 1 << n), dtype=np.uint32)
        ok = np.ones(masks.size, bool)
        for a, b in zip(u.tolist(), v.tolist()):
            ok &= ((masks >> np.uint32(a)) | (masks >> np.uint32(b))) & np.uint32(1) == 1
            if not ok.any():
                break
        if ok.any():
            best = min(best, int(_popcount(masks[ok]).min()))
    return best


def _adj_masks(g) -> list[int]:
    adj = [0] * g.n
    off = g.offsets.astype(np.int64)
    cols = g.cols.astype(np.int64)
    for x in range(g.n):
        m = 0
        for w in cols[off[x]:off[x + 1]].tolist():
            m |= 1 << w
        adj[x] = m
    return adj


def mis_bitset(g) -> int:
    """alpha(G) by bitmask branch and bound.

    A vertex of degree <= 1 inside the candidate set belongs to some maximum
    independent set, so it is taken without branching; otherwise branch on a
    vertex of maximum degree (exclude it / take it and drop its neighbours).
    The bound is |current| + |candidates|.
    """
    adj = _adj_masks(g)

    def component(P: int) -> int:
        """Bitmask of the connected component of G[P] holding P's lowest bit."""
        comp = P & -P
        frontier = comp
        while frontier:
            low = frontier & -frontier
            frontier ^= low
            x = low.bit_length() - 1
            new = adj[x] & P & ~comp
            comp |= new
            frontier |= new
        return comp

    def alpha(P: int) -> int:
        # alpha is additive over connected components
        total = 0
        while P:
            C = component(P)
            P &= ~C
            total += alpha_connected(C)
        return total

    def alpha_connected(P0: int) -> int:
        best = [0]
        rec(P0, 0, best)
        return best[0]

    def rec(P: int, size: int, best):
        # forced picks
        while P:
            if size + P.bit_count() <= best[0]:
                return
            pick = None
            maxd, maxv = -1, None
            Q = P
            while Q:
                low = Q & -Q
                x = low.bit_length() - 1
                Q ^= low
                d = (adj[x] & P).bit_count()
                if d <= 1:
                    pick = x
                    break
                if d > maxd:
                    maxd, maxv = d, x
            if pick is not None:
                P &= ~((1 << pick) | adj[pick])
                size += 1
                continue
            # branch on maxv: take it (solving what remains component-wise)
            # or leave it out
            t = alpha(P & ~((1 << maxv) | adj[maxv]))
            if size + 1 + t > best[0]:
                best[0] = size + 1 + t
            P &= ~(1 << maxv)
        if size > best[0]:
            best[0] = size

    return alpha((1 << g.n) - 1)


def koenig_mvc(g, left_mask: np.ndarray) -> int:
    """Maximum matching of a bipartite graph (left side given) = MVC."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_bipartite_matching
    left = np.flatnonzero(left_mask)
    right = np.flatnonzero(~left_mask)
    li = -np.ones(g.n, np.int64)
    ri = -np.ones(g.n, np.int64)
    li[left] = np.arange(left.size)
    ri[right] = np.arange(right.size)
    u, v = g.edges()
    a = np.where(left_mask[u], u, v)
    b = np.where(left_mask[u], v, u)
    assert np.all(left_mask[a]) and np.all(~left_mask[b]), "not bipartite"
    if a.size == 0:
        return 0
    m = csr_matrix((np.ones(a.size), (li[a], ri[b])),
                   shape=(left.size, right.size))
    match = maximum_bipartite_matching(m, perm_type="column")
    return int(np.sum(match >= 0))


def tree_mvc(g) -> int:
    """MVC of a forest by the take/skip dynamic program (iterative DFS)."""
    off = g.offsets.astype(np.int64)
    cols = g.cols.astype(np.int64)
    seen = np.zeros(g.n, bool)
    take = np.zeros(g.n, np.int64)
    skip = np.zeros(g.n, np.int64)
    total = 0
    for root in range(g.n):
        if seen[root]:
            continue
        order, parent = [], {root: -1}
        stack = [root]
        seen[root] = True
        while stack:
            x = stack.pop()
            order.append(x)
            for w in cols[off[x]:off[x + 1]].tolist():
                if not seen[w]:
                    seen[w] = True
                    parent[w] = x
                    stack.append(w)
                elif parent[x] != w:
                    raise ValueError("graph has a cycle")
        for x in reversed(order):
            take[x] += 1
            p = parent[x]
            if p >= 0:
                take[p] += min(take[x], skip[x])
                skip[p] += take[x]
        total += int(min(take[root], skip[root]))
    return total


def bipartition(g) -> np.ndarray:
    """Two-colouring by BFS (raises if the graph is not bipartite)."""
    off = g.offsets.astype(np.int64)
    cols = g.cols.astype(np.int64)
    colour = -np.ones(g.n, np.int64)
    for r in range(g.n):
        if colour[r] >= 0:
            continue
        colour[r] = 0
        q = [r]
        while q:
            x = q.pop()
            for w in cols[off[x]:off[x + 1]].tolist():
                if colour[w] < 0:
                    colour[w] = 1 - colour[x]
                    q.append(w)
                elif colour[w] == colour[x]:
                    raise ValueError("not bipartite")
    return colour == 0
