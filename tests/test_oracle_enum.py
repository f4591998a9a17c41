"""Pins of the oracle's enumeration of minimal vertex covers of size <= k.

Each pin is independent of the oracle's code: brute-force subset
enumeration from the definition (C covers every edge, and every vertex of C
has a neighbour outside C), closed forms, the product rule of disjoint
unions, and the minimum size equal to the (separately pinned) MVC.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2512_18334_amd import graphgen as gg


def brute_minimal(g, k):
    n = g.n
    nb = [set(g.cols[g.offsets[v]:g.offsets[v + 1]].tolist()) for v in range(n)]
    eu, ev = g.edges()
    edges = list(zip(eu.tolist(), ev.tolist()))
    out = set()
    for size in range(0, min(k, n) + 1):
        for c in itertools.combinations(range(n), size):
            cs = set(c)
            if all(a in cs or b in cs for a, b in edges) and all(nb[v] - cs for v in cs):
                out.add(frozenset(c))
    return out


@pytest.mark.parametrize("seed", range(40))
def test_enum_equals_brute_force(seed):
    r = np.random.default_rng(seed)
    n = int(r.integers(4, 13))
    g = gg.gnp(n, float(r.uniform(0.15, 0.6)), 900 + seed)
    for k in (0, 2, n // 2, n):
        assert oracle.enum_minimal(g, k)["covers"] == brute_minimal(g, k), (seed, k)


def star(m):
    return gg.from_edges(m + 1, [0] * m, list(range(1, m + 1)))


def kab(a, b):
    return gg.from_edges(a + b, [x for x in range(a) for _ in range(b)],
                         [a + y for _ in range(a) for y in range(b)])


def test_closed_forms():
    # a star: the centre, or all the leaves
    for m in (2, 3, 6):
        for k in range(0, m + 2):
            assert oracle.enum_minimal(star(m), k)["count"] == int(k >= 1) + int(k >= m)
    # K_{a,b}: exactly the two sides
    for a, b in ((2, 3), (3, 3), (2, 5)):
        for k in range(0, b + 1):
            want = {frozenset(range(a))} if a <= k else set()
            if b <= k:
                want.add(frozenset(range(a, a + b)))
            assert oracle.enum_minimal(kab(a, b), k)["covers"] == want
    # K_n: the n sets of n - 1 vertices
    for n in (3, 4, 6):
        g = gg.from_edges(n, *zip(*itertools.combinations(range(n), 2)))
        assert oracle.enum_minimal(g, n - 1)["count"] == n
        assert oracle.enum_minimal(g, n - 2)["count"] == 0
    # C_5: complements of its 5 maximal independent pairs; P_3: {1}, {0, 2}
    assert oracle.enum_minimal(gg.cycle(5), 3)["count"] == 5
    assert oracle.enum_minimal(gg.cycle(5), 2)["count"] == 0
    assert oracle.enum_minimal(gg.path(3), 2)["covers"] == {frozenset({1}), frozenset({0, 2})}


def union(*gs):
    us, vs, base = [], [], 0
    for g in gs:
        a, b = g.edges()
        us += (a + base).tolist()
        vs += (b + base).tolist()
        base += g.n
    return gg.from_edges(base, us, vs)


def test_disjoint_union_product():
    # minimal covers of a union are the unions of the parts' minimal covers
    p3, c5, s4 = gg.path(3), gg.cycle(5), star(4)
    g = union(p3, c5, s4)
    # sizes: P3 {1, 2} (one cover each), C5 {3} (five), star4 {1, 4} (one
    # each): totals 5, 6, 8, 9 with five combinations each
    for k, want in ((4, 0), (5, 5), (6, 10), (7, 10), (8, 15), (9, 20)):
        assert oracle.enum_minimal(g, k)["count"] == want, k
    assert oracle.enum_minimal(g, 9)["covers"] == brute_minimal(g, 9)


@pytest.mark.parametrize("seed", range(1, 6))
def test_minimum_equals_mvc(seed):
    g = gg.config1_gnp60(seed)
    m = oracle.mvc(g)["size"]
    assert oracle.enum_minimal(g, m - 1)["count"] == 0
    res = oracle.enum_minimal(g, m)
    assert res["count"] >= 1 and all(len(c) == m for c in res["covers"])
