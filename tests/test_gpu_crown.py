"""Crown reduction at the root (Sec. IV-B) through the C ABI.

The reduction is result-invariant, so every answer is compared with the
oracle exactly and every cover checked on every edge; the statistics show
that crowns were found (|H| put in the cover, |I| removed) where the graph
has them.
"""
import numpy as np
import pytest

from paper_2512_18334_amd import graphgen as gg
from paper_2512_18334_amd import vc
from tests.helpers import assert_cover

pytestmark = pytest.mark.gpu


def bipartite_union(blocks, a, b):
    """`blocks` disjoint copies of K_{a,b}: the degree rules fire on none of
    them (a, b >= 3), a crown takes each whole (H = the a side)."""
    us, vs = [], []
    for k in range(blocks):
        base = k * (a + b)
        for x in range(a):
            for y in range(b):
                us.append(base + x)
                vs.append(base + a + y)
    return gg.relabel(gg.from_edges(blocks * (a + b), us, vs), 7)


def hubs_with_fans(seed, groups=6):
    """Groups of a few hubs sharing many degree-3+ neighbours, the hubs also
    joined to a random core: crowns that the degree rules do not see."""
    r = np.random.default_rng(seed)
    core = gg.gnp(40, 0.12, seed)
    eu, ev = core.edges()
    us, vs = eu.tolist(), ev.tolist()
    n = core.n
    for _ in range(groups):
        a = int(r.integers(3, 5))
        b = int(r.integers(a + 2, 3 * a + 3))
        hubs = list(range(n, n + a))
        fans = list(range(n + a, n + a + b))
        n += a + b
        for x in fans:
            for h in hubs:
                if h == hubs[0] or h == hubs[1] or h == hubs[2] or r.random() < 0.5:
                    us.append(h)
                    vs.append(x)
        for h in hubs:
            us.append(h)
            vs.append(int(r.integers(0, core.n)))
    return gg.relabel(gg.from_edges(n, us, vs), seed)


@pytest.fixture(scope="module")
def crown_solver(libvc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    s = vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000, flags=vc.VC_OPT_CROWN)
    yield s
    s.close()


def test_crown_finds_and_keeps_answers(crown_solver, orc):
    found = 0
    for seed in range(12):
        g = hubs_with_fans(300 + seed)
        e = orc.mvc(g)["size"]
        r = crown_solver.mvc(g)
        assert r.size == e, (seed, r.size, e)
        assert_cover(g, r.cover, size=e)
        st = r.stats
        if st["crown_rounds"]:
            found += 1
            # every crown has |I| > |H| (H is matched into I, and I holds at
            # least one vertex the matching leaves free)
            assert st["crown_cover"] >= 1 and st["crown_removed"] > st["crown_cover"]
        for k in (e - 1, e):
            p = crown_solver.pvc(g, k)
            assert p.yes == (e <= k)
            if p.yes:
                assert_cover(g, p.cover, at_most=k)
    assert found >= 6, found


def test_crown_equals_no_crown_on_small_graphs(crown_solver, orc):
    with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000,
                   flags=vc.VC_OPT_NO_CROWN) as plain:
        for seed in range(1, 9):
            for g in (gg.config1_gnp60(seed), gg.gnp(48, 0.08, 70 + seed)):
                e = orc.mvc(g)["size"]
                a = crown_solver.mvc(g)
                b = plain.mvc(g)
                assert a.size == b.size == e
                assert_cover(g, a.cover, size=e)
                assert b.stats["crown_rounds"] == 0


def test_crown_takes_bipartite_union_beyond_lds(libvc):
    """9,900 vertices that the degree rules leave whole: the default
    (size-gated) crown solves it at the root; without it the search does,
    with its lists in HBM."""
    g = bipartite_union(900, 3, 8)
    with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000) as s:
        r = s.mvc(g)
        assert r.size == 2700
        assert_cover(g, r.cover, size=2700)
        assert r.stats["crown_rounds"] >= 1 and r.stats["crown_cover"] == 2700
        # M1 matches each 3-side, so I = the 5 other vertices of each 8-side;
        # the last 3 are isolated once H is gone and the degree rules drop them
        assert r.stats["crown_removed"] == 900 * 5
        assert s.pvc(g, 2699).yes is False and s.pvc(g, 2700).yes is True
    # without the crown the search takes the 9,900-vertex kernel itself, its
    # lists kept in HBM (they do not fit LDS)
    with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000,
                   flags=vc.VC_OPT_NO_CROWN) as s:
        r = s.mvc(g)
        assert r.size == 2700
        assert_cover(g, r.cover, size=2700)
        assert r.stats["crown_rounds"] == 0 and r.stats["lists_in_hbm"] == 1
