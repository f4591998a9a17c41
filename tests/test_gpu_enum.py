"""Enumeration of minimal vertex covers of size <= k (vc_param_enum) through
the C ABI, against the oracle's enumeration: the set of covers is unique, so
the two sets must be equal and the counts identical."""
import numpy as np
import pytest

from paper_2512_18334_amd import graphgen as gg
from paper_2512_18334_amd import vc
from tests.test_oracle_enum import kab, star, union

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver(libvc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    s = vc.Solver(0, watchdog_ms=60_000)
    yield s
    s.close()


def covers_set(covers):
    return {frozenset(c.tolist()) for c in covers}


def check(solver, orc, g, k, max_covers=200_000):
    count, covers = solver.enum_minimal(g, k, max_covers)
    o = orc.enum_minimal(g, k)
    assert count == o["count"], (g.name, k, count, o["count"])
    got = covers_set(covers)
    assert len(got) == len(covers) == min(count, max_covers)
    for c in covers:
        assert list(c) == sorted(c) and len(c) <= k
    if count <= max_covers:
        assert got == o["covers"], (g.name, k)
    else:
        assert got <= o["covers"]
    return count


def test_small_families(solver, orc):
    gs = [gg.path(3), gg.cycle(5), star(5), kab(2, 3), kab(3, 3),
          union(gg.path(3), gg.cycle(5), star(4)), gg.petersen()]
    for g in gs:
        for k in range(0, min(g.n, 9) + 1):
            check(solver, orc, g, k)


def test_random_small_graphs(solver, orc):
    r = np.random.default_rng(5)
    for i in range(40):
        g = gg.gnp(int(r.integers(5, 34)), float(r.uniform(0.05, 0.3)), 3000 + i)
        if g.nnz == 0:
            continue
        m = orc.mvc(g)["size"]
        for k in (m - 1, m, m + 2):
            if k >= 0:
                check(solver, orc, g, k)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_gnp60(solver, orc, seed):
    g = gg.config1_gnp60(seed)
    m = orc.mvc(g)["size"]
    assert check(solver, orc, g, m - 1) == 0
    assert check(solver, orc, g, m) >= 1
    check(solver, orc, g, m + 1)


def test_fewer_slots_than_covers(solver, orc):
    g = union(gg.cycle(5), gg.cycle(5), gg.path(3))
    k = 8
    o = orc.enum_minimal(g, k)
    assert o["count"] > 10
    count, covers = solver.enum_minimal(g, k, 10)
    assert count == o["count"] and len(covers) == 10
    assert covers_set(covers) <= o["covers"] and len(covers_set(covers)) == 10


def test_edge_cases(solver, orc):
    empty = gg.from_edges(5, [], [])
    assert solver.enum_minimal(empty, 3, 4)[0] == 1
    assert solver.enum_minimal(gg.path(4), 0, 4) == (0, [])
    big = gg.path(70)  # one component of 70 vertices
    with pytest.raises(vc.VCError) as e:
        solver.enum_minimal(big, 40, 4)
    assert e.value.status == vc.VC_ERANGE
    g = gg.config1_gnp60(9)
    m = orc.mvc(g)["size"]
    a = solver.enum_minimal(vc.DeviceGraph.from_graph(g), m)
    b = solver.enum_minimal(g, m)
    assert a[0] == b[0] and covers_set(a[1]) == covers_set(b[1])
