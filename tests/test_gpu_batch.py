"""Batches through the C ABI (vc_min_batch / vc_param_batch) against closed
forms and the CPU oracle.

Sizes and PVC answers must agree exactly with the expected value of each
instance; every returned cover is checked on every edge of its instance.
Expected values come only from closed forms and the oracle.
"""
import numpy as np
import pytest

from paper_2512_18334_amd import graphgen as gg
from paper_2512_18334_amd import vc
from tests.helpers import assert_cover

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver(libvc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    s = vc.Solver(0, node_limit=5_000_000, watchdog_ms=60_000)
    yield s
    s.close()


def mixed_graphs():
    """Closed forms, the worked example, empty and edgeless graphs."""
    cases = [(gg.path(7), 3), (gg.cycle(9), 5), (gg.complete(6), 5),
             (gg.complete_bipartite(3, 5), 3), (gg.star(12), 1), (gg.petersen(), 6),
             (gg.grid(4, 4), 8), (gg.hypercube(4), 8), (gg.fig1_tree(), 3),
             (gg.from_edges(0, [], []), 0), (gg.from_edges(5, [], []), 0),
             (gg.path(2), 1), (gg.disjoint_union([gg.cycle(5), gg.complete(4)]), 6)]
    return [(gg.relabel(g, 11), e) for g, e in cases]


def check_mvc(res, graphs, expected):
    assert list(res.status) == [vc.VC_OK] * len(graphs)
    for g, e, got, cov in zip(graphs, expected, res.sizes, res.covers):
        assert int(got) == e, (g.name, int(got), e)
        assert_cover(g, cov, size=e)


def test_batch_closed_forms(solver):
    gs, exp = zip(*mixed_graphs())
    check_mvc(solver.mvc_batch(list(gs)), gs, exp)


def test_batch_gnp60_and_hubs_vs_oracle(solver, orc):
    gs = [gg.config1_gnp60(s) for s in range(1, 65)]
    gs += [gg.config2_blocks_hubs(seed=30 + s, nblocks=4, bsize=32, nhubs=2, per_block=8)
           for s in range(4)]
    exp = [orc.mvc(g)["size"] for g in gs]
    check_mvc(solver.mvc_batch(gs), gs, exp)


def test_batch_pvc_thresholds(solver, orc):
    base = [gg.config1_gnp60(s) for s in range(1, 17)] + [g for g, _ in mixed_graphs()]
    mvc = [orc.mvc(g)["size"] for g in base]
    gs, ks, want = [], [], []
    for g, m in zip(base, mvc):
        for k in (m - 1, m, m + 1):
            if k < 0:
                continue
            gs.append(g)
            ks.append(k)
            want.append(k >= m)
    r = solver.pvc_batch(gs, ks)
    assert list(r.status) == [vc.VC_OK] * len(gs)
    for g, k, w, y, cov in zip(gs, ks, want, r.yes, r.covers):
        assert bool(y) == w, (g.name, k)
        if w:
            assert_cover(g, cov, at_most=k)
        else:
            assert cov.size == 0


def test_batch_device_resident(solver, orc):
    gs = [gg.config1_gnp60(s) for s in range(100, 132)]
    exp = [orc.mvc(g)["size"] for g in gs]
    b = vc.Batch.from_graphs(gs).to_device("cuda:0")
    check_mvc(solver.mvc_batch(b), gs, exp)


def test_batch_replay_and_plain_launch_agree(solver, orc):
    gs = [gg.config1_gnp60(s) for s in range(200, 216)]
    exp = [orc.mvc(g)["size"] for g in gs]
    b = vc.Batch.from_graphs(gs)
    for _ in range(3):  # the first call captures the launch, the others replay it
        check_mvc(solver.mvc_batch(b), gs, exp)
    with vc.Solver(0, node_limit=5_000_000, watchdog_ms=60_000,
                   flags=vc.VC_OPT_NO_GRAPH) as s2:
        check_mvc(s2.mvc_batch(b), gs, exp)


def test_batch_equals_single_solves(solver):
    """Each instance gets the same size in the batch as alone."""
    gs = [gg.config1_gnp60(s) for s in range(300, 316)]
    gs += [gg.config2_blocks_hubs(seed=40, nblocks=3, bsize=24, nhubs=2, per_block=6)]
    alone = [solver.mvc(g).size for g in gs]
    r = solver.mvc_batch(gs)
    assert [int(x) for x in r.sizes] == alone


def test_batch_device_validation_rejects(solver):
    good = gg.petersen()
    bad = gg.Graph(good.n, good.offsets.copy(), good.cols.copy())
    bad.cols[0] = 0  # self-loop
    b = vc.Batch.from_graphs([gg.cycle(5), bad, gg.path(4)]).to_device("cuda:0")
    with pytest.raises(vc.VCError) as e:
        solver.mvc_batch(b)
    assert e.value.status == vc.VC_EINVAL
    with pytest.raises(vc.VCError) as e:
        solver.mvc_batch([gg.cycle(5), bad])
    assert e.value.status == vc.VC_EINVAL


def test_batch_device_validation_finds_repeats_in_long_rows(solver):
    from tests.test_gpu_parity import long_row_graph
    good = long_row_graph(1500, seed=3)
    bad = long_row_graph(1500, dup=(7, 1300), seed=3)
    r = solver.mvc_batch(vc.Batch.from_graphs([gg.cycle(5), good]).to_device("cuda:0"))
    assert [int(x) for x in r.sizes] == [3, solver.mvc(good).size]
    b = vc.Batch.from_graphs([gg.cycle(5), bad, gg.path(4)]).to_device("cuda:0")
    with pytest.raises(vc.VCError) as e:
        solver.mvc_batch(b)
    assert e.value.status == vc.VC_EINVAL


def test_batch_node_limit_is_per_instance(libvc, orc):
    """A tiny limit stops the hard instances only; the easy ones still
    return exact sizes, and every cover is valid."""
    easy = [gg.path(9), gg.cycle(7), gg.star(5)]
    hard = [gg.gnp(160, 0.08, 9000 + i) for i in range(2)]
    gs = easy + hard
    with vc.Solver(0, node_limit=2_000, watchdog_ms=60_000) as s:
        r = s.mvc_batch(gs)
    for g, st, size, cov in zip(gs, r.status, r.sizes, r.covers):
        assert st in (vc.VC_OK, vc.VC_ETIMEDOUT)
        assert_cover(g, cov, size=int(size))
    assert list(r.status[:3]) == [vc.VC_OK] * 3
    assert [int(x) for x in r.sizes[:3]] == [4, 4, 1]
    for g, st, size in zip(hard, r.status[3:], r.sizes[3:]):
        if st == vc.VC_OK:
            assert int(size) == orc.mvc(g)["size"]


def test_batch_config4_sample(solver, orc):
    """Instances of the uneven 4096-graph batch: the batch runs a seeded
    sample of them; every instance the oracle finishes within its node
    limit must agree exactly."""
    gs = gg.config4_batch(count=96)
    r = solver.mvc_batch(gs)
    checked = 0
    for g, st, size, cov in zip(gs, r.status, r.sizes, r.covers):
        assert_cover(g, cov, size=int(size))
        try:
            o = orc.mvc(g, node_limit=50_000)
        except orc.OracleLimit:
            continue
        assert st == vc.VC_OK, g.name
        assert int(size) == o["size"], g.name
        checked += 1
    assert checked >= 10


def test_autotune_grid_keeps_exact_sizes(libvc):
    """The batch autotuner on a 2 x 2 grid (waves per CU x worklist depth):
    every configuration must give the same exact sizes (tune_batch raises
    otherwise), and the choice is one of the configurations swept."""
    from paper_2512_18334_amd import autotune
    graphs = [gg.config4_instance(i) for i in range(96)]
    grid = {"waves_per_cu": (1, 2), "worklist_cap": (1024, 4096), "donate_min": (48,)}
    out = autotune.tune_batch(graphs, node_limit=50_000, grid=grid, log=lambda m: None)
    assert len(out["table"]) == 4
    assert out["opts"] in [o for o, _ in out["table"]]
    assert out["ms"] == min(ms for _, ms in out["table"])
