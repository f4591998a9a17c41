"""GPU path vs the CPU oracle and closed forms, through the C ABI.

Every expected value comes from a closed form or from the oracle (never from
the GPU).  MVC sizes and PVC answers must agree exactly; every returned cover
is checked on every edge and for its size.  Which cover is returned is not
unique and is not compared.
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
    # a node limit turns a runaway search into a failed test, not a hang;
    # every complete search's registry end state is checked too
    s = vc.Solver(0, node_limit=50_000_000, watchdog_ms=60_000,
                  flags=vc.VC_OPT_CHECK_REGISTRY)
    yield s
    s.close()


def check_protocol(stats):
    """No worklist read saw an older payload, and after a search that ran to
    its end every registry entry was completed exactly once."""
    assert stats["stale_reads"] == 0, stats
    if stats["reg_checked"]:
        assert stats["reg_open"] == 0, stats


def gpu_mvc(solver, g, expected):
    try:
        r = solver.mvc(g)
    except vc.VCError:
        # the failed call's statistics name the stage it reached
        try:
            print("failed solve:", g.name, solver.stats(), flush=True)
        except vc.VCError:
            pass
        raise
    assert r.size == expected, (g.name, r.size, expected)
    assert_cover(g, r.cover, size=expected)
    check_protocol(r.stats)
    return r


def gpu_pvc_threshold(solver, g, mvc, ks=None):
    for k in (ks if ks is not None else [mvc - 1, mvc, mvc + 1]):
        if k < 0:
            continue
        r = solver.pvc(g, k)
        assert r.yes == (k >= mvc), (g.name, k, mvc, r.yes)
        check_protocol(r.stats)
        if r.yes:
            assert_cover(g, r.cover, at_most=k)
        else:
            assert r.cover.size == 0


# ----------------------------------------------------------- closed forms

def test_closed_forms(solver):
    cases = []
    cases += [(gg.path(n), n // 2) for n in range(1, 21)]
    cases += [(gg.cycle(n), (n + 1) // 2) for n in range(3, 21)]
    cases += [(gg.complete(n), max(n - 1, 0)) for n in range(1, 13)]
    cases += [(gg.complete_bipartite(a, b), min(a, b))
              for a, b in [(1, 1), (2, 5), (3, 3), (4, 7), (6, 6)]]
    cases += [(gg.star(k), 1) for k in (1, 3, 40)]
    cases += [(gg.petersen(), 6)]
    cases += [(gg.grid(a, b), a * b // 2) for a, b in [(2, 3), (4, 4), (5, 6)]]
    cases += [(gg.hypercube(d), 1 << (d - 1)) for d in range(1, 6)]
    for g, expect in cases:
        gpu_mvc(solver, gg.relabel(g, 7), expect)


def test_fig1_example(solver):
    g = gg.fig1_tree()
    r = gpu_mvc(solver, g, 3)
    assert sorted(r.cover.tolist()) == [1, 4, 7]  # {b, e, h}
    gpu_pvc_threshold(solver, g, 3)


def test_empty_and_edgeless(solver):
    for g in [gg.from_edges(0, [], []), gg.from_edges(1, [], []),
              gg.from_edges(33, [], [])]:
        r = solver.mvc(g)
        assert r.size == 0 and r.cover.size == 0
        assert solver.pvc(g, 0).yes


def test_disjoint_union_of_simple_components(solver, orc):
    g = gg.relabel(gg.disjoint_union([gg.cycle(9), gg.complete(6), gg.cycle(4),
                                      gg.petersen(), gg.complete(4), gg.cycle(12)]), 3)
    gpu_mvc(solver, g, 5 + 5 + 2 + 6 + 3 + 6)


# ------------------------------------------------------- G(60, 0.1) workload

@pytest.mark.parametrize("block", range(8))
def test_gnp60_parity(solver, orc, block):
    for seed in range(1 + 32 * block, 33 + 32 * block):
        g = gg.config1_gnp60(seed)
        gpu_mvc(solver, g, orc.mvc(g)["size"])


def test_gnp60_pvc(solver, orc):
    for seed in range(1, 33):
        g = gg.config1_gnp60(seed)
        gpu_pvc_threshold(solver, g, orc.mvc(g)["size"])


def test_random_small_graphs(solver, orc):
    r = gg.rng(777)
    for i in range(200):
        n = int(r.integers(6, 48))
        p = float(r.uniform(0.04, 0.5))
        g = gg.gnp(n, p, 5000 + i)
        gpu_mvc(solver, g, orc.mvc(g)["size"])


def test_device_resident_input(solver, orc):
    for seed in (1, 2, 3):
        g = gg.config1_gnp60(seed)
        dg = vc.DeviceGraph.from_graph(g)
        r = solver.mvc(dg)
        assert r.size == orc.mvc(g)["size"]
        assert_cover(g, r.cover, size=r.size)


def test_device_validation_rejects(solver):
    g = gg.petersen().with_cols(4)
    bad = gg.Graph(g.n, g.offsets.copy(), g.cols.copy())
    bad.cols[0] = 0  # self-loop
    with pytest.raises(vc.VCError) as e:
        solver.mvc(vc.DeviceGraph.from_graph(bad))
    assert e.value.status == vc.VC_EINVAL
    asym = gg.Graph(g.n, g.offsets.copy(), g.cols.copy())
    row = set(asym.cols[asym.offsets[0]:asym.offsets[1]].tolist())
    asym.cols[0] = next(x for x in range(1, g.n) if x not in row)
    with pytest.raises(vc.VCError) as e:
        solver.mvc(vc.DeviceGraph.from_graph(asym))
    assert e.value.status == vc.VC_EINVAL


def long_row_graph(deg, dup=None, seed=0):
    """Two adjacent hubs (0 and 1) joined to `deg` - 1 leaves that form a
    path; the hub rows are shuffled (not sorted).  dup=(p1, p2): hub 1 sits
    at positions p1 and p2 of hub 0's row, and hub 0 twice in hub 1's row --
    a symmetric repeat that only the check of long rows can catch."""
    r = np.random.default_rng(seed)
    n = deg + 1
    leaves = np.arange(2, n)
    h0 = [int(x) for x in r.permutation(leaves)]
    h1 = [int(x) for x in r.permutation(np.append(leaves, 0))]
    if dup is None:
        h0.insert(int(r.integers(0, len(h0) + 1)), 1)
    else:
        h0.insert(dup[0], 1)
        h0.insert(dup[1], 1)
        h1.insert(int(r.integers(0, len(h1) + 1)), 0)
    rows = [h0, h1]
    for x in range(2, n):
        rows.append([0, 1] + ([x - 1] if x > 2 else []) + ([x + 1] if x < n - 1 else []))
    offsets = np.zeros(n + 1, np.uint32)
    offsets[1:] = np.cumsum([len(a) for a in rows])
    return gg.Graph(n, offsets, np.concatenate(rows).astype(np.uint32), name=f"hubs2x{deg}")


@pytest.mark.parametrize("deg,dup", [(700, (3, 650)), (1500, (5, 1400)), (1500, (1100, 1300)),
                                     (2600, (2500, 2599))])
def test_device_validation_finds_repeats_in_long_unsorted_rows(solver, orc, deg, dup):
    good = long_row_graph(deg, seed=deg)
    r = solver.mvc(vc.DeviceGraph.from_graph(good))
    assert r.size == orc.mvc(good)["size"]
    bad = long_row_graph(deg, dup=dup, seed=deg)
    assert vc.DeviceGraph.from_graph(bad).n == good.n
    with pytest.raises(vc.VCError) as e:
        solver.mvc(vc.DeviceGraph.from_graph(bad))
    assert e.value.status == vc.VC_EINVAL
    with pytest.raises(vc.VCError) as e:  # the host check agrees
        solver.mvc(bad)
    assert e.value.status == vc.VC_EINVAL


# ------------------------------------------- component-splitting workload

def test_blocks_hubs_small(solver, orc):
    for seed in range(4):
        g = gg.config2_blocks_hubs(seed=10 + seed, nblocks=6, bsize=48, nhubs=3,
                                   per_block=12)
        gpu_mvc(solver, g, orc.mvc(g)["size"])


def test_blocks_hubs_full(solver, orc):
    g = gg.config2_blocks_hubs()
    expect = orc.mvc(g)["size"]
    assert expect == 1077
    r = gpu_mvc(solver, g, expect)
    st = r.stats
    assert st["deg_bytes"] == 2          # hub degree 600 needs 16 bits
    assert st["component_branches"] > 0  # hubs out -> the blocks split
    gpu_pvc_threshold(solver, g, expect)


def test_ablation_switches_agree(solver, orc, libvc):
    """Every switch and capacity gives the same exact answer.  Without
    component branching the search tree multiplies across blocks (the
    paper's ablation runs out of time), so that switch gets graphs where the
    plain vertex branching stays small."""
    small = [gg.config1_gnp60(s) for s in (1, 2, 3, 4)]
    small.append(gg.config2_blocks_hubs(seed=22, nblocks=3, bsize=16, nhubs=2,
                                        per_block=5))
    hubs = gg.config2_blocks_hubs(seed=21, nblocks=6, bsize=48, nhubs=3, per_block=12)
    exp_small = [orc.mvc(g)["size"] for g in small]
    exp_hubs = orc.mvc(hubs)["size"]
    for kw in [dict(flags=vc.VC_OPT_NO_COMPONENTS),
               dict(flags=vc.VC_OPT_NO_LOAD_BALANCE),
               dict(flags=vc.VC_OPT_NO_SMALL), dict(small_max=64),
               dict(flags=vc.VC_OPT_NO_COMPONENTS | vc.VC_OPT_NO_SMALL),
               dict(flags=vc.VC_OPT_NO_INDUCE), dict(flags=vc.VC_OPT_NO_COMPACT),
               dict(flags=vc.VC_OPT_NO_INDUCE | vc.VC_OPT_NO_COMPACT | vc.VC_OPT_NO_SMALL),
               dict(flags=vc.VC_OPT_CROWN), dict(flags=vc.VC_OPT_NO_CROWN),
               dict(workers=1), dict(workers=3),
               dict(registry_cap=64), dict(worklist_cap=8)]:
        with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000, **kw) as s2:
            for g, e in zip(small, exp_small):
                gpu_mvc(s2, g, e)
            if not kw.get("flags", 0) & vc.VC_OPT_NO_COMPONENTS:
                gpu_mvc(s2, hubs, exp_hubs)


def pendant_graph():
    """Blocks joined by hubs, with pendant paths (the degree-one rule fires
    at the root) and 5 isolated vertices."""
    g0 = gg.config2_blocks_hubs(seed=31, nblocks=4, bsize=24, nhubs=2, per_block=6)
    extra = 5
    us, vs = [], []
    for i in range(8):
        a = g0.n + extra + 2 * i
        us += [i * 3, a]
        vs += [a, a + 1]
    eu, ev = g0.edges()
    return gg.from_edges(g0.n + extra + 16, np.concatenate([eu, us]), np.concatenate([ev, vs]))


def test_no_induce_searches_the_input_graph(orc, libvc):
    """With the root reduction and induction off the search starts from the
    input in its own ids: nothing is forced at the root, every vertex
    (isolated ones included) keeps its id, and answers are unchanged."""
    g = pendant_graph()
    e = orc.mvc(g)["size"]
    with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000) as s0:
        r0 = gpu_mvc(s0, g, e)
    assert r0.stats["forced_root"] > 0
    for flags in (vc.VC_OPT_NO_INDUCE, vc.VC_OPT_NO_INDUCE | vc.VC_OPT_NO_COMPACT):
        with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000, flags=flags) as s:
            r = gpu_mvc(s, g, e)
            assert r.stats["forced_root"] == 0 and r.stats["root_rounds"] == 0
            assert r.stats["n_kernel"] == g.n
            for k in (e - 1, e):
                assert s.pvc(g, k).yes == (e <= k)


def test_poisoned_buffers_change_nothing(orc, libvc):
    """Every device buffer filled with 0xA7 bytes before use (VC_OPT_POISON):
    no step may read memory that the call did not write.  The root node's
    header flags were once left unwritten, and memory from earlier calls
    made the root scope induce a view of its own (wrong answers without the
    root rules)."""
    graphs = [pendant_graph(), gg.config1_gnp60(3),
              gg.config2_blocks_hubs(seed=22, nblocks=3, bsize=16, nhubs=2, per_block=5),
              gg.disjoint_union([gg.cycle(7), gg.complete(5), gg.petersen()])]
    exp = [orc.mvc(g)["size"] for g in graphs]
    P = vc.VC_OPT_POISON | vc.VC_OPT_CHECK_REGISTRY
    for flags in (0, vc.VC_OPT_NO_INDUCE, vc.VC_OPT_NO_INDUCE | vc.VC_OPT_NO_SMALL,
                  vc.VC_OPT_EAGER_INDUCE, vc.VC_OPT_NO_ROOT_CACHE, vc.VC_OPT_CROWN):
        with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000, flags=flags | P) as s:
            for g, e in zip(graphs, exp):
                gpu_mvc(s, g, e)
                gpu_pvc_threshold(s, g, e)
    with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000, flags=P) as s:
        res = s.mvc_batch(graphs)
        assert [int(x) for x in res.sizes] == exp
        for g, e, cov in zip(graphs, exp, res.covers):
            assert_cover(g, cov, size=e)


def test_context_reuse_after_worklist_wrap(orc, libvc):
    """A context keeps its worklist between calls.  With 8 slots the
    worklist wraps many times, so slot 0 (where the next call's root node
    goes) last held some earlier node, often a component child marked for
    induction; each call must start from its own root node only."""
    hubs = gg.config2_blocks_hubs(seed=21, nblocks=6, bsize=48, nhubs=3, per_block=12)
    g = pendant_graph()
    e_h, e_g = orc.mvc(hubs)["size"], orc.mvc(g)["size"]
    for flags in (vc.VC_OPT_NO_INDUCE, 0):
        with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000, worklist_cap=8,
                       flags=flags | vc.VC_OPT_CHECK_REGISTRY) as s:
            for _ in range(3):
                gpu_mvc(s, hubs, e_h)
                gpu_mvc(s, g, e_g)


def test_cycle_breakdown_counts_every_activity(solver, orc):
    """The per-activity shader-cycle counters (Fig. 4) are filled on a graph
    that branches on vertices and on components, and they add up to no more
    than the workers' lifetime."""
    g = gg.config2_blocks_hubs(seed=23, nblocks=8, bsize=64, nhubs=4, per_block=14)
    r = gpu_mvc(solver, g, orc.mvc(g)["size"])
    cyc = r.stats["cycles"]
    assert list(cyc) == vc.CYCLE_NAMES
    for k in ("fetch", "reduce", "components", "branch", "complete"):
        assert cyc[k] > 0, (k, cyc)
    assert r.stats["component_branches"] > 0
    # shader clock at most 2.4 GHz: the sum over workers is bounded by
    # workers x kernel time
    bound = r.stats["workers"] * r.stats["ms_search"] * 1e-3 * 2.5e9
    assert sum(cyc.values()) <= bound, (sum(cyc.values()), bound)


def _hub_graph(hub_degree, seed):
    """Cubic blocks plus one hub of exactly hub_degree neighbours, so that
    the hub survives the root reduction (the cover is far larger)."""
    r = gg.rng(seed)
    nblocks, bsize = 24, 48
    us, vs = [], []
    for b in range(nblocks):
        a, c = gg.random_regular(bsize, 3, r)
        us.append(a + b * bsize)
        vs.append(c + b * bsize)
    hub = nblocks * bsize
    t = r.choice(hub, size=hub_degree, replace=False)
    us.append(np.full(hub_degree, hub))
    vs.append(t)
    return gg.relabel(gg.from_edges(hub + 1, np.concatenate(us), np.concatenate(vs)), seed)


@pytest.mark.parametrize("hub_degree,deg_bytes", [(254, 1), (255, 2), (300, 2)])
def test_degree_type_boundary(solver, orc, hub_degree, deg_bytes):
    g = _hub_graph(hub_degree, 40 + hub_degree)
    r = gpu_mvc(solver, g, orc.mvc(g)["size"])
    if r.stats["n_kernel"]:
        assert r.stats["max_degree_kernel"] == hub_degree
        assert r.stats["deg_bytes"] == deg_bytes


# ----------------------------------------------- large sparse PVC workload

@pytest.fixture(scope="module")
def chung_lu_full():
    return gg.config3_chung_lu()


def test_planted_power_law_pvc_full(solver, orc, chung_lu_full):
    g = chung_lu_full
    o = orc.mvc(g)
    mvc = o["size"]
    assert mvc <= g.planted.size
    dg = vc.DeviceGraph.from_graph(g)
    for k in (mvc - 1, mvc):
        r = solver.pvc(dg, k)
        assert r.yes == (k >= mvc)
        if r.yes:
            assert_cover(g, r.cover, at_most=k)
    r = solver.mvc(dg)
    assert r.size == mvc
    assert_cover(g, r.cover, size=mvc)


def test_planted_power_law_scaled(solver, orc):
    for seed in (31, 32):
        g = gg.chung_lu_planted(100_000, 500_000, 2.1, 6_000, seed=seed)
        o = orc.mvc(g)
        gpu_mvc(solver, g, o["size"])
        gpu_pvc_threshold(solver, g, o["size"])


# ------------------------------------------------------ batch-config sample

def test_batch_config_tractable_sample(solver, orc):
    gs = gg.config4_batch(count=48)
    done = 0
    for g in gs:
        try:
            o = orc.mvc(g, node_limit=50_000)
        except orc.OracleLimit:
            continue
        gpu_mvc(solver, g, o["size"])
        done += 1
    assert done >= 10
