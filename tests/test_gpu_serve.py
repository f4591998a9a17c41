"""Serving through the C ABI (vc_submit / vc_poll / vc_cancel).

Requests of different kinds and sizes are submitted together so that they
are admitted into the resident search while others run; every answer must
equal the oracle's and the one the same request gets alone (exact integers),
and every cover is checked on every edge.
"""
import time

import pytest

from paper_2512_18334_amd import graphgen as gg
from paper_2512_18334_amd import vc
from tests.helpers import assert_cover

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver(libvc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    s = vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000)
    yield s
    s.close()


def request_mix():
    """(graph, kind, k) in arrival order: the served-stream recipe at
    reduced sizes plus small exact cases."""
    reqs = []
    for i, r in enumerate(gg.config5_stream(count=16, n_hi=20_000)):
        reqs.append((r["graph"], vc.VC_MIN if r["kind"] == "min" else vc.VC_PARAM, r["k"]))
    for s in range(1, 13):
        reqs.append((gg.config1_gnp60(s), vc.VC_MIN, 0))
    reqs.append((gg.config2_blocks_hubs(seed=50, nblocks=5, bsize=40, nhubs=3, per_block=10),
                 vc.VC_MIN, 0))
    reqs.append((gg.petersen(), vc.VC_PARAM, 5))
    reqs.append((gg.petersen(), vc.VC_PARAM, 6))
    reqs.append((gg.fig1_tree(), vc.VC_MIN, 0))
    reqs.append((gg.from_edges(4, [], []), vc.VC_MIN, 0))
    return reqs


def wait_idle_then(fn, timeout_s=30.0):
    """Run a blocking solve once the server has nothing in flight."""
    t0 = time.perf_counter()
    while True:
        try:
            return fn()
        except vc.VCError as e:
            if e.status != vc.VC_EAGAIN or time.perf_counter() - t0 > timeout_s:
                raise
            time.sleep(0.005)


def test_served_mix_matches_oracle_and_alone(solver, orc):
    reqs = request_mix()
    tickets = [solver.submit(g, kind, k) for g, kind, k in reqs]
    results = []
    for t, (g, _, _) in zip(tickets, reqs):
        print(f"serve: waiting for {g.name} (ticket {t})", flush=True)
        results.append(solver.wait(t, g.n))
    for (g, kind, k), (res, cov) in zip(reqs, results):
        assert res["status"] == vc.VC_OK, (g.name, res)
        mvc = orc.mvc(g)["size"]
        if kind == vc.VC_MIN:
            assert res["size"] == mvc, (g.name, res["size"], mvc)
            assert_cover(g, cov, size=mvc)
        else:
            assert bool(res["yes"]) == (mvc <= k), (g.name, k, mvc)
            if res["yes"]:
                assert_cover(g, cov, at_most=k)
            else:
                assert cov.size == 0
    # the same requests alone, one blocking solve each
    for (g, kind, k), (res, _) in zip(reqs, results):
        if kind == vc.VC_MIN:
            alone = wait_idle_then(lambda: solver.mvc(g)).size
            assert res["size"] == alone
        else:
            alone = wait_idle_then(lambda: solver.pvc(g, k)).yes
            assert bool(res["yes"]) == alone


def test_served_requests_overlap_in_one_launch(solver, orc):
    """Requests submitted back to back are in the resident search together:
    at least one is admitted while another is still unanswered."""
    gs = [gg.config2_blocks_hubs(seed=60 + s, nblocks=12, bsize=64, nhubs=4, per_block=16)
          for s in range(6)]
    tickets = [solver.submit(g) for g in gs]
    results = [solver.wait(t, g.n) for t, g in zip(tickets, gs)]
    for g, (res, cov) in zip(gs, results):
        e = orc.mvc(g)["size"]
        assert res["size"] == e
        assert_cover(g, cov, size=e)
    lat = [r["ms_latency"] for r, _ in results]
    queued = sorted(r["ms_queued"] for r, _ in results)
    # a second request was admitted before the first answer was ready
    assert queued[1] < min(lat), (queued, lat)


def test_cancel_and_unknown_ticket(solver):
    g = gg.gnp(220, 0.09, 4242)  # far too hard to finish quickly
    t = solver.submit(g)
    solver.cancel(t)
    with pytest.raises(vc.VCError) as e:
        solver.wait(t, g.n, timeout_s=60)
    assert e.value.status == vc.VC_ECANCELED
    with pytest.raises(vc.VCError) as e:
        solver.poll(t, g.n)
    assert e.value.status == vc.VC_EINVAL


def test_device_graph_submission(solver, orc):
    g = gg.config1_gnp60(77)
    dg = vc.DeviceGraph.from_graph(g)
    t = solver.submit(dg)
    del dg  # the request holds its own copy
    res, cov = solver.wait(t, g.n)
    e = orc.mvc(g)["size"]
    assert res["size"] == e
    assert_cover(g, cov, size=e)


def test_invalid_request_is_answered_with_einval(solver):
    good = gg.petersen()
    bad = gg.Graph(good.n, good.offsets.copy(), good.cols.copy())
    bad.cols[0] = 0  # self-loop
    t_bad = solver.submit(bad)
    t_good = solver.submit(good)
    res, cov = solver.wait(t_bad, bad.n)
    assert res["status"] == vc.VC_EINVAL and cov.size == 0
    res, cov = solver.wait(t_good, good.n)
    assert res["status"] == vc.VC_OK and res["size"] == 6


def test_served_requests_with_many_streams_alive(libvc, orc):
    """With many streams alive in the process, the runtime maps several of
    them onto one hardware queue, so the server's side stream may share a
    queue with its resident search launch.  A launch that waited for the
    host would then wait for work queued behind itself; served launches end
    when they run out of work, so requests still complete."""
    import torch
    streams = [torch.cuda.Stream(device=0) for _ in range(12)]
    for st in streams:
        with torch.cuda.stream(st):
            torch.zeros(16, device="cuda:0").add_(1)
    gs = [gg.config1_gnp60(s) for s in range(30, 42)]
    with vc.Solver(0, node_limit=20_000_000, watchdog_ms=60_000) as s:
        for rnd in range(3):
            tickets = [s.submit(g) for g in gs]
            for t, g in zip(tickets, gs):
                res, cov = s.wait(t, g.n, timeout_s=60)
                e = orc.mvc(g)["size"]
                assert res["status"] == vc.VC_OK and res["size"] == e, (rnd, g.name, res)
                assert_cover(g, cov, size=e)
    torch.cuda.synchronize()
    del streams


def test_device_graph_requests_through_the_ring(solver, orc):
    """Device graphs above 256 vertices are copied device to device into the
    server's request ring (64 MiB) and read there by the root steps.  Thirty
    copies of a 100,000-vertex graph (3.6 MB each) pass more than the ring
    holds, so pieces wrap around and a full ring sends requests through the
    host instead; a request of invalid structure is refused from the ring,
    one is cancelled on it, and the torch tensors are dropped right after
    each submission (the request owns its copy)."""
    big = gg.chung_lu_planted(100_000, 400_000, 2.3, 6_000, 99, col_bytes=None, name="big")
    mid = gg.config2_blocks_hubs(seed=71, nblocks=6, bsize=64, nhubs=3, per_block=12)
    e_big = orc.mvc(big)["size"]
    e_mid = orc.mvc(mid)["size"]
    bad = gg.Graph(mid.n, mid.offsets.copy(), mid.cols.copy(), name="self-loop")
    bad.cols[bad.offsets[5]] = 5  # a self-loop in row 5
    plan = []
    for i in range(30):
        if i % 3 == 2:
            plan.append((big, vc.VC_PARAM, e_big - (i % 2)))
        else:
            plan.append((big, vc.VC_MIN, 0))
        if i % 10 == 0:
            plan.append((mid, vc.VC_MIN, 0))
    plan.insert(7, (bad, vc.VC_MIN, 0))
    tickets = []
    for g, kind, k in plan:
        dg = vc.DeviceGraph.from_graph(g)
        tickets.append(solver.submit(dg, kind, k))
        del dg
    hard = vc.DeviceGraph.from_graph(gg.gnp(300, 0.09, 4343))
    t_hard = solver.submit(hard)
    del hard
    solver.cancel(t_hard)
    for t, (g, kind, k) in zip(tickets, plan):
        print(f"ring: waiting for {g.name} kind {kind} k {k} (ticket {t})", flush=True)
        res, cov = solver.wait(t, g.n, timeout_s=120)
        if g is bad:
            assert res["status"] == vc.VC_EINVAL and cov.size == 0
            continue
        assert res["status"] == vc.VC_OK, (g.name, res)
        e = e_big if g is big else e_mid
        if kind == vc.VC_MIN:
            assert res["size"] == e, (g.name, res["size"], e)
            assert_cover(g, cov, size=e)
        else:
            assert bool(res["yes"]) == (e <= k), (g.name, k, e)
            if res["yes"]:
                assert_cover(g, cov, at_most=k)
    with pytest.raises(vc.VCError) as ex:
        solver.wait(t_hard, 300, timeout_s=60)
    assert ex.value.status == vc.VC_ECANCELED
    # the ring is usable again afterwards
    t = solver.submit(vc.DeviceGraph.from_graph(mid))
    res, cov = solver.wait(t, mid.n)
    assert res["size"] == e_mid
    assert_cover(mid, cov, size=e_mid)
