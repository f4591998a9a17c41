#!/usr/bin/env python3
"""Benchmark of the exact vertex cover search on one MI355X.

Default workload (the headline line): exact MVC of the component-splitting
blocks-and-hubs graph -- 20 uniform random 3-regular blocks of 96 vertices
plus 8 hubs, each joined to 30 random vertices of every block; n = 1,928,
m = 7,680, CSR uint32 resident in HBM before the timed region.  One step is
one vc_min call on it (validation, degrees, greedy bound, root reduction,
induce, search, cover assembly, the cover copied back).  The line carries
the HBM-roofline view of the persistent search kernel and the CPU oracle
timed beside it, and (unless --no-legs) the metric's other parts as
sub-objects: "batch" (the uneven 4,096-graph batch in one launch),
"serve" (the 2,000-request served stream) and "serve_search_mix" (served
requests that reach the resident search), each beside the plain
one-graph-per-call solver and the oracle over the host's cores.

--workload batch: batched graphs/s on the uneven 4,096-graph batch (one
captured launch per step, a per-instance node limit), with the plain
one-graph-per-launch solver on a prefix of the batch for comparison.
--workload serve: a served stream of mixed MVC/PVC requests with Poisson
arrivals; p50/p99 latency and solves/s, against the plain solver serving
the same arrivals first come first served.
--workload ablation: each optimization switched off in turn (Table II) on
the blocks-and-hubs graph and on 20 G(60, 0.1) graphs.
--workload enum: enumeration of the minimal covers of size <= MVC + 1 on 20
G(60, 0.1) graphs (the enumeration variant of PVC).
--workload pvc_powerlaw: the two PVC queries (k = MVC - 1, MVC) on the
planted power-law graph with 10^6 vertices and 5*10^6 edges.

Prints one JSON line.  Only one GPU is supported: --gpus N with N > 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MVC time-to-solution & search-nodes/s; batched graphs/s; "
          "p50/p99 solve latency")
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "search_blocks_hubs_traffic.json")


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in ("search_worker.hpp", "search_deg.hip", "search.hip", "dev_common.hpp",
              "internal.hpp"):
        with open(os.path.join(ROOT, "paper_2512_18334_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_counters():
    """The committed rocprofv3 counter figures of the search kernel (HBM
    bytes, device-scope atomics and waves per launch), or None if they are
    missing or were taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_source_sha():
        return None
    return t


def cpu_baseline(g, budget_s: float):
    import oracle
    reps, t0, nodes = 0, time.perf_counter(), 0
    while True:
        r = oracle.mvc(g)
        nodes += r["nodes"]
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": nodes / el, "unit": "nodes/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} full sequential solves of the same graph "
                      f"({el:.1f} s; MVC {r['size']}, {r['nodes']} tree nodes each, "
                      f"{el / reps * 1e3:.1f} ms per solve)"}


HOST_CORES_MAX = 16  # a one-GPU machine's share of the host's cores


def host_info():
    """The host's CPU model and the cores a CPU pool may use here (the cores
    this process may run on, at most a one-GPU machine's share)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, min(cores, HOST_CORES_MAX)


def _oracle_batch_instance(i):
    from paper_2512_18334_amd import graphgen as gg
    import oracle
    g = gg.config4_instance(i)
    t0 = time.perf_counter()
    try:
        oracle.mvc(g, node_limit=200_000)
    except oracle.OracleLimit:
        pass
    return time.perf_counter() - t0


def _served_request(i):
    from paper_2512_18334_amd import graphgen as gg
    return gg.config5_request(i)


def _oracle_served_request(i):
    from paper_2512_18334_amd import graphgen as gg
    import oracle
    r = gg.config5_request(i)
    t0 = time.perf_counter()
    if r["kind"] == "min":
        oracle.mvc(r["graph"])
    else:
        oracle.pvc(r["graph"], r["k"])
    return time.perf_counter() - t0


def pool_map(fn, items, procs):
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(procs) as pool:
        return pool.map(fn, items, chunksize=4)


def roofline(stats_list, search_ms):
    """HBM view of the search kernel: algorithmic bytes per launch (node
    slots written and read back once, the root slot, registry entries,
    cover bitmaps and per-component graphs, all counted on the device) over
    the kernel's time."""
    alg_bytes = sum(2 * s["bytes_nodes"] + s["slot_bytes"] + s["bytes_registry"]
                    + s["bytes_rows"] for s in stats_list) / len(stats_list)
    achieved = alg_bytes / (search_ms * 1e-3) / 1e9
    t = measured_counters()
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS,
           "traffic": t.get("hbm_bytes_per_launch") if t else None,
           "alg_bytes_per_launch": alg_bytes}
    # copies of component subgraphs into the workers' LDS graph caches (a
    # view is read again each time a worker switches to it): not counted
    # as algorithmic bytes, reported beside them
    out["view_copy_bytes_per_launch"] = sum(s.get("bytes_views", 0)
                                            for s in stats_list) / len(stats_list)
    # the secondary view: per-node work is latency and atomic bound
    s0 = stats_list[-1]
    out["waves_per_cu"] = s0["workers"] / 256.0
    if t:
        if t.get("atomics_per_launch") is not None:
            out["device_atomics_per_s"] = t["atomics_per_launch"] / (search_ms * 1e-3)
            out["device_atomics_per_launch"] = t["atomics_per_launch"]
        if t.get("wave_occupancy") is not None:
            out["wave_occupancy"] = t["wave_occupancy"]
    return out


def cycle_breakdown(stats):
    """Share of the search workers' shader cycles per activity (Fig. 4):
    fetching nodes, reduction rules, component detection and branching,
    vertex branching, registry completion, idle."""
    tot = {}
    for s in stats:
        for k, v in s["cycles"].items():
            tot[k] = tot.get(k, 0) + v
    all_ = sum(tot.values()) or 1
    return {k: round(100.0 * v / all_, 2) for k, v in tot.items()}


def bench_blocks_hubs(args, torch, gg, vc):
    g = gg.config2_blocks_hubs()
    dg = vc.DeviceGraph.from_graph(g, "cuda:0")
    torch.cuda.synchronize()
    solver = vc.Solver(0, flags=args.flags, workers=args.workers, donate_min=args.donate_min,
                       donate_slack=args.donate_slack, small_max=args.small_max)
    for _ in range(args.warmup):
        solver.mvc(dg)
    torch.cuda.synchronize()

    stats, per_call = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        r = solver.mvc(dg)
        per_call.append(time.perf_counter() - t1)
        stats.append(r.stats)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    size = r.size
    # time to solution from host memory: upload, solve, cover copied back
    # (outside the timed steps)
    import numpy as np
    host_ms = []
    for _ in range(50):
        t1 = time.perf_counter()
        solver.mvc(g)
        host_ms.append((time.perf_counter() - t1) * 1e3)
    dev_ms = np.array(per_call) * 1e3

    nodes = sum(s["tree_nodes"] for s in stats)
    ms_step = el * 1e3 / args.steps
    search_ms = sum(s["ms_search"] for s in stats) / len(stats)
    s0 = stats[-1]
    out = {
        "metric": METRIC,
        "value": nodes / el,
        "unit": "search-nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "mvc_blocks_hubs_n1928", "graph": g.name, "n": g.n,
                   "m": g.m, "mvc": size, "time_to_solution_ms": ms_step,
                   "tree_nodes_per_solve": nodes / args.steps,
                   "search_kernel_ms": search_ms, "workers": s0["workers"],
                   "deg_bytes": s0["deg_bytes"],
                   "component_branches_per_solve":
                       sum(s["component_branches"] for s in stats) / len(stats),
                   "tts_resident_ms_p50": float(np.percentile(dev_ms, 50)),
                   "tts_resident_ms_p90": float(np.percentile(dev_ms, 90)),
                   "tts_host_input_ms_p50": float(np.percentile(host_ms, 50)),
                   "tts_host_input_ms_p90": float(np.percentile(host_ms, 90)),
                   "idle_pct": cycle_breakdown(stats).get("idle", 0.0),
                   "components_per_branch_hist": s0["comp_hist"],
                   "cycle_breakdown_pct": cycle_breakdown(stats)},
        "roofline": roofline(stats, search_ms),
    }
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["config"]["calibration_copy_mib"] = args.copy_mib
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds)
        model, cores = host_info()
        out["cpu_baseline"]["host_cpu"] = model
        out["cpu_baseline"]["host_cores"] = cores
    solver.close()
    if not args.no_legs:
        # the metric's other parts: batched graphs/s and served p50/p99
        print("bench: batch leg", file=sys.stderr, flush=True)
        out["batch"] = leg_batch(args, torch, gg, vc)
        print("bench: served stream leg", file=sys.stderr, flush=True)
        items = served_stream_items(vc)
        out["serve"] = leg_serve(args, torch, gg, vc, items, "served_stream_2000")
        if not args.no_cpu_baseline:
            model, cores = host_info()
            t0 = time.perf_counter()
            pool_map(_oracle_served_request, list(range(len(items))), cores)
            dt = time.perf_counter() - t0
            out["serve"]["cpu_pool_baseline"] = {
                "value": len(items) / dt, "unit": "solves/s", "cores": cores,
                "kind": "oracle",
                "sample": f"all {len(items)} requests, one process per core ({dt:.1f} s)"}
        del items
        print("bench: served search-mix leg", file=sys.stderr, flush=True)
        out["serve_search_mix"] = leg_serve(args, torch, gg, vc, search_mix_items(gg, vc),
                                            "served_gnp60_and_blocks_mix_300")
    return out


GOLDEN_BATCH = os.path.join(ROOT, "tests", "golden", "batch4096_oracle.txt")


def leg_batch(args, torch, gg, vc):
    """The uneven 4,096-graph batch in one captured persistent launch, each
    instance capped at 200,000 tree nodes (the oracle's stored answers under
    the same cap give the agreement), beside the plain one-graph-per-launch
    solver on a prefix and the oracle over the host's cores on a sample."""
    import numpy as np
    cap = 200_000
    gs = gg.config4_batch()
    b = vc.Batch.from_graphs(gs).to_device("cuda:0")
    torch.cuda.synchronize()
    with vc.Solver(0, node_limit=cap, watchdog_ms=120_000) as s:
        t0 = time.perf_counter()
        r = s.mvc_batch(b, want_cover=False)
        el = time.perf_counter() - t0
        st = r.stats
    ok = r.status == vc.VC_OK
    gold = {}
    try:
        with open(GOLDEN_BATCH) as f:
            for line in f:
                if not line.startswith("#"):
                    x = line.split()
                    gold[int(x[0])] = (x[4], int(x[5]))
    except OSError:
        pass
    both = sum(1 for i in range(len(gs)) if ok[i] and gold.get(i, ("", 0))[0] == "exact")
    agree = sum(1 for i in range(len(gs))
                if ok[i] and gold.get(i, ("", 0))[0] == "exact" and int(r.sizes[i]) == gold[i][1])
    nplain = 256
    dgs = [vc.DeviceGraph.from_graph(g, "cuda:0") for g in gs[:nplain]]
    torch.cuda.synchronize()
    with vc.Solver(0, node_limit=cap, watchdog_ms=120_000) as plain:
        t1 = time.perf_counter()
        for dg in dgs:
            try:
                plain.mvc(dg, want_cover=False)
            except vc.VCError as e:
                if e.status != vc.VC_ETIMEDOUT:
                    raise
        pel = time.perf_counter() - t1
    out = {"workload": "mvc_batch_4096_uneven", "count": len(gs),
           "node_limit_per_instance": cap, "graphs_per_s": len(gs) / el,
           "exact_graphs_per_s": int(ok.sum()) / el, "s_per_launch": el,
           "instances_exact": int(ok.sum()), "instances_at_limit": int((~ok).sum()),
           "oracle_exact_under_same_limit": sum(1 for v in gold.values() if v[0] == "exact"),
           "agree_with_oracle": f"{agree}/{both}",
           "search_nodes_per_s": st["tree_nodes"] / (st["ms_search"] * 1e-3),
           "plain_graphs_per_s": nplain / pel, "plain_prefix": nplain}
    if not args.no_cpu_baseline:
        model, cores = host_info()
        sample = list(range(128))
        t0 = time.perf_counter()
        pool_map(_oracle_batch_instance, sample, cores)
        dt = time.perf_counter() - t0
        out["cpu_pool_baseline"] = {"value": len(sample) / dt, "unit": "graphs/s",
                                    "cores": cores, "kind": "oracle",
                                    "sample": f"instances 0-127, same node limit, "
                                              f"one process per core ({dt:.1f} s)"}
    return out


def _fifo_plain(solver, dev, items, arrive, vc):
    """The plain solver serving the same arrivals first come first served,
    measured: each request starts when it has arrived and the previous one
    is done."""
    import numpy as np
    lat, answers = [], []
    t0 = time.perf_counter()
    for j, (g, kind, k) in enumerate(items):
        while time.perf_counter() - t0 < arrive[j]:
            pass
        if kind == vc.VC_MIN:
            answers.append(solver.mvc(dev[j]).size)
        else:
            answers.append(bool(solver.pvc(dev[j], k).yes))
        lat.append((time.perf_counter() - t0 - arrive[j]) * 1e3)
    return np.array(lat), answers, time.perf_counter() - t0


def _serve_stream(solver, dev, items, arrive, vc):
    """Submit at the arrival times, poll until every request is answered;
    returns latencies (ms), answers and the span (first arrival to last
    completion, s)."""
    import numpy as np
    served = [None] * len(items)
    pending = {}
    t0 = time.perf_counter()
    i = 0
    while i < len(items) or pending:
        now = time.perf_counter() - t0
        while i < len(items) and arrive[i] <= now:
            _, kind, k = items[i]
            pending[solver.submit(dev[i], kind, k)] = i
            i += 1
        for tk in list(pending):
            r = solver.poll(tk, items[pending[tk]][0].n)
            if r is not None:
                j = pending.pop(tk)
                served[j] = (r[0], time.perf_counter() - t0)
        time.sleep(0.0001)
    lat = np.array([served[j][1] - arrive[j] for j in range(len(items))]) * 1e3
    ans = [s[0]["size"] if items[j][1] == vc.VC_MIN else bool(s[0]["yes"])
           for j, s in enumerate(served)]
    span = max(s[1] for s in served) - arrive[0]
    return lat, ans, span


def _wait_idle(solver, gg, vc):
    while True:  # until the resident launch is closed
        try:
            solver.mvc(gg.path(3), want_cover=False)
            return
        except vc.VCError as e:
            if e.status != vc.VC_EAGAIN:
                raise
            time.sleep(0.002)


def leg_serve(args, torch, gg, vc, items, label, calib=None):
    """A served stream at a fixed Poisson rate: 0.8 x the plain solver's
    measured solves/s on the first `calib` requests (all of them by default;
    the rate taken from a 200-request prefix varied by a third between runs).  p50/p99 latency and
    solves/s, served (continuous batching) and plain first come first served
    under the same arrivals, both measured; answers compared."""
    import numpy as np
    dev = [vc.DeviceGraph.from_graph(g, "cuda:0") for g, _, _ in items]
    torch.cuda.synchronize()
    if calib is None:
        calib = len(items)
    with vc.Solver(0, node_limit=20_000_000, watchdog_ms=120_000) as s:
        t0 = time.perf_counter()
        for j in range(min(calib, len(items))):
            g, kind, k = items[j]
            if kind == vc.VC_MIN:
                s.mvc(dev[j], want_cover=False)
            else:
                s.pvc(dev[j], k, want_cover=False)
        plain_rate = min(calib, len(items)) / (time.perf_counter() - t0)
        rate = 0.8 * plain_rate
        arrive = np.cumsum(np.random.default_rng(12345).exponential(1.0 / rate, len(items)))
        arrive -= arrive[0]
        t = s.submit(dev[0], items[0][1], items[0][2])  # warm up the server
        s.wait(t, items[0][0].n)
        _wait_idle(s, gg, vc)
        lat, ans, span = _serve_stream(s, dev, items, arrive, vc)
        _wait_idle(s, gg, vc)
        plat, pans, pspan = _fifo_plain(s, dev, items, arrive, vc)
    same = sum(int(a == b) for a, b in zip(ans, pans))
    return {"workload": label, "requests": len(items), "rate_per_s": rate,
            "rate_rule": f"0.8 x plain solves/s on {min(calib, len(items))} requests",
            "solves_per_s": len(items) / span,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "plain_fifo_solves_per_s": len(items) / pspan,
            "plain_fifo_p50_ms": float(np.percentile(plat, 50)),
            "plain_fifo_p99_ms": float(np.percentile(plat, 99)),
            "same_answer_served_and_plain": f"{same}/{len(items)}"}


def served_stream_items(vc, count=2000):
    """The served stream's requests, generated over the host's cores."""
    model, cores = host_info()
    reqs = pool_map(_served_request, list(range(count)), min(cores, 16))
    return [(r["graph"], vc.VC_MIN if r["kind"] == "min" else vc.VC_PARAM, r["k"])
            for r in reqs]


def search_mix_items(gg, vc, count=300):
    """Requests that reach the resident search: G(60, p) graphs (p from 0.08
    to 0.12) and small blocks-and-hubs graphs (4 blocks of 48, 2 hubs), all
    MVC, in a seeded order."""
    import numpy as np
    r = np.random.default_rng(77)
    items = []
    for i in range(count):
        if r.random() < 0.8:
            g = gg.gnp(60, float(r.uniform(0.08, 0.12)), seed=1000 + i)
        else:
            g = gg.config2_blocks_hubs(seed=2000 + i, nblocks=4, bsize=48, nhubs=2,
                                       per_block=10)
        items.append((g, vc.VC_MIN, 0))
    return items


def bench_batch(args, torch, gg, vc):
    """Batched graphs/s on the uneven 4096-graph batch: one captured launch
    per step, each instance capped at --node-limit tree nodes; the plain
    one-graph-per-launch solver runs a prefix of the batch beside it."""
    import numpy as np
    gs = gg.config4_batch(count=args.batch_count)
    b = vc.Batch.from_graphs(gs).to_device("cuda:0")
    opts = {}
    if args.autotune:
        from paper_2512_18334_amd import autotune
        sample = vc.Batch.from_graphs(gs[:min(512, len(gs))]).to_device("cuda:0")
        tuned = autotune.tune_batch(sample, node_limit=args.node_limit, cache=args.tune_cache,
                                    log=lambda m: print(m, file=sys.stderr, flush=True))
        opts = tuned["opts"]
    solver = vc.Solver(0, node_limit=args.node_limit, watchdog_ms=120_000, **opts)
    for _ in range(args.warmup):
        solver.mvc_batch(b, want_cover=False)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = solver.mvc_batch(b, want_cover=False)
        stats.append(r.stats)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    capped = int((r.status != vc.VC_OK).sum())
    # plain per-graph solver on a prefix, same node limit
    nplain = min(args.plain_count, len(gs))
    dgs = [vc.DeviceGraph.from_graph(g, "cuda:0") for g in gs[:nplain]]
    agree = checked = 0
    with vc.Solver(0, node_limit=args.node_limit, watchdog_ms=120_000, **opts) as plain:
        t1 = time.perf_counter()
        psz = []
        for dg in dgs:
            try:
                psz.append(plain.mvc(dg, want_cover=False).size)
            except vc.VCError as e:
                if e.status != vc.VC_ETIMEDOUT:
                    raise
                psz.append(None)
        pel = time.perf_counter() - t1
    for i, ps in enumerate(psz):
        if ps is not None and r.status[i] == vc.VC_OK:
            checked += 1
            agree += int(ps == int(r.sizes[i]))
    search_ms = sum(s["ms_search"] for s in stats) / len(stats)
    out = {
        "metric": METRIC, "value": len(gs) * args.steps / el, "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"mvc_batch_{len(gs)}_uneven", "count": len(gs),
                   "node_limit_per_instance": args.node_limit,
                   "instances_at_limit": capped,
                   "tree_nodes_per_step": stats[-1]["tree_nodes"],
                   "search_nodes_per_s": stats[-1]["tree_nodes"] / (search_ms * 1e-3),
                   "plain_graphs_per_s": nplain / pel, "plain_prefix": nplain,
                   "plain_agree": f"{agree}/{checked}", "opts": opts},
        "roofline": roofline(stats, search_ms),
    }
    solver.close()
    return out


def bench_serve(args, torch, gg, vc):
    """Served stream: Poisson arrivals at --rate of mixed MVC/PVC requests;
    p50/p99 latency and solves/s, against the plain per-graph solver serving
    the same arrivals first come first served (its queueing computed from
    its measured service times)."""
    import numpy as np
    reqs = gg.config5_stream(count=args.serve_count)
    rng = np.random.default_rng(12345)
    arrive = np.cumsum(rng.exponential(1.0 / args.rate, len(reqs)))
    items = [(r["graph"], vc.VC_MIN if r["kind"] == "min" else vc.VC_PARAM, r["k"])
             for r in reqs]
    # every request's CSR is resident in HBM before the timed region, for
    # the served stream and the plain solver alike
    dev = [vc.DeviceGraph.from_graph(g, "cuda:0") for g, _, _ in items]
    torch.cuda.synchronize()
    solver = vc.Solver(0, node_limit=args.node_limit, watchdog_ms=120_000)
    # warm up the server (first launch, buffers)
    t = solver.submit(items[0][0], items[0][1], items[0][2])
    solver.wait(t, items[0][0].n)
    while True:  # until the warm-up launch is closed
        try:
            solver.mvc(gg.path(3), want_cover=False)
            break
        except vc.VCError as e:
            if e.status != vc.VC_EAGAIN:
                raise
            time.sleep(0.002)
    served = [None] * len(items)
    pending = {}
    t0 = time.perf_counter()
    i = 0
    while i < len(items) or pending:
        now = time.perf_counter() - t0
        while i < len(items) and arrive[i] <= now:
            _, kind, k = items[i]
            pending[solver.submit(dev[i], kind, k)] = i
            i += 1
        for tk in list(pending):
            r = solver.poll(tk, items[pending[tk]][0].n)
            if r is not None:
                j = pending.pop(tk)
                served[j] = (r[0], time.perf_counter() - t0)
        time.sleep(0.0001)
    lat = np.array([served[j][1] - arrive[j] for j in range(len(items))]) * 1e3
    span = max(s[1] for s in served) - arrive[0]
    # plain solver, FIFO at the same arrivals
    while True:
        try:
            solver.mvc(gg.path(3), want_cover=False)
            break
        except vc.VCError as e:
            if e.status != vc.VC_EAGAIN:
                raise
            time.sleep(0.002)
    free_at, plat, agree = 0.0, [], 0
    for j, (g, kind, k) in enumerate(items):
        g = dev[j]
        t1 = time.perf_counter()
        if kind == vc.VC_MIN:
            ans = solver.mvc(g, want_cover=True).size
            same = ans == served[j][0]["size"]
        else:
            ans = solver.pvc(g, k, want_cover=True).yes
            same = bool(ans) == bool(served[j][0]["yes"])
        svc = time.perf_counter() - t1
        start = max(arrive[j], free_at)
        free_at = start + svc
        plat.append((free_at - arrive[j]) * 1e3)
        agree += int(same)
    plat = np.array(plat)
    solver.close()
    return {
        "metric": METRIC, "value": len(items) / span, "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": span * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
        "config": {"workload": f"served_stream_{len(items)}", "rate_per_s": args.rate,
                   "p50_ms": float(np.percentile(lat, 50)),
                   "p99_ms": float(np.percentile(lat, 99)),
                   "plain_fifo_p50_ms": float(np.percentile(plat, 50)),
                   "plain_fifo_p99_ms": float(np.percentile(plat, 99)),
                   "plain_solves_per_s": len(items) / (free_at - arrive[0]),
                   "same_answer_served_and_plain": f"{agree}/{len(items)}"},
    }


ABLATIONS = [("proposed", 0), ("no_components", 1), ("no_reduce_induce", 32),
             ("no_compaction", 64), ("no_load_balance", 2), ("no_small_solver", 16),
             ("crown_forced", 128), ("eager_induce", 2048), ("no_root_cache", 4096)]


def bench_ablation(args, torch, gg, vc):
    """Each optimization switched off in turn (Table II's columns plus this
    design's own switches) on the blocks-and-hubs graph and on 20 G(60, 0.1)
    graphs: time per solve (best of --steps) and search-tree nodes.  A run
    that reaches --node-limit tree nodes is reported as such (the paper's
    '>6 hrs')."""
    import numpy as np
    workloads = [("blocks_hubs_n1928", [vc.DeviceGraph.from_graph(gg.config2_blocks_hubs(),
                                                                  "cuda:0")]),
                 ("gnp60_x20", [vc.DeviceGraph.from_graph(gg.config1_gnp60(s), "cuda:0")
                                for s in range(1, 21)])]
    torch.cuda.synchronize()
    table, ref = {}, {}
    for wname, graphs in workloads:
        for aname, flags in ABLATIONS:
            solver = vc.Solver(0, flags=flags, node_limit=args.node_limit, watchdog_ms=120_000)
            best, nodes, sizes, hit = float("inf"), 0, [], False
            for rep in range(args.warmup + args.steps):
                t0 = time.perf_counter()
                nodes_rep, sizes = 0, []
                for g in graphs:
                    try:
                        sizes.append(solver.mvc(g, want_cover=False).size)
                    except vc.VCError as e:
                        if e.status != vc.VC_ETIMEDOUT:
                            raise
                        hit = True
                        sizes.append(None)
                    solver_stats_last = solver.stats()
                    nodes_rep += solver_stats_last["tree_nodes"]
                el = (time.perf_counter() - t0) * 1e3
                if hit:  # time and nodes up to the limit, once
                    best, nodes = el, nodes_rep
                    break
                if rep >= args.warmup and el < best:
                    best, nodes = el, nodes_rep
            solver.close()
            if aname == "proposed":
                ref[wname] = sizes
            elif not hit and sizes != ref[wname]:
                raise RuntimeError(f"{aname} changed an answer on {wname}")
            table.setdefault(wname, {})[aname] = {
                "ms": round(best, 3), "tree_nodes": nodes,
                "node_limit_reached": hit}
            if aname == "proposed":
                # Table III/IV-style counters of the last solve
                st = solver_stats_last
                table[wname][aname].update({
                    "components_per_branch_hist": st["comp_hist"],
                    "component_branches": st["component_branches"],
                    "n_kernel": st["n_kernel"], "max_degree_kernel": st["max_degree_kernel"],
                    "deg_bytes": st["deg_bytes"], "workers": st["workers"]})
            print(f"ablation {wname} {aname}: {best:.2f} ms, {nodes} nodes"
                  + (" (node limit)" if hit else ""), file=sys.stderr, flush=True)
    p = table["blocks_hubs_n1928"]["proposed"]
    return {
        "metric": METRIC, "value": p["tree_nodes"] / p["ms"] * 1e3, "unit": "search-nodes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": p["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "ablation_blocks_hubs_n1928_and_gnp60_x20",
                   "node_limit": args.node_limit, "ablation": table},
    }


def bench_pvc_powerlaw(args, torch, gg, vc):
    """PVC on the planted power-law graph (n = 10^6, m = 5*10^6, gamma 2.1,
    |S| = 60,000; CSR uint32 resident in HBM): one step is the two queries
    k = MVC - 1 (no) and k = MVC (yes, with a cover), MVC taken from vc_min
    on the same graph; each call runs to solution (validation, greedy bound,
    root reduction, induce, search if anything is left, cover)."""
    import numpy as np
    g = gg.config3_chung_lu()
    dg = vc.DeviceGraph.from_graph(g, "cuda:0")
    torch.cuda.synchronize()
    solver = vc.Solver(0, watchdog_ms=120_000)
    m = solver.mvc(dg).size
    for _ in range(args.warmup):
        solver.pvc(dg, m - 1)
        solver.pvc(dg, m)
    torch.cuda.synchronize()
    t_no, t_yes, st = [], [], None
    for _ in range(args.steps):
        t0 = time.perf_counter()
        no = solver.pvc(dg, m - 1)
        t1 = time.perf_counter()
        yes = solver.pvc(dg, m)
        t2 = time.perf_counter()
        assert not no.yes and yes.yes and yes.cover.size <= m
        t_no.append(t1 - t0)
        t_yes.append(t2 - t1)
        st = yes.stats
    t0 = time.perf_counter()
    r = solver.mvc(dg)
    t_mvc = time.perf_counter() - t0
    solver.close()
    el = sum(t_no) + sum(t_yes)
    out = {
        "metric": METRIC, "value": 2 * args.steps / el, "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "pvc_chung_lu_n1e6_m5e6", "n": g.n, "m": g.m, "mvc": m,
                   "ms_k_mvc_minus_1": float(np.median(t_no)) * 1e3,
                   "ms_k_mvc": float(np.median(t_yes)) * 1e3, "ms_mvc": t_mvc * 1e3,
                   "greedy_size": st["greedy_size"], "forced_root": st["forced_root"],
                   "n_kernel": st["n_kernel"], "root_rounds": st["root_rounds"],
                   "ms_root_device": st["ms_root"]},
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        o1 = oracle.pvc(g, m - 1)
        o2 = oracle.pvc(g, m)
        dt = time.perf_counter() - t0
        assert not o1["yes"] and o2["yes"]
        out["cpu_baseline"] = {"value": 2 / dt, "unit": "queries/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the same two queries ({dt:.2f} s)"}
    return out


def bench_enum(args, torch, gg, vc):
    """Enumeration of the minimal vertex covers of size <= MVC + 1 on 20
    G(60, 0.1) graphs (vc_param_enum; k from vc_min on the same graph), with
    the oracle's enumeration timed beside it on the same graphs."""
    graphs = [gg.config1_gnp60(s) for s in range(1, 21)]
    dev = [vc.DeviceGraph.from_graph(g, "cuda:0") for g in graphs]
    torch.cuda.synchronize()
    solver = vc.Solver(0, watchdog_ms=120_000)
    ks = [solver.mvc(d, want_cover=False).size + 1 for d in dev]
    for _ in range(args.warmup):
        for d, k in zip(dev, ks):
            solver.enum_minimal(d, k, 4096)
    torch.cuda.synchronize()
    covers = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        covers = 0
        for d, k in zip(dev, ks):
            covers += solver.enum_minimal(d, k, 4096)[0]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    solver.close()
    out = {
        "metric": METRIC, "value": len(graphs) * args.steps / el, "unit": "graphs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "enum_minimal_gnp60_x20_k_mvc_plus_1",
                   "minimal_covers_per_step": covers,
                   "covers_per_s": covers * args.steps / el},
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        done, ocov = 0, 0
        while done < len(graphs) and time.perf_counter() - t0 < args.cpu_seconds:
            ocov += oracle.enum_minimal(graphs[done], ks[done])["count"]
            done += 1
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": done / dt, "unit": "graphs/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{done} of the 20 graphs enumerated ({dt:.1f} s, "
                                         f"{ocov} minimal covers)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["blocks_hubs", "batch", "serve", "ablation", "enum",
                             "pvc_powerlaw"],
                    default="blocks_hubs")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--flags", type=int, default=0,
                    help="vc_opts.flags for the default workload (ablation switches)")
    ap.add_argument("--workers", type=int, default=0, help="vc_opts.workers (0: default)")
    ap.add_argument("--donate-min", type=int, default=0, help="vc_opts.donate_min (0: default)")
    ap.add_argument("--donate-slack", type=int, default=0, help="vc_opts.donate_slack")
    ap.add_argument("--small-max", type=int, default=0, help="vc_opts.small_max (0: default)")
    ap.add_argument("--no-legs", action="store_true",
                    help="default workload only: skip the batch and served legs")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed steps, copy this many MiB device to "
                         "device once: a kernel of known traffic that scales "
                         "the HBM byte counters of a profiler run")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--node-limit", type=int, default=200_000)
    ap.add_argument("--plain-count", type=int, default=256)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--serve-count", type=int, default=200)
    ap.add_argument("--rate", type=float, default=100.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the search shards across GPUs only by instance, see the design notes",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_18334_amd import graphgen as gg
    from paper_2512_18334_amd import vc

    if not os.path.exists(vc.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    fn = {"blocks_hubs": bench_blocks_hubs, "batch": bench_batch, "serve": bench_serve,
          "ablation": bench_ablation, "enum": bench_enum,
          "pvc_powerlaw": bench_pvc_powerlaw}
    out = fn[args.workload](args, torch, gg, vc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
