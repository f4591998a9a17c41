"""Autotuner for batched solves (vc_min_batch).

Sweeps the three knobs that shape a batched launch and keeps the fastest:
  workers       waves per CU x CUs (a worker is one 64-lane wave, the GPU's
                block size here),
  worklist_cap  capacity of the shared worklist (its depth),
  donate_min    the live-vertex size below which a node is never handed to
                another worker (the split threshold of the work sharing).
Every configuration must give identical sizes on every instance that finished
below the node limit, or the sweep stops with an error.  Results are cached
in a JSON file keyed by the batch's shape, so a later run reuses them.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

import numpy as np

from . import vc

DEFAULT_GRID = {
    "waves_per_cu": (1, 2, 3),
    "worklist_cap": (1024, 4096, 16384),
    "donate_min": (16, 48, 96),
}


def batch_key(b: "vc.Batch", node_limit: int) -> str:
    h = hashlib.sha256()
    for a in (b.n, b.nnz, b.offs_base, b.cols_base):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(str((b.col_bytes, node_limit)).encode())
    return h.hexdigest()[:24]


def _cus() -> int:
    import torch
    return int(torch.cuda.get_device_properties(0).multi_processor_count)


def tune_batch(batch, node_limit: int = 100_000, grid: dict | None = None,
               cache: str | None = None, reps: int = 1, log=print) -> dict:
    """Return {"opts": best Solver keyword arguments, "ms": its time,
    "table": [(opts, ms), ...]} for vc_min_batch over `batch` (a vc.Batch or
    a list of graphs)."""
    b = batch if isinstance(batch, vc.Batch) else vc.Batch.from_graphs(batch)
    key = batch_key(b, node_limit)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            saved = json.load(f)
        if key in saved:
            return saved[key]
    grid = grid or DEFAULT_GRID
    cus = _cus()
    table, ref = [], None
    for wpc, cap, dmin in itertools.product(grid["waves_per_cu"], grid["worklist_cap"],
                                            grid["donate_min"]):
        opts = {"workers": wpc * cus, "worklist_cap": cap, "donate_min": dmin}
        with vc.Solver(0, node_limit=node_limit, watchdog_ms=120_000, **opts) as s:
            s.mvc_batch(b, want_cover=False)  # captures the launch
            best = float("inf")
            for _ in range(reps):
                t0 = time.perf_counter()
                r = s.mvc_batch(b, want_cover=False)
                best = min(best, (time.perf_counter() - t0) * 1e3)
        exact = r.status == vc.VC_OK
        if ref is None:
            ref = (r.sizes.copy(), exact.copy())
        else:
            both = exact & ref[1]
            if not np.array_equal(r.sizes[both], ref[0][both]):
                raise RuntimeError(f"configuration {opts} changed an exact size")
        table.append((opts, best))
        log(f"autotune {opts}: {best:.1f} ms")
    opts, ms = min(table, key=lambda t: t[1])
    out = {"opts": opts, "ms": ms, "table": table}
    if cache:
        saved = {}
        if os.path.exists(cache):
            with open(cache) as f:
                saved = json.load(f)
        saved[key] = out
        with open(cache, "w") as f:
            json.dump(saved, f, indent=1)
    return out
