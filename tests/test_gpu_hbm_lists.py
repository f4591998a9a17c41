"""Induced subgraphs whose search lists do not fit LDS (Sec. IV-A: the
search falls back to global memory): the lists go to HBM and the answers
must still equal the oracle's.  The degree rules leave these graphs whole
(3-regular components: no degree-one or degree-two vertices), so the kernel
keeps every vertex."""
import numpy as np
import pytest

from paper_2512_18334_amd import graphgen as gg
from paper_2512_18334_amd import vc
from tests.helpers import assert_cover

pytestmark = pytest.mark.gpu


def cubic_union(count: int, size: int, seed: int):
    r = gg.rng(seed)
    parts = []
    for _ in range(count):
        u, v = gg.random_regular(size, 3, r)
        parts.append(gg.from_edges(size, u, v))
    return gg.relabel(gg.disjoint_union(parts, name=f"cubic{count}x{size}"), seed)


@pytest.fixture(scope="module")
def big_union(orc):
    g = cubic_union(250, 84, 41)          # 21,000 vertices, 31,500 edges
    return g, orc.mvc(g)["size"]


def test_kernel_beyond_lds_matches_oracle(libvc, big_union):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    g, want = big_union
    print(f"hbm lists: {g.name} n={g.n} mvc={want}", flush=True)
    with vc.Solver(0, flags=vc.VC_OPT_NO_CROWN | vc.VC_OPT_CHECK_REGISTRY,
                   node_limit=50_000_000, watchdog_ms=60_000) as s:
        r = s.mvc(g)
        assert r.size == want
        assert_cover(g, r.cover, size=want)
        st = r.stats
        assert st["n_kernel"] >= 20_000 and st["lists_in_hbm"] == 1, st
        assert st["reg_checked"] == 1 and st["reg_open"] == 0
        assert st["stale_reads"] == 0
        assert not s.pvc(g, want - 1).yes
        y = s.pvc(g, want)
        assert y.yes
        assert_cover(g, y.cover, at_most=want)


def test_kernel_beyond_lds_one_worker_and_device_input(libvc, big_union):
    g, want = big_union
    with vc.Solver(0, workers=8, flags=vc.VC_OPT_NO_CROWN, node_limit=50_000_000,
                   watchdog_ms=60_000) as s:
        r = s.mvc(vc.DeviceGraph.from_graph(g, "cuda:0"))
        assert r.size == want
        assert_cover(g, r.cover, size=want)
        assert r.stats["lists_in_hbm"] == 1
