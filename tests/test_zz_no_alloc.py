"""vc_min_static (the entry point that allocates no device memory) against
vc_min, through the C ABI: two calls in a row, the second on a smaller
graph, each equal to vc_min's answer and to the oracle's, with valid
covers; then the size limits."""
import ctypes

import numpy as np
import pytest

from paper_2512_18334_amd import graphgen as gg
from paper_2512_18334_amd import vc
from tests.helpers import assert_cover

pytestmark = pytest.mark.gpu


def _static(lib, h, g):
    c, keep = vc.host_csr(g)
    size = ctypes.c_uint32(0)
    clen = ctypes.c_uint32(0)
    cov = np.zeros(max(g.n, 1), np.uint32)
    st = lib.vc_min_static(h, ctypes.byref(c), ctypes.byref(size),
                           cov.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                           ctypes.byref(clen))
    return st, int(size.value), cov[:clen.value].copy()


def test_static_matches_vc_min_on_two_calls(libvc, orc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    big = gg.config2_blocks_hubs()                      # n = 1928, MVC 1077
    small = gg.config1_gnp60(3)                         # n = 60
    with vc.Solver(0, node_limit=50_000_000, watchdog_ms=60_000) as s:
        for g in (big, small):
            print(f"static: {g.name} n={g.n}", flush=True)
            want = orc.mvc(g)["size"]
            ref = s.mvc(g)
            st, size, cover = _static(libvc, s._h, g)
            assert st == vc.VC_OK, vc.status_str(st)
            assert size == ref.size == want, (g.name, size, ref.size, want)
            assert_cover(g, cover, size=want)
            # the device-resident form of the same graph
            r = s.mvc_static(vc.DeviceGraph.from_graph(g, "cuda:0"))
            assert r.size == want
            assert_cover(g, r.cover, size=want)


def test_static_limits_and_edge_cases(libvc, orc):
    with vc.Solver(0, node_limit=50_000_000, watchdog_ms=60_000) as s:
        st, size, cover = _static(libvc, s._h, gg.from_edges(0, [], []))
        assert st == vc.VC_OK and size == 0 and cover.size == 0
        g = gg.relabel(gg.disjoint_union([gg.cycle(9), gg.complete(6), gg.petersen()]), 4)
        st, size, cover = _static(libvc, s._h, g)
        assert st == vc.VC_OK and size == orc.mvc(g)["size"]
        assert_cover(g, cover, size=size)
        # more vertices than the scratch is sized for: rejected before any work
        off = np.zeros((1 << 20) + 2, np.uint32)
        c = vc.vc_csr((1 << 20) + 1, 0, off.ctypes.data, None, 4, 0)
        zero = ctypes.c_uint32(0)
        assert libvc.vc_min_static(s._h, ctypes.byref(c), ctypes.byref(zero), None,
                                   ctypes.byref(zero)) == vc.VC_ERANGE
