"""Context plumbing through the C ABI: a caller-owned arena (every device
buffer carved from a PyTorch uint8 tensor), PyTorch streams, and device
inputs written by PyTorch asynchronously just before the call.  Answers
must equal the oracle's, with valid covers."""
import numpy as np
import pytest

from paper_2512_18334_amd import graphgen as gg
from paper_2512_18334_amd import vc
from tests.helpers import assert_cover

pytestmark = pytest.mark.gpu


def _graphs():
    return [gg.config1_gnp60(5), gg.config2_blocks_hubs(seed=7, nblocks=4, bsize=48,
                                                         nhubs=2, per_block=10),
            gg.relabel(gg.disjoint_union([gg.petersen(), gg.cycle(11), gg.grid(4, 5)]), 3)]


def test_arena_backed_context(libvc, orc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    arena = torch.empty(512 << 20, dtype=torch.uint8, device="cuda:0")
    with vc.Solver(0, arena=arena, node_limit=50_000_000, watchdog_ms=60_000) as s:
        for g in _graphs():
            want = orc.mvc(g)["size"]
            print(f"arena: {g.name} n={g.n}", flush=True)
            r = s.mvc(g)
            assert r.size == want
            assert_cover(g, r.cover, size=want)
            assert s.pvc(g, want).yes and not s.pvc(g, want - 1).yes
        rb = s.mvc_batch(_graphs())
        for g, size, cov in zip(_graphs(), rb.sizes, rb.covers):
            want = orc.mvc(g)["size"]
            assert int(size) == want
            assert_cover(g, cov, size=want)
    # an arena too small for the buffers: out of memory, not a fault
    tiny = torch.empty(1 << 16, dtype=torch.uint8, device="cuda:0")
    with vc.Solver(0, arena=tiny, watchdog_ms=60_000) as s:
        with pytest.raises(vc.VCError) as e:
            s.mvc(gg.config2_blocks_hubs())
        assert e.value.status == vc.VC_ENOMEM


def test_explicit_torch_stream_and_async_inputs(libvc, orc):
    import torch
    g = gg.config2_blocks_hubs(seed=11, nblocks=6, bsize=48, nhubs=3, per_block=8)
    want = orc.mvc(g)["size"]
    st = torch.cuda.Stream(device=0)
    off_h = torch.from_numpy(np.asarray(g.offsets, np.uint32).view(np.int32)).pin_memory()
    col_h = torch.from_numpy(np.asarray(g.cols, np.uint32).view(np.int32)).pin_memory()
    with torch.cuda.stream(st):
        with vc.Solver(0, stream=st, node_limit=50_000_000, watchdog_ms=60_000) as s:
            for _ in range(3):
                # written on the solver's stream right before the call, with
                # asynchronous copies: the call is ordered after them
                off = torch.empty_like(off_h, device="cuda:0")
                col = torch.empty_like(col_h, device="cuda:0")
                off.copy_(off_h, non_blocking=True)
                col.copy_(col_h, non_blocking=True)
                dg = vc.DeviceGraph(g.n, g.nnz, off, col, 4)
                r = s.mvc(dg)
                assert r.size == want
                assert_cover(g, r.cover, size=want)


def test_default_stream_inputs_with_own_stream(libvc, orc):
    """The default Solver (PyTorch's default stream, handle 0): the library
    runs on its own stream, which waits for the default stream before it
    reads device inputs that a torch kernel has just written there."""
    import torch
    g = gg.config1_gnp60(9)
    want = orc.mvc(g)["size"]
    with vc.Solver(0, node_limit=50_000_000, watchdog_ms=60_000) as s:
        for _ in range(3):
            base = torch.from_numpy(np.asarray(g.cols, np.int32)).to("cuda:0")
            # a chain of torch kernels on the default stream ends with the
            # true columns (x + 7 - 7), so a read before they finish is wrong
            col = ((base + 7) * 3) // 3 - 7
            col = col.to(torch.int32)
            off = torch.from_numpy(np.asarray(g.offsets, np.uint32).view(np.int32)).to(
                "cuda:0", non_blocking=True)
            r = s.mvc(vc.DeviceGraph(g.n, g.nnz, off, col, 4))
            assert r.size == want
            assert_cover(g, r.cover, size=want)
