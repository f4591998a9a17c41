"""Exact minimum / parameterized vertex cover on AMD Instinct MI355X.

The solver is libvc.so (HIP, gfx950) behind the C ABI in include/vc.h; the
binding is paper_2512_18334_amd.vc.  Seeded workload generators live in
paper_2512_18334_amd.graphgen.
"""
__all__ = ["graphgen", "vc", "build"]
