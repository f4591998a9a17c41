"""CPU oracle for MVC / PVC (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The solver library never does: the
oracle and the GPU path share no code.  The C source ``vc_oracle.c`` states
what is computed and which passages of the paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile vc_oracle.c with gcc into liboracle.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra",
                           "-shared", "-fPIC", _SRC, "-o", tmp])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_mvc.restype = ctypes.c_int64
    lib.oracle_mvc.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint64,
                               u32p, u32p, u64p, u32p]
    lib.oracle_pvc.restype = ctypes.c_int
    lib.oracle_pvc.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint32,
                               ctypes.c_uint64, u32p, u32p, u64p, u32p]
    lib.oracle_greedy.restype = ctypes.c_int64
    lib.oracle_greedy.argtypes = [ctypes.c_uint32, u32p, u32p, u32p, u32p]
    lib.oracle_enum_minimal.restype = ctypes.c_int64
    lib.oracle_enum_minimal.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint32,
                                        ctypes.c_uint64, u32p, u32p, ctypes.c_uint64]
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


class OracleLimit(RuntimeError):
    """The node limit was reached before the search finished."""


def _prep(offsets, cols):
    off = np.ascontiguousarray(offsets, dtype=np.uint32)
    col = np.ascontiguousarray(cols, dtype=np.uint32)
    return off, col


def mvc(g, node_limit: int = 0):
    """Minimum vertex cover of g -> dict(size, cover, nodes, kernel_n, seconds)."""
    off, col = _prep(g.offsets, g.cols)
    n = int(g.n)
    cover = np.zeros(max(n, 1), np.uint32)
    clen = ctypes.c_uint32(0)
    nodes = ctypes.c_uint64(0)
    kn = ctypes.c_uint32(0)
    t0 = time.perf_counter()
    r = _load().oracle_mvc(n, _ptr(off), _ptr(col), node_limit, _ptr(cover),
                           ctypes.byref(clen), ctypes.byref(nodes),
                           ctypes.byref(kn))
    dt = time.perf_counter() - t0
    if r == -2:
        raise OracleLimit(f"node limit {node_limit} reached")
    if r < 0:
        raise MemoryError("oracle allocation failed")
    return {"size": int(r), "cover": cover[:clen.value].copy(),
            "nodes": int(nodes.value), "kernel_n": int(kn.value), "seconds": dt}


def pvc(g, k: int, node_limit: int = 0):
    """Is there a vertex cover of size <= k?  -> dict(yes, cover, nodes, ...)."""
    off, col = _prep(g.offsets, g.cols)
    n = int(g.n)
    cover = np.zeros(max(n, 1), np.uint32)
    clen = ctypes.c_uint32(0)
    nodes = ctypes.c_uint64(0)
    kn = ctypes.c_uint32(0)
    t0 = time.perf_counter()
    r = _load().oracle_pvc(n, _ptr(off), _ptr(col), int(k), node_limit,
                           _ptr(cover), ctypes.byref(clen), ctypes.byref(nodes),
                           ctypes.byref(kn))
    dt = time.perf_counter() - t0
    if r == -2:
        raise OracleLimit(f"node limit {node_limit} reached")
    if r < 0:
        raise MemoryError("oracle allocation failed")
    return {"yes": bool(r), "cover": cover[:clen.value].copy(),
            "nodes": int(nodes.value), "kernel_n": int(kn.value), "seconds": dt}


def greedy(g):
    """The max-degree greedy cover the oracle starts from."""
    off, col = _prep(g.offsets, g.cols)
    n = int(g.n)
    cover = np.zeros(max(n, 1), np.uint32)
    clen = ctypes.c_uint32(0)
    r = _load().oracle_greedy(n, _ptr(off), _ptr(col), _ptr(cover),
                              ctypes.byref(clen))
    return {"size": int(r), "cover": cover[:clen.value].copy()}


def enum_minimal(g, k: int, cap: int = 1_000_000, node_limit: int = 0):
    """All minimal vertex covers of g with at most k vertices, as a set of
    frozensets of vertex ids (exactly the first `cap` found are returned;
    "count" is the total)."""
    off, col = _prep(g.offsets, g.cols)
    n = int(g.n)
    kk = max(int(k), 1)
    ids = np.zeros(max(cap * kk, 1), np.uint32)
    lens = np.zeros(max(cap, 1), np.uint32)
    r = _load().oracle_enum_minimal(n, _ptr(off), _ptr(col), int(k), cap, _ptr(ids),
                                    _ptr(lens), node_limit)
    if r == -2:
        raise OracleLimit(f"node limit {node_limit} reached")
    if r < 0:
        raise MemoryError("oracle allocation failed")
    got = min(int(r), cap)
    covers = {frozenset(ids[c * kk:c * kk + int(lens[c])].tolist()) for c in range(got)}
    return {"count": int(r), "covers": covers}
