"""Python binding of libvc (include/vc.h): argument marshalling only.

Every step of a solve runs in the HIP kernels of libvc.so; this module only
builds the C structs, passes pointers and turns status codes into
exceptions.  PyTorch is used for device memory (graphs made resident in HBM)
and for streams.  There is no fallback: if libvc.so is missing or cannot be
loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvc.so")

VC_OK, VC_EINVAL, VC_ENOMEM, VC_EDEVICE = 0, -1, -2, -3
VC_EAGAIN, VC_ETIMEDOUT, VC_ECANCELED, VC_ERANGE = -4, -5, -6, -7
VC_CSR_DEVICE = 1
VC_OPT_NO_COMPONENTS = 1
VC_OPT_NO_LOAD_BALANCE = 2
VC_OPT_VALIDATE_SKIP = 4
VC_OPT_NO_GRAPH = 8
VC_OPT_NO_SMALL = 16
VC_OPT_NO_INDUCE = 32
VC_OPT_NO_COMPACT = 64
VC_OPT_CROWN = 128
VC_OPT_NO_CROWN = 256
VC_OPT_STRONG_ORDER = 512
VC_OPT_CHECK_REGISTRY = 1024
VC_OPT_EAGER_INDUCE = 2048
VC_OPT_NO_ROOT_CACHE = 4096
VC_OPT_POISON = 8192
VC_MIN, VC_PARAM = 0, 1

CYCLE_NAMES = ["fetch", "reduce", "components", "branch", "complete", "idle"]
COMP_HIST_BUCKETS = ["2", "3-4", "5-8", "9-16", "17-32", "33-64", "65-128", ">128"]

EXPORTS = ["vc_ctx_create", "vc_ctx_destroy", "vc_validate", "vc_min",
           "vc_param", "vc_min_batch", "vc_param_batch", "vc_submit", "vc_poll",
           "vc_cancel", "vc_last_stats", "vc_status_str", "vc_param_enum",
           "vc_min_static"]


class vc_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("nnz", ctypes.c_uint64),
                ("offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p),
                ("col_bytes", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class vc_batch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint32), ("offs_base", ctypes.c_void_p),
                ("cols_base", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("nnz", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("cols", ctypes.c_void_p), ("col_bytes", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class vc_opts(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_uint32), ("donate_slack", ctypes.c_uint32),
                ("worklist_cap", ctypes.c_uint32), ("registry_cap", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64), ("node_limit", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("watchdog_ms", ctypes.c_uint32),
                ("donate_min", ctypes.c_uint32), ("gcache_words", ctypes.c_uint32),
                ("serve_n_max", ctypes.c_uint32), ("serve_slots", ctypes.c_uint32),
                ("small_max", ctypes.c_uint32)]


class vc_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("size", ctypes.c_uint32), ("yes", ctypes.c_int32),
                ("cover_len", ctypes.c_uint32), ("n", ctypes.c_uint32),
                ("tree_nodes", ctypes.c_uint64), ("ms_queued", ctypes.c_double),
                ("ms_latency", ctypes.c_double)]


class vc_stats(ctypes.Structure):
    _fields_ = [("tree_nodes", ctypes.c_uint64),
                ("component_branches", ctypes.c_uint64),
                ("components", ctypes.c_uint64), ("donations", ctypes.c_uint64),
                ("pushes", ctypes.c_uint64), ("local_views", ctypes.c_uint64),
                ("bytes_nodes", ctypes.c_uint64), ("bytes_registry", ctypes.c_uint64),
                ("cycles", ctypes.c_uint64 * 6),
                ("n_input", ctypes.c_uint32), ("n_kernel", ctypes.c_uint32),
                ("nnz_kernel", ctypes.c_uint64), ("forced_root", ctypes.c_uint32),
                ("greedy_size", ctypes.c_uint32),
                ("max_degree_kernel", ctypes.c_uint32),
                ("deg_bytes", ctypes.c_uint32), ("workers", ctypes.c_uint32),
                ("root_rounds", ctypes.c_uint32), ("slot_bytes", ctypes.c_uint32),
                ("bitmap_bytes", ctypes.c_uint32), ("ms_root", ctypes.c_double),
                ("ms_induce", ctypes.c_double), ("ms_search", ctypes.c_double),
                ("ms_total", ctypes.c_double),
                ("crown_cover", ctypes.c_uint32), ("crown_removed", ctypes.c_uint32),
                ("crown_rounds", ctypes.c_uint32),
                ("stale_reads", ctypes.c_uint64), ("reg_entries", ctypes.c_uint32),
                ("reg_checked", ctypes.c_uint32), ("reg_open", ctypes.c_uint32),
                ("reg_parents", ctypes.c_uint32), ("reg_depth", ctypes.c_uint32),
                ("lists_in_hbm", ctypes.c_uint32), ("bytes_rows", ctypes.c_uint64),
                ("comp_hist", ctypes.c_uint32 * 8), ("bytes_views", ctypes.c_uint64)]


class VCError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"libvc {what}: {status_str(status)} ({status})")


_lib = None


def load():
    """Load libvc.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first "
                          "(python -m paper_2512_18334_amd.build)")
    # libvc and PyTorch must share one HIP runtime: importing torch first
    # loads its libamdhip64, which libvc then binds to (same soname)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    p = ctypes.c_void_p
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.vc_ctx_create.restype = ctypes.c_int
    lib.vc_ctx_create.argtypes = [ctypes.c_int, p, p, ctypes.c_uint64,
                                  ctypes.POINTER(vc_opts), ctypes.POINTER(p)]
    lib.vc_ctx_destroy.restype = ctypes.c_int
    lib.vc_ctx_destroy.argtypes = [p]
    lib.vc_validate.restype = ctypes.c_int
    lib.vc_validate.argtypes = [p, ctypes.POINTER(vc_csr)]
    lib.vc_min.restype = ctypes.c_int
    lib.vc_min.argtypes = [p, ctypes.POINTER(vc_csr), u32p, u32p, u32p]
    lib.vc_min_static.restype = ctypes.c_int
    lib.vc_min_static.argtypes = [p, ctypes.POINTER(vc_csr), u32p, u32p, u32p]
    lib.vc_param.restype = ctypes.c_int
    lib.vc_param.argtypes = [p, ctypes.POINTER(vc_csr), ctypes.c_uint32,
                             ctypes.POINTER(ctypes.c_int), u32p, u32p]
    i32p = ctypes.POINTER(ctypes.c_int32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.vc_min_batch.restype = ctypes.c_int
    lib.vc_min_batch.argtypes = [p, ctypes.POINTER(vc_batch), u32p, i32p, u32p, u64p]
    lib.vc_param_batch.restype = ctypes.c_int
    lib.vc_param_batch.argtypes = [p, ctypes.POINTER(vc_batch), u32p,
                                   ctypes.POINTER(ctypes.c_int), i32p, u32p, u64p]
    lib.vc_submit.restype = ctypes.c_int
    lib.vc_submit.argtypes = [p, ctypes.POINTER(vc_csr), ctypes.c_int, ctypes.c_uint32,
                              u64p]
    lib.vc_poll.restype = ctypes.c_int
    lib.vc_poll.argtypes = [p, ctypes.c_uint64, ctypes.POINTER(vc_result), u32p]
    lib.vc_cancel.restype = ctypes.c_int
    lib.vc_cancel.argtypes = [p, ctypes.c_uint64]
    lib.vc_last_stats.restype = ctypes.c_int
    lib.vc_last_stats.argtypes = [p, ctypes.POINTER(vc_stats)]
    lib.vc_param_enum.restype = ctypes.c_int
    lib.vc_param_enum.argtypes = [p, ctypes.POINTER(vc_csr), ctypes.c_uint32, ctypes.c_uint64,
                                  u32p, u32p, u64p]
    lib.vc_status_str.restype = ctypes.c_char_p
    lib.vc_status_str.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def status_str(s: int) -> str:
    return load().vc_status_str(int(s)).decode()


def _check(st: int, what: str):
    if st != VC_OK:
        raise VCError(st, what)


@dataclass
class DeviceGraph:
    """A CSR graph resident in device memory (torch tensors keep it alive)."""
    n: int
    nnz: int
    offsets: object       # torch.int32 tensor, bytes of uint32 offsets
    cols: object          # torch.int16 / torch.int32 tensor
    col_bytes: int

    @classmethod
    def from_graph(cls, g, device="cuda"):
        import torch
        off = torch.from_numpy(np.ascontiguousarray(g.offsets, np.uint32).view(np.int32))
        cdt = np.int16 if g.col_bytes == 2 else np.int32
        col = torch.from_numpy(np.ascontiguousarray(g.cols).view(cdt))
        return cls(g.n, g.nnz, off.to(device), col.to(device), g.col_bytes)

    def csr(self) -> vc_csr:
        return vc_csr(self.n, self.nnz, self.offsets.data_ptr(),
                      self.cols.data_ptr() if self.nnz else None,
                      self.col_bytes, VC_CSR_DEVICE)


def host_csr(g):
    """vc_csr for a host graph plus the arrays that must stay alive."""
    off = np.ascontiguousarray(g.offsets, dtype=np.uint32)
    cols = np.ascontiguousarray(g.cols)
    if cols.dtype not in (np.uint16, np.uint32):
        cols = cols.astype(np.uint32)
    c = vc_csr(int(g.n), int(off[-1]) if off.size else 0,
               off.ctypes.data, cols.ctypes.data if cols.size else None,
               int(cols.dtype.itemsize), 0)
    return c, (off, cols)


@dataclass
class Batch:
    """Graphs packed into one offsets and one cols buffer (vc_batch).  The
    descriptor arrays stay on the host; offsets and cols are numpy arrays,
    or torch tensors on the device after to_device()."""
    n: np.ndarray          # uint32 [count]
    nnz: np.ndarray        # uint64 [count]
    offs_base: np.ndarray  # uint64 [count]
    cols_base: np.ndarray  # uint64 [count]
    offsets: object        # uint32 [sum(n+1)]
    cols: object           # uint16 or uint32 [sum(nnz)]
    col_bytes: int
    device: bool = False

    @classmethod
    def from_graphs(cls, graphs, col_bytes: int = 0):
        graphs = list(graphs)
        cb = col_bytes or (2 if all(g.n <= 65536 for g in graphs) else 4)
        ns = np.array([g.n for g in graphs], np.uint32)
        nnz = np.array([g.nnz for g in graphs], np.uint64)
        ob = np.zeros(len(graphs), np.uint64)
        cbase = np.zeros(len(graphs), np.uint64)
        if len(graphs) > 1:
            ob[1:] = np.cumsum(ns[:-1].astype(np.uint64) + 1)
            cbase[1:] = np.cumsum(nnz[:-1])
        cdt = np.uint16 if cb == 2 else np.uint32
        offsets = (np.concatenate([np.asarray(g.offsets, np.uint32) for g in graphs])
                   if graphs else np.zeros(1, np.uint32))
        cols = (np.concatenate([np.asarray(g.cols).astype(cdt) for g in graphs])
                if graphs else np.zeros(1, cdt))
        return cls(ns, nnz, ob, cbase, offsets, cols, cb)

    @property
    def count(self) -> int:
        return int(self.n.size)

    def to_device(self, device="cuda"):
        import torch
        off = torch.from_numpy(self.offsets.view(np.int32)).to(device)
        cdt = np.int16 if self.col_bytes == 2 else np.int32
        col = torch.from_numpy(np.ascontiguousarray(self.cols).view(cdt)).to(device)
        return Batch(self.n, self.nnz, self.offs_base, self.cols_base, off, col,
                     self.col_bytes, True)

    def c_struct(self) -> vc_batch:
        if self.device:
            op, cp = self.offsets.data_ptr(), self.cols.data_ptr()
        else:
            op, cp = self.offsets.ctypes.data, self.cols.ctypes.data
        return vc_batch(self.count, self.offs_base.ctypes.data, self.cols_base.ctypes.data,
                        self.n.ctypes.data, self.nnz.ctypes.data, op, cp,
                        self.col_bytes, VC_CSR_DEVICE if self.device else 0)


@dataclass
class BatchResult:
    sizes: np.ndarray | None   # MVC per instance (None for PVC)
    yes: np.ndarray | None     # PVC answers (None for MVC)
    status: np.ndarray         # VC_OK or VC_ETIMEDOUT per instance
    covers: list               # ascending local ids per instance
    stats: dict


@dataclass
class Result:
    size: int | None      # MVC size (None for PVC)
    yes: bool | None      # PVC answer (None for MVC)
    cover: np.ndarray     # cover vertex ids, ascending
    stats: dict


class Solver:
    """One libvc context on a HIP device.

    stream: a torch.cuda.Stream or a raw hipStream_t handle; by default
    PyTorch's current stream on the device (its handle is 0 for the default
    stream, and the library then orders its own stream after the default
    one).  arena: optional uint8 device tensor all device buffers are carved
    from (the library then allocates no device memory); it is kept alive by
    the Solver."""

    def __init__(self, device: int = 0, stream=None, workers: int = 0,
                 donate_slack: int = 0, worklist_cap: int = 0,
                 registry_cap: int = 0, hbm_budget: int = 0,
                 node_limit: int = 0, flags: int = 0, watchdog_ms: int = 0,
                 donate_min: int = 0, gcache_words: int = 0, serve_n_max: int = 0,
                 serve_slots: int = 0, small_max: int = 0, arena=None):
        lib = load()
        self._opts = vc_opts(workers, donate_slack, worklist_cap, registry_cap,
                             hbm_budget, node_limit, flags, watchdog_ms,
                             donate_min, gcache_words, serve_n_max, serve_slots,
                             small_max)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        handle = getattr(stream, "cuda_stream", stream)
        self._arena = arena
        a_ptr, a_bytes = (None, 0)
        if arena is not None:
            a_ptr, a_bytes = arena.data_ptr(), arena.numel() * arena.element_size()
        h = ctypes.c_void_p()
        st = lib.vc_ctx_create(int(device), handle or None, a_ptr, int(a_bytes),
                               ctypes.byref(self._opts), ctypes.byref(h))
        _check(st, "vc_ctx_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().vc_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def _csr(g):
        if isinstance(g, DeviceGraph):
            return g.csr(), (g,)
        return host_csr(g)

    def validate(self, g) -> int:
        c, keep = self._csr(g)
        return load().vc_validate(self._h, ctypes.byref(c))


    def stats(self) -> dict:
        s = vc_stats()
        _check(load().vc_last_stats(self._h, ctypes.byref(s)), "vc_last_stats")
        out = {f: getattr(s, f) for f, _ in vc_stats._fields_}
        out["cycles"] = dict(zip(CYCLE_NAMES, list(s.cycles)))
        out["comp_hist"] = dict(zip(COMP_HIST_BUCKETS, list(s.comp_hist)))
        return out

    def mvc(self, g, want_cover: bool = True) -> Result:
        c, keep = self._csr(g)
        n = int(c.n)
        size = ctypes.c_uint32(0)
        clen = ctypes.c_uint32(0)
        cov = np.zeros(max(n, 1), np.uint32)
        cp = cov.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if want_cover else None
        st = load().vc_min(self._h, ctypes.byref(c), ctypes.byref(size), cp,
                           ctypes.byref(clen))
        _check(st, "vc_min")
        return Result(int(size.value), None, cov[:clen.value].copy(), self.stats())

    def mvc_static(self, g, want_cover: bool = True) -> Result:
        """vc_min_static: vc_min on the library's static scratch (no device
        memory is allocated by the call)."""
        c, keep = self._csr(g)
        n = int(c.n)
        size = ctypes.c_uint32(0)
        clen = ctypes.c_uint32(0)
        cov = np.zeros(max(n, 1), np.uint32)
        cp = cov.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if want_cover else None
        st = load().vc_min_static(self._h, ctypes.byref(c), ctypes.byref(size), cp,
                                  ctypes.byref(clen))
        _check(st, "vc_min_static")
        return Result(int(size.value), None, cov[:clen.value].copy(), self.stats())

    def pvc(self, g, k: int, want_cover: bool = True) -> Result:
        c, keep = self._csr(g)
        n = int(c.n)
        yes = ctypes.c_int(0)
        clen = ctypes.c_uint32(0)
        cov = np.zeros(max(n, 1), np.uint32)
        cp = cov.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if want_cover else None
        st = load().vc_param(self._h, ctypes.byref(c), int(k), ctypes.byref(yes),
                             cp, ctypes.byref(clen))
        _check(st, "vc_param")
        return Result(None, bool(yes.value), cov[:clen.value].copy(), self.stats())

    def enum_minimal(self, g, k: int, max_covers: int = 100_000):
        """vc_param_enum: (count, list of the first min(count, max_covers)
        minimal covers of size <= k, each an ascending id array)."""
        c, keep = self._csr(g)
        kk = int(k)
        covers = np.zeros(max(max_covers * kk, 1), np.uint32)
        sizes = np.zeros(max(max_covers, 1), np.uint32)
        cnt = ctypes.c_uint64(0)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        st = load().vc_param_enum(self._h, ctypes.byref(c), kk, int(max_covers),
                                  covers.ctypes.data_as(u32p), sizes.ctypes.data_as(u32p),
                                  ctypes.byref(cnt))
        _check(st, "vc_param_enum")
        got = min(int(cnt.value), int(max_covers))
        out = [covers[t * kk:t * kk + int(sizes[t])].copy() for t in range(got)]
        return int(cnt.value), out


    def submit(self, g, kind: int = VC_MIN, k: int = 0) -> int:
        """vc_submit: returns the ticket (the graph is copied)."""
        c, keep = self._csr(g)
        t = ctypes.c_uint64(0)
        _check(load().vc_submit(self._h, ctypes.byref(c), int(kind), int(k),
                                ctypes.byref(t)), "vc_submit")
        return int(t.value)

    def poll(self, ticket: int, n: int):
        """vc_poll: None while pending, else (vc_result fields dict, cover).
        Raises VCError for a cancelled or unknown ticket."""
        r = vc_result()
        cov = np.zeros(max(int(n), 1), np.uint32)
        st = load().vc_poll(self._h, int(ticket), ctypes.byref(r),
                            cov.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        if st == VC_EAGAIN:
            return None
        _check(st, "vc_poll")
        out = {f: getattr(r, f) for f, _ in vc_result._fields_}
        return out, cov[:r.cover_len].copy()

    def cancel(self, ticket: int):
        _check(load().vc_cancel(self._h, int(ticket)), "vc_cancel")

    def wait(self, ticket: int, n: int, timeout_s: float = 120.0):
        """Poll until the request is answered (or raise after timeout_s)."""
        import time
        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket, n)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"request {ticket} still pending")
            time.sleep(0.0002)

    def mvc_batch(self, batch, want_cover: bool = True) -> BatchResult:
        """vc_min_batch over a Batch (or a list of graphs, packed here)."""
        b = _as_batch(batch)
        c = b.c_struct()
        cnt = b.count
        sizes = np.zeros(max(cnt, 1), np.uint32)
        status = np.zeros(max(cnt, 1), np.int32)
        flat = np.zeros(max(int(b.n.sum()), 1), np.uint32)
        offs = np.zeros(cnt + 1, np.uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        st = load().vc_min_batch(
            self._h, ctypes.byref(c), sizes.ctypes.data_as(u32p),
            status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            flat.ctypes.data_as(u32p) if want_cover else None,
            offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if want_cover else None)
        _check(st, "vc_min_batch")
        covers = _split_covers(flat, offs, cnt) if want_cover else []
        return BatchResult(sizes[:cnt].copy(), None, status[:cnt].copy(), covers, self.stats())


    def pvc_batch(self, batch, ks, want_cover: bool = True) -> BatchResult:
        """vc_param_batch with one bound per instance."""
        b = _as_batch(batch)
        c = b.c_struct()
        cnt = b.count
        kk = np.ascontiguousarray(np.asarray(ks, np.uint32).reshape(-1))
        if kk.size != cnt:
            raise ValueError("one k per instance")
        yes = np.zeros(max(cnt, 1), np.int32)
        status = np.zeros(max(cnt, 1), np.int32)
        flat = np.zeros(max(int(b.n.sum()), 1), np.uint32)
        offs = np.zeros(cnt + 1, np.uint64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        st = load().vc_param_batch(
            self._h, ctypes.byref(c), kk.ctypes.data_as(u32p),
            yes.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            flat.ctypes.data_as(u32p) if want_cover else None,
            offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if want_cover else None)
        _check(st, "vc_param_batch")
        covers = _split_covers(flat, offs, cnt) if want_cover else []
        return BatchResult(None, yes[:cnt].astype(bool), status[:cnt].copy(), covers,
                           self.stats())

def _as_batch(b):
    return b if isinstance(b, Batch) else Batch.from_graphs(b)


def _split_covers(flat, offs, count):
    return [flat[offs[i]:offs[i + 1]].copy() for i in range(count)]




def validate_host(g) -> int:
    """Exact host-side CSR check (no device or context needed)."""
    c, keep = host_csr(g)
    return load().vc_validate(None, ctypes.byref(c))
