"""The C-ABI boundary on the CPU: the library loads, exports every entry
point include/vc.h declares, its structs have the header's layout, and the
exact host-side CSR validation accepts simple symmetric graphs and rejects
the malformed ones the header lists."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2512_18334_amd import graphgen as gg
from paper_2512_18334_amd import vc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["vc_ctx_create", "vc_ctx_destroy", "vc_min", "vc_param",
              "vc_min_batch", "vc_param_batch", "vc_submit", "vc_poll", "vc_cancel",
              "vc_validate", "vc_last_stats", "vc_status_str"]:
        assert f in names


def test_library_exports_every_declared_symbol(libvc):
    out = subprocess.run(["nm", "-D", "--defined-only", vc.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(vc_\w+)", out))
    for f in declared_functions():
        assert f in exported, f
        getattr(libvc, f)
    assert set(vc.EXPORTS) <= exported


def test_struct_layout_matches_header(tmp_path, libvc):
    prog = tmp_path / "layout.c"
    fields = {
        "vc_csr": [f for f, _ in vc.vc_csr._fields_],
        "vc_opts": [f for f, _ in vc.vc_opts._fields_],
        "vc_stats": [f for f, _ in vc.vc_stats._fields_],
        "vc_batch": [f for f, _ in vc.vc_batch._fields_],
        "vc_result": [f for f, _ in vc.vc_result._fields_],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vc.h"',
             "int main(void) {"]
    for s, fs in fields.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0; }")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"),
                    str(prog), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run(
        [str(exe)], capture_output=True, text=True, check=True).stdout.splitlines())
    for s, cls in [("vc_csr", vc.vc_csr), ("vc_opts", vc.vc_opts),
                   ("vc_stats", vc.vc_stats), ("vc_batch", vc.vc_batch),
                   ("vc_result", vc.vc_result)]:
        assert int(got[s]) == ctypes.sizeof(cls), s
        for f, _ in cls._fields_:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)


def test_status_strings(libvc):
    for code in range(0, -8, -1):
        assert vc.status_str(code) != "unknown status"


def _mutate(g, fn):
    h = gg.Graph(g.n, g.offsets.copy(), g.cols.copy(), g.name)
    fn(h)
    return h


@pytest.mark.parametrize("g", [gg.petersen(), gg.fig1_tree(), gg.config1_gnp60(3),
                               gg.config2_blocks_hubs(),
                               gg.from_edges(5, [], []), gg.from_edges(0, [], [])])
def test_host_validation_accepts(libvc, g):
    assert vc.validate_host(g) == vc.VC_OK


def test_host_validation_rejects(libvc):
    g = gg.petersen().with_cols(4)
    # self-loop: vertex 0 lists itself
    assert vc.validate_host(_mutate(g, lambda h: h.cols.__setitem__(0, 0))) == vc.VC_EINVAL
    # out of range id
    assert vc.validate_host(_mutate(g, lambda h: h.cols.__setitem__(1, 99))) == vc.VC_EINVAL
    # asymmetric: 0's first neighbour replaced by a non-neighbour
    def asym(h):
        row = set(h.cols[h.offsets[0]:h.offsets[1]].tolist())
        other = next(x for x in range(1, h.n) if x not in row)
        h.cols[0] = other
    assert vc.validate_host(_mutate(g, asym)) == vc.VC_EINVAL
    # repeated entry in a row
    assert vc.validate_host(_mutate(g, lambda h: h.cols.__setitem__(1, h.cols[0]))) == vc.VC_EINVAL
    # offsets not starting at 0 / not monotone
    assert vc.validate_host(_mutate(g, lambda h: h.offsets.__setitem__(0, 1))) == vc.VC_EINVAL
    def nonmono(h):
        h.offsets[3], h.offsets[4] = h.offsets[4], h.offsets[3]
    assert vc.validate_host(_mutate(g, nonmono)) == vc.VC_EINVAL


def test_host_validation_rejects_bad_widths(libvc):
    g = gg.petersen()
    c, keep = vc.host_csr(g)
    c.col_bytes = 3
    assert libvc.vc_validate(None, ctypes.byref(c)) == vc.VC_EINVAL
    big = vc.vc_csr(70000, 0, keep[0].ctypes.data, None, 2, 0)
    assert libvc.vc_validate(None, ctypes.byref(big)) == vc.VC_EINVAL


def test_batch_entry_points_reject_missing_context(libvc):
    b = vc.Batch.from_graphs([gg.petersen(), gg.fig1_tree()])
    c = b.c_struct()
    sizes = np.zeros(2, np.uint32)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    assert libvc.vc_min_batch(None, ctypes.byref(c), sizes.ctypes.data_as(u32p),
                              None, None, None) == vc.VC_EINVAL
    k = np.array([6, 3], np.uint32)
    yes = np.zeros(2, np.int32)
    assert libvc.vc_param_batch(None, ctypes.byref(c), k.ctypes.data_as(u32p),
                                yes.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                None, None, None) == vc.VC_EINVAL


def test_batch_packing_layout():
    gs = [gg.petersen(), gg.from_edges(0, [], []), gg.fig1_tree(), gg.cycle(5)]
    b = vc.Batch.from_graphs(gs)
    assert b.count == 4 and b.col_bytes == 2
    for i, g in enumerate(gs):
        ob, cb = int(b.offs_base[i]), int(b.cols_base[i])
        assert np.array_equal(b.offsets[ob:ob + g.n + 1], g.offsets)
        assert int(b.offsets[ob]) == 0 and int(b.offsets[ob + g.n]) == g.nnz
        assert np.array_equal(b.cols[cb:cb + g.nnz], np.asarray(g.cols))


def test_serving_entry_points_reject_missing_context(libvc):
    g = gg.petersen()
    c, keep = vc.host_csr(g)
    t = ctypes.c_uint64(0)
    assert libvc.vc_submit(None, ctypes.byref(c), vc.VC_MIN, 0, ctypes.byref(t)) == vc.VC_EINVAL
    r = vc.vc_result()
    assert libvc.vc_poll(None, 1, ctypes.byref(r), None) == vc.VC_EINVAL
    assert libvc.vc_cancel(None, 1) == vc.VC_EINVAL


def test_python_constants_match_the_header():
    """Every #define and vc_status value in include/vc.h has the same value in
    the Python binding."""
    text = open(HEADER).read()
    found = dict(re.findall(r"^#define (VC_[A-Z_]+) (\d+)u?\b", text, re.M))
    found.update(re.findall(r"^\s+(VC_[A-Z]+) = (-?\d+),", text, re.M))
    assert {"VC_OPT_NO_INDUCE", "VC_OPT_NO_COMPACT", "VC_EINVAL", "VC_MIN"} <= set(found)
    for name, val in found.items():
        assert getattr(vc, name) == int(val), name
