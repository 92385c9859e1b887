"""C-ABI checks that need no GPU: the library loads, exports every entry point
the header declares, lays out grids as documented, and rejects misuse before
any HIP call (context state machine of Section 4, Fig. 2b)."""
import ctypes
import os
import re

import pytest

import paper_1207_1746_amd as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(gscl_\w+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = G.lib()
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    # and the binding types every one of them
    assert set(G._SIGS) == names


def test_grid_layout_defaults_and_bytes():
    d = G.make_desc((64, 64, 64), G.F64, halo=1)
    assert G.lib().gscl_grid_layout(ctypes.byref(d)) == G.OK
    assert (d.pitch[0], d.pitch[1]) == (64, 64 * 64)
    assert G.lib().gscl_grid_bytes(ctypes.byref(d)) == 64 ** 3 * 8
    d = G.make_desc((5, 7, 37), G.F32)
    G.lib().gscl_grid_layout(ctypes.byref(d))
    assert d.pitch[0] == 48 and d.pitch[1] == 48 * 7
    assert G.lib().gscl_grid_bytes(ctypes.byref(d)) == 48 * 7 * 5 * 4
    d = G.make_desc((4, 8192, 8192), G.U8, halo=2, bc=G.CLAMP, ndim=2)
    G.lib().gscl_grid_layout(ctypes.byref(d))
    assert d.n[2] == 4 and d.pitch[0] == 8192


@pytest.mark.parametrize("bad,code", [
    (dict(ndim=4), G.ERR_SHAPE), (dict(dtype=17), G.ERR_DTYPE), (dict(halo=9), G.ERR_HALO),
    (dict(bc=5), G.ERR_ARG), (dict(pitch=(3, 0)), G.ERR_SHAPE),
])
def test_layout_rejects_bad_descriptors(bad, code):
    d = G.make_desc((8, 8, 8), G.F32)
    for k, v in bad.items():
        if k == "pitch":
            d.pitch[0], d.pitch[1] = v
        else:
            setattr(d, k, v)
    assert G.lib().gscl_grid_layout(ctypes.byref(d)) == code
    assert G.lib().gscl_grid_bytes(ctypes.byref(d)) == 0
    assert G.lib().gscl_last_error()


def test_context_state_machine_before_begin():
    L = G.lib()
    h = ctypes.c_void_p()
    assert L.gscl_init(0, ctypes.byref(h)) == G.OK
    sd = G.StencilDesc()
    sd.kind = G.K_WJACOBI
    arr = (ctypes.c_void_p * 1)(None)
    # iteration spaces outside begin/end are an error (the paper aborts; we return)
    assert L.gscl_do_all(h, ctypes.byref(sd), arr, 1, arr, 1, None, None) == G.ERR_STATE
    assert L.gscl_do_all_noalloc(h, ctypes.byref(sd), arr, 1, arr, 1, None, None) == G.ERR_STATE
    rd = G.ReduceDesc()
    res = ctypes.c_double()
    assert L.gscl_do_reduce(h, ctypes.byref(rd), None, None, ctypes.byref(res)) == G.ERR_STATE
    assert L.gscl_end(h) == G.ERR_STATE
    assert L.gscl_graph_begin(h) == G.ERR_STATE
    assert L.gscl_finalize(h) == G.OK


def test_null_and_invalid_handles():
    L = G.lib()
    assert L.gscl_init(0, None) == G.ERR_ARG
    assert L.gscl_init(-1, ctypes.byref(ctypes.c_void_p())) == G.ERR_ARG
    assert L.gscl_begin(None, None) == G.ERR_ARG
    assert L.gscl_grid_destroy(None) == G.ERR_ARG
    assert L.gscl_graph_destroy(None) == G.ERR_ARG
    assert L.gscl_version().startswith(b"gscl")


def test_begin_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = G.lib()
    h = ctypes.c_void_p()
    L.gscl_init(0, ctypes.byref(h))
    assert L.gscl_begin(h, None) == G.ERR_HIP
    assert b"hip" in L.gscl_last_error().lower()
    L.gscl_finalize(h)


_STRUCTS = {
    "gscl_grid_desc": G.GridDesc, "gscl_term": G.Term, "gscl_stencil_desc": G.StencilDesc,
    "gscl_reduce_desc": G.ReduceDesc, "gscl_tile": G.Tile, "gscl_solve_desc": G.SolveDesc,
    "gscl_solve_stats": G.SolveStats, "gscl_batch_desc": G.BatchDesc, "gscl_slot_stats": G.SlotStats,
}


def test_binding_structs_match_header_layout(tmp_path):
    """Every descriptor the binding passes by pointer has the size and field
    offsets the C compiler gives the header's struct (compiled here with gcc)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "gscl.h"', "int main(void) {"]
    for cname, py in _STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, what, val = line.split()
        got[(cname, what)] = int(val)
    for cname, py in _STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
