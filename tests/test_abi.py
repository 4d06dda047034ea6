"""The C ABI library loads and exports every symbol include/les.h declares;
argument errors are reported as codes without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2003_08746_amd import lesmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="les.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(les_[a-z_]+)\s*\(", src)))


def _exported_by_library():
    """Names of the les_* functions the shared library defines in its dynamic
    symbol table (listed with binutils' nm)."""
    import shutil
    import subprocess
    if shutil.which("nm") is None:
        pytest.skip("binutils nm is not installed")
    out = subprocess.run(["nm", "-D", "--defined-only", lesmi.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    return sorted({ln.split()[-1] for ln in out.splitlines() if " T les_" in ln})


def test_header_symbols_exported():
    names = _declared()
    assert "les_create" in names and "les_rk_step" in names and "les_adjoint_step" in names
    L = lesmi.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(lesmi.EXPORTED) == set(names)


def test_every_export_is_declared():
    """Every les_* symbol of the library is declared in include/les.h or, for
    the instrumentation entry points, include/les_debug.h (and vice versa)."""
    declared = set(_declared()) | set(_declared("les_debug.h"))
    assert set(_exported_by_library()) == declared


def test_layout_for():
    st, o, fe, gh = lesmi.les_layout_for(256, 128, 128)
    assert gh == 2  # two ghost layers per side
    assert st[0] == 1 and st[1] % 16 == 0 and st[1] >= 9 + 256 + 2
    assert st[2] == st[1] * (128 + 4)
    # interior i = 0 sits 9 elements into a row, so node i = -1 (the first
    # node a stage-kernel tile copies) starts on a 64-byte boundary
    assert o == 9 + 2 * st[1] + 2 * st[2]
    assert (o - 1) % 8 == 0
    assert fe >= st[2] * (128 + 4) and fe % 32 == 0
    # every node of the padded box lies inside [0, fe)
    assert o - 2 - 2 * st[1] - 2 * st[2] >= 0
    assert o + 257 + 129 * st[1] + 129 * st[2] < fe
    with pytest.raises(lesmi.LesError) as e:
        lesmi.les_layout_for(4, 10, 10)
    assert e.value.code == lesmi.LES_ERR_ARG


def test_create_rejects_bad_arguments():
    L = lesmi.lib()
    ctx = ctypes.c_void_p()
    g = lesmi.LesGrid()
    g.ni, g.nj, g.nk = 16, 16, 16
    p = lesmi.flow_params_struct(__import__("paper_2003_08746_amd.inputs", fromlist=["x"]).flow_params())
    assert L.les_create(None, ctypes.byref(g), None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    assert L.les_create(ctypes.byref(ctx), None, None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    # no coordinates and no metrics (also with an empty les_metrics)
    assert L.les_create(ctypes.byref(ctx), ctypes.byref(g), None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    m = lesmi.LesMetrics()
    assert L.les_create(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(m), ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    g.xyz = 1234  # never dereferenced: the checks below fail first
    g.ni = 4
    assert L.les_create(ctypes.byref(ctx), ctypes.byref(g), None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    assert b"5" in L.les_last_create_error()
    g.ni = 16
    g.bc[1] = 7
    assert L.les_create(ctypes.byref(ctx), ctypes.byref(g), None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    g.bc[1] = 0
    p.gamma = 1.0
    assert L.les_create(ctypes.byref(ctx), ctypes.byref(g), None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    p.gamma = 1.4
    p.prec = 9
    assert L.les_create(ctypes.byref(ctx), ctypes.byref(g), None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    assert ctx.value is None


def test_null_context_calls():
    L = lesmi.lib()
    assert L.les_residual(None, None, None, None) == lesmi.LES_ERR_ARG
    assert L.les_rk_step(None, None, 0.0, None, None, None) == lesmi.LES_ERR_ARG
    assert L.les_adjoint_step(None, None, 1.0, None, None) == lesmi.LES_ERR_ARG
    assert L.les_set_forcing(None, None, 0) == lesmi.LES_ERR_ARG
    assert L.les_stats_accumulate(None, None, None) == lesmi.LES_ERR_ARG
    assert L.les_stats_profiles(None, None, 1.0, 1.0, 0.95, None, None) == lesmi.LES_ERR_ARG
    assert L.les_set_face(None, 0, 1, None, 0.0) == lesmi.LES_ERR_ARG
    assert L.les_debug_stream_copy(None, None, 16, None) == lesmi.LES_ERR_ARG
    assert L.les_debug_stream_copy(16, 32, 24, None) == lesmi.LES_ERR_ARG  # not a multiple of 16 (no launch)
    L.les_destroy(None)


def test_create_size_limit():
    """The stage kernel takes 32-bit element offsets from a 64-bit base per
    segment of k planes, and a segment spans at least seven planes: a block
    whose padded k plane times 7 reaches 2^29 elements is refused before
    anything is allocated, whatever nk is.  9000 x 9000 is over that limit;
    8200 x 8200 is under it, as is an 800 x 800 x 815 block whose fields
    exceed 2^29 elements (both fail on the missing coordinates instead)."""
    L = lesmi.lib()
    ctx = ctypes.c_void_p()
    p = lesmi.flow_params_struct(__import__("paper_2003_08746_amd.inputs", fromlist=["x"]).flow_params())
    g = lesmi.LesGrid()
    g.ni, g.nj, g.nk = 9000, 9000, 5
    assert 7 * lesmi.les_layout_for(9000, 9000, 5)[0][2] >= (1 << 29)
    assert L.les_create(ctypes.byref(ctx), ctypes.byref(g), None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
    assert b"too large" in L.les_last_create_error()
    for n in ((8200, 8200, 5), (800, 800, 815)):
        g.ni, g.nj, g.nk = n
        assert L.les_create(ctypes.byref(ctx), ctypes.byref(g), None, ctypes.byref(p), None) == lesmi.LES_ERR_ARG
        assert b"too large" not in L.les_last_create_error()
    assert 7 * lesmi.les_layout_for(8200, 8200, 5)[0][2] < (1 << 29)
    assert lesmi.les_layout_for(800, 800, 815)[2] >= (1 << 29)
    assert ctx.value is None
