"""The C-ABI library loads and exports every entry point include/dpg.h
declares; host-only entry points work without a GPU."""
import os
import re

import pytest

from paper_2609_03155_amd import dpg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "dpg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpg_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert declared_entry_points() == sorted(dpg.EXPORTS)


@pytest.mark.skipif(not os.path.exists(dpg.LIB_PATH), reason="libdpgmi.so not built")
def test_library_exports_every_declared_symbol():
    L = dpg.lib()
    for name in declared_entry_points():
        assert hasattr(L, name), name


@pytest.mark.skipif(not os.path.exists(dpg.LIB_PATH), reason="libdpgmi.so not built")
def test_local_dims_host_only():
    from paper_2609_03155_amd import workloads as W
    for p in range(1, 5):
        for dp in (1, 2):
            assert dpg.dpg_local_dims(p, dp) == W.local_dims(p, dp)
    with pytest.raises(dpg.DPGError):
        dpg.dpg_local_dims(5, 1)
    with pytest.raises(dpg.DPGError):
        dpg.dpg_local_dims(2, 0)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(dpg, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(dpg, "_lib", None)
    with pytest.raises(dpg.DPGError):
        dpg.lib()


@pytest.mark.skipif(not os.path.exists(dpg.LIB_PATH), reason="libdpgmi.so not built")
def test_global_solve_entry_points_reject_bad_arguments_on_the_host():
    """Argument errors of the global-solve entry points are returned
    synchronously, before any device call (so they need no GPU); empty
    inputs are no-ops."""
    import ctypes as C
    L = dpg.lib()
    it, rr = C.c_int64(7), C.c_double(7.0)
    cg = lambda n, tol, mi, iters=True: L.dpg_cg_solve(n, None, None, None, None, None, tol, mi,
                                                      C.byref(it) if iters else None, C.byref(rr), None)
    assert cg(-1, 1e-8, 10) == dpg.DPG_ERR_ARG
    assert cg(5, 1e-8, 10) == dpg.DPG_ERR_ARG          # null device pointers
    assert cg(0, -1.0, 10) == dpg.DPG_ERR_ARG
    assert cg(0, float("nan"), 10) == dpg.DPG_ERR_ARG
    assert cg(0, 1e-8, -1) == dpg.DPG_ERR_ARG
    assert cg(0, 1e-8, 10, iters=False) == dpg.DPG_ERR_ARG
    assert cg(0, 1e-8, 10) == dpg.DPG_OK and it.value == 0 and rr.value == 0.0
    assert L.dpg_trace_system_cg(None, None, None, None, 1e-8, 10, C.byref(it), C.byref(rr), None) == dpg.DPG_ERR_ARG
    mark = lambda n, fr, fc: L.dpg_dorfler_mark(n, None, fr, fc, None, None, 0, None)
    ws = C.c_size_t(7)
    assert L.dpg_dorfler_mark_workspace_size(-1, C.byref(ws)) == dpg.DPG_ERR_ARG
    assert L.dpg_dorfler_mark_workspace_size(4, None) == dpg.DPG_ERR_ARG
    assert L.dpg_dorfler_mark_workspace_size(0, C.byref(ws)) == dpg.DPG_OK and ws.value == 0
    assert mark(-1, 0.3, 0.05) == dpg.DPG_ERR_ARG
    assert mark(2 ** 31, 0.3, 0.05) == dpg.DPG_ERR_ARG
    assert mark(4, 0.3, 0.05) == dpg.DPG_ERR_ARG        # null device pointers
    assert mark(0, 1.5, 0.05) == dpg.DPG_ERR_ARG
    assert mark(0, 0.3, float("nan")) == dpg.DPG_ERR_ARG
    assert mark(0, 0.3, 0.05) == dpg.DPG_OK
    assert L.dpg_reconstruct(None, None, None, None, None, None, None) == dpg.DPG_ERR_ARG
    assert L.dpg_power_dissipation(None, None, None, None, None) == dpg.DPG_ERR_ARG
    assert L.dpg_trace_system_scatter(None, None, None, None) == dpg.DPG_ERR_ARG
