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
