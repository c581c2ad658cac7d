"""Host logic of the condensed trace system: the library's native numbering
(dpg_trace_numbering, C++) equals the oracle's, id for id, on structured
meshes with the waveguide boundary conditions, all-Robin boundaries, mixed
degrees (minimum rule) and perturbed vertices; both reject a mesh whose
cells disagree on an edge direction.  Host only (no device calls)."""
import numpy as np
import pytest

from oracle import dpg_assembly as A
from paper_2609_03155_amd import dpg
from paper_2609_03155_amd import workloads as W


def _oracle(cells, fk, deg):
    glob, n = A.trace_numbering(cells, fk, deg)
    return np.concatenate(glob), n


@pytest.mark.parametrize("shape,degs", [((2, 2, 2), [1]), ((3, 2, 2), [2]), ((2, 3, 1), [3]), ((1, 1, 2), [4]),
                                        ((3, 3, 2), [1, 2, 3]), ((2, 2, 3), [2, 3])])
def test_native_numbering_equals_oracle(shape, degs):
    nx, ny, nz = shape
    V, cells, fk, _ = W.box_mesh(nx, ny, nz, 1.0, 1.0, 1.0)
    rng = np.random.default_rng(sum(shape) * 10 + len(degs))
    deg = rng.choice(np.array(degs, np.int8), size=cells.shape[0])
    for kinds in (fk, np.where(fk != 0, 3, 0).astype(np.int8)):
        g_or, n_or = _oracle(cells, kinds, deg)
        g_lib, n_lib = dpg.trace_numbering(cells, kinds, deg)
        assert n_lib == n_or
        assert np.array_equal(g_lib, g_or)


def test_workload_numbering_matches_on_c1_and_small_c3():
    for w in (W.config1(), W.config3(nx=3, ny=2, nz=3)):
        g_or, n_or = _oracle(w.cells, w.face_kind, w.degree)
        g_lib, n_lib = dpg.trace_numbering(w.cells, w.face_kind, w.degree)
        assert n_lib == n_or and np.array_equal(g_lib, g_or)


def test_inconsistent_orientation_is_rejected():
    V, cells, fk, _ = W.box_mesh(2, 1, 1, 1.0, 1.0, 1.0)
    bad = cells.copy()
    bad[1] = bad[1][[3, 2, 1, 0, 7, 6, 5, 4]]        # second cell turned by 180 degrees about z
    with pytest.raises(ValueError):
        A.trace_numbering(bad, fk, np.array([1, 1]))
    with pytest.raises(dpg.DPGError):
        dpg.trace_numbering(bad, fk, np.array([1, 1]))
