"""Host logic of the adaptive loop (paper_2609_03155_amd/adapt.py): the
degree update after a marking.  No GPU."""
import numpy as np
import pytest

from paper_2609_03155_amd.adapt import AdaptPass, next_degrees


def test_next_degrees_refines_coarsens_and_clamps():
    deg = np.array([1, 2, 3, 4, 1, 4, 2, 2], np.int8)
    flags = np.array([1, 1, -1, 1, -1, -1, 0, 0], np.int8)
    assert next_degrees(deg, flags).tolist() == [2, 3, 2, 4, 1, 3, 2, 2]
    assert next_degrees(deg, flags, p_min=2, p_max=3).tolist() == [2, 3, 2, 3, 2, 3, 2, 2]
    # no marks: unchanged (dtype int8, what the plan takes)
    out = next_degrees(deg, np.zeros(8, np.int8))
    assert out.dtype == np.int8 and np.array_equal(out, deg)


def test_next_degrees_rejects_bad_input():
    with pytest.raises(ValueError):
        next_degrees(np.ones(3, np.int8), np.zeros(4, np.int8))
    with pytest.raises(ValueError):
        next_degrees(np.ones(3, np.int8), np.zeros(3, np.int8), p_min=3, p_max=2)
    with pytest.raises(ValueError):
        next_degrees(np.ones(3, np.int8), np.zeros(3, np.int8), p_max=5)


def test_eta_total_is_the_global_residual_norm():
    ap = AdaptPass(degree=np.ones(3, np.int8), n_dofs=0, cg_iterations=0, relres=0.0,
                   eta=np.array([3.0, 4.0, 0.0]), flags=np.zeros(3, np.int8))
    assert ap.eta_total == 5.0
