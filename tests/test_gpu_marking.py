"""GPU parity of the Dörfler marking (dpg_dorfler_mark, §4.2) against the
oracle (oracle/dpg_marking.py), through the C ABI, on seeded synthetic
indicators: heavy-tailed values of the 5120-cell and 262144-cell workloads'
sizes (the ranking and the flags are integer results: bit-exact, except that
a cell whose prefix sum lies within 1e-9 of a threshold could go either way
under another summation order -- the test checks that no such cell exists
before comparing), small integers with many ties (sums exact in FP64, so
bit-exact with ties ranked by cell index), and the edge cases."""
import sys

import numpy as np
import pytest

from paper_2609_03155_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gpu_mark(v, fr, fc):
    torch = _torch()
    from paper_2609_03155_amd import dpg
    vd = torch.from_numpy(np.ascontiguousarray(v, np.float64)).cuda()
    f = dpg.dorfler_mark(vd, fr, fc)
    torch.cuda.synchronize()
    return f.cpu().numpy()[:len(v)]


def _margin_ok(v, fr, fc):
    """No cell's decision is within 1e-9 T of a threshold (sums in ranking order)."""
    order = np.lexsort((np.arange(len(v)), -v))
    s = np.concatenate([[0.0], np.cumsum(v[order])[:-1]])
    T = float(np.sum(v[order]))
    tol = 1e-9 * T
    return np.all(np.abs(s - fr * T) > tol) and np.all(np.abs((T - s) - fc * T) > tol)


@pytest.mark.parametrize("n", [5120, 100003, 262144])
def test_marking_matches_oracle_heavy_tailed(n):
    from oracle import dpg_marking as OM
    _say(f"case: dpg_dorfler_mark lognormal n={n}")
    rng = np.random.default_rng(W.SEED_BASE + 51 + n)
    v = np.exp(rng.normal(-6.0, 2.0, n))
    for fr, fc in ((0.30, 0.05), (0.5, 0.2)):
        assert _margin_ok(v, fr, fc)
        fo = OM.dorfler_mark(v, fr, fc)
        fg = _gpu_mark(v, fr, fc)
        assert np.array_equal(fg, fo), (fr, fc, np.count_nonzero(fg != fo))
        assert np.array_equal(_gpu_mark(v, fr, fc), fg)   # deterministic


def test_marking_ties_and_edge_cases():
    torch = _torch()
    from oracle import dpg_marking as OM
    from paper_2609_03155_amd import dpg
    _say("case: dpg_dorfler_mark ties, zeros, fractions 0 and 1, n = 0 and 1, bad arguments")
    rng = np.random.default_rng(W.SEED_BASE + 52)
    for n in (1, 7, 1024, 1025, 40000):
        v = rng.integers(0, 10, n).astype(np.float64)
        for fr, fc in ((0.30, 0.05), (0.0, 0.0), (1.0, 0.0), (0.25, 0.25)):
            assert np.array_equal(_gpu_mark(v, fr, fc), OM.dorfler_mark(v, fr, fc)), (n, fr, fc)
    z = np.zeros(300)
    z[17] = -0.0
    assert np.array_equal(_gpu_mark(z, 0.3, 0.05), OM.dorfler_mark(z, 0.3, 0.05))
    # with a caller's workspace: the same flags, no allocation by the library;
    # a workspace that is too small is refused before anything runs
    for n in (1, 5120, 100003):
        v = np.exp(rng.normal(-6.0, 2.0, n))
        vd = torch.from_numpy(v).cuda()
        nb = dpg.dorfler_mark_workspace_size(n)
        assert nb > 0
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        fw = dpg.dorfler_mark(vd, 0.3, 0.05, workspace=ws)
        fa = dpg.dorfler_mark(vd, 0.3, 0.05)
        torch.cuda.synchronize()
        assert torch.equal(fw[:n], fa[:n]), n
        with pytest.raises(dpg.DPGError):
            dpg.dorfler_mark(vd, 0.3, 0.05, workspace=ws[:nb - 256])
    f = dpg.dorfler_mark(torch.zeros(0, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    vd = torch.ones(10, dtype=torch.float64, device="cuda")
    for fr, fc in ((-0.1, 0.05), (0.3, 1.5), (float("nan"), 0.05)):
        with pytest.raises(dpg.DPGError):
            dpg.dorfler_mark(vd, fr, fc)
