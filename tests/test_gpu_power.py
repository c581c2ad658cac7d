"""GPU parity of the per-cell power dissipation (dpg_power_dissipation, §3.2
heat source) against the oracle (oracle/dpg_power.py), through the C ABI, on
seeded random coefficient vectors: the cube (p = 1, one lossy cell), a
perturbed lossy piece of the WR340 guide (p = 2), mixed degrees 1..4, p = 4
with dp = 2, and the full 5120-cell WR340 workload (sampled cells; every
cell's |E|^2 and |H|^2 integrals positive).  Bar: 1e-12 of the cell's value
(the integrands are quadratic forms of the coefficients with positive
weights, so both sides round at that level)."""
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


def _gpu_power(w, x):
    torch = _torch()
    from paper_2609_03155_amd import dpg
    plan = dpg.Plan(w.degree, w.dp)
    prob = dpg.DeviceProblem.from_workload(w)
    out = plan.power_dissipation(prob, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    res = out.cpu().numpy()[:w.n_cells]
    plan.close()
    return res


def _check(w, x, off, cells):
    from oracle import dpg_oracle as O
    from oracle import dpg_power as OP
    g = _gpu_power(w, x)
    om = O.omega_dimensionless(w.freq_hz)
    for c in cells:
        p = int(w.degree[c])
        o = OP.cell_power(w.cell_vertices(c), p, x[off[c]:off[c + 1]], complex(w.eps[c]), complex(w.mu[c]), om)
        for k in range(3):
            assert abs(g[c, k] - o[k]) <= 1e-12 * max(abs(o[1]), abs(o[2]), 1e-300) * max(1.0, om), (c, k, g[c], o)
    return g


def _mixed():
    w = W.config3(nx=3, ny=2, nz=2)
    w.degree[:] = np.array([1, 2, 3, 4, 2, 1] * 2, np.int8)[: w.n_cells]
    w.eps[:] = w.eps * (1.0 + 0.2j)
    return w


@pytest.mark.parametrize("name", ["config1", "config2_3x2x2", "mixed_p1to4", "config4_p4_dp2"])
def test_power_matches_oracle(name):
    w = {"config1": W.config1, "config2_3x2x2": lambda: W.config2(nx=3, ny=2, nz=2), "mixed_p1to4": _mixed,
         "config4_p4_dp2": lambda: W.config4(n=2)}[name]()
    _say(f"case: dpg_power_dissipation {w.name}")
    x, off = W.random_coefficients(w, seed=61)
    _check(w, x, off, range(w.n_cells))


def test_power_config2_full_size_sampled():
    w = W.config2()
    _say(f"case: dpg_power_dissipation {w.name} (full size, sampled)")
    x, off = W.random_coefficients(w, seed=62)
    rng = np.random.default_rng(W.SEED_BASE + 63)
    cells = sorted(set([0, w.n_cells - 1] + list(rng.choice(w.n_cells, 6, replace=False))))
    g = _check(w, x, off, cells)
    assert np.all(g[:, 1] > 0) and np.all(g[:, 2] > 0) and np.all(g[:, 0] >= 0)
