"""Waveguide checks of the oracle (§4.1): the TE10 mode, projected onto the
local trial and trace spaces, is nearly a discrete solution -- its residual
indicator eta -> 0 under h-refinement at the rate of the paper's L2
convergence (p+1) times the h^{3/2} cell-volume factor; and in the 2x2x2
cube with one eps = 4 + 0.5i cell, the vacuum TE10 mode has its largest
residual in that cell."""
import math

import numpy as np
import pytest

from oracle import dpg_oracle as O
from paper_2609_03155_amd import workloads as W


@pytest.mark.parametrize("p", [1, 2])
def test_te10_residual_converges(p):
    om = O.omega_dimensionless(2.45e9)
    pm = O.PortMode(0.25, 0.25, 1, 0, om)
    Ef = lambda x: pm.fields(x)[0]
    Hf = lambda x: pm.fields(x)[1]
    etas = []
    for h in (0.03125, 0.015625):
        x0 = np.array([0.07, 0.09, 0.31])
        X = np.array([x0 + h * np.array([i, j, k]) for k in (0, 1) for j in (0, 1) for i in (0, 1)])
        cp = O.CellProblem(X=X, p=p, dp=1, eps=1.0, mu=1.0, omega=om)
        G, Bf, l = O.cell_forms(cp)
        _, _, eta = O.local_solve(G, Bf, l, O.projected_solution(X, p, Ef, Hf))
        etas.append(eta)
    rate = math.log2(etas[0] / etas[1])
    assert rate > p + 2.0, (p, etas, rate)


def test_config1_inclusion_has_largest_residual():
    w = W.config1()
    om = O.omega_dimensionless(w.freq_hz)
    pt = w.port
    pm = O.PortMode(pt["a"], pt["b"], pt["m"], pt["n"], om, pt["eps"], pt["mu"])
    Ef = lambda x: pm.fields(x)[0]
    Hf = lambda x: pm.fields(x)[1]
    etas = []
    for c in range(w.n_cells):
        X = w.cell_vertices(c)
        cp = O.CellProblem(X=X, p=int(w.degree[c]), dp=w.dp, eps=w.eps[c], mu=w.mu[c], omega=om,
                           face_kind=tuple(int(k) for k in w.face_kind[c]), zinv=tuple(w.zinv[c]), port=pm)
        G, Bf, l = O.cell_forms(cp)
        _, _, eta = O.local_solve(G, Bf, l, O.projected_solution(X, int(w.degree[c]), Ef, Hf))
        etas.append(eta)
    etas = np.array(etas)
    assert int(np.argmax(etas)) == 0
    assert etas[0] > 2 * np.max(etas[1:])


def test_workload_port_admittance_matches_oracle():
    """The Robin admittance the workload generator stores equals k3/(omega mu)
    of the oracle's TE_mn mode."""
    for cfg in (W.config1, W.config2):
        w = cfg()
        om = O.omega_dimensionless(w.freq_hz)
        pt = w.port
        y = O.PortMode(pt["a"], pt["b"], pt["m"], pt["n"], om, pt["eps"], pt["mu"]).zinv()
        robin = (w.face_kind == W.FACE_PORT) | (w.face_kind == W.FACE_ROBIN0)
        assert np.allclose(w.zinv[robin], y, rtol=1e-14, atol=0)
        assert np.all(w.zinv[~robin] == 0)


def test_workload_meshes_are_valid():
    """Every cell of the perturbed and curved meshes has det J > 0 at its
    quadrature points (the meshes are legal inputs)."""
    pts, _ = O.volume_rule(3)
    for cfg, kw in ((W.config2, {}), (W.config3, dict(nx=10, ny=10, nz=12)), (W.config5, dict(n=12))):
        w = cfg(**kw)
        for c in range(0, w.n_cells, max(1, w.n_cells // 200)):
            _, J = O.trilinear_map(w.cell_vertices(c), pts)
            assert np.linalg.det(J).min() > 0
