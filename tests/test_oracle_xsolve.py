"""Pins of the oracle's extended-precision solve (oracle/xsolve.c) and of its
second formation route (cell_forms_blocks, App. A's real block matrices).

* xsolve returns the exact answer of systems built from integers: with L
  lower triangular with integer entries and W0 integer, G = L L^H and
  B = L W0 are exact in FP64, and K_e = W0^H W0, l_e and eta are integers.
* xsolve agrees with an independent extended-precision Gaussian elimination
  (numpy long double, partial pivoting) to far below FP64 accuracy.
* the block route gives the same G, B_f, l as the pointwise route to
  roundoff, and it solves the exact polynomial manufactured solution of §2.2
  (B_f x_exact - l = 0) with port, impedance and PEC faces and complex
  coefficients.
"""
import math

import numpy as np
import pytest

from oracle import dpg_oracle as O
from oracle import xsolve as X

from test_oracle_forms import _affine_cell, _cell, _elim_extended, _manufactured


def test_xsolve_is_exact_on_integer_systems():
    rng = np.random.default_rng(11)
    n, k = 23, 7
    L = np.tril(rng.integers(-3, 4, (n, n)) + 1j * rng.integers(-3, 4, (n, n)), -1)
    L += np.diag(rng.integers(1, 4, n)).astype(complex)
    W0 = rng.integers(-4, 5, (n, k + 2)) + 1j * rng.integers(-4, 5, (n, k + 2))
    G = L @ L.conj().T                  # integers below 2^53: exact
    R = L @ W0
    B, l, r = R[:, :k], R[:, k], R[:, k + 1]
    K, le, eta, ynorm = X.local_solve_ext(G, B, l, r, with_ynorm=True)
    Wb, wl, wr = W0[:, :k], W0[:, k], W0[:, k + 1]
    assert np.array_equal(K, Wb.conj().T @ Wb)
    assert np.array_equal(le, Wb.conj().T @ wl)
    assert eta == math.sqrt(float(np.real(wr.conj() @ wr)))
    assert ynorm == math.sqrt(float(np.real(wl.conj() @ wl)))


def test_xsolve_rejects_an_indefinite_matrix():
    G = np.diag([1.0, -1.0, 2.0]).astype(complex)
    with pytest.raises(ValueError):
        X.local_solve_ext(G, np.eye(3, dtype=complex), np.zeros(3, complex))


@pytest.mark.skipif(np.finfo(np.longdouble).eps > 1e-18, reason="no extended precision long double on this host")
def test_xsolve_agrees_with_an_independent_extended_elimination():
    cp = _cell(2, p=1)
    cp.port = O.PortMode(0.1, 0.1, 1, 0, cp.omega)
    cp.face_kind = (0, 0, 0, 0, O.FACE_PORT, 0)
    G, Bf, l = O.cell_forms(cp)
    Xe = _elim_extended(G, np.concatenate([Bf, l[:, None]], axis=1))
    Bh = np.conj(Bf).T.astype(np.clongdouble)
    Ke = (Bh @ Xe[:, :-1]).astype(np.complex128)
    le = (Bh @ Xe[:, -1]).astype(np.complex128)
    K, lx, _ = X.local_solve_ext(G, Bf, l)
    assert np.linalg.norm(K - Ke) < 1e-12 * np.linalg.norm(Ke)
    assert np.linalg.norm(lx - le) < 1e-12 * np.linalg.norm(le)
    # and the FP64 oracle is within its condition-number bound of it
    Kf, lf, _ = O.local_solve(G, Bf, l)
    d = 1 / np.sqrt(np.real(np.diag(G)))
    kappa = np.linalg.cond(G * d[:, None] * d[None, :])
    assert np.linalg.norm(Kf - K) < 50 * kappa * 1e-16 * np.linalg.norm(K)


@pytest.mark.parametrize("p,dp", [(1, 1), (2, 1), (3, 1), (2, 2)])
def test_block_route_matches_pointwise_forms(p, dp):
    cp = _cell(p + 7, p=p, dp=dp, robin=((4, 0.79 + 0.1j), (1, 1.2 - 0.3j)))
    cp.eps, cp.mu = 3.5 + 0.8j, 1.2 + 0.05j
    cp.port = O.PortMode(0.1, 0.1, 1, 0, cp.omega)
    cp.face_kind = (O.FACE_PEC, O.FACE_ROBIN0, 0, 0, O.FACE_PORT, 0)
    G1, B1, l1 = O.cell_forms(cp)
    G2, B2, l2 = O.cell_forms_blocks(cp)
    d = np.sqrt(np.real(np.diag(G1)))
    assert (np.abs(G2 - G1) / np.outer(d, d)).max() < 1e-13
    assert np.abs(B2 - B1).max() < 1e-13 * np.abs(B1).max()
    assert np.abs(l2 - l1).max() < 1e-13 * np.abs(l1).max()


@pytest.mark.parametrize("p,dp", [(1, 1), (2, 2)])
def test_block_route_solves_the_manufactured_solution(p, dp):
    om, eps, mu = 23.0, 2.5 + 0.7j, 1.3 - 0.1j
    Ef, Hf, Jf = _manufactured(p, om, eps, mu, seed=p + 10 * dp)
    Xv = _affine_cell(p)
    fk = (O.FACE_PEC, O.FACE_ROBIN0, 0, 0, O.FACE_PORT, O.FACE_ROBIN0)
    zi = (0, 0.6 + 0.2j, 0, 0, 0.83 - 0.1j, 1.1 + 0.4j)

    def g(f, xx, n):
        E, H = Ef(xx), Hf(xx)
        return np.cross(n, H) + zi[f] * np.cross(n, np.cross(E, n))
    cp = O.CellProblem(X=Xv, p=p, dp=dp, eps=eps, mu=mu, omega=om, face_kind=fk, zinv=zi, J_src=Jf, g_src=g)
    _, Bf, l = O.cell_forms_blocks(cp)
    xe = O.projected_solution(Xv, p, Ef, Hf)
    assert np.linalg.norm(Bf @ xe - l) < 1e-11 * (np.linalg.norm(Bf @ xe) + np.linalg.norm(l))
