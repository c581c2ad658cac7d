"""Pins of the global-solve oracle (oracle/dpg_assembly.py: cg, scatter,
reconstruct; §2.3: the condensed system solved by CG without a
preconditioner, then the interior unknowns recovered cell by cell).

* cg: a Hermitian matrix with three distinct eigenvalues is solved in three
  iterations (the Krylov space is then complete); every iterate satisfies the
  Galerkin condition of CG, V_k^H (b - A x_k) = 0 on an orthonormal basis V_k
  of the Krylov space K_k(A, b) built independently here; the converged
  iterate equals a direct solve;
* everything together: for an exact polynomial solution on a sheared mesh
  (Robin data on every boundary face), CG on the assembled system returns the
  exact traces, reconstruction the exact interior coefficients, and the local
  residual indicator of the reconstructed coefficients vanishes (without a
  preconditioner CG needs several times n iterations here: 2373 for the 360
  unknowns at p = 1, 7023 for the 828 at p = 2, to 1e-12);
* plausible mistakes planted in the oracle (an unconjugated inner product in
  CG, a sign in the reconstruction) fail these pins.
"""
import numpy as np
import pytest

from oracle import dpg_assembly as A
from oracle import dpg_oracle as O
from paper_2609_03155_amd import workloads as W

from test_oracle_forms import _manufactured


def _unitary(n, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return Q


def test_cg_three_distinct_eigenvalues_three_iterations():
    rng = np.random.default_rng(11)
    n = 30
    Q = _unitary(n, rng)
    lam = np.repeat([1.0, 3.5, 10.0], n // 3)
    M = (Q * lam) @ Q.conj().T
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist = A.cg(M, b, 1e-12, 50)
    assert it == 3, hist
    assert hist[2] > 1e-3
    assert np.linalg.norm(M @ x - b) <= 1e-12 * np.linalg.norm(b)


def _krylov_basis(M, b, k):
    """Orthonormal basis of span{b, M b, ..., M^{k-1} b} (Gram-Schmidt twice)."""
    V = np.zeros((len(b), k), complex)
    v = b / np.linalg.norm(b)
    for j in range(k):
        for _ in range(2):
            v = v - V[:, :j] @ (V[:, :j].conj().T @ v)
        V[:, j] = v / np.linalg.norm(v)
        v = M @ V[:, j]
    return V


def test_cg_iterates_satisfy_galerkin_condition_and_converge():
    rng = np.random.default_rng(12)
    n = 40
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    M = X @ X.conj().T / n + 0.5 * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for k in range(1, 7):
        xk, it, _ = A.cg(M, b, 0.0, k)
        assert it == k
        V = _krylov_basis(M, b, k)
        # x_k in K_k and its residual orthogonal to K_k
        assert np.linalg.norm(xk - V @ (V.conj().T @ xk)) <= 1e-10 * np.linalg.norm(xk)
        assert np.linalg.norm(V.conj().T @ (b - M @ xk)) <= 1e-10 * np.linalg.norm(b)
    x, it, hist = A.cg(M, b, 1e-13, 500)
    assert hist[-1] <= 1e-13 and it < 500
    xd = np.linalg.solve(M, b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # a zero right-hand side needs no iteration
    x0, it0, _ = A.cg(M, np.zeros(n, complex), 1e-12, 10)
    assert it0 == 0 and not np.any(x0)


def test_cg_planted_unconjugated_inner_product_fails(monkeypatch):
    def bad(M, b, tol, max_iter, x0=None):
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        rr = r @ r
        it = 0
        while it < max_iter:
            q = M @ p
            alpha = rr / (p @ q)
            x = x + alpha * p
            r = r - alpha * q
            rn = r @ r
            p = r + (rn / rr) * p
            rr = rn
            it += 1
        return x, it, None
    monkeypatch.setattr(A, "cg", bad)
    with pytest.raises(AssertionError):
        test_cg_iterates_satisfy_galerkin_condition_and_converge()


def _manufactured_global(p):
    """The exact-polynomial problem of the assembly pin: per-cell forms,
    K_e, l_e, the exact coefficient vectors, the assembled system and the
    numbering."""
    om, eps, mu, dp = 23.0, 2.5 + 0.7j, 1.3 - 0.1j, 1
    Ef, Hf, Jf = _manufactured(p, om, eps, mu, seed=40 + p)
    V, cells, fk, _ = W.box_mesh(2, 2, 2, 0.1, 0.1, 0.1)
    rng = np.random.default_rng(7 + p)
    Mt = np.eye(3) + 0.15 * rng.standard_normal((3, 3))
    V = V @ Mt.T + np.array([0.01, -0.02, 0.03])
    nc = cells.shape[0]
    bnd = fk != 0
    fk = np.where(bnd, O.FACE_ROBIN0, 0).astype(np.int8)
    zi = np.where(bnd, 0.7 + 0.25j + 0.1 * np.arange(6)[None, :], 0).astype(complex)
    nu = 6 * (p + 1) ** 3
    glob, n = A.trace_numbering(cells, fk, np.full(nc, p))
    cells_out = []
    for c in range(nc):
        X = V[cells[c]]
        z = tuple(zi[c])

        def g(f, xx, nrm, z=z):
            E, H = Ef(xx), Hf(xx)
            return np.cross(nrm, H) + z[f] * np.cross(nrm, np.cross(E, nrm))
        cp = O.CellProblem(X=X, p=p, dp=dp, eps=eps, mu=mu, omega=om, face_kind=tuple(fk[c]), zinv=z,
                           J_src=Jf, g_src=g)
        G, Bf, l = O.cell_forms(cp)
        K, le, _ = O.local_solve(G, Bf, l, None)
        cells_out.append(dict(G=G, Bf=Bf, l=l, K=K, le=le, x=O.projected_solution(X, p, Ef, Hf)))
    Ak = [A.condense(c["K"], c["le"], nu) for c in cells_out]
    Ag, bg = A.assemble([a for a, _ in Ak], [b for _, b in Ak], glob, n)
    return nu, glob, n, cells_out, Ag, bg


@pytest.mark.parametrize("p", [1, 2])
def test_global_solve_recovers_exact_solution(p):
    nu, glob, n, cells, Ag, bg = _manufactured_global(p)
    t, it, hist = A.cg(Ag, bg, 1e-12, 20 * n)
    assert hist[-1] <= 1e-12, (it, hist[-1])
    scale = max(np.abs(c["x"]).max() for c in cells)
    for c, g in zip(cells, glob):
        tK = A.scatter(t, g)
        keep = g >= 0
        # the exact traces, where kept (removed ones are not unknowns)
        assert np.abs(tK[keep] - c["x"][nu:][keep]).max() <= 1e-8 * scale
        x = A.reconstruct(c["K"], c["le"], nu, c["x"][nu:] * keep)
        assert np.abs(x[:nu] - c["x"][:nu]).max() <= 1e-9 * scale
        xr = A.reconstruct(c["K"], c["le"], nu, tK)
        assert np.abs(xr[:nu] - c["x"][:nu]).max() <= 1e-7 * scale
        _, _, eta = O.local_solve(c["G"], c["Bf"], c["l"], xr)
        _, _, eta0 = O.local_solve(c["G"], c["Bf"], c["l"], 0 * xr)
        assert eta <= 1e-8 * eta0, (eta, eta0)


def test_reconstruction_planted_sign_fails(monkeypatch):
    def bad(K, le, nu, t_local):
        u = np.linalg.solve(K[:nu, :nu], le[:nu] + K[:nu, nu:] @ t_local)
        return np.concatenate([u, t_local])
    monkeypatch.setattr(A, "reconstruct", bad)
    with pytest.raises(AssertionError):
        test_global_solve_recovers_exact_solution(1)
