"""Pins of the oracle's local forms G, B_f, l and of its local solve.

* G on axis-aligned boxes against a closed form built from exact 1D Legendre
  integrals (no quadrature), through the block form of the adjoint graph
  inner product -- an independent route from the oracle's pointwise one.
* B_f and l against an exact polynomial manufactured solution: with E of total
  degree <= p, H = curl E / (i w mu), J = curl H + i w eps E and Robin data
  g = n x H + Z^{-1} n x (E x n), the discrete residual B_f x_exact - l vanishes
  for every test function on affine cells (integration by parts, §2.2).
* K_e: Hermitian positive semidefinite with the null space left by the Robin
  faces (§2.3, unconstrained H-hat DOFs); LU and Cholesky routes agree; the
  FP64 solve agrees with an extended-precision elimination; eta, K_e and l_e
  satisfy eta^2 = x^H K x - 2 Re(x^H l_e) + l^H G^{-1} l.
"""
import math

import numpy as np
import pytest
import sympy as sp

from oracle import dpg_oracle as O


# ------------------------------------------------------------------ box G
def _eps3(a, b, c):
    return (a - b) * (b - c) * (c - a) / 2


def _test_enum(s):
    out = []
    for a in range(3):
        hi = [s, s, s]
        hi[a] = s - 1
        for d2 in range(hi[2] + 1):
            for d1 in range(hi[1] + 1):
                for d0 in range(hi[0] + 1):
                    out.append((a, (d0, d1, d2)))
    return out


def _i1d(m, n, dm, dn):
    c = math.sqrt((2 * m + 1) * (2 * n + 1))
    if dm == 0 and dn == 0:
        return 1.0 if m == n else 0.0
    if dm == 1 and dn == 0:
        return c * 2.0 if (n < m and (m + n) % 2 == 1) else 0.0
    if dm == 0 and dn == 1:
        return _i1d(n, m, 1, 0)
    k = min(m, n)
    return 2.0 * c * k * (k + 1) if (m + n) % 2 == 0 else 0.0


def _pend(m, side):
    return math.sqrt(2 * m + 1) * (1.0 if side else (-1.0) ** m)


def box_gram_closed_form(h, s, om, eps, mu, alpha, robin):
    """Closed-form G for the box [0,hx]x[0,hy]x[0,hz] (J = diag h) in the
    orthonormal Legendre Nedelec basis: block algebra of the adjoint graph
    inner product with M, S, C and the Robin face matrices from exact 1D
    integrals."""
    idx = _test_enum(s)
    N = len(idx)
    V = h[0] * h[1] * h[2]
    M = np.zeros((N, N)); S = np.zeros((N, N)); C = np.zeros((N, N))
    face = {f: (np.zeros((N, N)), np.zeros((N, N))) for f in robin}
    for i, (ai, di) in enumerate(idx):
        for j, (aj, dj) in enumerate(idx):
            if ai == aj and di == dj:
                M[i, j] = V / h[ai] ** 2
            # S_ij = sum_b h_b^2 / V int chat_ib chat_jb ; chat_b = sum_c eps(b,c,a) d_c f
            sv = 0.0
            for b in range(3):
                for c in range(3):
                    e1 = _eps3(b, c, ai)
                    if e1 == 0:
                        continue
                    for c2 in range(3):
                        e2 = _eps3(b, c2, aj)
                        if e2 == 0:
                            continue
                        sv += h[b] ** 2 / V * e1 * e2 * np.prod(
                            [_i1d(di[x], dj[x], int(x == c), int(x == c2)) for x in range(3)])
            S[i, j] = sv
            # C_ij = int curl psi_i . psi_j = sum_c eps(a_j, c, a_i) int d_c f_i f_j
            C[i, j] = sum(_eps3(aj, c, ai) * np.prod([_i1d(di[x], dj[x], int(x == c), 0) for x in range(3)])
                          for c in range(3))
            for f in robin:
                nax, side = f // 2, f % 2
                tr = np.prod([_i1d(di[x], dj[x], 0, 0) for x in range(3) if x != nax]) \
                    * _pend(di[nax], side) * _pend(dj[nax], side) * V / h[nax]
                Mt, Xt = face[f]
                if ai == aj and ai != nax:
                    Mt[i, j] = tr / h[ai] ** 2
                Xt[i, j] = (2 * side - 1) * _eps3(ai, nax, aj) * tr / (h[ai] * h[aj])
    GFF = S + (om ** 2 * abs(eps) ** 2 + alpha) * M
    GII = S + (om ** 2 * abs(mu) ** 2 + alpha) * M
    GFI = 1j * om * np.conj(mu) * C + 1j * om * eps * C.T
    for f, z in robin.items():
        Mt, Xt = face[f]
        GFF = GFF + abs(z) ** 2 * Mt
        GII = GII + Mt
        GFI = GFI + z * Xt
    return np.block([[GFF, GFI], [np.conj(GFI).T, GII]])


@pytest.mark.parametrize("p,dp", [(1, 1), (2, 1)])
def test_gram_on_box_matches_closed_form(p, dp):
    h = np.array([0.3, 0.5, 0.7])
    X = np.array([[i * h[0], j * h[1], k * h[2]] for k in (0, 1) for j in (0, 1) for i in (0, 1)])
    om, eps, mu, alpha = 7.3, 3.0 + 0.8j, 1.4 + 0.2j, 0.7
    robin = {4: 0.8 - 0.3j, 1: 0.5 + 0.25j}
    fk = [0] * 6
    zi = [0j] * 6
    for f, z in robin.items():
        fk[f] = O.FACE_ROBIN0
        zi[f] = z
    cp = O.CellProblem(X=X, p=p, dp=dp, eps=eps, mu=mu, omega=om, face_kind=fk, zinv=zi, alpha=alpha)
    G, _, _ = O.cell_forms(cp)
    Gc = box_gram_closed_form(h, p + dp + 1, om, eps, mu, alpha, robin)
    assert np.abs(G - Gc).max() < 1e-12 * np.abs(Gc).max()
    assert np.abs(G - np.conj(G).T).max() < 1e-13 * np.abs(G).max()


def test_gram_positive_definite_and_translation_invariant():
    rng = np.random.default_rng(1)
    X = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], float) * 0.1
    X = X + 0.012 * rng.uniform(-1, 1, X.shape)
    kw = dict(p=1, dp=1, eps=2 + 0.4j, mu=1.0, omega=30.0, face_kind=(0, 0, 0, 0, 3, 0), zinv=(0, 0, 0, 0, 0.7, 0))
    G1, B1, _ = O.cell_forms(O.CellProblem(X=X, **kw))
    G2, B2, _ = O.cell_forms(O.CellProblem(X=X + np.array([3.0, -2.0, 5.0]), **kw))
    assert np.linalg.eigvalsh(G1).min() > 0
    assert np.abs(G1 - G2).max() < 1e-11 * np.abs(G1).max()
    assert np.abs(B1 - B2).max() < 1e-11 * np.abs(B1).max()


# ------------------------------------------------------ manufactured solution
def _manufactured(p, om, eps, mu, seed):
    x, y, z = sp.symbols('x y z')
    rng = np.random.default_rng(seed)
    mons = [x ** a * y ** b * z ** c for a in range(p + 1) for b in range(p + 1) for c in range(p + 1)
            if a + b + c <= p]
    E = [sum((rng.standard_normal() + 1j * rng.standard_normal()) * m for m in mons) for _ in range(3)]

    def curl(F):
        return [sp.diff(F[2], y) - sp.diff(F[1], z), sp.diff(F[0], z) - sp.diff(F[2], x),
                sp.diff(F[1], x) - sp.diff(F[0], y)]
    H = [sp.expand(c / (sp.I * om * mu)) for c in curl(E)]
    Jv = [sp.expand(a + sp.I * om * eps * b) for a, b in zip(curl(H), E)]

    def vec(F):
        fs = [sp.lambdify((x, y, z), c, 'numpy') for c in F]

        def ev(P):
            P = np.asarray(P, float)
            return np.stack([np.broadcast_to(np.asarray(f(P[:, 0], P[:, 1], P[:, 2]), complex), (P.shape[0],))
                             for f in fs], axis=1)
        return ev
    return vec(E), vec(H), vec(Jv)


def _affine_cell(seed):
    rng = np.random.default_rng(seed)
    A = np.diag([0.09, 0.07, 0.11]) + 0.02 * rng.standard_normal((3, 3))
    base = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], float)
    return base @ A.T + np.array([0.02, -0.01, 0.03])


@pytest.mark.parametrize("p,dp", [(1, 1), (2, 1), (3, 1), (2, 2)])
def test_manufactured_solution_residual_vanishes(p, dp):
    om, eps, mu = 23.0, 2.5 + 0.7j, 1.3 - 0.1j
    Ef, Hf, Jf = _manufactured(p, om, eps, mu, seed=p + 10 * dp)
    X = _affine_cell(p)
    fk = (O.FACE_PEC, O.FACE_ROBIN0, 0, 0, O.FACE_PORT, O.FACE_ROBIN0)
    zi = (0, 0.6 + 0.2j, 0, 0, 0.83 - 0.1j, 1.1 + 0.4j)

    def g(f, xx, n):
        E, H = Ef(xx), Hf(xx)
        return np.cross(n, H) + zi[f] * np.cross(n, np.cross(E, n))
    cp = O.CellProblem(X=X, p=p, dp=dp, eps=eps, mu=mu, omega=om, face_kind=fk, zinv=zi,
                       J_src=Jf, g_src=g)
    G, Bf, l = O.cell_forms(cp)
    xe = O.projected_solution(X, p, Ef, Hf)
    r = Bf @ xe - l
    scale = np.linalg.norm(Bf @ xe) + np.linalg.norm(l)
    assert np.linalg.norm(r) < 1e-11 * scale
    # eta of the exact solution vanishes as well
    _, _, eta = O.local_solve(G, Bf, l, xe)
    K, le, _ = O.local_solve(G, Bf, l, None)
    assert eta < 1e-9 * math.sqrt(abs(np.real(np.conj(xe) @ K @ xe)))


@pytest.mark.parametrize("flip", ["conj_eps", "sign_trace", "robin_sign"])
def test_manufactured_solution_detects_planted_mistakes(flip, monkeypatch):
    """A plausible mistake planted in the oracle (on the CPU) breaks the identity."""
    p, dp = 1, 1
    om, eps, mu = 23.0, 2.5 + 0.7j, 1.3 - 0.1j
    Ef, Hf, Jf = _manufactured(p, om, eps, mu, seed=3)
    X = _affine_cell(5)
    fk = (0, 0, 0, 0, O.FACE_ROBIN0, 0)
    zi = (0, 0, 0, 0, 0.83 - 0.1j, 0)

    def g(f, xx, n):
        E, H = Ef(xx), Hf(xx)
        return np.cross(n, H) + zi[f] * np.cross(n, np.cross(E, n))
    e2, z2 = eps, list(zi)
    if flip == "conj_eps":
        e2 = np.conj(eps)
    elif flip == "robin_sign":
        z2[4] = -zi[4]
    cp = O.CellProblem(X=X, p=p, dp=dp, eps=e2, mu=mu, omega=om, face_kind=fk, zinv=z2, J_src=Jf, g_src=g)
    if flip == "sign_trace":
        real_cross = np.cross
        monkeypatch.setattr(O.np, "cross", lambda a, b, *k, **kw: real_cross(b, a, *k, **kw))
    G, Bf, l = O.cell_forms(cp)
    if flip == "sign_trace":
        monkeypatch.undo()
    xe = O.projected_solution(X, p, Ef, Hf)
    r = Bf @ xe - l
    assert np.linalg.norm(r) > 1e-4 * (np.linalg.norm(Bf @ xe) + np.linalg.norm(l))


# ------------------------------------------------------------- local solve
def _cell(seed, p=1, dp=1, robin=((4, 0.79),)):
    rng = np.random.default_rng(seed)
    X = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], float) * 0.05
    X = X + 0.004 * rng.uniform(-1, 1, X.shape)
    fk = [0] * 6
    zi = [0j] * 6
    for f, z in robin:
        fk[f] = O.FACE_ROBIN0
        zi[f] = z
    om = O.omega_dimensionless(2.45e9)
    return O.CellProblem(X=X, p=p, dp=dp, eps=3.0 + 0.6j, mu=1.0, omega=om, face_kind=fk, zinv=zi)


@pytest.mark.parametrize("p,robin,nullity", [
    (1, ((4, 0.79),), 4),
    (2, ((4, 0.79), (5, 0.79)), 24),
    (2, ((4, 0.79), (1, 0.6)), 27),       # faces z- and x+ share an edge: + r
    (1, (), 0),
])
def test_Ke_hermitian_psd_with_robin_null_space(p, robin, nullity):
    G, Bf, l = O.cell_forms(_cell(p, p=p, robin=robin))
    K, le, _ = O.local_solve(G, Bf, l)
    # the LU route is Hermitian up to the solve's accuracy, ~ kappa(D G D) * u
    assert np.abs(K - np.conj(K).T).max() < 1e-10 * np.abs(K).max()
    ev = np.linalg.eigvalsh(0.5 * (K + np.conj(K).T))
    tol = 1e-12 * ev.max()
    assert ev.min() > -tol
    assert int(np.sum(ev < tol)) == nullity
    zero_cols = np.where(np.abs(Bf).max(axis=0) < 1e-13 * np.abs(Bf).max())[0]
    assert len(zero_cols) == nullity


def test_lu_and_cholesky_routes_agree():
    cp = _cell(11, p=2)
    cp.port = O.PortMode(0.1, 0.1, 1, 0, cp.omega)
    cp.face_kind = (0, 0, 0, 0, O.FACE_PORT, 0)
    G, Bf, l = O.cell_forms(cp)
    x = np.random.default_rng(0).standard_normal(Bf.shape[1]) * (1 + 0.5j)
    K1, l1, e1 = O.local_solve(G, Bf, l, x)
    K2, l2, e2 = O.local_solve_cholesky(G, Bf, l, x)
    assert np.linalg.norm(K1 - K2) < 1e-10 * np.linalg.norm(K1)
    assert np.linalg.norm(l1 - l2) < 1e-10 * np.linalg.norm(l1)
    assert abs(e1 - e2) < 1e-10 * e1


def _elim_extended(G, R):
    """Gaussian elimination with partial pivoting in extended precision (x87
    long double, ~19 digits), vectorised over rows."""
    A = np.concatenate([G, R], axis=1).astype(np.clongdouble)
    n = G.shape[0]
    for c in range(n):
        piv = c + int(np.argmax(np.abs(A[c:, c])))
        if piv != c:
            A[[c, piv]] = A[[piv, c]]
        A[c + 1:, c:] -= np.outer(A[c + 1:, c] / A[c, c], A[c, c:])
    X = np.zeros((n, R.shape[1]), dtype=np.clongdouble)
    for c in range(n - 1, -1, -1):
        X[c] = (A[c, n:] - A[c, c + 1:n] @ X[c + 1:]) / A[c, c]
    return X


def test_fp64_solve_against_extended_precision():
    if np.finfo(np.longdouble).eps > 1e-18:
        pytest.skip("no extended precision long double on this host")
    cp = _cell(2, p=1)
    cp.port = O.PortMode(0.1, 0.1, 1, 0, cp.omega)
    cp.face_kind = (0, 0, 0, 0, O.FACE_PORT, 0)
    G, Bf, l = O.cell_forms(cp)
    K, le, _ = O.local_solve(G, Bf, l)
    X = _elim_extended(G, np.concatenate([Bf, l[:, None]], axis=1))
    Bh = np.conj(Bf).T.astype(np.clongdouble)
    Kx = (Bh @ X[:, :-1]).astype(np.complex128)
    lx = (Bh @ X[:, -1]).astype(np.complex128)
    d = 1 / np.sqrt(np.real(np.diag(G)))
    kappa = np.linalg.cond(G * d[:, None] * d[None, :])
    assert np.linalg.norm(K - Kx) < 50 * kappa * 1e-16 * np.linalg.norm(Kx)
    assert np.linalg.norm(le - lx) < 50 * kappa * 1e-16 * np.linalg.norm(lx)


def test_eta_expansion_identity():
    cp = _cell(4, p=2, robin=((4, 0.79),))
    cp.port = O.PortMode(0.1, 0.1, 1, 0, cp.omega)
    cp.face_kind = (0, 0, 0, 0, O.FACE_PORT, 0)
    G, Bf, l = O.cell_forms(cp)
    x = np.random.default_rng(9).standard_normal(Bf.shape[1]) + 1j * np.random.default_rng(8).standard_normal(Bf.shape[1])
    K, le, eta = O.local_solve(G, Bf, l, x)
    lGl = np.real(np.conj(l) @ np.linalg.solve(G, l))
    e2 = np.real(np.conj(x) @ K @ x) - 2 * np.real(np.conj(x) @ le) + lGl
    assert abs(eta ** 2 - e2) < 1e-9 * (np.real(np.conj(x) @ K @ x) + lGl)


def test_degenerate_cell_reports_info():
    cp = _cell(0)
    X = cp.X.copy()
    X[[0, 1]] = X[[1, 0]]          # inverted: det J < 0
    cp.X = X
    assert O.solve_cell(cp)["info"] == -1
