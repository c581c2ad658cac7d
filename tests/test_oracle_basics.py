"""Pins of the oracle's building blocks against closed forms, library special
cases and numbers printed in the paper (tests/golden/paper_values.json)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import dpg_oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_legendre_exact_on_monomials(n):
    x, w = O.gauss_legendre_01(n)
    for k in range(2 * n):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-14
    # special case of a library routine: numpy's Gauss-Legendre on [-1,1]
    t, v = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, 0.5 * (t + 1), atol=1e-15) and np.allclose(w, 0.5 * v, atol=1e-15)


def test_gauss_lobatto_closed_forms():
    assert np.allclose(O.gauss_lobatto_nodes_01(2), [0, 1])
    assert np.allclose(O.gauss_lobatto_nodes_01(3), [0, 0.5, 1])
    s5 = 1 / math.sqrt(5)
    assert np.allclose(O.gauss_lobatto_nodes_01(4), [0, (1 - s5) / 2, (1 + s5) / 2, 1], atol=1e-15)
    s37 = math.sqrt(3 / 7)
    assert np.allclose(O.gauss_lobatto_nodes_01(5), [0, (1 - s37) / 2, 0.5, (1 + s37) / 2, 1], atol=1e-15)


def test_onb_legendre_against_closed_forms():
    """Orthonormality and the classical derivative integrals
    int P_m' P_n = 2 [n<m, m+n odd], int P_m' P_n' = min(m,n)(min+1) [m+n even]."""
    x, w = O.gauss_legendre_01(12)
    v, d = O.onb_legendre(6, x)
    assert np.allclose((v * w) @ v.T, np.eye(7), atol=1e-13)
    for m in range(7):
        for n in range(7):
            c = math.sqrt((2 * m + 1) * (2 * n + 1))
            i10 = c * (2.0 if (n < m and (m + n) % 2 == 1) else 0.0)
            mn = min(m, n)
            i11 = 2 * c * (mn * (mn + 1) if (m + n) % 2 == 0 else 0.0)
            assert abs(np.dot(w, d[m] * v[n]) - i10) < 1e-11
            assert abs(np.dot(w, d[m] * d[n]) - i11) < 1e-10
    assert np.allclose(O.onb_legendre(4, np.array(0.0))[0], [math.sqrt(2 * k + 1) * (-1) ** k for k in range(5)])


def test_bubbles_vanish_and_lagrange_nodal():
    for m in range(2, 6):
        assert abs(O.lobatto_bubble(m, np.array(0.0))) < 1e-15
        assert abs(O.lobatto_bubble(m, np.array(1.0))) < 1e-15
    for p in range(1, 5):
        z = O.gauss_lobatto_nodes_01(p + 1)
        assert np.allclose(O.lagrange_gll(p, z), np.eye(p + 1), atol=1e-13)


# ---------------------------------------------------------------- spaces
@pytest.mark.parametrize("p,dp", [(1, 1), (2, 1), (3, 1), (4, 1), (4, 2)])
def test_space_dimensions(p, dp):
    s, r = p + dp + 1, p + 1
    N, nv, nu, nt = O.dims(p, dp)
    assert N == len(O.test_index_list(s)) == 3 * s * (s + 1) ** 2
    assert nu == 6 * (p + 1) ** 3 and nt == 24 * r * r
    assert len(O.trace_index_list(r)) == 12 * r * r


def test_global_dof_counts_printed_in_paper():
    g = GOLD["waveguide_coarse_dofs"]
    nx, ny, nz = g["mesh"]
    assert g["real_fields"] * O.nedelec_global_dofs(nx, ny, nz, g["trial_degree"] + 1) == g["value"]
    g = GOLD["waveguide_finest_dofs"]
    n = g["real_fields"] * O.nedelec_global_dofs(*g["mesh"], g["trial_degree"] + 1)
    assert float(f"{n:.{g['significant_digits']}g}") == g["value"]
    # p = 3 at level 3 (8x8x32) vs p = 1 at level 5 (32x32x128): "about eight times"
    r3 = 4 * O.nedelec_global_dofs(8, 8, 32, 4)
    r1 = 4 * O.nedelec_global_dofs(32, 32, 128, 2)
    assert round(r1 / r3) == GOLD["dof_ratio_p3_level3_vs_p1_level5"]["approx"]
    d = GOLD["dg_cell_dofs"]
    assert O.trial_basis_ref(3, np.zeros((1, 3))).shape[0] == d["p3_cell"]
    assert 64 * O.trial_basis_ref(1, np.zeros((1, 3))).shape[0] == d["p1_cell_refined_twice"]


def test_test_space_contains_gradients_and_is_nedelec():
    """The first-kind Nedelec space of FEEC index s contains grad Q_s: check that
    the gradient of a random Q_s polynomial is reproduced by the test basis."""
    s = 3
    rng = np.random.default_rng(0)
    pts = rng.uniform(size=(80, 3))
    coef = rng.standard_normal((s + 1, s + 1, s + 1))
    v = [O.onb_legendre(s, pts[:, a]) for a in range(3)]
    grad = np.zeros((80, 3))
    for i in range(s + 1):
        for j in range(s + 1):
            for k in range(s + 1):
                c = coef[i, j, k]
                grad[:, 0] += c * v[0][1][i] * v[1][0][j] * v[2][0][k]
                grad[:, 1] += c * v[0][0][i] * v[1][1][j] * v[2][0][k]
                grad[:, 2] += c * v[0][0][i] * v[1][0][j] * v[2][1][k]
    val, curl = O.test_basis_ref(s, pts)
    A = val.transpose(1, 2, 0).reshape(-1, val.shape[0])
    c, res, *_ = np.linalg.lstsq(A, grad.ravel(), rcond=None)
    assert np.linalg.norm(A @ c - grad.ravel()) < 1e-10 * np.linalg.norm(grad)
    # ... and the curl of that combination vanishes
    C = curl.transpose(1, 2, 0).reshape(-1, val.shape[0])
    assert np.linalg.norm(C @ c) < 1e-9 * np.linalg.norm(grad)


# ---------------------------------------------------------------- geometry
def _perturbed_cell(rng, amp=0.15, affine=False):
    base = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], float)
    if affine:
        A = np.eye(3) + amp * rng.standard_normal((3, 3))
        if np.linalg.det(A) < 0:
            A[:, 0] *= -1
        return base @ A.T + rng.standard_normal(3)
    return base * np.array([0.7, 1.1, 0.9]) + amp * rng.uniform(-1, 1, size=(8, 3))


@pytest.mark.parametrize("seed", range(4))
def test_volume_by_divergence_theorem(seed):
    """int det J equals (1/3) sum_faces int x.n dS, both exact for trilinear cells
    (checks face normals' orientation and area elements against det J)."""
    X = _perturbed_cell(np.random.default_rng(seed))
    pts, w = O.volume_rule(3)
    _, J = O.trilinear_map(X, pts)
    vol = np.dot(w, np.linalg.det(J))
    flux = 0.0
    for f in range(6):
        fp, fw = O.face_rule(3, f)
        x, _, n, dS = O.face_geometry(X, f, fp)
        flux += np.dot(fw * dS, np.einsum('qa,qa->q', x, n)) / 3.0
    assert abs(vol - flux) < 1e-13 * vol
    Xa = _perturbed_cell(np.random.default_rng(seed), affine=True)
    _, J = O.trilinear_map(Xa, pts)
    A = np.stack([Xa[1] - Xa[0], Xa[2] - Xa[0], Xa[4] - Xa[0]], axis=1)
    assert abs(np.dot(w, np.linalg.det(J)) - np.linalg.det(A)) < 1e-13


def test_outward_normals():
    X = _perturbed_cell(np.random.default_rng(5))
    cen = X.mean(axis=0)
    for f in range(6):
        fp, _ = O.face_rule(3, f)
        x, _, n, _ = O.face_geometry(X, f, fp)
        assert np.all(np.einsum('qa,qa->q', x - cen, n) > 0)


def test_trace_tangential_conformity_across_shared_face():
    """Two trilinear cells sharing the face x+ / x-: the tangential traces of the
    shared edge and face functions agree pointwise from both sides, and every
    other trace function has zero tangential trace on that face."""
    rng = np.random.default_rng(3)
    base = np.array([[i, j, k] for k in (0, 1) for j in (0, 1) for i in (0, 1)], float)
    grid = {}
    for i in range(3):
        for j in range(2):
            for k in range(2):
                grid[(i, j, k)] = np.array([i, j, k], float) + (0.12 * rng.uniform(-1, 1, 3) if i == 1 else 0)
    XA = np.array([grid[(i, j, k)] for k in (0, 1) for j in (0, 1) for i in (0, 1)])
    XB = np.array([grid[(i + 1, j, k)] for k in (0, 1) for j in (0, 1) for i in (0, 1)])
    for r in (1, 2, 3):
        idx = O.trace_index_list(r)
        pa, _ = O.face_rule(4, 1)
        pb, _ = O.face_rule(4, 0)
        xa, Ja, na, _ = O.face_geometry(XA, 1, pa)
        xb, Jb, nb, _ = O.face_geometry(XB, 0, pb)
        assert np.allclose(xa, xb, atol=1e-14) and np.allclose(na, -nb, atol=1e-14)
        ta = np.cross(na[None], np.einsum('qba,nqb->nqa', np.linalg.inv(Ja), O.trace_basis_ref(r, pa)))
        tb = np.cross(na[None], np.einsum('qba,nqb->nqa', np.linalg.inv(Jb), O.trace_basis_ref(r, pb)))
        matched = 0
        for n_, (a, i, (bax, bk), (cax, ck)) in enumerate(idx):
            on_face_a = (bax == 0 and bk == ('v', 1)) or (cax == 0 and ck == ('v', 1))
            if not on_face_a:
                assert np.abs(ta[n_]).max() < 1e-13
                continue
            key = (a, i, (bax, ('v', 0) if bax == 0 else bk), (cax, ('v', 0) if cax == 0 else ck))
            m_ = idx.index(key)
            assert np.abs(ta[n_] - tb[m_]).max() < 1e-12
            matched += 1
        assert matched == 4 * r + 2 * r * (r - 1)      # 4 edges + 1 face of the shared face


# ---------------------------------------------------------------- port data
def test_port_admittance_printed_in_paper():
    g = GOLD["wr430_port_admittance"]
    om = O.omega_dimensionless(g["freq_hz"])
    pm = O.PortMode(g["a_m"], g["b_m"], *g["mode"], om)
    # agreement to 5e-11 relative: the printed value carries the rounding of
    # the constants used to form omega; any formula error is far larger
    assert abs(pm.zinv() - g["value"]) < 1e-10 * g["value"]
    f = GOLD["fichera_frequency"]
    assert abs(O.omega_dimensionless(f["freq_hz"]) - f["omega"]) < 1e-8
    w = GOLD["waveguide_wavenumber"]
    assert round(O.omega_dimensionless(w["freq_hz"]) / math.pi) == w["approx_over_pi"]


def test_te_mode_solves_maxwell_and_outlet_condition():
    """Central differences of the TE_mn fields: curl E - i w mu H = 0 and
    curl H + i w eps E = 0; the outlet Robin datum of the travelling mode is 0."""
    om = O.omega_dimensionless(2.45e9)
    for (m, n, eps, mu) in [(1, 0, 1.0, 1.0), (1, 1, 2.0 + 0.3j, 1.2), (2, 1, 1.5, 1.0 + 0.1j)]:
        pm = O.PortMode(0.25, 0.2, m, n, om, eps, mu)
        rng = np.random.default_rng(m + n)
        x = rng.uniform(0, 0.2, size=(10, 3))
        h = 1e-6

        def curl(fun):
            c = np.zeros((10, 3), complex)
            d = []
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                d.append((fun(x + e) - fun(x - e)) / (2 * h))
            c[:, 0] = d[1][:, 2] - d[2][:, 1]
            c[:, 1] = d[2][:, 0] - d[0][:, 2]
            c[:, 2] = d[0][:, 1] - d[1][:, 0]
            return c
        E, H = pm.fields(x)
        sc = np.abs(om * mu * H).max()
        assert np.abs(curl(lambda y: pm.fields(y)[0]) - 1j * om * mu * H).max() < 1e-6 * sc
        assert np.abs(curl(lambda y: pm.fields(y)[1]) + 1j * om * eps * E).max() < 1e-6 * sc
        nrm = np.tile([0, 0, 1.0], (10, 1))
        assert np.abs(pm.robin_data(x, nrm, pm.zinv())).max() < 1e-12 * sc
