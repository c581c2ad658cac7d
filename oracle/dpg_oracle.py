"""Plain FP64 CPU oracle for the DPG per-cell local solve of the ultraweak
time-harmonic Maxwell system (Marquis, Maier, Blais, arXiv 2609.03155).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product path
(the HIP library and its Python binding) never calls it, and shares no code,
tables or constants with it.

What it computes, per hexahedral cell K (all complex, FP64):

* G   = [(psi_i, psi_j)_V]                 test-space Gram matrix, §2.2 adjoint
                                            graph inner product (eq. test_inner_product)
* B_f = [b_h(psi_i, phi_j) | <psi_i, phihat_j>_h]
                                            §2.2 ultraweak bilinear form and trace
                                            pairing; entries as in §2.3
* l   = [l_h(psi_i)]                         §2.2 linear form
* K_e = B_f^H G^{-1} B_f,  l_e = B_f^H G^{-1} l       §2.3, elimination of Psi
* eta = ||Psi||_V = sqrt(r^H G^{-1} r),  r = B_f x - l  §2.3, error representation

The forms are evaluated *directly from their definitions*: every test, trial and
trace function is mapped to the physical cell and the integrands of §2.2 are
formed pointwise at Gauss points, with conjugation in the first argument.
No block decomposition of G or B is used here; the solve is the plain
definition X = G^{-1}[B_f l] via LU (numpy.linalg.solve), with a Cholesky route
offered only as a cross-check.

Readings of points the paper leaves open:
  * spaces (§2.3): trial E,H = discontinuous tensor Lagrange of degree p per
    Cartesian component at Gauss-Lobatto nodes; trace = tangential traces of
    first-kind Nedelec functions of FEEC index r=p+1 with interior functions
    dropped (12 r^2 per field); test = first-kind Nedelec of FEEC index
    s = p+dp+1 (3 s (s+1)^2 per field).  Pinned by the DOF counts the paper
    prints for the waveguide meshes (§4.1) and the 64-DOF p=3 cell.
  * test basis: tensor products of L2-orthonormal shifted Legendre
    polynomials; K_e, l_e and eta do not depend on this choice.
  * trace basis: hierarchical -- orthonormal Legendre along the component
    direction times {1-xi, xi, normalised integrated-Legendre bubbles}.
  * quadrature: Gauss-Legendre with n1 = p+dp+2 points per direction.
  * non-dimensional units with reference length L = 1 m (App. A).
  * conjugation in the first argument of every form (§2.1, §2.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

# Speed of light in vacuum (exact SI value) used by the non-dimensional
# frequency of App. A: omega = L * omega_dim / c0.
SPEED_OF_LIGHT = 299_792_458.0

FACE_INTERIOR = 0   # interior skeleton face (trace pairing only)
FACE_PEC = 1        # n x E = 0, imposed on the global trace DOFs, not locally
FACE_PORT = 2       # Robin face with g from the TE_mn port mode
FACE_ROBIN0 = 3     # Robin face with g = 0 (impedance outlet)


# --------------------------------------------------------------------------
# App. A: non-dimensional frequency
# --------------------------------------------------------------------------
def omega_dimensionless(freq_hz: float, length_m: float = 1.0) -> float:
    """App. A: omega = L * (2 pi f) / c0."""
    return 2.0 * math.pi * freq_hz * length_m / SPEED_OF_LIGHT


# --------------------------------------------------------------------------
# 1D polynomials and quadrature
# --------------------------------------------------------------------------
def legendre_table(nmax: int, t):
    """Legendre P_0..P_nmax on [-1,1] and their first derivatives, by Bonnet's
    three-term recurrence.  Returns arrays of shape (nmax+1,) + t.shape."""
    t = np.asarray(t, dtype=np.float64)
    P = np.zeros((nmax + 1,) + t.shape)
    dP = np.zeros_like(P)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = t
        dP[1] = 1.0
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * t * P[n] - n * P[n - 1]) / (n + 1)
        dP[n + 1] = dP[n - 1] + (2 * n + 1) * P[n]
    return P, dP


def gauss_legendre_01(n: int):
    """n-point Gauss-Legendre rule on [0,1]: Newton iteration on P_n."""
    x = np.cos(np.pi * (np.arange(1, n + 1) - 0.25) / (n + 0.5))
    for _ in range(100):
        P, dP = legendre_table(n, x)
        dx = P[n] / dP[n]
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    P, dP = legendre_table(n, x)
    w = 2.0 / ((1.0 - x * x) * dP[n] ** 2)
    order = np.argsort(x)
    return 0.5 * (x[order] + 1.0), 0.5 * w[order]


def gauss_lobatto_nodes_01(n: int):
    """n Gauss-Lobatto nodes on [0,1] (endpoints plus the roots of P'_{n-1})."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs n >= 2")
    m = n - 1
    x = np.cos(np.pi * np.arange(n) / m)          # Chebyshev-Lobatto start
    inner = x[1:-1].copy()
    for _ in range(100):
        P, dP = legendre_table(m, inner)
        # P''_m from the Legendre ODE: (1-t^2) P'' = 2 t P' - m(m+1) P
        d2P = (2 * inner * dP[m] - m * (m + 1) * P[m]) / (1.0 - inner ** 2)
        dx = dP[m] / d2P
        inner = inner - dx
        if inner.size == 0 or np.max(np.abs(dx)) < 1e-16:
            break
    x = np.concatenate([[-1.0], np.sort(inner), [1.0]])
    return 0.5 * (x + 1.0)


def onb_legendre(nmax: int, xi):
    """L2([0,1])-orthonormal shifted Legendre p_n(xi) = sqrt(2n+1) P_n(2xi-1),
    n = 0..nmax, with derivatives d/dxi."""
    P, dP = legendre_table(nmax, 2.0 * np.asarray(xi) - 1.0)
    sc = np.sqrt(2.0 * np.arange(nmax + 1) + 1.0).reshape((-1,) + (1,) * np.ndim(xi))
    return sc * P, 2.0 * sc * dP


def lobatto_bubble(m: int, xi):
    """Normalised integrated Legendre bubble of degree m >= 2 on [0,1]:
    (P_m(2xi-1) - P_{m-2}(2xi-1)) / sqrt(2(2m-1)); vanishes at xi = 0 and 1."""
    P, _ = legendre_table(m, 2.0 * np.asarray(xi) - 1.0)
    return (P[m] - P[m - 2]) / math.sqrt(2.0 * (2 * m - 1))


def lagrange_gll(p: int, xi):
    """Lagrange polynomials of degree p at the p+1 Gauss-Lobatto nodes."""
    z = gauss_lobatto_nodes_01(p + 1)
    xi = np.asarray(xi, dtype=np.float64)
    out = np.ones((p + 1,) + xi.shape)
    for i in range(p + 1):
        for j in range(p + 1):
            if j != i:
                out[i] = out[i] * (xi - z[j]) / (z[i] - z[j])
    return out


# --------------------------------------------------------------------------
# Space dimensions (§2.3; FEEC indices as read from the DOF counts of §4.1)
# --------------------------------------------------------------------------
def dims(p: int, dp: int):
    """Returns (N, n_test, n_interior, n_trace): N test functions per field,
    n_test = 2N (F and I), n_interior = 6 (p+1)^3 (E and H), n_trace = 24 (p+1)^2."""
    s = p + dp + 1
    r = p + 1
    N = 3 * s * (s + 1) ** 2
    return N, 2 * N, 6 * (p + 1) ** 3, 24 * r * r


def nedelec_global_dofs(nx: int, ny: int, nz: int, r: int) -> int:
    """Number of first-kind Nedelec DOFs of FEEC index r on an nx x ny x nz hex
    mesh, counting edge (r each), face (2r(r-1) each) and cell-interior
    (3 r (r-1)^2 each) functions."""
    edges = nx * (ny + 1) * (nz + 1) + (nx + 1) * ny * (nz + 1) + (nx + 1) * (ny + 1) * nz
    faces = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)
    cells = nx * ny * nz
    return edges * r + faces * 2 * r * (r - 1) + cells * 3 * r * (r - 1) ** 2


# --------------------------------------------------------------------------
# Reference basis functions on [0,1]^3
# --------------------------------------------------------------------------
def test_index_list(s: int):
    """(component, (d0,d1,d2)) for the 3 s (s+1)^2 first-kind Nedelec test
    functions of FEEC index s: component a has degree <= s-1 along axis a and
    <= s along the other two.  Ordering: component-major, then x-degree
    fastest, then y, then z."""
    out = []
    for a in range(3):
        hi = [s, s, s]
        hi[a] = s - 1
        for d2 in range(hi[2] + 1):
            for d1 in range(hi[1] + 1):
                for d0 in range(hi[0] + 1):
                    out.append((a, (d0, d1, d2)))
    return out


def test_basis_ref(s: int, pts):
    """Reference test functions psi_hat_i = p_d0(x) p_d1(y) p_d2(z) e_a and their
    curls at points pts (npts,3).  Returns (val, curl), each (N, npts, 3)."""
    pts = np.asarray(pts, dtype=np.float64)
    v = [onb_legendre(s, pts[:, ax]) for ax in range(3)]   # (val, der) per axis
    idx = test_index_list(s)
    val = np.zeros((len(idx), pts.shape[0], 3))
    curl = np.zeros_like(val)
    for n, (a, d) in enumerate(idx):
        f = v[0][0][d[0]] * v[1][0][d[1]] * v[2][0][d[2]]
        grad = np.stack([v[0][1][d[0]] * v[1][0][d[1]] * v[2][0][d[2]],
                         v[0][0][d[0]] * v[1][1][d[1]] * v[2][0][d[2]],
                         v[0][0][d[0]] * v[1][0][d[1]] * v[2][1][d[2]]], axis=-1)
        e = np.zeros(3)
        e[a] = 1.0
        val[n, :, a] = f
        curl[n] = np.cross(grad, e)          # curl(f e_a) = grad f x e_a
    return val, curl


def trace_index_list(r: int):
    """Boundary functions of the first-kind Nedelec space of FEEC index r
    (12 r^2 per field).  Each entry is (component a, along-degree i,
    (axis_b, kind_b), (axis_c, kind_c)) with the function
        p_i(xi_a) * t_b(xi_b) * t_c(xi_c) * e_a,
    where kind 'v0' = 1-xi, 'v1' = xi, ('b', m) = bubble of degree m.
    Ordering: 12 edges x r, then 6 faces x 2 r (r-1).
      edges 0-3 along x at (y,z) = (0,0),(1,0),(0,1),(1,1)
      edges 4-7 along y at (x,z) = (0,0),(1,0),(0,1),(1,1)
      edges 8-11 along z at (x,y) = (0,0),(1,0),(0,1),(1,1)
      faces x-,x+,y-,y+,z-,z+ ; on each face first the functions with the
      lower tangential axis as component (bubble along the higher one), then
      the other; inside each group the along-degree i is fastest."""
    out = []
    for a in range(3):
        b, c = [ax for ax in range(3) if ax != a]
        for vc in range(2):
            for vb in range(2):
                for i in range(r):
                    out.append((a, i, (b, ('v', vb)), (c, ('v', vc))))
    for f in range(6):
        nax, side = f // 2, f % 2
        t1, t2 = [ax for ax in range(3) if ax != nax]
        for comp, other in ((t1, t2), (t2, t1)):
            for m in range(2, r + 1):
                for i in range(r):
                    out.append((comp, i, (nax, ('v', side)), (other, ('b', m))))
    return out


def _transverse(kind, xi):
    if kind[0] == 'v':
        return (1.0 - xi) if kind[1] == 0 else xi
    return lobatto_bubble(kind[1], xi)


def trace_basis_ref(r: int, pts):
    """Reference trace functions (full 3D Nedelec fields, of which only the
    tangential trace on faces is used) at pts.  Returns (12 r^2, npts, 3)."""
    pts = np.asarray(pts, dtype=np.float64)
    idx = trace_index_list(r)
    out = np.zeros((len(idx), pts.shape[0], 3))
    for n, (a, i, (bax, bk), (cax, ck)) in enumerate(idx):
        pa, _ = onb_legendre(r - 1, pts[:, a])
        out[n, :, a] = pa[i] * _transverse(bk, pts[:, bax]) * _transverse(ck, pts[:, cax])
    return out


def trial_basis_ref(p: int, pts):
    """Scalar DG Lagrange functions phi_m, m = i + (p+1)(j + (p+1)k), at pts."""
    pts = np.asarray(pts, dtype=np.float64)
    lx, ly, lz = (lagrange_gll(p, pts[:, ax]) for ax in range(3))
    n = p + 1
    out = np.zeros((n ** 3, pts.shape[0]))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                out[i + n * (j + n * k)] = lx[i] * ly[j] * lz[k]
    return out


# --------------------------------------------------------------------------
# Geometry: trilinear hexahedron, vertex v(i,j,k) at index 4k+2j+i
# --------------------------------------------------------------------------
def trilinear_map(X, pts):
    """Physical points x(xi) and Jacobians J_ab = dx_a/dxi_b at pts."""
    X = np.asarray(X, dtype=np.float64).reshape(8, 3)
    pts = np.asarray(pts, dtype=np.float64)
    x = np.zeros((pts.shape[0], 3))
    J = np.zeros((pts.shape[0], 3, 3))
    for k in range(2):
        for j in range(2):
            for i in range(2):
                v = X[4 * k + 2 * j + i]
                fx = pts[:, 0] if i else 1.0 - pts[:, 0]
                fy = pts[:, 1] if j else 1.0 - pts[:, 1]
                fz = pts[:, 2] if k else 1.0 - pts[:, 2]
                dfx = 1.0 if i else -1.0
                dfy = 1.0 if j else -1.0
                dfz = 1.0 if k else -1.0
                x += np.outer(fx * fy * fz, v)
                J[:, :, 0] += np.outer(dfx * fy * fz, v)
                J[:, :, 1] += np.outer(fx * dfy * fz, v)
                J[:, :, 2] += np.outer(fx * fy * dfz, v)
    return x, J


def volume_rule(n1: int):
    g, w = gauss_legendre_01(n1)
    Z, Y, Xg = np.meshgrid(g, g, g, indexing='ij')
    WZ, WY, WX = np.meshgrid(w, w, w, indexing='ij')
    pts = np.stack([Xg.ravel(), Y.ravel(), Z.ravel()], axis=1)   # x fastest
    return pts, (WX * WY * WZ).ravel()


def face_rule(n1: int, f: int):
    """Gauss points on reference face f (x-,x+,y-,y+,z-,z+) as 3D points."""
    g, w = gauss_legendre_01(n1)
    nax, side = f // 2, f % 2
    t1, t2 = [ax for ax in range(3) if ax != nax]
    B, A = np.meshgrid(g, g, indexing='ij')
    WB, WA = np.meshgrid(w, w, indexing='ij')
    pts = np.zeros((n1 * n1, 3))
    pts[:, t1] = A.ravel()
    pts[:, t2] = B.ravel()
    pts[:, nax] = float(side)
    return pts, (WA * WB).ravel()


def face_geometry(X, f: int, pts):
    """Outward unit normal n and area element factor |t1 x t2| on face f."""
    x, J = trilinear_map(X, pts)
    nax, side = f // 2, f % 2
    t1, t2 = [ax for ax in range(3) if ax != nax]
    N = np.cross(J[:, :, t1], J[:, :, t2])
    # orient outward: along +dx/dxi_nax on the side-1 face, against it on side 0
    sgn = np.sign(np.einsum('qa,qa->q', N, J[:, :, nax])) * (1.0 if side else -1.0)
    nrm = np.linalg.norm(N, axis=1)
    n = N * (sgn / nrm)[:, None]
    return x, J, n, nrm


# --------------------------------------------------------------------------
# TE_mn rectangular-waveguide mode (§4.1) and port data
# --------------------------------------------------------------------------
@dataclass
class PortMode:
    """TE_mn mode travelling in +x3 in a guide [0,a] x [0,b] filled with
    (eps, mu); coordinates are non-dimensional (units of L = 1 m)."""
    a: float
    b: float
    m: int
    n: int
    omega: float
    eps: complex = 1.0
    mu: complex = 1.0

    @property
    def k1(self):
        return self.m * math.pi / self.a

    @property
    def k2(self):
        return self.n * math.pi / self.b

    @property
    def k3(self):
        kc2 = self.k1 ** 2 + self.k2 ** 2
        return np.sqrt(complex(self.omega ** 2 * self.eps * self.mu - kc2))

    def zinv(self):
        """Port admittance Z_s^{-1} = k_x3 / (omega mu_r) (§4.1 port condition)."""
        return self.k3 / (self.omega * self.mu)

    def fields(self, x):
        """E_sol, H_sol of §4.1 at points x (npts,3)."""
        x = np.asarray(x, dtype=np.float64)
        k1, k2, k3 = self.k1, self.k2, self.k3
        kc2 = k1 ** 2 + k2 ** 2
        c1, s1 = np.cos(k1 * x[:, 0]), np.sin(k1 * x[:, 0])
        c2, s2 = np.cos(k2 * x[:, 1]), np.sin(k2 * x[:, 1])
        ph = np.exp(1j * k3 * x[:, 2])
        E = np.zeros((x.shape[0], 3), dtype=complex)
        H = np.zeros((x.shape[0], 3), dtype=complex)
        pre = 1j * self.omega * self.mu / kc2
        E[:, 0] = pre * (-k2 * c1 * s2) * ph
        E[:, 1] = pre * (k1 * s1 * c2) * ph
        H[:, 0] = -1j * k3 * k1 / kc2 * s1 * c2 * ph
        H[:, 1] = -1j * k3 * k2 / kc2 * c1 * s2 * ph
        H[:, 2] = c1 * c2 * ph
        return E, H

    def robin_data(self, x, n, zinv):
        """g = n x H_TE + Z^{-1} n x (E_TE x n) at the port (§4.1 inlet condition)."""
        E, H = self.fields(x)
        return np.cross(n, H) + zinv * np.cross(n, np.cross(E, n))


# --------------------------------------------------------------------------
# The local forms (§2.2 / §2.3) evaluated from their definitions
# --------------------------------------------------------------------------
@dataclass
class CellProblem:
    X: np.ndarray                   # (8,3) vertices, v(i,j,k) at 4k+2j+i
    p: int
    dp: int
    eps: complex
    mu: complex
    omega: float
    face_kind: Sequence[int] = (0, 0, 0, 0, 0, 0)
    zinv: Sequence[complex] = (0, 0, 0, 0, 0, 0)
    alpha: float = 1.0
    port: Optional[PortMode] = None
    J_src: Optional[Callable] = None        # x -> (npts,3) complex current density
    g_src: Optional[Callable] = None        # (face, x, n) -> (npts,3) complex Robin data
    quad_extra: int = 0                     # extra Gauss points (tests only)


def _robin(kind):
    return kind in (FACE_PORT, FACE_ROBIN0)


def cell_forms(cp: CellProblem):
    """Returns (G, B_f, l) for one cell, or raises ValueError on a degenerate
    cell (det J <= 0 at a quadrature point).

    Rows: F-block test functions (N), then I-block (N).
    Columns of B_f: E_x,E_y,E_z,H_x,H_y,H_z blocks of (p+1)^3 DG functions,
    then E-hat (12 r^2) and H-hat (12 r^2) trace functions."""
    p, dp = cp.p, cp.dp
    s, r = p + dp + 1, p + 1
    n1 = p + dp + 2 + cp.quad_extra
    N = 3 * s * (s + 1) ** 2
    m1 = (p + 1) ** 3
    om, eps, mu, alpha = cp.omega, complex(cp.eps), complex(cp.mu), cp.alpha

    # ---- volume terms -------------------------------------------------
    pts, w = volume_rule(n1)
    x, J = trilinear_map(cp.X, pts)
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0.0):
        raise ValueError("degenerate cell: det J <= 0")
    Jinv = np.linalg.inv(J)
    wd = w * detJ
    val, curl = test_basis_ref(s, pts)
    psi = np.einsum('qba,nqb->nqa', Jinv, val)                 # J^{-T} psi_hat
    cpsi = np.einsum('qab,nqb->nqa', J, curl) / detJ[None, :, None]
    Z = np.zeros_like(psi)
    F, I = np.concatenate([psi, Z]), np.concatenate([Z, psi])      # v_i = (F_i, I_i)
    cF, cI = np.concatenate([cpsi, Z]), np.concatenate([Z, cpsi])

    def ip(u, v, wt):
        """sum_q wt_q conj(u_i(q)) . v_j(q)  ->  (nu, nv)"""
        nu, nv = u.shape[0], v.shape[0]
        return np.conj(u).reshape(nu, -1) @ (v * wt[None, :, None]).reshape(nv, -1).T

    # adjoint graph inner product (§2.2, test inner product)
    A1 = cF + 1j * om * np.conj(mu) * I
    A2 = cI - 1j * om * np.conj(eps) * F
    G = ip(A1, A1, wd) + ip(A2, A2, wd) + alpha * (ip(F, F, wd) + ip(I, I, wd))

    # trial functions u_j = (E_j, H_j): phi_m e_c
    phi = trial_basis_ref(p, pts)
    nq = pts.shape[0]
    Et = np.zeros((6 * m1, nq, 3), dtype=complex)
    Ht = np.zeros_like(Et)
    for c in range(3):
        Et[c * m1:(c + 1) * m1, :, c] = phi
        Ht[(3 + c) * m1:(4 + c) * m1, :, c] = phi
    # ultraweak bilinear form (§2.2): (curl I,E) - (I, i w mu H) + (curl F,H) + (F, i w eps E)
    B = (ip(cI, Et, wd) - ip(I, 1j * om * mu * Ht, wd)
         + ip(cF, Ht, wd) + ip(F, 1j * om * eps * Et, wd))

    # linear form volume part: (F, J)
    l = np.zeros(2 * N, dtype=complex)
    if cp.J_src is not None:
        Jx = np.asarray(cp.J_src(x), dtype=complex)
        l += ip(F, Jx[None], wd)[:, 0]

    # ---- face terms ---------------------------------------------------
    nt = 12 * r * r
    Bh = np.zeros((2 * N, 2 * nt), dtype=complex)
    for f in range(6):
        kind = cp.face_kind[f]
        fpts, fw = face_rule(n1, f)
        xf, Jf, n, dS = face_geometry(cp.X, f, fpts)
        wf = fw * dS
        Jfinv = np.linalg.inv(Jf)
        fval, _ = test_basis_ref(s, fpts)
        fpsi = np.einsum('qba,nqb->nqa', Jfinv, fval)
        Zf = np.zeros_like(fpsi)
        Ff, If = np.concatenate([fpsi, Zf]), np.concatenate([Zf, fpsi])
        th = np.einsum('qba,nqb->nqa', Jfinv, trace_basis_ref(r, fpts))   # covariant Piola
        Zt = np.zeros_like(th)
        Eh, Hh = np.concatenate([th, Zt]), np.concatenate([Zt, th])        # uhat_j = (Ehat_j, Hhat_j)
        nb = n[None]
        # trace pairing (§2.2): <I, n x Ehat>_{dK} + <F, n x Hhat>_{dK \ Gamma_R}
        Bh += ip(If, np.cross(nb, Eh), wf)
        if not _robin(kind):
            Bh += ip(Ff, np.cross(nb, Hh), wf)
            continue
        zi = complex(cp.zinv[f])
        # Robin part of the test norm: (n x I + conj(Z^{-1}) n x (F x n), same)_{Gamma_R}
        Cr = np.cross(nb, If) + np.conj(zi) * np.cross(nb, np.cross(Ff, nb))
        G += ip(Cr, Cr, wf)
        # Robin part of b_h: - <F, Z^{-1} n x (E x n)>_{Gamma_R}
        phif = trial_basis_ref(p, fpts)
        Etf = np.zeros((6 * m1, fpts.shape[0], 3), dtype=complex)
        for c in range(3):
            Etf[c * m1:(c + 1) * m1, :, c] = phif
        B -= ip(Ff, zi * np.cross(nb, np.cross(Etf, nb)), wf)
        # Robin part of l_h: - <F, g>_{Gamma_R}
        g = None
        if cp.g_src is not None:
            g = cp.g_src(f, xf, n)
        elif kind == FACE_PORT and cp.port is not None:
            g = cp.port.robin_data(xf, n, zi)
        if g is not None:
            l -= ip(Ff, np.asarray(g, dtype=complex)[None], wf)[:, 0]
    Bf = np.concatenate([B, Bh], axis=1)
    return G, Bf, l


def cell_forms_blocks(cp: CellProblem):
    """The same (G, B_f, l) as cell_forms by a second route: the real volume
    matrices of the mapped test functions (psi, curl psi) and trial functions
    (phi e_c),
        M = (psi, psi), S = (curl psi, curl psi), C_ij = (curl psi_i, psi_j),
        D_i,(c,a) = ((psi_i)_c, phi_a), R_i,(c,a) = ((curl psi_i)_c, phi_a),
    per Robin face the tangential ones
        Mt = (psi_t, psi_t), Rt_ij = (psi_i, n x psi_j), Dt_i,(c,a) = ((psi_i,t)_c, phi_a),
    and the trace pairing T_ij = (psi_i, n x theta_j), combined with the
    coefficients by expanding the forms of §2.2 on the basis (psi_i, 0),
    (0, psi_i) (conjugation in the first argument):
        G_FF = S + (w^2 |eps|^2 + alpha) M + sum_R |z|^2 Mt,
        G_II = S + (w^2 |mu|^2 + alpha) M + sum_R Mt,
        G_FI = i w conj(mu) C + i w eps C^T + sum_R z Rt,   G_IF = G_FI^H,
        B_FE = i w eps D - sum_R z Dt,  B_FH = R,  B_IE = R,  B_IH = -i w mu D,
        Bhat_IEhat = T (all faces),  Bhat_FHhat = T (non-Robin faces),
        l_F = (psi, J) - sum_R (psi, g),  l_I = 0,
    with z the face's Z^{-1}.  The arithmetic differs from the pointwise
    route (real contractions first, coefficients after), so the exact solves
    of the two FP64 systems differ by what FP64 formation roundoff moves
    K_e, l_e and eta: the floor any independent FP64 implementation has."""
    p, dp = cp.p, cp.dp
    s, r = p + dp + 1, p + 1
    n1 = p + dp + 2 + cp.quad_extra
    N = 3 * s * (s + 1) ** 2
    m1 = (p + 1) ** 3
    om, eps, mu, alpha = cp.omega, complex(cp.eps), complex(cp.mu), cp.alpha

    def rip(u, v, wt):
        """sum_q wt_q u_i(q) . v_j(q) for real fields -> (nu, nv)"""
        return u.reshape(u.shape[0], -1) @ (v * wt[None, :, None]).reshape(v.shape[0], -1).T

    def dg(u, phi, wt):
        """[i, c*m1 + a] = sum_q wt_q u_i,c(q) phi_a(q)"""
        return np.einsum('iqc,aq,q->ica', u, phi, wt).reshape(u.shape[0], 3 * phi.shape[0])

    pts, w = volume_rule(n1)
    x, J = trilinear_map(cp.X, pts)
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0.0):
        raise ValueError("degenerate cell: det J <= 0")
    Jinv = np.linalg.inv(J)
    wd = w * detJ
    val, curl = test_basis_ref(s, pts)
    psi = np.einsum('qba,nqb->nqa', Jinv, val)
    cpsi = np.einsum('qab,nqb->nqa', J, curl) / detJ[None, :, None]
    phi = trial_basis_ref(p, pts)
    M, S, C = rip(psi, psi, wd), rip(cpsi, cpsi, wd), rip(cpsi, psi, wd)
    D, R = dg(psi, phi, wd), dg(cpsi, phi, wd)
    cF = om * om * abs(eps) ** 2 + alpha
    cI = om * om * abs(mu) ** 2 + alpha
    GFF = S + cF * M + 0j
    GII = S + cI * M + 0j
    GFI = 1j * om * np.conj(mu) * C + 1j * om * eps * C.T
    BFE = 1j * om * eps * D
    nt = 12 * r * r
    TI = np.zeros((N, nt))
    TF = np.zeros((N, nt))
    lF = np.zeros(N, dtype=complex)
    if cp.J_src is not None:
        Jx = np.asarray(cp.J_src(x), dtype=complex)
        lF += np.einsum('iqa,qa,q->i', psi, Jx, wd)
    for f in range(6):
        kind = cp.face_kind[f]
        fpts, fw = face_rule(n1, f)
        xf, Jf, n, dS = face_geometry(cp.X, f, fpts)
        wf = fw * dS
        Jfinv = np.linalg.inv(Jf)
        fval, _ = test_basis_ref(s, fpts)
        fpsi = np.einsum('qba,nqb->nqa', Jfinv, fval)
        th = np.einsum('qba,nqb->nqa', Jfinv, trace_basis_ref(r, fpts))
        Tf = rip(fpsi, np.cross(n[None], th), wf)
        TI += Tf
        if not _robin(kind):
            TF += Tf
            continue
        z = complex(cp.zinv[f])
        pt = fpsi - np.einsum('nqa,qa->nq', fpsi, n)[:, :, None] * n[None]      # tangential part
        GFF += abs(z) ** 2 * rip(pt, pt, wf)
        GII += rip(pt, pt, wf)
        GFI += z * rip(fpsi, np.cross(n[None], fpsi), wf)
        BFE -= z * dg(pt, trial_basis_ref(p, fpts), wf)
        g = None
        if cp.g_src is not None:
            g = cp.g_src(f, xf, n)
        elif kind == FACE_PORT and cp.port is not None:
            g = cp.port.robin_data(xf, n, z)
        if g is not None:
            lF -= np.einsum('iqa,qa,q->i', fpsi, np.asarray(g, dtype=complex), wf)
    G = np.block([[GFF, GFI], [GFI.conj().T, GII]])
    Z3 = np.zeros((N, nt))
    B = np.block([[BFE, R + 0j, Z3, TF], [R + 0j, -1j * om * mu * D, TI, Z3]])
    l = np.concatenate([lF, np.zeros(N, dtype=complex)])
    return G, B, l


# --------------------------------------------------------------------------
# The local solve (§2.3): elimination of Psi, error representation
# --------------------------------------------------------------------------
def local_solve(G, Bf, l, x=None, r=None):
    """K_e = B_f^H G^{-1} B_f, l_e = B_f^H G^{-1} l and, if x is given,
    eta = sqrt(r^H G^{-1} r) with r = B_f x - l (or with the residual r
    itself, when it is given instead of x).  Plain definition: the G-solves
    are LU solves (numpy.linalg.solve)."""
    k = Bf.shape[1]
    rhs = np.concatenate([Bf, l[:, None]], axis=1)
    if r is None and x is not None:
        r = Bf @ x - l
    if r is not None:
        rhs = np.concatenate([rhs, np.asarray(r)[:, None]], axis=1)
    X = np.linalg.solve(G, rhs)
    K = np.conj(Bf).T @ X[:, :k]
    le = np.conj(Bf).T @ X[:, k]
    eta = None
    if r is not None:
        rr = rhs[:, k + 1]
        eta = math.sqrt(max(0.0, float(np.real(np.conj(rr) @ X[:, k + 1]))))
    return K, le, eta


def local_solve_cholesky(G, Bf, l, x=None):
    """Cross-check route: Jacobi scaling, G = L L^H, W = L^{-1} D B_f,
    K_e = W^H W, l_e = W^H y, eta = ||W x - y||."""
    import scipy.linalg as sla
    d = 1.0 / np.sqrt(np.real(np.diag(G)))
    Gs = G * d[:, None] * d[None, :]
    L = np.linalg.cholesky(Gs)
    W = sla.solve_triangular(L, Bf * d[:, None], lower=True)
    y = sla.solve_triangular(L, l * d, lower=True)
    K = np.conj(W).T @ W
    le = np.conj(W).T @ y
    eta = None
    if x is not None:
        eta = float(np.linalg.norm(W @ x - y))
    return K, le, eta


def solve_cell(cp: CellProblem, x=None):
    """Forms and local solve for one cell.  Returns dict with K, l, eta, info
    (info = 0 ok, -1 degenerate geometry)."""
    try:
        G, Bf, l = cell_forms(cp)
    except ValueError:
        return dict(K=None, l=None, eta=None, info=-1)
    K, le, eta = local_solve(G, Bf, l, x)
    return dict(K=K, l=le, eta=eta, info=0)


# --------------------------------------------------------------------------
# Projections onto the local trial and trace spaces (for manufactured data)
# --------------------------------------------------------------------------
def interpolate_trial(X, p, E_fun, H_fun):
    """DG Lagrange interpolant (nodal values at the mapped Gauss-Lobatto nodes)
    of physical fields E, H -> coefficient vector of length 6 (p+1)^3."""
    z = gauss_lobatto_nodes_01(p + 1)
    n = p + 1
    Zg, Yg, Xg = np.meshgrid(z, z, z, indexing='ij')
    nodes = np.stack([Xg.ravel(), Yg.ravel(), Zg.ravel()], axis=1)
    x, _ = trilinear_map(X, nodes)
    E, H = np.asarray(E_fun(x), complex), np.asarray(H_fun(x), complex)
    return np.concatenate([E[:, 0], E[:, 1], E[:, 2], H[:, 0], H[:, 1], H[:, 2]])


def project_trace(X, r, fun, extra=2):
    """Coefficients c (12 r^2) minimising sum_faces int |n x (sum c_j theta_j - u)|^2 dS:
    the L2 projection of the tangential trace of u onto the trace space."""
    nt = 12 * r * r
    A = np.zeros((nt, nt))
    b = np.zeros(nt, dtype=complex)
    n1 = r + 2 + extra
    for f in range(6):
        fpts, fw = face_rule(n1, f)
        xf, Jf, n, dS = face_geometry(X, f, fpts)
        th = np.einsum('qba,nqb->nqa', np.linalg.inv(Jf), trace_basis_ref(r, fpts))
        nth = np.cross(n[None], th)
        nu = np.cross(n, np.asarray(fun(xf), complex))
        wt = fw * dS
        A += np.einsum('iqa,jqa,q->ij', nth, nth, wt)
        b += np.einsum('iqa,qa,q->i', nth, nu, wt)
    return np.linalg.solve(A, b)


def projected_solution(X, p, E_fun, H_fun):
    """x_e = [Pi E, Pi H, Pi Ehat, Pi Hhat] for the local solve's eta."""
    r = p + 1
    u = interpolate_trial(X, p, E_fun, H_fun)
    ce = project_trace(X, r, E_fun)
    ch = project_trace(X, r, H_fun)
    return np.concatenate([u, ce, ch])
