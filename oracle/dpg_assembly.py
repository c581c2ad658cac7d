"""Plain FP64 CPU oracle for the condensed trace system (Marquis, Maier,
Blais, arXiv 2609.03155, §2.3: static condensation of the interior unknowns
and the linear system solved by CG).

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` may import this module.  It shares
no code with the HIP library or its host code.

* condense:        A_K = M3 - M2^H M1^{-1} M2,  b_K = (M5 - M2^H M1^{-1} M4) l
                   with K_e = [[M1, M2], [M2^H, M3]] over [interior u ; trace t]
                   and l_e = [M4 l ; M5 l]  (§2.3, the condensed system).
* trace_numbering: global trace unknowns of a conforming hexahedral mesh.
* assemble:        A = sum_K P_K^T A_K P_K,  b = sum_K P_K^T b_K  (scipy.sparse).
* cg:              the condensed system A t = b solved by conjugate gradients
                   without a preconditioner (§2.3; A is Hermitian positive
                   definite); textbook Hestenes-Stiefel recursion.
* scatter:         t_K = P_K t, the cell's local trace coefficients (zero where
                   removed or constrained).
* reconstruct:     the interior unknowns recovered cell by cell,
                   u_K = M1^{-1} (M4 l - M2 t_K)  (§2.3), returned with t_K as
                   the cell's whole coefficient vector [u_K ; t_K].

Numbering rule (the library's host numbering follows the same rule, written
independently):
  * a trace function of a cell lives on an edge (12 r per field) or a face
    (2 r (r-1) per field), in the local order of ``trace_index_list``; Ehat
    functions come before Hhat functions;
  * edges are keyed by their (start, end) global vertices along the local
    component axis, faces by their vertex set; every cell must see an edge in
    the same direction and a face with the same (t1, t2) axes (structured
    meshes do), else ValueError;
  * mixed degrees follow the minimum rule on shared edges and faces: an
    entity keeps the hierarchical functions of the smallest r among its
    cells; a cell's higher functions on it are constrained to zero;
  * removed (Dirichlet) unknowns: Ehat on every edge or face that lies in a
    PEC boundary face (n x E = 0, §2.2); Hhat face functions of Robin faces
    and Hhat edge functions whose cell faces are all Robin (excluded from the
    trace pairing there, §2.2, so they have zero rows in K_e);
  * kept unknowns are numbered in order of first appearance, scanning cells
    in order and each cell's trace functions in local order.
"""
from __future__ import annotations

import numpy as np

from .dpg_oracle import FACE_PEC, FACE_PORT, FACE_ROBIN0, trace_index_list


def condense(K, le, nu: int):
    """The §2.3 condensed cell matrix and right-hand side from K_e, l_e."""
    K = np.asarray(K, complex)
    le = np.asarray(le, complex)
    M1, M2, M3 = K[:nu, :nu], K[:nu, nu:], K[nu:, nu:]
    X = np.linalg.solve(M1, np.concatenate([M2, le[:nu, None]], axis=1))   # M1^{-1} [M2 | M4 l]
    A = M3 - M2.conj().T @ X[:, :-1]
    b = le[nu:] - M2.conj().T @ X[:, -1]
    return A, b


# local edge e -> (component axis a, transverse vertex indices): edges 0-3 along
# x at (y,z) = (0,0),(1,0),(0,1),(1,1); 4-7 along y at (x,z); 8-11 along z at (x,y)
def _edge_vertices(e):
    a = e // 4
    vb, vc = e % 2, (e % 4) // 2
    b, c = [ax for ax in range(3) if ax != a]
    ends = []
    for t in (0, 1):
        ijk = [0, 0, 0]
        ijk[a], ijk[b], ijk[c] = t, vb, vc
        ends.append(4 * ijk[2] + 2 * ijk[1] + ijk[0])
    return a, ends


def _face_vertices(f):
    """Local vertex ids of face f at (t1, t2) = (0,0), (1,0), (0,1), (1,1)."""
    nax, side = f // 2, f % 2
    t1, t2 = [ax for ax in range(3) if ax != nax]
    out = []
    for u2 in (0, 1):
        for u1 in (0, 1):
            ijk = [0, 0, 0]
            ijk[nax], ijk[t1], ijk[t2] = side, u1, u2
            out.append(4 * ijk[2] + 2 * ijk[1] + ijk[0])
    return out


# faces of the cell containing local edge e (both contain it)
def _edge_faces(e):
    a, ends = _edge_vertices(e)
    return [f for f in range(6) if set(ends) <= set(_face_vertices(f))]


def trace_numbering(cells, face_kind, degree):
    """Global ids of every cell's local trace functions.

    cells [n][8] global vertex ids (v(i,j,k) at 4k+2j+i), face_kind [n][6],
    degree [n] (p; r = p+1).  Returns (glob, n_dofs) with glob a list of
    int64 arrays, glob[c] of length 24 r_c^2 (Ehat then Hhat), -1 where the
    function is removed or constrained."""
    cells = np.asarray(cells)
    face_kind = np.asarray(face_kind)
    n = cells.shape[0]
    # entities, their minimum r, orientation and boundary kinds
    edge_r, face_r = {}, {}
    edge_pec, face_pec, face_robin = set(), set(), set()
    edge_allrobin = {}
    face_orient = {}
    for c in range(n):
        r = int(degree[c]) + 1
        V = cells[c]
        for e in range(12):
            _, ends = _edge_vertices(e)
            key = (int(V[ends[0]]), int(V[ends[1]]))
            if (key[1], key[0]) in edge_r:
                raise ValueError("edge seen in opposite directions")
            edge_r[key] = min(edge_r.get(key, r), r)
            fs = _edge_faces(e)
            kinds = [int(face_kind[c, f]) for f in fs]
            allrobin = all(k in (FACE_PORT, FACE_ROBIN0) for k in kinds)
            edge_allrobin[key] = edge_allrobin.get(key, True) and allrobin
            if any(k == FACE_PEC for k in kinds):
                edge_pec.add(key)
        for f in range(6):
            fv = [int(V[v]) for v in _face_vertices(f)]
            key = frozenset(fv)
            if key in face_orient and face_orient[key] != tuple(fv[:3]):
                raise ValueError("face seen with different axes")
            face_orient[key] = tuple(fv[:3])
            face_r[key] = min(face_r.get(key, r), r)
            k = int(face_kind[c, f])
            if k == FACE_PEC:
                face_pec.add(key)
            if k in (FACE_PORT, FACE_ROBIN0):
                face_robin.add(key)
    ids = {}
    glob = []
    for c in range(n):
        r = int(degree[c]) + 1
        V = cells[c]
        idx = trace_index_list(r)
        nt1 = 12 * r * r
        g = np.full(2 * nt1, -1, dtype=np.int64)
        for field in (0, 1):
            for lt in range(nt1):
                if lt < 12 * r:
                    e, i = lt // r, lt % r
                    _, ends = _edge_vertices(e)
                    key = (int(V[ends[0]]), int(V[ends[1]]))
                    rmin = edge_r[key]
                    if i >= rmin:
                        continue
                    if field == 0 and key in edge_pec:
                        continue
                    if field == 1 and edge_allrobin[key]:
                        continue
                    gid = ('e', field, key, i)
                else:
                    q = lt - 12 * r
                    f, w = q // (2 * r * (r - 1)), q % (2 * r * (r - 1))
                    grp, rest = w // (r * (r - 1)), w % (r * (r - 1))
                    m, i = 2 + rest // r, rest % r
                    key = frozenset(int(V[v]) for v in _face_vertices(f))
                    rmin = face_r[key]
                    if m > rmin or i >= rmin:
                        continue
                    if field == 0 and key in face_pec:
                        continue
                    if field == 1 and key in face_robin:
                        continue
                    gid = ('f', field, key, grp, m, i)
                if gid not in ids:
                    ids[gid] = len(ids)
                g[field * nt1 + lt] = ids[gid]
        glob.append(g)
    return glob, len(ids)


def assemble(A_cells, b_cells, glob, n_dofs):
    """A = sum_K P_K^T A_K P_K, b = sum_K P_K^T b_K over the kept unknowns
    (scipy.sparse CSR, duplicates summed)."""
    import scipy.sparse as sps
    rows, cols, vals = [], [], []
    b = np.zeros(n_dofs, complex)
    for A, bk, g in zip(A_cells, b_cells, glob):
        keep = np.nonzero(g >= 0)[0]
        gg = g[keep]
        rows.append(np.repeat(gg, len(gg)))
        cols.append(np.tile(gg, len(gg)))
        vals.append(np.asarray(A)[np.ix_(keep, keep)].ravel())
        np.add.at(b, gg, np.asarray(bk)[keep])
    A = sps.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n_dofs, n_dofs)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A, b


def cg(A, b, tol: float, max_iter: int, x0=None):
    """Conjugate gradients for the Hermitian positive definite A (any object
    with ``@``), as the condensed trace system is solved in §2.3: no
    preconditioner, start x0 (zero if None), stop once the recursively updated
    residual satisfies ||r||_2 <= tol ||b||_2 or after max_iter iterations.
    Each iteration:
        q = A p,  alpha = (r^H r) / (p^H q),  x += alpha p,  r -= alpha q,
        beta = (r_new^H r_new) / (r^H r),     p = r + beta p.
    Returns (x, iterations, history of ||r||_2 / ||b||_2, one entry per
    iteration plus the initial one)."""
    b = np.asarray(b, complex)
    x = np.zeros_like(b) if x0 is None else np.array(x0, complex)
    bn = float(np.linalg.norm(b))
    r = b - A @ x
    p = r.copy()
    rr = float(np.real(np.vdot(r, r)))
    hist = [np.sqrt(rr) / bn if bn > 0 else 0.0]
    it = 0
    while it < max_iter and bn > 0 and np.sqrt(rr) > tol * bn:
        q = A @ p
        alpha = rr / float(np.real(np.vdot(p, q)))
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.real(np.vdot(r, r)))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr) / bn)
    return x, it, np.array(hist)


def scatter(t, glob_cell):
    """P_K t: the cell's local trace coefficients from the global ones."""
    g = np.asarray(glob_cell)
    out = np.zeros(len(g), complex)
    keep = g >= 0
    out[keep] = np.asarray(t, complex)[g[keep]]
    return out


def reconstruct(K, le, nu: int, t_local):
    """The cell's interior unknowns from its traces (§2.3),
    u = M1^{-1} (M4 l - M2 t), with M1 = K_e[:nu, :nu], M2 = K_e[:nu, nu:] and
    M4 l = l_e[:nu]; returns [u ; t]."""
    K = np.asarray(K, complex)
    le = np.asarray(le, complex)
    t_local = np.asarray(t_local, complex)
    u = np.linalg.solve(K[:nu, :nu], le[:nu] - K[:nu, nu:] @ t_local)
    return np.concatenate([u, t_local])
