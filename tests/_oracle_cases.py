"""Helpers that run the oracle on cells of a seeded workload (tests only)."""
import numpy as np

from oracle import dpg_oracle as O


def port_mode(w):
    om = O.omega_dimensionless(w.freq_hz)
    pt = w.port
    return O.PortMode(pt["a"], pt["b"], pt["m"], pt["n"], om, pt["eps"], pt["mu"])


def cell_problem(w, c):
    om = O.omega_dimensionless(w.freq_hz)
    return O.CellProblem(X=w.cell_vertices(c), p=int(w.degree[c]), dp=w.dp, eps=complex(w.eps[c]),
                         mu=complex(w.mu[c]), omega=om, face_kind=tuple(int(k) for k in w.face_kind[c]),
                         zinv=tuple(complex(z) for z in w.zinv[c]), port=port_mode(w))


def oracle_cell(w, c, x=None):
    """(G, B_f, l, K_e, l_e, eta) of cell c."""
    G, Bf, l = O.cell_forms(cell_problem(w, c))
    K, le, eta = O.local_solve(G, Bf, l, x)
    return G, Bf, l, K, le, eta


U64 = 2.0 ** -53


def kappa_scaled(G):
    """2-norm condition number of the Jacobi-scaled Gram matrix D G D."""
    d = 1.0 / np.sqrt(np.real(np.diag(G)))
    return float(np.linalg.cond(G * d[:, None] * d[None, :]))


def fp64_tol(G, floor=1e-10):
    """Parity bar of the FP64 path for one cell: 1e-10, or 4 kappa(D G D) u
    where the FP64 forward-error floor of the local solve itself is larger
    (both the oracle and the GPU path carry ~kappa u error)."""
    return max(floor, 4.0 * kappa_scaled(G) * U64)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


# ------------------------------------------------------------------ element-wise parity
# K_e is Hermitian positive semidefinite, K_e = W^H W, so |K_ab| <= sqrt(K_aa K_bb)
# and |l_e,a| <= sqrt(K_aa) ||y|| (y = L^{-1} D l).  The parity metrics compare
# every entry on that scale: blocks whose entries are orders of magnitude
# below the trace block (the interior block M1, which the condensation
# inverts) count as much as the largest ones.

# edges of the reference cell (order of the trace basis) -> their two faces
_EDGE_FACES = ((2, 4), (3, 4), (2, 5), (3, 5), (0, 4), (1, 4), (0, 5), (1, 5), (0, 2), (1, 2), (0, 3), (1, 3))


def robin_null(w, c):
    """Indices (K_e order) of the H-hat functions that live only on Robin
    faces of cell c: the pairing excludes H-hat there (§2.2), so their rows
    and columns of K_e and their entries of l_e are zero."""
    p = int(w.degree[c])
    r = p + 1
    nu, nt1 = 6 * (p + 1) ** 3, 12 * r * r
    rob = [int(k) in (2, 3) for k in w.face_kind[c]]
    base = nu + nt1
    idx = []
    for e, (fa, fb) in enumerate(_EDGE_FACES):
        if rob[fa] and rob[fb]:
            idx += range(base + e * r, base + (e + 1) * r)
    nf = 2 * r * (r - 1)
    for f in range(6):
        if rob[f]:
            idx += range(base + 12 * r + f * nf, base + 12 * r + (f + 1) * nf)
    return np.array(sorted(idx), np.int64)


def _keep(k, null):
    keep = np.ones(k, bool)
    keep[null] = False
    return keep


def k_scaled_err(K, Kref, null, rows=None, cols=None):
    """max |K_ab - Kref_ab| / sqrt(Kref_aa Kref_bb) over a, b outside the null
    set (optionally restricted to a row and a column range)."""
    k = Kref.shape[0]
    d = np.sqrt(np.maximum(np.real(np.diag(Kref)), 0.0))
    keep = _keep(k, null)
    ra = np.zeros(k, bool)
    ca = np.zeros(k, bool)
    ra[rows if rows is not None else slice(None)] = True
    ca[cols if cols is not None else slice(None)] = True
    ra &= keep
    ca &= keep
    if not ra.any() or not ca.any():
        return 0.0
    E = np.abs(K - Kref)[np.ix_(ra, ca)] / np.outer(d[ra], d[ca])
    return float(E.max())


def l_scaled_err(l, lref, Kref, ynorm, null, rows=None):
    """max |l_a - lref_a| / (sqrt(Kref_aa) ||y||) outside the null set."""
    k = Kref.shape[0]
    if ynorm == 0.0:
        return float(np.abs(l).max()) if len(l) else 0.0
    d = np.sqrt(np.maximum(np.real(np.diag(Kref)), 0.0))
    ra = np.zeros(k, bool)
    ra[rows if rows is not None else slice(None)] = True
    ra &= _keep(k, null)
    if not ra.any():
        return 0.0
    return float((np.abs(l - lref)[ra] / (d[ra] * ynorm)).max())


def null_exact(K, l, null):
    """The null rows and columns of K and entries of l are exactly zero."""
    if len(null) == 0:
        return True
    return bool(np.all(K[null, :] == 0) and np.all(K[:, null] == 0) and np.all(l[null] == 0))


def block_errs(K, l, Kref, lref, ynorm, null, nu):
    """Element-wise scaled errors per block: M1 (interior x interior), M2
    (interior x trace), M3 (trace x trace), l_u, l_t."""
    k = Kref.shape[0]
    iu, it = np.arange(nu), np.arange(nu, k)
    return dict(M1=k_scaled_err(K, Kref, null, iu, iu), M2=k_scaled_err(K, Kref, null, iu, it),
                M3=k_scaled_err(K, Kref, null, it, it), l_u=l_scaled_err(l, lref, Kref, ynorm, null, iu),
                l_t=l_scaled_err(l, lref, Kref, ynorm, null, it))


class OracleRef:
    """Oracle-side references of one cell for the element-wise parity bars.

    K, l, eta     -- the oracle's FP64 solve (LU) of its FP64 system;
    Kx, lx, ex    -- the exact solve of that FP64 system (extended precision),
    yx            -- ||y|| = sqrt(l^H G^{-1} l), the scale of l_e;
    e_or          -- the larger FP64 error against Kx of the oracle's two solve
                     routes (LU; Jacobi scaling, Cholesky and triangular
                     solves): the FP64 floor of the solve (a single route's
                     error varies several-fold with the BLAS build);
    s_form        -- how far the exact answer moves between the oracle's two
                     FP64 formations of the same forms (pointwise, and by
                     App. A's real block matrices): the floor set by formation
                     roundoff, which any independent FP64 implementation has.
    Everything here comes from oracle/ alone."""

    def __init__(self, w, c, x=None):
        from oracle import dpg_oracle as O
        from oracle import xsolve as X
        p = int(w.degree[c])
        self.cell, self.p = int(c), p
        self.nu = 6 * (p + 1) ** 3
        self.null = robin_null(w, c)
        cp = cell_problem(w, c)
        G, B, l = O.cell_forms(cp)
        self.kappa = kappa_scaled(G)
        r = None if x is None else B @ x - l
        self.K, self.l, self.eta = O.local_solve(G, B, l, r=r)
        self.Kx, self.lx, self.ex, self.yx = X.local_solve_ext(G, B, l, r, with_ynorm=True)
        # the oracle's second solve route (Jacobi scaling, Cholesky, triangular solves)
        Kc, lc, ec = O.local_solve_cholesky(G, B, l, x)
        G2, B2, l2 = O.cell_forms_blocks(cp)
        r2 = None if x is None else B2 @ x - l2
        Kx2, lx2, ex2 = X.local_solve_ext(G2, B2, l2, r2)
        self.e_or = dict(K=max(k_scaled_err(self.K, self.Kx, self.null), k_scaled_err(Kc, self.Kx, self.null)),
                         l=max(l_scaled_err(self.l, self.lx, self.Kx, self.yx, self.null),
                               l_scaled_err(lc, self.lx, self.Kx, self.yx, self.null)),
                         eta=max(abs(self.eta - self.ex), abs(ec - self.ex)) / self.ex if x is not None else 0.0)
        self.s_form = dict(K=k_scaled_err(Kx2, self.Kx, self.null),
                           l=l_scaled_err(lx2, self.lx, self.Kx, self.yx, self.null),
                           eta=abs(ex2 - self.ex) / self.ex if x is not None else 0.0)

    def fp64_bar(self, q):
        """Bar of the FP64 path for output q (K, l or eta):
        max(1e-10, 2 (e_or + s_form))."""
        return max(1e-10, 2.0 * (self.e_or[q] + self.s_form[q]))

    def errors(self, Kg, lg, eg):
        """Element-wise scaled errors of GPU outputs against the oracle's FP64
        solve (K, l, eta) and against the exact solve (K_x, ...), per block,
        and whether the Robin null rows are exactly zero."""
        out = dict(K=k_scaled_err(Kg, self.K, self.null), l=l_scaled_err(lg, self.l, self.Kx, self.yx, self.null),
                   K_x=k_scaled_err(Kg, self.Kx, self.null), l_x=l_scaled_err(lg, self.lx, self.Kx, self.yx, self.null),
                   K_frob=rel(Kg, self.K), null_exact=null_exact(Kg, lg, self.null),
                   blocks=block_errs(Kg, lg, self.K, self.l, self.yx, self.null, self.nu))
        if eg is not None and self.eta is not None:
            out["eta"] = abs(eg - self.eta) / self.eta
            out["eta_x"] = abs(eg - self.ex) / self.ex
        return out

    def summary(self):
        return dict(cell=self.cell, p=self.p, kappa=self.kappa, e_or=self.e_or, s_form=self.s_form,
                    bars={q: self.fp64_bar(q) for q in ("K", "l", "eta")})


SPLIT_TOL = 1e-6    # required element-wise bar of the split path on K_e and l_e (eta stays FP64)


def check_fp64(ref, Kg, lg, eg, what=""):
    """FP64 path: every entry of K_e and l_e and eta within the oracle-derived
    bar; the Robin null rows exactly zero.  Returns the errors."""
    e = ref.errors(Kg, lg, eg)
    info = (what, ref.summary(), e)
    assert e["null_exact"], info
    assert e["K"] <= ref.fp64_bar("K"), info
    assert e["l"] <= ref.fp64_bar("l"), info
    if "eta" in e:
        assert e["eta"] <= ref.fp64_bar("eta"), info
    return e


def check_split(ref, Kg, lg, eg, what=""):
    """Split path: K_e and l_e element-wise within SPLIT_TOL (plus the FP64
    bar), eta (FP64) within the FP64 bar; the Robin null rows exactly zero."""
    e = ref.errors(Kg, lg, eg)
    info = (what, ref.summary(), e)
    assert e["null_exact"], info
    assert e["K"] <= SPLIT_TOL + ref.fp64_bar("K"), info
    assert e["l"] <= SPLIT_TOL + ref.fp64_bar("l"), info
    if "eta" in e:
        assert e["eta"] <= ref.fp64_bar("eta"), info
    return e


def oracle_global_solve(w):
    """The oracle's whole global solve of workload w (every cell's K_e, its
    condensation, the assembled trace system solved densely, reconstruction,
    and the residual indicator of the reconstructed cell vectors).  Returns
    (traces, cell vectors, eta per cell, cond(A))."""
    from oracle import dpg_assembly as OA
    from oracle import dpg_oracle as O
    cells = []
    for c in range(w.n_cells):
        G, Bf, l, K, le, _ = oracle_cell(w, c)
        cells.append((G, Bf, l, K, le, 6 * (int(w.degree[c]) + 1) ** 3))
    cond = [OA.condense(K, le, nu) for (_, _, _, K, le, nu) in cells]
    glob, n = OA.trace_numbering(w.cells, w.face_kind, w.degree)
    Ao, bo = OA.assemble([a for a, _ in cond], [b for _, b in cond], glob, n)
    Ad = Ao.toarray()
    to = np.linalg.solve(Ad, bo)
    ev = np.linalg.eigvalsh(Ad)
    xs, etas = [], []
    for (G, Bf, l, K, le, nu), g in zip(cells, glob):
        x = OA.reconstruct(K, le, nu, OA.scatter(to, g))
        xs.append(x)
        etas.append(O.local_solve(G, Bf, l, x)[2])
    return to, xs, np.array(etas), ev.max() / ev.min()
