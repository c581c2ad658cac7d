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
