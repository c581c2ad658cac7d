"""Adaptive loop on the residual indicator (Sec. 4.2): solve, estimate, mark,
refine, repeated.

Each pass runs the whole global solve of Algorithm 1 on the GPU through the
C ABI: the local solve, condensation, numbering and assembly of the trace
system, CG without a preconditioner, reconstruction of the interior
unknowns, the residual indicator eta_K of the global solution (a local solve
with that solution), and Doerfler marking on eta_K (the cells that carry the
first 30% of the summed indicators are refined, those within the last 5%
coarsened).

Refinement here raises the cell's trial degree p (coarsening lowers it),
within [p_min, p_max]; the mesh stays fixed.  The paper refines the mesh
(h-refinement with hanging nodes), which this library does not build; with
p-refinement the trace space stays conforming under the minimum rule on
shared edges and faces, which the trace numbering applies to cells of mixed
degree.  The enrichment dp is the same for every cell.

Only host bookkeeping lives here (the degree update and the loop); every
step of the solve runs in the library's kernels.
"""
from dataclasses import dataclass, field

import numpy as np

from . import dpg


@dataclass
class AdaptPass:
    """One pass of the loop: the solve on `degree` and its marking."""
    degree: np.ndarray            # (n_cells,) int8, the degrees this pass solved with
    n_dofs: int                   # global trace unknowns
    cg_iterations: int
    relres: float                 # ||r|| / ||b|| of the condensed system at the end of CG
    eta: np.ndarray               # (n_cells,) residual indicator of the global solution
    flags: np.ndarray             # (n_cells,) int8 marking: +1 refine, -1 coarsen, 0 keep
    failed_cells: int = 0         # cells with a nonzero info in any stage
    meta: dict = field(default_factory=dict)

    @property
    def eta_total(self) -> float:
        """(sum_K eta_K^2)^(1/2), the global residual norm."""
        return float(np.sqrt(np.sum(self.eta.astype(np.float64) ** 2)))


def next_degrees(degree, flags, p_min: int = 1, p_max: int = 4) -> np.ndarray:
    """The degrees after one marking: p + 1 where flagged for refinement, p - 1
    where flagged for coarsening, clamped to [p_min, p_max]."""
    d = np.asarray(degree, np.int16)
    f = np.asarray(flags, np.int16)
    if d.shape != f.shape:
        raise ValueError("degree and flags differ in length")
    if not (1 <= p_min <= p_max <= 4):
        raise ValueError("need 1 <= p_min <= p_max <= 4")
    return np.clip(d + np.sign(f), p_min, p_max).astype(np.int8)


def solve_and_mark(w, degree, refine_fraction: float = 0.30, coarsen_fraction: float = 0.05,
                   cg_tol: float = 1e-10, max_iter: int = 400000, device: str = "cuda:0") -> AdaptPass:
    """One pass on workload `w` (its mesh, materials and boundary data) with
    per-cell degrees `degree`."""
    import torch
    degree = np.ascontiguousarray(np.asarray(degree, np.int8))
    nc = int(degree.shape[0])
    plan = dpg.Plan(degree, w.dp)
    prob = dpg.DeviceProblem.from_workload(w, device)
    ts = None
    try:
        K, l, eta, info = plan.alloc_outputs(device)
        plan.local_solve(prob, None, K, l, eta, info)
        A, b, cinfo = plan.condense(K, l)
        ts = dpg.TraceSystem(plan, w.cells, w.face_kind)
        vals, rhs = ts.assemble(A, b)
        t = torch.zeros(max(ts.n_dofs, 1), dtype=torch.complex128, device=K.device)
        it, rr = ts.solve(vals, rhs, t, cg_tol, max_iter)
        x, rinfo = plan.reconstruct(K, l, ts.scatter(t))
        K2, l2, eta2, info2 = plan.alloc_outputs(device)
        plan.local_solve(prob, x, K2, l2, eta2, info2)
        mark_ws = torch.empty(dpg.dorfler_mark_workspace_size(nc), dtype=torch.uint8, device=K.device)
        flags = dpg.dorfler_mark(eta2[:nc], refine_fraction, coarsen_fraction, workspace=mark_ws)
        torch.cuda.synchronize(K.device)
        failed = sum(int(np.count_nonzero(a.cpu().numpy()[:nc])) for a in (info, cinfo, rinfo, info2))
        return AdaptPass(degree=degree.copy(), n_dofs=int(ts.n_dofs), cg_iterations=int(it), relres=float(rr),
                         eta=eta2.cpu().numpy()[:nc].copy(), flags=flags.cpu().numpy()[:nc].copy(),
                         failed_cells=failed)
    finally:
        if ts is not None:
            ts.close()
        plan.close()


def p_adapt(w, passes: int, degree=None, refine_fraction: float = 0.30, coarsen_fraction: float = 0.05,
            p_min: int = 1, p_max: int = 4, cg_tol: float = 1e-10, max_iter: int = 400000,
            device: str = "cuda:0", on_pass=None):
    """`passes` passes of solve -> estimate -> mark -> refine, starting from
    `degree` (default: the workload's).  Returns the list of AdaptPass; the
    degrees for a further pass are next_degrees(last.degree, last.flags)."""
    if passes < 0:
        raise ValueError("passes must be >= 0")
    deg = np.asarray(w.degree if degree is None else degree, np.int8).copy()
    out = []
    for _ in range(passes):
        ap = solve_and_mark(w, deg, refine_fraction, coarsen_fraction, cg_tol, max_iter, device)
        out.append(ap)
        if on_pass is not None:
            on_pass(ap)
        deg = next_degrees(ap.degree, ap.flags, p_min, p_max)
    return out
