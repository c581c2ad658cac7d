"""Plain CPU oracle of the electromagnetic power dissipated in each cell
(§3.2, the heat source of the enthalpy equation: Q_em = sigma |E|^2 / 2 +
omega eps0 eps_im |E|^2 / 2 + omega mu0 mu_im |H|^2 / 2, the time average of
minus the divergence of the Poynting vector).

TEST INFRASTRUCTURE ONLY.  Only ``tests/`` may import this module.  It shares
no code with the HIP library.

In the non-dimensional variables of the solver (lengths in units of L, E in
units of E0, H in units of E0/Z0, omega = 2 pi f L / c0) the density is
q = omega (eps_im |E|^2 + mu_im |H|^2) / 2 and Q_em = q E0^2 / (Z0 L); the
conductivity is part of eps_im.  Per cell this returns
  (integral of q, integral of |E|^2, integral of |H|^2)
over the cell for its DG coefficient vector u = [E_x, E_y, E_z, H_x, H_y, H_z]
(each on the (p+1)^3 Lagrange-GLL functions), by Gauss quadrature exact for
the integrand on trilinear cells (p + 2 points per axis).
"""
from __future__ import annotations

import numpy as np

from .dpg_oracle import trial_basis_ref, trilinear_map, volume_rule


def cell_power(X, p: int, u, eps: complex, mu: complex, omega: float):
    pts, w = volume_rule(p + 2)
    _, J = trilinear_map(X, pts)
    dV = w * np.abs(np.linalg.det(J))
    phi = trial_basis_ref(p, pts)                       # [m1, npts]
    m1 = (p + 1) ** 3
    u = np.asarray(u, complex)[:6 * m1].reshape(6, m1)
    F = u @ phi                                         # [6, npts] field components at the points
    e2 = np.sum(np.abs(F[:3]) ** 2, axis=0)
    h2 = np.sum(np.abs(F[3:]) ** 2, axis=0)
    IE, IH = float(dV @ e2), float(dV @ h2)
    return 0.5 * omega * (complex(eps).imag * IE + complex(mu).imag * IH), IE, IH
