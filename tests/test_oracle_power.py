"""Pins of the power-dissipation oracle (oracle/dpg_power.py): closed-form
integrals -- a constant field over a sheared parallelepiped (|E|^2 times the
volume |det A|), E_x = x1 over a box (a^3 b c / 3), H_y = x2 x3 over a box
(a b^3 c^3 / 9) -- and the density's weights (omega/2, eps_im, mu_im); a
dropped Jacobian is detected."""
import numpy as np
import pytest

from oracle import dpg_oracle as O
from oracle import dpg_power as P


def _coeffs(X, p, Ef, Hf):
    return O.interpolate_trial(X, p, Ef, Hf)


def _box(a, b, c, x0=(0.0, 0.0, 0.0)):
    return np.array([[x0[0] + a * i, x0[1] + b * j, x0[2] + c * k] for k in (0, 1) for j in (0, 1) for i in (0, 1)])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_power_closed_forms(p):
    rng = np.random.default_rng(p)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    X = _box(1.0, 1.0, 1.0) @ A.T + np.array([0.2, -0.1, 0.4])
    E0 = np.array([1.0 + 2.0j, -0.5j, 0.25])
    H0 = np.array([0.0, 0.3, -1.0 + 1.0j])
    u = _coeffs(X, p, lambda x: np.tile(E0, (len(x), 1)), lambda x: np.tile(H0, (len(x), 1)))
    q, IE, IH = P.cell_power(X, p, u, 2.0 + 0.7j, 1.0 + 0.2j, 3.0)
    vol = abs(np.linalg.det(A))
    assert np.isclose(IE, np.sum(np.abs(E0) ** 2) * vol, rtol=1e-12)
    assert np.isclose(IH, np.sum(np.abs(H0) ** 2) * vol, rtol=1e-12)
    assert np.isclose(q, 0.5 * 3.0 * (0.7 * IE + 0.2 * IH), rtol=1e-12)
    a, b, c = 0.3, 0.5, 0.7
    X = _box(a, b, c)
    z = lambda x: np.zeros((len(x), 3), complex)

    def ex(x):
        out = np.zeros((len(x), 3), complex)
        out[:, 0] = x[:, 0]
        return out

    def hy(x):
        out = np.zeros((len(x), 3), complex)
        out[:, 1] = x[:, 1] * x[:, 2]
        return out
    _, IE, IH = P.cell_power(X, p, _coeffs(X, p, ex, z), 1.0, 1.0, 1.0)
    assert np.isclose(IE, a ** 3 * b * c / 3.0, rtol=1e-12) and IH == 0.0
    if p >= 2:
        _, IE, IH = P.cell_power(X, p, _coeffs(X, p, z, hy), 1.0, 1.0, 1.0)
        assert np.isclose(IH, a * b ** 3 * c ** 3 / 9.0, rtol=1e-12)
    # lossless materials dissipate nothing
    assert P.cell_power(X, p, _coeffs(X, p, ex, ex), 4.0, 1.0, 2.0)[0] == 0.0


def test_power_planted_missing_jacobian_fails(monkeypatch):
    orig = P.trilinear_map

    def unit_jac(X, pts):
        x, J = orig(X, pts)
        return x, np.broadcast_to(np.eye(3), J.shape)
    monkeypatch.setattr(P, "trilinear_map", unit_jac)
    with pytest.raises(AssertionError):
        test_power_closed_forms(1)
