"""Pins of the oracle's kernel functions U and T against what the mathematics fixes.

* Static limit s -> 0: the Kelvin solution (textbook closed form).
* U solves the Laplace-domain Navier equation  mu Lap u + (lam + mu) grad div u - rho s^2 u = 0
  away from the source (checked by finite differences of the oracle's own U).
* U equals the textbook Laplace-domain form U = (psi d_ij - chi rh_i rh_j) / (4 pi rho c2^2)
  with psi, chi evaluated in 50-digit arithmetic (mpmath), on both series and closed-form
  branches of the oracle.
* T equals the traction of the finite-difference stress of U (stress law of Sec. 2.1).
* Conjugate symmetry U(conj s) = conj U(s) (real kernel coefficients; Sec. 4.1 uses it).
"""
import mpmath as mp
import numpy as np
import pytest

import oracle

RHO, C1, C2 = 1.0, 1.0, 0.5


def U(x, y, s, rho=RHO, c1=C1, c2=C2):
    return oracle.kernel_point(0, x, y, None, s, rho, c1, c2)


def T(x, y, n, s, rho=RHO, c1=C1, c2=C2):
    return oracle.kernel_point(1, x, y, n, s, rho, c1, c2)


def kelvin(rv, rho, c1, c2):
    r = np.linalg.norm(rv)
    rh = rv / r
    return ((1 / c1**2 + 1 / c2**2) * np.eye(3) + (1 / c2**2 - 1 / c1**2) * np.outer(rh, rh)) / (8 * np.pi * rho * r)


@pytest.mark.parametrize("rv", [[0.3, 0.2, 0.1], [-1.2, 0.4, 2.0], [1e-3, -2e-3, 5e-4]])
def test_static_limit_is_kelvin(rv):
    rv = np.array(rv)
    for rho, c1, c2 in [(1.0, 1.0, 0.5), (2.5, 3.0, 1.1)]:
        Uo = U(np.zeros(3), rv, 1e-13, rho, c1, c2)
        Ke = kelvin(rv, rho, c1, c2)
        assert np.abs(Uo - Ke).max() <= 1e-11 * np.abs(Ke).max()


def _mp_textbook_U(rv, s, rho, c1, c2):
    mp.mp.dps = 50
    rv = [mp.mpf(float(v)) for v in rv]
    r = mp.sqrt(sum(v * v for v in rv))
    rh = [v / r for v in rv]
    s = mp.mpc(s.real, s.imag)
    k1, k2 = s / c1, s / c2
    e1, e2 = mp.exp(-k1 * r), mp.exp(-k2 * r)
    q = (mp.mpf(c2) / c1) ** 2
    psi = e2 / r * (1 + 1 / (k2 * r) + 1 / (k2 * r) ** 2) - q * e1 / r * (1 / (k1 * r) + 1 / (k1 * r) ** 2)
    chi = e2 / r * (1 + 3 / (k2 * r) + 3 / (k2 * r) ** 2) - q * e1 / r * (1 + 3 / (k1 * r) + 3 / (k1 * r) ** 2)
    out = np.zeros((3, 3), dtype=np.complex128)
    for i in range(3):
        for j in range(3):
            v = (psi * (1 if i == j else 0) - chi * rh[i] * rh[j]) / (4 * mp.pi * rho * c2**2)
            out[i, j] = complex(v)
    return out


@pytest.mark.parametrize("s", [0.7 + 0.2j, 6.45, 13.8 - 9.7j, 1.78 + 30j, 0.05 + 0.01j])
@pytest.mark.parametrize("rlen", [0.01, 0.3, 1.9])
def test_U_matches_textbook_form(s, rlen):
    rv = np.array([0.48, -0.6, 0.64]) * rlen
    for rho, c1, c2 in [(1.0, 1.0, 0.5), (2660.0, 5994.26, 3204.07), (1.0, 1.0, 0.55)]:
        Uo = U(np.zeros(3), rv, s, rho, c1, c2)
        Ut = _mp_textbook_U(rv, complex(s), rho, c1, c2)
        assert np.abs(Uo - Ut).max() <= 1e-13 * np.abs(Ut).max(), (s, rlen, c1)


def test_branch_boundary_both_sides_exact():
    # the oracle switches from series to closed form at |s r| / c2 = 2: both sides must
    # agree with the 50-digit textbook value
    s = 3.0 + 4.0j  # |s| = 5
    rb = 2.0 * C2 / 5.0
    d = np.array([0.6, 0.0, 0.8])
    for f in (1 - 1e-12, 1 + 1e-12):
        rv = d * rb * f
        a = U(np.zeros(3), rv, s)
        t = _mp_textbook_U(rv, s, RHO, C1, C2)
        assert np.abs(a - t).max() <= 1e-14 * np.abs(t).max()


@pytest.mark.parametrize("s", [0.9 + 0.4j, 6.45, 11.5 - 16.7j])
def test_U_solves_navier_equation(s):
    rho, c1, c2 = RHO, C1, C2
    mu = rho * c2**2
    lam = rho * c1**2 - 2 * mu
    y0 = np.array([0.41, -0.23, 0.32])
    h = 2e-4

    def u(y):
        return U(np.zeros(3), y, s)  # row i = load direction, column j = component

    e = np.eye(3)
    H = np.zeros((3, 3, 3, 3), dtype=np.complex128)  # d2 u_ij / dy_a dy_b
    for a in range(3):
        for b in range(3):
            if a == b:
                H[:, :, a, a] = (u(y0 + h * e[a]) - 2 * u(y0) + u(y0 - h * e[a])) / h**2
            else:
                H[:, :, a, b] = (u(y0 + h * e[a] + h * e[b]) - u(y0 + h * e[a] - h * e[b])
                                 - u(y0 - h * e[a] + h * e[b]) + u(y0 - h * e[a] - h * e[b])) / (4 * h * h)
    u0 = u(y0)
    lap = np.einsum("ijaa->ij", H)
    grad_div = np.einsum("ikkj->ij", H)  # d/dy_j (sum_k d u_ik / dy_k)
    res = mu * lap + (lam + mu) * grad_div - rho * s * s * u0
    scale = max(np.abs(mu * lap).max(), np.abs(rho * s * s * u0).max())
    assert np.abs(res).max() <= 2e-5 * scale


@pytest.mark.parametrize("s", [0.9 + 0.4j, 6.45, 25.9, 11.5 - 16.7j, 1e-9])
def test_T_is_traction_of_fd_stress(s):
    rho, c1, c2 = RHO, C1, C2
    mu = rho * c2**2
    lam = rho * c1**2 - 2 * mu
    x = np.array([0.1, 0.2, -0.1])
    y = np.array([0.5, -0.1, 0.3])
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    h = 1e-5
    G = np.zeros((3, 3, 3), dtype=np.complex128)  # d U_ij / d y_k
    for k in range(3):
        d = np.zeros(3)
        d[k] = h
        G[:, :, k] = (U(x, y + d, s) - U(x, y - d, s)) / (2 * h)
    Tfd = np.zeros((3, 3), dtype=np.complex128)
    for i in range(3):
        eps = 0.5 * (G[i] + G[i].T)
        sig = lam * np.trace(G[i]) * np.eye(3) + 2 * mu * eps
        Tfd[i] = sig @ n
    To = T(x, y, n, s)
    assert np.abs(To - Tfd).max() <= 1e-7 * np.abs(To).max()


def test_static_traction_is_kelvin_traction():
    # textbook static traction of the Kelvin solution (nu from c1, c2)
    c1, c2 = C1, C2
    nu = (c1**2 - 2 * c2**2) / (2 * (c1**2 - c2**2))
    x = np.zeros(3)
    y = np.array([0.3, -0.4, 0.5])
    n = np.array([0.2, 0.9, -0.4])
    n /= np.linalg.norm(n)
    rv = y - x
    r = np.linalg.norm(rv)
    rh = rv / r
    drdn = rh @ n
    Tk = np.zeros((3, 3))
    for i in range(3):
        for j in range(3):
            Tk[i, j] = -1.0 / (8 * np.pi * (1 - nu) * r**2) * (
                drdn * ((1 - 2 * nu) * (i == j) + 3 * rh[i] * rh[j]) - (1 - 2 * nu) * (rh[i] * n[j] - rh[j] * n[i]))
    To = T(x, y, n, 1e-13)
    assert np.abs(To - Tk).max() <= 1e-10 * np.abs(Tk).max()


@pytest.mark.parametrize("s", [6.45 + 3.1j, 0.2 - 0.7j, 20.0 + 15.0j])
def test_conjugate_symmetry(s):
    x = np.array([0.0, 0.1, 0.2])
    y = np.array([0.7, -0.3, 0.4])
    n = np.array([0.0, 0.6, 0.8])
    for which in (0, 1):
        a = oracle.kernel_point(which, x, y, n, s)
        b = oracle.kernel_point(which, x, y, n, np.conj(s))
        assert np.abs(a - np.conj(b)).max() <= 1e-14 * np.abs(a).max()


def test_U_symmetric():
    a = U(np.zeros(3), np.array([0.3, -0.7, 0.2]), 4.0 - 2.0j)
    assert np.abs(a - a.T).max() <= 1e-15 * np.abs(a).max()
