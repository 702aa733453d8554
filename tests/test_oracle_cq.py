"""Pins of the oracle's convolution quadrature (oracle/cq.py): the weights of K(s) = s and
K(s) = 1 are the BDF2 coefficients and the identity, the weights of K(s) = 1/s are the
series of dt / delta(z), convolution with K(s) = 1/(s + a) converges to the exact
convolution at second order, and marching on in time inverts the convolution."""
import numpy as np

from oracle import cq


def _setup(L, T=1.0):
    dt = T / L
    R = 1e-10 ** (1.0 / (2 * L))
    z, s = cq.contour(L, dt, R)
    return dt, R, s


def test_weights_of_s_are_the_bdf2_coefficients():
    L = 32
    dt, R, s = _setup(L)
    om = cq.weights(s, R)
    ref = np.zeros(L)
    ref[:3] = np.array([1.5, -2.0, 0.5]) / dt
    assert np.abs(om - ref).max() <= 1e-6 / dt  # aliasing R^L = 1e-5 times at most 2 / dt
    om1 = cq.weights(np.ones(L), R)
    assert abs(om1[0] - 1) < 1e-12 and np.abs(om1[1:]).max() < 1e-9


def test_inverse_weights_are_the_series_of_dt_over_delta():
    # K(s) = 1/s: omega_k are the Taylor coefficients of dt / delta(z), from the recurrence
    # 1.5 c_k - 2 c_{k-1} + 0.5 c_{k-2} = [k = 0]
    L = 64
    dt, R, s = _setup(L)
    om = cq.weights(1.0 / s, R)
    c = np.zeros(L)
    for k in range(L):
        c[k] = ((1.0 if k == 0 else 0.0) + 2.0 * (c[k - 1] if k >= 1 else 0.0)
                - 0.5 * (c[k - 2] if k >= 2 else 0.0)) / 1.5
    assert np.abs(om - dt * c).max() <= 1e-4 * dt  # aliasing: R^L = 1e-5 times the sum of |c|


def test_convolution_converges_at_second_order():
    # y(t) = int_0^t exp(-a (t - tau)) tau dtau = (a t - 1 + exp(-a t)) / a^2
    a, T = 2.0, 1.0
    errs = []
    for L in (16, 32, 64):
        dt, R, s = _setup(L, T)
        tn = dt * np.arange(L)
        y = cq.convolve(cq.weights(1.0 / (s + a), R), tn)
        ex = (a * tn - 1 + np.exp(-a * tn)) / a ** 2
        errs.append(np.abs(y - ex).max())
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0, errs


def test_marching_inverts_the_convolution():
    rng = np.random.default_rng(2)
    L, M = 16, 5
    dt, R, s = _setup(L)
    # a matrix-valued K(s) = A + s B with A, B well conditioned
    A = np.eye(M) * 3 + 0.3 * rng.standard_normal((M, M))
    Bm = 0.1 * rng.standard_normal((M, M))
    V = A[None] + s[:, None, None] * Bm[None]
    t_true = rng.standard_normal((L, M)) + 1j * rng.standard_normal((L, M))
    g = cq.convolve(cq.weights(V, R), t_true)
    t = cq.dirichlet(V, None, g, R)
    assert np.abs(t - t_true).max() < 1e-8 * np.abs(t_true).max()
