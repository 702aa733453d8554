"""Convolution quadrature in time (oracle, numpy, FP64).  TEST INFRASTRUCTURE ONLY.

Multistep convolution quadrature of Sec. 2.4 in its uniform-step form with the BDF2
generating function delta(z) = 3/2 - 2 z + z^2 / 2: the weights are the Taylor coefficients
of K(delta(z) / dt) = sum_k omega_k z^k, computed from the values at the contour points
s_l = delta(z_l) / dt, z_l = R exp(2 pi i l / L), by the trapezoidal rule of Cauchy's integral:
omega_k = R^-k / L sum_l K(s_l) exp(-2 pi i k l / L), k < L.

The discrete convolution (eq. (matvec)) is y_n = sum_{j <= n} omega_{n-j} g_j; the Dirichlet
problem of the collocation system of Sec. 2.3 in time asks for tractions t_n with
sum_{j <= n} omega_{n-j}(V) t_j = sum_{j <= n} omega_{n-j}(I/2 + K) g_j, solved step by step
(marching on in time) by forward substitution with omega_0(V).
"""
from __future__ import annotations

import numpy as np


def bdf2_delta(z):
    """BDF2 generating function delta(z) = (1 - z) + (1 - z)^2 / 2."""
    return 1.5 - 2.0 * z + 0.5 * z * z


def contour(L, dt, R):
    """Contour points z_l and s_l = delta(z_l) / dt of the trapezoidal rule."""
    z = R * np.exp(2j * np.pi * np.arange(L) / L)
    return z, bdf2_delta(z) / dt


def weights(Ks, R):
    """omega_k, k < L, from samples Ks[l] = K(s_l) (scalars or arrays of any shape)."""
    Ks = np.asarray(Ks, dtype=np.complex128)
    L = Ks.shape[0]
    k = np.arange(L)
    F = np.exp(-2j * np.pi * np.outer(k, np.arange(L)) / L) / L  # [k, l]
    om = np.tensordot(F, Ks, axes=(1, 0))
    scale = R ** (-k.astype(np.float64))
    return om * scale.reshape((L,) + (1,) * (Ks.ndim - 1))


def convolve(om, g):
    """y_n = sum_{j <= n} omega_{n-j} g_j for scalar weights om[k] and samples g[n, ...], or
    matrix weights om[k, M, M] and vectors g[n, M]."""
    om = np.asarray(om)
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[0]
    y = np.zeros_like(g)
    for n in range(N):
        for j in range(n + 1):
            y[n] += om[n - j] @ g[j] if om.ndim == 3 else om[n - j] * g[j]
    return y


def dirichlet(V, H, g, R):
    """Marching on in time for sum_j omega_{n-j}(V) t_j = sum_j omega_{n-j}(H) g_j.
    V, H: dense operators at the contour points [L, M, M] (H = None: right-hand side g);
    g: [N, M] with N <= L.  Returns t [N, M]."""
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[0]
    wV = weights(V, R)
    b = convolve(weights(H, R), g) if H is not None else g
    t = np.zeros_like(g)
    for n in range(N):
        hist = np.zeros(g.shape[1], dtype=np.complex128)
        for j in range(n):
            hist += wV[n - j] @ t[j]
        t[n] = np.linalg.solve(wV[0], b[n] - hist)
    return t
