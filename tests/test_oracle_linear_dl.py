"""Pins of the oracle's double layer against continuous piecewise-linear shape functions
(Sec. 2.3, eqs. (subspace), (basis): the Dirichlet data of eq. (discreteCollo) are nodal,
and K of eq. (discrVK) integrates T times the hat function of each node).

* Partition of unity: the three barycentric weights of an element sum to one, so the three
  vertex-weighted operators add up to the piecewise-constant double layer, entry by entry, in
  every rule (regular, near subdivision, self principal value).
* Static rigid rotation u = w x x: a linear field, so the linear basis reproduces it on the
  flat elements of the cube exactly and (C + K) u = 0 at the centroids (the rigid-body identity
  of the double layer) up to the quadrature; the piecewise-constant basis cannot (O(h)).
* Static uniform strain u = E x (a solution of the static Navier equations, traction
  sigma(E) n constant per flat face): the Somigliana identity I/2 u(x_i) + (K u)(x_i) =
  (V t)(x_i) holds up to the quadrature with the linear basis.
* The point-source field of Sec. 4.1 (dynamic, s = 2 + i): the same identity converges at
  second order in h with nodal data, first order with centroid data.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15292_amd import workloads as W


def _cube(n):
    X, T = W.cube_grid(n, 1.0)
    C = X[T].mean(axis=1)
    nrm = np.cross(X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    return X, T, C, nrm


def test_vertex_weights_sum_to_the_constant_basis():
    X, T, _, _ = _cube(2)
    P = oracle.Problem(X, T, [1e-12, 2.0 + 1.0j, 0.7 - 3.0j], near_on=True)
    Ksum = sum(P.dense(oracle.OP_KL0 + v) for v in range(3))
    Kc = P.dense(oracle.OP_K)
    assert np.abs(Ksum - Kc).max() < 1e-13 * np.abs(Kc).max()
    # each vertex operator differs from a third of the constant one (the weights vary)
    D0 = P.dense(oracle.OP_KL0)
    assert np.abs(D0 - Kc / 3.0).max() > 1e-3 * np.abs(Kc).max()


@pytest.mark.parametrize("n", [2, 4])
def test_static_rigid_rotation(n):
    X, T, C, _ = _cube(n)
    P = oracle.Problem(X, T, [1e-12], near_on=True)
    w = np.array([0.3, -0.7, 0.5])
    ref = np.abs(np.cross(w, C)).max()
    r_lin = P.dense_linear_dl(free_term=True)[0] @ np.cross(w, X).ravel()
    r_const = P.dense(oracle.OP_HK)[0] @ np.cross(w, C).ravel()
    assert np.abs(r_lin).max() < 1e-4 * ref
    assert np.abs(r_const).max() > 100 * np.abs(r_lin).max()


@pytest.mark.parametrize("n", [2, 4])
def test_static_uniform_strain_somigliana(n):
    X, T, C, nrm = _cube(n)
    rho, cp, cs = 1.0, 1.0, 0.5
    P = oracle.Problem(X, T, [1e-12], rho, cp, cs, near_on=True)
    E = np.array([[0.2, 0.1, -0.05], [0.1, -0.3, 0.15], [-0.05, 0.15, 0.4]])
    lam, mu = rho * (cp**2 - 2 * cs**2), rho * cs**2
    sig = lam * np.trace(E) * np.eye(3) + 2 * mu * E
    t = (nrm @ sig).ravel()
    res = P.dense_linear_dl(free_term=True)[0] @ (X @ E.T).ravel() - P.dense(oracle.OP_V)[0] @ t
    assert np.abs(res).max() < 1e-4 * np.abs(C @ E.T).max()


def test_free_term_is_half_of_the_nodal_average():
    X, T, _, _ = _cube(2)
    P = oracle.Problem(X, T, [2.0 + 1.0j], near_on=True)
    Cfree = P.dense_linear_dl(free_term=True) - P.dense_linear_dl(free_term=False)
    g = np.random.default_rng(3).standard_normal((len(X), 3))
    y = (Cfree[0] @ g.ravel()).reshape(-1, 3)
    assert np.allclose(y, 0.5 * g[T].mean(axis=1), atol=1e-15)


@pytest.mark.slow
def test_point_source_second_order():
    p, dvec, s = np.array([1.5, 1.2, 1.2]), np.array([1.0, 1.0, 1.0]), 2.0 + 1.0j
    errs = []
    for n in (2, 4, 8):
        X, T, C, nrm = _cube(n)
        P = oracle.Problem(X, T, [s], near_on=True)
        un = np.array([dvec @ oracle.kernel_point(0, p, x, None, s) for x in X])
        uc = np.array([dvec @ oracle.kernel_point(0, p, c, None, s) for c in C])
        tc = np.array([dvec @ oracle.kernel_point(1, p, C[j], nrm[j], s) for j in range(len(T))])
        Vt = P.dense(oracle.OP_V)[0] @ tc.ravel()
        e_lin = np.abs(P.dense_linear_dl()[0] @ un.ravel() - Vt).max() / np.abs(uc).max()
        e_const = np.abs(P.dense(oracle.OP_HK)[0] @ uc.ravel() - Vt).max() / np.abs(uc).max()
        errs.append((e_lin, e_const))
    (l2, c2), (l4, c4), (l8, c8) = errs
    assert l2 / l4 > 3.0 and l4 / l8 > 3.0      # second order with nodal data
    assert c4 / c8 < 3.0 and l8 < 0.1
