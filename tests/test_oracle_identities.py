"""Pins of the oracle's single and double layer entries through identities of elastodynamics.

* Rigid-body translation (static limit): sum_j K[i, j] = -I/2 at every centroid of a closed
  polyhedral surface (the solid angle at a flat-element centroid is 2 pi), which pins the
  principal-value self term, the near rule and the sign and index order of T.
* Somigliana identity (eq. (rep) in the Laplace domain) with the full-space field of a point
  load at p = [1.5, 1.2, 1.2] in direction d = [1, 1, 1] (the source of Sec. 4.1 / App. A):
  u(x) = int U t - int T u inside the body, 0 outside, at second order in h.
* Collocation form at the centroids (eq. (SBIE), C = I/2): converges under refinement.
* Pulsating sphere (exterior domain, normals into the sphere): radial field u = A grad phi,
  phi = exp(-k r)/r, k = s/c1, with traction from the stress law of Sec. 2.1.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15292_amd import workloads

P_SRC = np.array([1.5, 1.2, 1.2])
D_SRC = np.array([1.0, 1.0, 1.0])


def _geom(X, T):
    C = X[T].mean(axis=1)
    n = np.cross(X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]])
    n /= np.linalg.norm(n, axis=1)[:, None]
    return C, n


def _dense_blocks(P, op, l=0):
    K = P.K
    ii, jj = np.meshgrid(np.arange(K), np.arange(K), indexing="ij")
    return P.entries(op, ii.ravel(), jj.ravel(), l).reshape(K, K, 3, 3)


@pytest.mark.parametrize("mesh", ["ico1", "ico2", "cube4"])
def test_rigid_body_static_double_layer(mesh):
    X, T = {"ico1": lambda: workloads.icosphere(1), "ico2": lambda: workloads.icosphere(2),
            "cube4": lambda: workloads.cube_grid(4, 1.0)}[mesh]()
    P = oracle.Problem(X, T, [1e-12], near_on=True)
    S = _dense_blocks(P, oracle.OP_K).sum(axis=1)
    assert np.abs(S + 0.5 * np.eye(3)).max() < 5e-5
    # the free term variant is the rigid-body null operator
    S2 = _dense_blocks(P, oracle.OP_HK).sum(axis=1)
    assert np.abs(S2).max() < 5e-5


def _point_source_data(X, T, s):
    C, n = _geom(X, T)
    u = np.array([D_SRC @ oracle.kernel_point(0, P_SRC, C[j], None, s) for j in range(len(T))])
    t = np.array([D_SRC @ oracle.kernel_point(1, P_SRC, C[j], n[j], s) for j in range(len(T))])
    return u, t


@pytest.mark.slow
def test_somigliana_interior_and_exterior_points():
    s = 2.0 + 1.0j
    pts_in = np.array([[0.1, 0.2, -0.1], [0.0, 0.0, 0.0], [0.3, -0.3, 0.4]])
    pts_out = np.array([[0.2, 1.6, -0.3], [-2.0, 0.1, 0.5]])
    errs = []
    for lvl in (1, 2):
        X, T = workloads.icosphere(lvl)
        K = len(T)
        u, t = _point_source_data(X, T, s)
        P = oracle.Problem(X, T, [s], near_on=True)
        e_in = 0.0
        for q in range(len(pts_in)):
            rep = (np.einsum("jab,jb->a", P.point_entries(0, pts_in, q, np.arange(K), 0), t)
                   - np.einsum("jab,jb->a", P.point_entries(1, pts_in, q, np.arange(K), 0), u))
            ex = D_SRC @ oracle.kernel_point(0, P_SRC, pts_in[q], None, s)
            e_in = max(e_in, np.abs(rep - ex).max() / np.abs(ex).max())
        errs.append(e_in)
        for q in range(len(pts_out)):
            rep = (np.einsum("jab,jb->a", P.point_entries(0, pts_out, q, np.arange(K), 0), t)
                   - np.einsum("jab,jb->a", P.point_entries(1, pts_out, q, np.arange(K), 0), u))
            assert np.abs(rep).max() < 0.1 * np.abs(u).max()
    assert errs[0] < 0.06 and errs[1] < 0.016
    assert errs[0] / errs[1] > 3.0  # second order in h


@pytest.mark.slow
def test_somigliana_collocation_converges():
    s = 2.0 + 1.0j
    res = []
    for lvl in (1, 2):
        X, T = workloads.icosphere(lvl)
        u, t = _point_source_data(X, T, s)
        P = oracle.Problem(X, T, [s], near_on=True)
        V = _dense_blocks(P, oracle.OP_V)
        Kk = _dense_blocks(P, oracle.OP_K)
        r = 0.5 * u - (np.einsum("ijab,jb->ia", V, t) - np.einsum("ijab,jb->ia", Kk, u))
        res.append(np.abs(r).max() / np.abs(u).max())
    assert res[0] < 0.03 and res[1] < 0.01
    assert res[1] < 0.5 * res[0]


def _pulsating_sphere(points, normals, s, rho=1.0, c1=1.0, c2=0.5, a=2.5):
    """Exact displacement and traction of the radially pulsating unit sphere."""
    mu = rho * c2**2
    lam = rho * c1**2 - 2 * mu
    k = s / c1
    G = a**4 * 24.0 / (s + a) ** 5  # Laplace transform of (a t)^4 exp(-a t)
    dphi1 = -(1 + k) * np.exp(-k)   # phi'(1) for phi = exp(-k r)/r
    A = G / dphi1
    u = np.zeros((len(points), 3), dtype=np.complex128)
    t = np.zeros_like(u)
    for q, (x, n) in enumerate(zip(points, normals)):
        r = np.linalg.norm(x)
        rh = x / r
        e = np.exp(-k * r)
        phi = e / r
        d1 = -(1 + k * r) * e / r**2
        d2 = (2 + 2 * k * r + (k * r) ** 2) * e / r**3
        u[q] = A * d1 * rh
        grad = A * (d2 * np.outer(rh, rh) + d1 / r * (np.eye(3) - np.outer(rh, rh)))
        sig = lam * A * k * k * phi * np.eye(3) + 2 * mu * grad
        t[q] = sig @ n
    return u, t


@pytest.mark.slow
def test_pulsating_sphere_collocation_converges():
    s = 1.78 + 0.9j
    res = []
    for lvl in (1, 2):
        X, T = workloads.icosphere(lvl)
        T = T[:, [0, 2, 1]].copy()  # exterior domain: normals point into the sphere
        C, n = _geom(X, T)
        u, t = _pulsating_sphere(C, n, s)
        P = oracle.Problem(X, T, [s], near_on=True)
        V = _dense_blocks(P, oracle.OP_V)
        Kk = _dense_blocks(P, oracle.OP_K)
        r = 0.5 * u - (np.einsum("ijab,jb->ia", V, t) - np.einsum("ijab,jb->ia", Kk, u))
        res.append(np.abs(r).max() / np.abs(u).max())
    assert res[1] < 0.03
    assert res[1] < 0.6 * res[0]


def test_oracle_solve_pulsating_sphere_converges():
    """The oracle's dense solve of V t = (I/2 + K) u (Sec. 2.3 collocation system at one
    contour point) recovers the exact traction of the pulsating sphere, with the error
    falling under refinement."""
    s = 1.78 + 0.9j
    err = []
    for lvl in (1, 2):
        X, T = workloads.icosphere(lvl)
        T = T[:, [0, 2, 1]].copy()
        C, n = _geom(X, T)
        u, t = _pulsating_sphere(C, n, s)
        P = oracle.Problem(X, T, [s], near_on=True)
        x = P.solve(oracle.OP_V, u.reshape(1, 1, -1), rhs_op=oracle.OP_HK)
        err.append(np.linalg.norm(x[0, 0] - t.ravel()) / np.linalg.norm(t))
    assert err[1] < 0.05
    assert err[1] < 0.6 * err[0]


def test_oracle_solve_is_inverse():
    """solve(op, A x) = x for the dense operator itself (two right-hand sides, two
    frequencies), and the right-hand-side operator is applied before the solve."""
    X, T = workloads.icosphere(1)
    s = [1.5 + 0.5j, 4.0 - 2.0j]
    P = oracle.Problem(X, T, s, near_on=True)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 2, 3 * P.K)) + 1j * rng.standard_normal((2, 2, 3 * P.K))
    V = P.dense(oracle.OP_V)
    H = P.dense(oracle.OP_HK)
    b = np.einsum("lij,rlj->rli", V, x)
    assert np.abs(P.solve(oracle.OP_V, b) - x).max() < 1e-9 * np.abs(x).max()
    c = np.einsum("lij,rlj->rli", np.linalg.inv(H), b)  # H^-1 V x, so V^-1 H c = x
    assert np.abs(P.solve(oracle.OP_V, c, rhs_op=oracle.OP_HK) - x).max() < 1e-8 * np.abs(x).max()
