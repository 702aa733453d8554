"""GPU parity of the time stepping by BDF2 convolution quadrature (bem_cq_dirichlet): against
the oracle's marching on in time with the dense operators (oracle/cq.py), with dense and
compressed operators, and against the convolution quadrature of the pulsating sphere's
closed-form traction (the same time discretisation, so the two differ by the spatial error
only)."""
import numpy as np
import pytest

import oracle
from oracle import cq
from paper_2607_15292_amd import binding as B
from paper_2607_15292_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _sphere(level):
    X, T = W.icosphere(level)
    return X, T[:, [0, 2, 1]].copy()  # exterior domain: normals into the sphere


def _ctx(X, T, s):
    c = B.Context(0)
    c.set_mesh(X, T)
    c.set_material(1.0, 1.0, 0.5)
    c.set_frequencies(s)
    c.set_quadrature(near_on=True)
    return c


def _contour(L, dt):
    return W.bdf2_contour(L, dt), 1e-10 ** (1.0 / (2 * L))


@pytest.mark.parametrize("compressed", [False, True])
def test_cq_matches_oracle_marching(torch, compressed):
    X, T = _sphere(1)
    L, dt = 16, 0.1
    s, R = _contour(L, dt)
    c = _ctx(X, T, s)
    if compressed:
        V = c.compress(B.OP_V, eps3d=1e-10, leaf=16, prec=B.PREC_F64)
        H = c.compress(B.OP_HK, eps3d=1e-10, leaf=16, prec=B.PREC_F64)
    else:
        V = c.assemble_dense(B.OP_V)
        H = c.assemble_dense(B.OP_HK)
    N = 12
    g = W.random_rhs(80, (N, 3 * len(T)))
    t, st = V.cq_dirichlet(torch.tensor(g, device="cuda"), dt, R, H=H, tol=1e-12, restart=60)
    assert st["converged"] == 1 and st["rc"] == 0
    P = oracle.Problem(X, T, s, near_on=True)
    ref = cq.dirichlet(P.dense(oracle.OP_V), P.dense(oracle.OP_HK), g, R)
    err = np.abs(t.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < (1e-7 if compressed else 1e-9), err
    # without H the right-hand side is g itself
    t2, _ = V.cq_dirichlet(g, dt, R, tol=1e-12, restart=60)
    ref2 = cq.dirichlet(P.dense(oracle.OP_V), None, g, R)
    assert np.abs(t2 - ref2).max() / np.abs(ref2).max() < (1e-7 if compressed else 1e-9)


def test_cq_pulsating_sphere(torch):
    X, T = _sphere(2)
    L, dt = 32, 0.1
    s, R = _contour(L, dt)
    C = X[T].mean(axis=1)
    n = np.cross(X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]])
    n /= np.linalg.norm(n, axis=1)[:, None]
    a = 2.5
    Gs = a ** 4 * 24.0 / (s + a) ** 5
    U = np.empty((L, 3 * len(T)), dtype=np.complex128)
    Tr = np.empty_like(U)
    for l in range(L):
        u, tr = W.pulsating_sphere(C, n, s[l], a=a)
        U[l], Tr[l] = u.ravel() / Gs[l], tr.ravel() / Gs[l]
    tn = dt * np.arange(L)
    phi = (a * tn) ** 4 * np.exp(-a * tn)  # the pulse whose transform is G(s)
    g = cq.convolve(cq.weights(U, R), phi[:, None] * np.ones((1, 3 * len(T))))
    t_ref = cq.convolve(cq.weights(Tr, R), phi[:, None] * np.ones((1, 3 * len(T))))
    c = _ctx(X, T, s)
    V = c.compress(B.OP_V, eps3d=1e-8, leaf=32, prec=B.PREC_F64)
    H = c.compress(B.OP_HK, eps3d=1e-8, leaf=32, prec=B.PREC_F64)
    t, st = V.cq_dirichlet(torch.tensor(g, device="cuda"), dt, R, H=H, tol=1e-8)
    assert st["converged"] == 1
    err = np.abs(t.cpu().numpy() - t_ref).max() / np.abs(t_ref).max()
    assert err < 0.06, err  # spatial discretisation error at 320 triangles (3.8e-2 per frequency)


def test_cq_argument_errors(torch):
    X, T = _sphere(1)
    L, dt = 8, 0.1
    s, R = _contour(L, dt)
    c = _ctx(X, T, s)
    V = c.assemble_dense(B.OP_V)
    g = W.random_rhs(1, (L + 1, 3 * len(T)))
    with pytest.raises(B.BemError):
        V.cq_dirichlet(g, dt, R)  # N > L
    with pytest.raises(B.BemError) as e:
        V.cq_dirichlet(g[:4], 2 * dt, R)  # contour of another step
    assert e.value.code == -4  # BEM_ERR_FREQ
