"""GPU parity of the double layer against continuous piecewise-linear shape functions (Sec. 2.3,
eqs. (subspace), (basis); K of eq. (discrVK) with the nodal hat functions), through the C-ABI.

* Entries: the vertex-weighted blocks int_{gamma_j} T(x_i, y) lambda_v(y) dy (BEM_OP_KL0..2)
  of every pair of a cube mesh with the near rule on (regular, near level 1 and 2 and self
  pairs) equal the oracle's element by element (1e-11 of the largest block, the principal
  value's tolerance of the piecewise-constant double layer).
* Matrix-free product (bem_apply_linear_dl) with and without the free term: equal to the
  oracle's dense linear-basis operator applied to nodal data (1e-12), host and device buffers,
  five right-hand sides (two passes of the kernel's right-hand-side loop).
* The static rigid rotation of the cube: (C + K) u = 0 up to the quadrature (1e-4).
"""
import numpy as np
import pytest

import oracle
from paper_2607_15292_amd import binding as B
from paper_2607_15292_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def ctx_for(X, T, s, near_on=True):
    c = B.Context(0)
    c.set_mesh(X, T)
    c.set_material(1.0, 1.0, 0.5)
    c.set_frequencies(s)
    c.set_quadrature(near_on=near_on)
    return c


S3 = np.array([2.0 + 1.0j, 0.7 - 3.0j, 6.4])


@pytest.mark.parametrize("near_on", [False, True])
def test_linear_dl_entries(torch, near_on):
    X, T = W.cube_grid(2, 1.0)
    K = len(T)
    c = ctx_for(X, T, S3, near_on)
    P = oracle.Problem(X, T, S3, 1.0, 1.0, 0.5, near_on=near_on)
    ii, jj, ll = (a.ravel() for a in np.meshgrid(np.arange(K), np.arange(K), np.arange(len(S3)), indexing="ij"))
    for v in range(3):
        eg = c.entries(B.OP_KL0 + v, ii, jj, ll)
        eo = P.entries(oracle.OP_KL0 + v, ii, jj, ll)
        assert np.abs(eg - eo).max() < 1e-11 * np.abs(eo).max(), v


@pytest.mark.parametrize("free_term", [False, True])
def test_linear_dl_product(torch, free_term):
    X, T = W.cube_grid(3, 1.0)  # 108 elements
    K, N, L = len(T), len(X), len(S3)
    c = ctx_for(X, T, S3)
    D = oracle.Problem(X, T, S3, 1.0, 1.0, 0.5, near_on=True).dense_linear_dl(free_term=free_term)
    g = W.random_rhs(11, (5, L, 3 * N))
    yo = np.einsum("lij,rlj->rli", D, g)
    y = c.apply_linear_dl(g, free_term=free_term)
    assert np.abs(y - yo).max() < 1e-12 * np.abs(yo).max()
    yd = c.apply_linear_dl(torch.tensor(g, device="cuda"), free_term=free_term).cpu().numpy()
    assert np.abs(yd - yo).max() < 1e-12 * np.abs(yo).max()


def test_linear_dl_static_rigid_rotation(torch):
    X, T = W.cube_grid(4, 1.0)
    c = ctx_for(X, T, np.array([1e-12]))
    w = np.array([0.3, -0.7, 0.5])
    g = np.cross(w, X).reshape(1, 1, -1).astype(np.complex128)
    r = c.apply_linear_dl(g, free_term=True)
    C = X[T].mean(axis=1)
    assert np.abs(r).max() < 1e-4 * np.abs(np.cross(w, C)).max()


def test_linear_dl_errors(torch):
    X, T = W.cube_grid(2, 1.0)
    c = ctx_for(X, T, S3)
    with pytest.raises(B.BemError):
        c.entries(B.OP_KL0, [0], [1], [0], prec=B.PREC_MIXED)
    with pytest.raises(B.BemError):
        c.entries(7, [0], [1], [0])
