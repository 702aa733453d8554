"""GPU parity of the per-slice ACA + recompression (Sec. 3.1, eq. (ACA)) with the numpy
oracle, through bem_aca_matrix, and of the compressed product when every admissible face
goes through that pass (far_dense_max = 0).

For one matrix the two sides take the same pivots (same rules, ties to the smallest
index), so the ACA column count kc and the recompressed rank kk must agree exactly; the
reconstructions agree to the tolerance.  The failure rules (column cap, no memory saving)
give the same outcome on both sides.
"""
import numpy as np
import pytest

import oracle
from oracle import aca3d as A3
from paper_2607_15292_amd import binding as B
from paper_2607_15292_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return B.Context(0)


def _kernel_face(L=4, l=0, grid=8, nr=48, nc=40, op=oracle.OP_V):
    X, T = W.cube_grid(grid, 1.0)
    s = W.bdf2_contour(L, 0.1)
    P = oracle.Problem(X, T, s)
    C = X[T].mean(axis=1)
    rows = np.flatnonzero(C[:, 0] < -0.99)[:nr]
    cols = np.flatnonzero(C[:, 0] > 0.99)[:nc]
    ii, jj = np.meshgrid(rows, cols, indexing="ij")
    E = P.entries(op, ii.ravel(), jj.ravel(), np.full(ii.size, l)).reshape(len(rows), len(cols), 3, 3)
    return A3.blocks_to_matrix(E)


def _lowrank(rng, m, n, r):
    a = rng.standard_normal((3 * m, r)) + 1j * rng.standard_normal((3 * m, r))
    b = rng.standard_normal((r, 3 * n)) + 1j * rng.standard_normal((r, 3 * n))
    return a @ b


def _oracle(A, tol, max_cols=A3.KMAX_ACA):
    m, n = A.shape[0] // 3, A.shape[1] // 3
    U, V, ok = A3.aca_matrix(A, tol, min(max_cols, A3.face_aca_cap(m, n)))
    if not ok:
        return -1, 0, None
    Ub, Vb = A3.recompress(U, V, tol)
    kk = Ub.shape[1] if Ub.shape[1] * (m + n) < 3 * m * n else 0
    return U.shape[1], kk, (Ub @ Vb.conj().T if kk else None)


@pytest.mark.parametrize("m,n,r", [(20, 15, 6), (24, 30, 12), (33, 17, 9)])
def test_exact_low_rank(ctx, m, n, r):
    A = _lowrank(np.random.default_rng(m * n + r), m, n, r)
    tol = 1e-10 * np.linalg.norm(A)
    kc, kk, U, V = ctx.aca_matrix(A, tol)
    okc, okk, _ = _oracle(A, tol)
    assert (kc, kk) == (okc, okk) == (r, r)
    assert np.linalg.norm(U @ V.conj().T - A) < 1e-9 * np.linalg.norm(A)


@pytest.mark.parametrize("rtol", [1e-3, 1e-5, 1e-7])
@pytest.mark.parametrize("l", [0, 3])
def test_kernel_face_matches_oracle(ctx, rtol, l):
    A = _kernel_face(l=l)
    tol = rtol * np.linalg.norm(A)
    kc, kk, U, V = ctx.aca_matrix(A, tol)
    okc, okk, Ao = _oracle(A, tol)
    assert (kc, kk) == (okc, okk)
    if kk:
        Ag = U @ V.conj().T
        assert np.linalg.norm(Ag - A) <= 3 * tol
        assert np.linalg.norm(Ag - Ao) <= 2 * tol


def test_mixed_precision_face(ctx):
    """complex64 storage: the pass runs on the rounded matrix; the same rounded matrix in
    complex128 gives the oracle's ranks, and the factors (complex64) reproduce it."""
    A = _kernel_face(l=1).astype(np.complex64)
    tol = 1e-4 * np.linalg.norm(A)
    kc, kk, U, V = ctx.aca_matrix(A, tol, prec=B.PREC_MIXED)
    okc, okk, _ = _oracle(A.astype(np.complex128), tol)
    assert (kc, kk) == (okc, okk) and kk > 0
    assert U.dtype == np.complex64
    err = np.linalg.norm(U.astype(np.complex128) @ V.astype(np.complex128).conj().T - A)
    assert err <= 3 * tol + 1e-6 * np.linalg.norm(A)


def test_failure_rules(ctx):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 24)) + 1j * rng.standard_normal((30, 24))
    tol = 1e-12 * np.linalg.norm(A)
    # column cap short of 3 min(m, n): not resolved
    assert ctx.aca_matrix(A, tol, max_cols=9)[:2] == (-1, 0)
    assert _oracle(A, tol, max_cols=9)[:2] == (-1, 0)
    # full interpolation resolves, but full rank saves no memory: kept dense
    kc, kk, _, _ = ctx.aca_matrix(A, tol)
    assert (kc, kk) == _oracle(A, tol)[:2] == (24, 0)
    # zero matrix
    assert ctx.aca_matrix(np.zeros((6, 9), complex), 1.0)[:2] == (-1, 0)


def test_argument_errors(ctx):
    with pytest.raises(B.BemError):
        ctx.aca_matrix(np.zeros((6, 6), complex), -1.0)
    with pytest.raises(B.BemError):
        ctx.aca_matrix(np.zeros((6, 6), complex), 1.0, prec=7)


@pytest.mark.parametrize("prec,eps,bound", [(B.PREC_F64, 1e-5, 5e-5), (B.PREC_MIXED, 1e-5, 1e-4)])
def test_compressed_apply_with_aca_faces(ctx, prec, eps, bound):
    """Every admissible face goes through the ACA pass; rows sampled against the oracle."""
    X, T = W.icosphere(3)  # 1280 triangles
    K, L = len(T), 8
    s = W.bdf2_contour(L, 0.1)
    c = B.Context(0)
    c.set_mesh(X, T)
    c.set_material(1.0, 1.0, 0.5)
    c.set_frequencies(s)
    c.set_quadrature(near_on=True)
    op = c.compress(B.OP_V, eps3d=eps, eps_aca=eps / 100, leaf=32, prec=prec, far_dense_max=0)
    st = op.stats()
    assert st["n_far_faces"] > 0, st
    x = W.random_rhs(9, (1, L, 3 * K))
    y = op.apply(x)
    rows = np.sort(np.random.default_rng(4).choice(K, size=24, replace=False))
    P = oracle.Problem(X, T, s, near_on=True)
    yo = P.matvec_rows(B.OP_V, rows, x)
    yg = y.reshape(1, L, K, 3)[:, :, rows, :].reshape(1, L, -1)
    err = float((np.linalg.norm(yg - yo, axis=-1) / np.linalg.norm(yo, axis=-1)).max())
    assert err < bound, (err, st)
