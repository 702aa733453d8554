"""Pins of the numpy 3D-ACA / ACA oracle (Algorithm 1, eq. (FrobNorm), eq. (ACA)).

* A tensor of exact face-fibre rank r is recovered with rank r and to rounding.
* Interpolation: the chosen slices k_d and fibres (i_d, j_d) are reproduced exactly.
* The recursive matrix-valued Frobenius norm equals the explicit norm of the approximation.
* On a well-separated kernel block the error is a small multiple of eps, the first slice is
  k = 0 and the next ones are the small-Re(s) conjugate pairs (Sec. 4.1 observes this).
* Blocks without a regular 3x3 pivot (sigma_3 = 0 everywhere) fall back to dense storage.
* Per-slice ACA recovers exact low-rank matrices; recompression removes redundant columns
  and respects its tolerance.
"""
import numpy as np
import pytest

import oracle
from oracle import aca3d as A3
from paper_2607_15292_amd import workloads


def _rand_blocks(rng, *shape):
    return rng.standard_normal(shape + (3, 3)) + 1j * rng.standard_normal(shape + (3, 3))


def _lowrank_tensor(rng, L, m, n, r):
    C = np.zeros((L, m, n, 3, 3), dtype=np.complex128)
    for _ in range(r):
        H = _rand_blocks(rng, m, n)
        g = _rand_blocks(rng, L)
        C += np.einsum("ijab,kbc->kijac", H, g)
    return C


@pytest.mark.parametrize("r", [1, 2, 5])
def test_exact_rank_recovery(r):
    rng = np.random.default_rng(7 + r)
    C = _lowrank_tensor(rng, 12, 6, 5, r)
    ap = A3.aca3d(C, 1e-10)
    assert not ap.dense
    assert ap.rank == r
    err = np.linalg.norm(ap.tensor() - C) / np.linalg.norm(C)
    assert err < 1e-12


def _kernel_block(L=16, op=oracle.OP_V, grid=4, nr=12, nc=10):
    X, T = workloads.cube_grid(grid, 1.0)
    s = workloads.bdf2_contour(L, 0.1)
    P = oracle.Problem(X, T, s)
    C = X[T].mean(axis=1)
    rows = np.flatnonzero(C[:, 0] < -0.99)[:nr]      # on the -x face
    cols = np.flatnonzero(C[:, 0] > 0.99)[:nc]       # on the +x face
    ii, jj, ll = np.meshgrid(rows, cols, np.arange(L), indexing="ij")
    E = P.entries(op, ii.ravel(), jj.ravel(), ll.ravel()).reshape(len(rows), len(cols), L, 3, 3)
    return E.transpose(2, 0, 1, 3, 4).copy()


def test_interpolation_and_norm_on_kernel_block():
    C = _kernel_block()
    ap = A3.aca3d(C, 1e-6)
    assert not ap.dense and 1 <= ap.rank < C.shape[0]
    Ct = ap.tensor()
    scale = np.abs(C).max()
    for k, (i, j) in zip(ap.ks, ap.pivots):
        assert np.abs(Ct[k] - C[k]).max() < 1e-12 * scale            # slice k_d reproduced
        assert np.abs(Ct[:, i, j] - C[:, i, j]).max() < 1e-12 * scale  # fibre (i_d, j_d) reproduced
    # recursive norm of the kept pairs equals the explicit norm
    G = 0.0
    for a in range(ap.rank):
        for b in range(ap.rank):
            Gab = np.einsum("ijba,ijbc->ac", ap.faces[a].conj(), ap.faces[b])
            Fba = np.einsum("kab,kcb->ac", ap.fibres[b], ap.fibres[a].conj())
            G += np.real(np.trace(Gab @ Fba))
    assert abs(np.sqrt(G) - A3.frobenius_explicit(ap)) < 1e-12 * A3.frobenius_explicit(ap)
    err = np.linalg.norm(Ct - C) / np.linalg.norm(C)
    assert err < 1e-5
    # first slice is the first contour point, the next are small-Re(s) conjugate pairs
    assert ap.ks[0] == 0
    assert set(ap.ks[1:3]) <= {1, 15, 2, 14}


def test_dense_fallback_without_regular_pivot():
    rng = np.random.default_rng(3)
    L, m, n = 6, 4, 4
    a = rng.standard_normal((L, m, n, 3, 2)) + 1j * rng.standard_normal((L, m, n, 3, 2))
    b = rng.standard_normal((L, m, n, 2, 3)) + 1j * rng.standard_normal((L, m, n, 2, 3))
    C = a @ b  # every 3x3 block has rank 2: sigma_3 = 0
    ap = A3.aca3d(C, 1e-6)
    assert ap.dense and ap.rank == L
    assert np.abs(ap.tensor() - C).max() == 0.0


def test_aca_exact_low_rank_and_recompression():
    rng = np.random.default_rng(11)
    m, n, r = 20, 15, 6  # matrix-valued ACA captures rank in steps of 3
    A = (rng.standard_normal((3 * m, r)) + 1j * rng.standard_normal((3 * m, r))) @ \
        (rng.standard_normal((r, 3 * n)) + 1j * rng.standard_normal((r, 3 * n)))
    U, V, ok = A3.aca_matrix(A, 1e-12 * np.linalg.norm(A))
    assert ok and U.shape[1] == r
    assert np.linalg.norm(U @ V.conj().T - A) < 1e-10 * np.linalg.norm(A)
    # recompression of a redundant factorisation (rank 4 written with 9 columns)
    B = rng.standard_normal((3 * m, 4)) + 1j * rng.standard_normal((3 * m, 4))
    Cm = rng.standard_normal((3 * n, 4)) + 1j * rng.standard_normal((3 * n, 4))
    mix = rng.standard_normal((4, 9))
    U9, V9 = B @ mix, Cm @ np.linalg.pinv(mix).conj().T
    M = U9 @ V9.conj().T
    Ub, Vb = A3.recompress(U9, V9, 1e-10 * np.linalg.norm(M))
    assert Ub.shape[1] == 4
    assert np.linalg.norm(Ub @ Vb.conj().T - M) < 1e-10 * np.linalg.norm(M)


def test_aca_on_kernel_face_meets_tolerance():
    C = _kernel_block(L=4, grid=8, nr=48, nc=40)
    Amat = A3.blocks_to_matrix(C[0])
    for eps in (1e-4, 1e-8):
        tol = eps * np.linalg.norm(Amat)
        U, V, ok = A3.aca_matrix(Amat, tol)
        assert ok
        Ub, Vb = A3.recompress(U, V, tol)
        err = np.linalg.norm(Ub @ Vb.conj().T - Amat) / np.linalg.norm(Amat)
        assert err < 20 * eps
        assert Ub.shape[1] <= U.shape[1]


def test_aca3d_with_aca_faces_error():
    """The ACA pass over the faces (tol_d = eps_aca ||C|| / ||f_d||) keeps the tensor error
    within a small multiple of eps + rank * eps_aca, and every face it keeps as factors
    takes less memory than the dense face."""
    C = _kernel_block(L=16, grid=8, nr=48, nc=40)
    ap = A3.aca3d(C, 1e-4)
    exact = ap.tensor()
    A3.compress_faces(ap, 1e-6)
    nf = sum(uv is not None for uv in ap.factors)
    assert nf > 0
    m, n = C.shape[1:3]
    for uv in ap.factors:
        if uv is not None:
            assert uv[0].shape[1] * (m + n) < 3 * m * n
    err = np.linalg.norm(ap.tensor() - C) / np.linalg.norm(C)
    assert err < 1e-3
    # each face-fibre term moves by at most about eps_aca ||C||
    dev = np.linalg.norm(ap.tensor() - exact) / np.linalg.norm(C)
    assert dev < 2e-6 * ap.rank


def test_aca_cap_and_failure_rules():
    """A full-rank face does not resolve within a small column cap (ok False: kept dense);
    an all-zero face is kept dense; the cap is twice the break-even rank."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((30, 24)) + 1j * rng.standard_normal((30, 24))
    U, V, ok = A3.aca_matrix(A, 1e-12 * np.linalg.norm(A), max_cols=9)
    assert not ok and U.shape[1] == 9
    U, V, ok = A3.aca_matrix(A, 1e-12 * np.linalg.norm(A))
    assert ok and np.linalg.norm(U @ V.conj().T - A) < 1e-9 * np.linalg.norm(A)
    assert A3.compress_face(np.zeros((4, 5, 3, 3), complex), 1.0) == (None, -1)
    assert A3.face_aca_cap(80, 80) == 240 and A3.face_aca_cap(160, 80) == 240
    assert A3.face_aca_cap(2, 2) == 6  # at most 3 min(m, n)
    # factors that would not save memory are dropped: random 10 x 10 blocks need full rank
    H = A3.matrix_to_blocks(rng.standard_normal((30, 30)) + 1j * rng.standard_normal((30, 30)))
    uv, kc = A3.compress_face(H, 1e-10)
    assert uv is None
