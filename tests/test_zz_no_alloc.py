"""bem_aca_matrix_noalloc (the allocation-free variant of bem_aca_matrix, for callers that
cannot allocate) against bem_aca_matrix through the C-ABI: two calls in a row on the same
GPU, the second with a smaller matrix, in both precisions.  The two entry points run the
same kernels on the same input, so the column counts and ranks agree exactly and the
factors to rounding (bit-identical in practice).  The library-held scratch keeps the
previous call's contents, which must not leak into the next result."""
import numpy as np
import pytest

import oracle
from oracle import aca3d as A3
from paper_2607_15292_amd import binding as B
from paper_2607_15292_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_ctx():
    import torch
    assert torch.cuda.is_available()
    return torch, B.Context(0)


def _kernel_face(nr, nc, l=1):
    X, T = W.cube_grid(8, 1.0)
    P = oracle.Problem(X, T, W.bdf2_contour(4, 0.1))
    C = X[T].mean(axis=1)
    rows = np.flatnonzero(C[:, 0] < -0.99)[:nr]
    cols = np.flatnonzero(C[:, 0] > 0.99)[:nc]
    ii, jj = np.meshgrid(rows, cols, indexing="ij")
    E = P.entries(oracle.OP_V, ii.ravel(), jj.ravel(), np.full(ii.size, l)).reshape(len(rows), len(cols), 3, 3)
    return A3.blocks_to_matrix(E)


def _same(torch, ctx, A, rtol):
    tol = rtol * np.linalg.norm(A)
    kc, kk, U, V = ctx.aca_matrix(A, tol, prec=B.PREC_MIXED if A.dtype == np.complex64 else B.PREC_F64)
    kc2, kk2, U2, V2 = ctx.aca_matrix_noalloc(torch.tensor(A, device="cuda"), tol)
    assert (kc2, kk2) == (kc, kk)
    assert kk > 0
    U2, V2 = U2.cpu().numpy(), V2.cpu().numpy()
    assert U2.dtype == A.dtype and U2.shape == U.shape and V2.shape == V.shape
    su, sv = np.abs(U).max(), np.abs(V).max()
    assert np.abs(U2 - U).max() <= 1e-14 * su and np.abs(V2 - V).max() <= 1e-14 * sv
    return kc, kk


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_noalloc_matches_allocating_entry(torch_ctx, dtype):
    torch, ctx = torch_ctx
    big = _kernel_face(48, 40).astype(dtype)
    small = _kernel_face(20, 15, l=2).astype(dtype)
    rtol = 1e-5 if dtype == np.complex128 else 1e-4
    r1 = _same(torch, ctx, big, rtol)
    r2 = _same(torch, ctx, small, rtol)
    assert r2[0] <= r1[0]


def test_noalloc_exact_low_rank_and_limits(torch_ctx):
    torch, ctx = torch_ctx
    rng = np.random.default_rng(17)
    m, n, r = 128, 96, 9
    A = (rng.standard_normal((3 * m, r)) + 1j * rng.standard_normal((3 * m, r))) @ \
        (rng.standard_normal((r, 3 * n)) + 1j * rng.standard_normal((r, 3 * n)))
    kc, kk, U, V = ctx.aca_matrix_noalloc(torch.tensor(A, device="cuda"), 1e-10 * np.linalg.norm(A))
    assert (kc, kk) == (r, r)
    Ag = U.cpu().numpy() @ V.cpu().numpy().conj().T
    assert np.linalg.norm(Ag - A) < 1e-9 * np.linalg.norm(A)
    # beyond the largest size: rejected before any work
    too_big = torch.zeros((3 * 129, 6), dtype=torch.complex128, device="cuda")
    with pytest.raises(B.BemError):
        ctx.aca_matrix_noalloc(too_big, 1.0)
    # host buffers are rejected
    kk_t = torch.zeros(2, dtype=torch.int32, device="cuda")
    Ah = np.zeros((6, 6), dtype=np.complex128)
    Ud = torch.zeros(36, dtype=torch.complex128, device="cuda")
    rc = B.lib().bem_aca_matrix_noalloc(ctx.h, B.PREC_F64, 2, 2, Ah.ctypes.data, 1.0, 0, kk_t.data_ptr(),
                                        Ud.data_ptr(), Ud.data_ptr())
    assert rc == -1
