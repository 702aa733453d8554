"""Pin of the oracle's matrix-free rows of the products (the reference of every check on
meshes too large for a dense oracle) against the dense operator of eq. (discrVK) at the
contour points: y[r, l, 3 q + a] = (A(s_l) x[r, l])[3 rows[q] + a].

The dense operator is assembled entry by entry and multiplied by numpy; the rows are summed
inside the C oracle without storing the operator.  A mistake in the row, frequency,
right-hand-side or component indexing of the matrix-free sum fails here."""
import numpy as np
import pytest

import oracle
from paper_2607_15292_amd import workloads as W


@pytest.mark.parametrize("op", [oracle.OP_V, oracle.OP_K, oracle.OP_HK])
@pytest.mark.parametrize("near_on", [False, True])
def test_matvec_rows_equals_dense_rows(op, near_on):
    X, T = W.cube_grid(2, 1.0)          # 48 triangles
    K, L, nrhs = len(T), 3, 2
    P = oracle.Problem(X, T, W.bdf2_contour(L, 0.1), near_on=near_on)
    D = P.dense(op)                      # [L, 3K, 3K]
    x = W.random_rhs(31, (nrhs, L, 3 * K))
    rows = np.array([0, 7, 8, 23, 47, 7], dtype=np.int32)  # unsorted, repeated, both ends
    y = P.matvec_rows(op, rows, x)
    dof = (3 * rows[:, None] + np.arange(3)[None, :]).ravel()
    yd = np.einsum("lij,rlj->rli", D[:, dof, :], x)
    assert y.shape == (nrhs, L, 3 * rows.size)
    assert np.abs(y - yd).max() < 1e-12 * np.abs(yd).max()


def test_free_term_of_hk_rows():
    """(I/2 + K) x - K x = x / 2 on the sampled rows (eq. (SBIE) at smooth points)."""
    X, T = W.icosphere(1)                # 80 triangles
    K, L = len(T), 2
    P = oracle.Problem(X, T, W.bdf2_contour(L, 0.1), near_on=True)
    x = W.random_rhs(32, (1, L, 3 * K))
    rows = np.array([3, 40, 79], dtype=np.int32)
    dof = (3 * rows[:, None] + np.arange(3)[None, :]).ravel()
    d = P.matvec_rows(oracle.OP_HK, rows, x) - P.matvec_rows(oracle.OP_K, rows, x)
    assert np.abs(d - 0.5 * x[:, :, dof]).max() < 1e-13 * np.abs(x).max()
