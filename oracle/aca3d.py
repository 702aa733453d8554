"""Matrix-valued 3D-ACA (Algorithm 1, Sec. 3) and per-slice matrix-valued ACA with QR/SVD
recompression (Sec. 3.1, eq. (ACA)) in plain numpy, for small tensors.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Tensor convention: ``C[k, i, j]`` is the 3x3 block ENTRY(i, j, k) of an array of m x n
blocks over L frequencies; an approximation is C[k, i, j] ~= sum_d H_d[i, j] @ f_d[k]
(face block on the left, as in the fibre line of Algorithm 1).

Readings of the paper taken here (the same readings bind the GPU library):
  * k_1 = 0 is the first contour point; the loop is a do-while (the test needs a pair).
  * The next frequency is the argmax of sigma_3(f_d[k]) over frequencies not yet used
    (f_d[k_d] = I, so without the exclusion the argmax repeats k_d).
  * The norm of eq. (FrobNorm) in its matrix-valued form:
        ||C^(d)||_F^2 = sum_{a,b<=d} tr[(sum_ij H_a[i,j]^H H_b[i,j]) (sum_k f_b[k] f_a[k]^H)],
    ||f_d|| is the Frobenius norm over all L blocks.
  * r = d - 1 when the test of eq. (precision) fails (the sub-tolerance pair is dropped);
    r = L when every frequency has been used.
  * No regular pivot (max sigma_3 <= pivot_rtol * max block norm) -> the block is kept
    dense: one face per frequency with a selector fibre; except when d > 1 and the residual
    face itself is below eps ||C^(d-1)||_F, which means the tensor is already reproduced
    (then r = d - 1).
  * Ties of an argmax go to the smallest index (row-major (i, j); smallest k).
  * Per-slice ACA (Sec. 3.1) is a pass over the faces of the finished 3D-ACA: the 3D-ACA
    runs on exact residual faces, then each face H_d of an admissible block is compressed
    by the matrix-valued ACA + QR/SVD recompression with the absolute tolerance
        tol_d = eps_aca ||C^(r)||_F / ||f_d||_F,
    i.e. each face-fibre term errs by at most about eps_aca ||C^(r)||_F (the paper sets
    eps = 100 eps_aca, room for the errors of many terms).  ||C^(r)||_F is the recursive
    norm of the last step (it includes a dropped sub-tolerance pair).
  * The ACA stops when ||U_k||_F ||V_k||_F <= tol for the newest 3 columns, or when a
    residual row without a regular block is itself below tol.  It fails (the face stays
    dense) when it reaches its column cap short of 3 min(m, n) columns, after MAX_FAIL rows in a row without a regular
    pivot, or when every row was visited and a skipped row remains.  The cap is
    3 ceil(2 m n / (m + n)) columns (ACA columns at twice the memory of the dense face:
    rank-3 steps overshoot the recompressed rank about twofold), at most 3 min(m, n) and
    KMAX_ACA; recompressed factors that do not take less memory than the dense face are
    dropped as well (kk (m + n) >= 3 m n).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

PIVOT_RTOL = 1e-14
MAX_FAIL = 8
KMAX_ACA = 96
QRCP_FRAC = 0.25


def sigma3(B):
    """Smallest singular value of each 3x3 block of B[..., 3, 3]."""
    return np.linalg.svd(B, compute_uv=False)[..., -1]


def _fro2(A):
    return float(np.sum(np.abs(A) ** 2))


class Approx3D:
    """Result of 3D-ACA on one block: faces H[d] (m, n, 3, 3) and fibres f[d] (L, 3, 3)."""

    def __init__(self, faces, fibres, pivots, ks, dense, norm2=0.0):
        self.faces = faces
        self.fibres = fibres
        self.pivots = pivots
        self.ks = ks
        self.dense = dense
        self.norm2 = norm2          # recursive ||C^(r)||_F^2 of the last step
        self.factors = [None] * len(faces)  # per face: (Ubar, Vbar) after the ACA pass, or None

    @property
    def rank(self):
        return len(self.faces)

    def tensor(self, L=None):
        if not self.faces:
            return None
        m, n = self.faces[0].shape[:2]
        L = self.fibres[0].shape[0]
        C = np.zeros((L, m, n, 3, 3), dtype=np.complex128)
        for H, f, uv in zip(self.faces, self.fibres, self.factors):
            if uv is not None:
                H = matrix_to_blocks(uv[0] @ uv[1].conj().T)
            C += np.einsum("ijab,kbc->kijac", H, f)
        return C


def aca3d(C, eps):
    """Algorithm 1 on a dense block tensor C[L, m, n, 3, 3] (exact residual faces)."""
    L, m, n = C.shape[:3]
    faces, fibres, pivots, ks = [], [], [], []
    G = {}  # G[(a, b)] = sum_ij H_a^H H_b
    F = {}  # F[(b, a)] = sum_k f_b f_a^H
    norm2 = 0.0
    used = np.zeros(L, dtype=bool)
    k = 0
    d = 0
    blocknorm = np.sqrt(np.max(np.sum(np.abs(C) ** 2, axis=(-2, -1))))
    while True:
        d += 1
        # face at k_d: entries minus the current approximation
        R = C[k].copy()
        for Ha, fa in zip(faces, fibres):
            R -= np.einsum("ijab,bc->ijac", Ha, fa[k])
        Hd = R
        s3 = sigma3(Hd)
        flat = int(np.argmax(s3))
        i_d, j_d = divmod(flat, n)
        if not (s3[i_d, j_d] > PIVOT_RTOL * blocknorm):
            if blocknorm == 0.0:
                return Approx3D([], [], [], [], dense=False)
            if d > 1 and np.sqrt(_fro2(Hd)) <= eps * np.sqrt(max(norm2, 0.0)):
                # the residual face vanishes: the tensor is reproduced, stop with r = d - 1
                return Approx3D(faces, fibres, pivots, ks, dense=False, norm2=norm2)
            return dense_fallback(C)
        P = Hd[i_d, j_d]
        # fibre at (i_d, j_d) over all frequencies, residual, times the pivot inverse
        Fib = C[:, i_d, j_d].copy()
        for Ha, fa in zip(faces, fibres):
            Fib -= np.einsum("ab,kbc->kac", Ha[i_d, j_d], fa)
        fd = np.einsum("ab,kbc->kac", np.linalg.inv(P), Fib)
        used[k] = True
        faces.append(Hd)
        fibres.append(fd)
        pivots.append((i_d, j_d))
        ks.append(k)
        # recursive Frobenius norm
        b = d - 1
        for a in range(d):
            G[(a, b)] = np.einsum("ijba,ijbc->ac", faces[a].conj(), Hd)
            F[(b, a)] = np.einsum("kab,kcb->ac", fd, fibres[a].conj())
        cross = sum(np.trace(G[(a, b)] @ F[(b, a)]) for a in range(b))
        norm2 += 2.0 * np.real(cross) + np.real(np.trace(G[(b, b)] @ F[(b, b)]))
        hn = np.sqrt(max(np.real(np.trace(G[(b, b)])), 0.0))
        fn = np.sqrt(max(np.real(np.trace(F[(b, b)])), 0.0))
        if not (hn * fn > eps * np.sqrt(max(norm2, 0.0))):
            faces.pop(), fibres.pop(), pivots.pop(), ks.pop()
            return Approx3D(faces, fibres, pivots, ks, dense=False, norm2=norm2)
        if used.all():
            return Approx3D(faces, fibres, pivots, ks, dense=False, norm2=norm2)
        s3f = sigma3(fd)
        s3f[used] = -1.0
        k = int(np.argmax(s3f))


def dense_fallback(C):
    L = C.shape[0]
    faces, fibres = [], []
    for k in range(L):
        faces.append(C[k].copy())
        f = np.zeros((L, 3, 3), dtype=np.complex128)
        f[k] = np.eye(3)
        fibres.append(f)
    return Approx3D(faces, fibres, [None] * L, list(range(L)), dense=True)


def frobenius_explicit(approx):
    T = approx.tensor()
    return 0.0 if T is None else np.sqrt(_fro2(T))


# ------------------------------------------------------------------ per-slice ACA

def blocks_to_matrix(H):
    """(m, n, 3, 3) blocks -> (3m, 3n) matrix."""
    m, n = H.shape[:2]
    return H.transpose(0, 2, 1, 3).reshape(3 * m, 3 * n)


def matrix_to_blocks(A):
    m3, n3 = A.shape
    return A.reshape(m3 // 3, 3, n3 // 3, 3).transpose(0, 2, 1, 3)


def face_aca_cap(m, n):
    """Column cap of the per-slice ACA of an m x n (elements) face."""
    s = -(-2 * m * n // (m + n))
    return 3 * min(s, m, n)


def aca_matrix(A, tol, max_cols=None):
    """Matrix-valued partial-pivot ACA of A (3m x 3n) with rank-3 steps and sigma_3 pivots.

    Rows and columns of the residual are read from A minus the current approximation
    U V^H; the pivot block of a row is its block of largest sigma_3, and the next row is
    the unused row whose new U block has the largest sigma_3.  Returns (U, V, ok) with
    A ~= U V^H; see the module docstring for the stopping and failure rules.
    """
    m, n = A.shape[0] // 3, A.shape[1] // 3
    if max_cols is None:
        max_cols = 3 * min(m, n)
    Us, Vs = [], []
    used_rows = np.zeros(m, dtype=bool)
    scale = np.abs(A).max() if A.size else 0.0
    i, kc, fails, skipped = 0, 0, 0, 0

    def result(ok):
        if not Us:
            return np.zeros((3 * m, 0), dtype=A.dtype), np.zeros((3 * n, 0), dtype=A.dtype), ok
        return np.concatenate(Us, axis=1), np.concatenate(Vs, axis=1), ok

    while True:
        if kc + 3 > max_cols:
            # all min(m, n) block rows or columns interpolated: the residual is zero
            return result(kc >= 3 * min(m, n))
        row = A[3 * i:3 * i + 3].copy()
        for Uk, Vk in zip(Us, Vs):
            row -= Uk[3 * i:3 * i + 3] @ Vk.conj().T
        used_rows[i] = True
        s3 = sigma3(row.reshape(3, n, 3).transpose(1, 0, 2))
        j = int(np.argmax(s3))
        if not (s3[j] > PIVOT_RTOL * scale):
            if np.linalg.norm(row) <= tol:
                return result(True)
            skipped += 1
            fails += 1
            free = np.flatnonzero(~used_rows)
            if fails >= MAX_FAIL or free.size == 0:
                return result(False)
            i = int(free[0])
            continue
        fails = 0
        P = row[:, 3 * j:3 * j + 3]
        col = A[:, 3 * j:3 * j + 3].copy()
        for Uk, Vk in zip(Us, Vs):
            col -= Uk @ Vk[3 * j:3 * j + 3].conj().T
        Un = col @ np.linalg.inv(P)
        Vn = row.conj().T
        Us.append(Un)
        Vs.append(Vn)
        kc += 3
        if np.linalg.norm(Un) * np.linalg.norm(Vn) <= tol:
            return result(True)
        s3u = sigma3(Un.reshape(m, 3, 3))
        s3u[used_rows] = -1.0
        if used_rows.all():
            return result(skipped == 0)
        i = int(np.argmax(s3u))


def recompress(U, V, tol):
    """eq. (ACA): U V^H = Q_U M Q_V^H with M = R_U R_V^H, and the SVD approximation of M.

    The SVD of M is taken through a QR with column pivoting, M P = Q_M R, cut at the first
    step whose remaining rows R[j:, j:] have Frobenius norm rest <= QRCP_FRAC tol; the SVD
    of the kept rows R[:j] P^T = X S Y^H gives M ~ (Q_M[:, :j] X) S Y^H, truncated to the
    smallest k with sqrt(rest^2 + sum_{i>=k} s_i^2) <= tol (at least 1 when M != 0).
    Returns Ubar = Q_U Q_M X_k S_k (3m x k) and Vbar = Q_V Y_k (3n x k)."""
    if U.shape[1] == 0:
        return U, V
    QU, RU = np.linalg.qr(U)
    QV, RV = np.linalg.qr(V)
    M = RU @ RV.conj().T
    QM, R, perm = scipy.linalg.qr(M, pivoting=True)
    n = M.shape[1]
    trail = [float(np.sum(np.abs(R[j:, j:]) ** 2)) for j in range(n)] + [0.0]
    kq = next(j for j in range(n + 1) if np.sqrt(trail[j]) <= QRCP_FRAC * tol)
    if kq == 0:
        return U[:, :0], V[:, :0]
    B = np.zeros((kq, n), dtype=M.dtype)
    B[:, perm] = R[:kq]
    X, S, Yh = np.linalg.svd(B, full_matrices=False)
    rest2 = trail[kq]
    tot = np.sqrt(rest2 + np.sum(S**2))
    k = len(S)
    while k > 0 and np.sqrt(rest2 + np.sum(S[k - 1:] ** 2)) <= tol:
        k -= 1
    k = max(k, 1) if tot > 0 else 0
    return (QU @ (QM[:, :kq] @ X[:, :k])) * S[:k], QV @ Yh[:k].conj().T


def compress_face(H, tol, max_cols=KMAX_ACA):
    """Per-slice ACA + recompression of one face H (m, n, 3, 3) with absolute tolerance tol.
    Returns (Ubar, Vbar, kc): the factors, or None when the face stays dense, and the ACA
    column count (-1 when the ACA failed)."""
    m, n = H.shape[:2]
    A = blocks_to_matrix(H)
    if not np.any(A):
        return None, -1
    U, V, ok = aca_matrix(A, tol, min(max_cols, face_aca_cap(m, n)))
    if not ok:
        return None, -1
    Ub, Vb = recompress(U, V, tol)
    if Ub.shape[1] == 0 or Ub.shape[1] * (m + n) >= 3 * m * n:
        return None, U.shape[1]
    return (Ub, Vb), U.shape[1]


def compress_faces(ap, eps_aca, max_cols=KMAX_ACA):
    """The per-slice ACA pass over the faces of a 3D-ACA result (in place); returns ap."""
    if ap.dense:
        return ap
    cn = np.sqrt(max(ap.norm2, 0.0))
    for d, (H, f) in enumerate(zip(ap.faces, ap.fibres)):
        fn = np.sqrt(_fro2(f))
        tol = eps_aca * cn / fn if fn > 0 else 0.0
        ap.factors[d] = compress_face(H, tol, max_cols)[0]
    return ap
