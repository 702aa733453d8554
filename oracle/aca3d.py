"""Matrix-valued 3D-ACA (Algorithm 1, Sec. 3) and the H-matrix ACA of the faces (Sec. 3.1:
matrix-valued ACA of a face, QR/SVD recompression of eq. (ACA), pivot found on the
reconstruction) in plain numpy, for small tensors.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Tensor convention: ``C[k, i, j]`` is the 3x3 block ENTRY(i, j, k) of an array of m x n
blocks over L frequencies; an approximation is C[k, i, j] ~= sum_d H_d[i, j] @ f_d[k]
(face block on the left, as in the fibre line of Algorithm 1).

Readings of the paper taken here:
  * k_1 = 0 is the first contour point; the loop is a do-while (the test needs a pair).
  * The next frequency is the argmax of sigma_3(f_d[k]) over frequencies not yet used
    (f_d[k_d] = I, so without the exclusion the argmax repeats k_d).
  * The norm of eq. (FrobNorm) in its matrix-valued form:
        ||C^(d)||_F^2 = sum_{a,b<=d} tr[(sum_ij H_a[i,j]^H H_b[i,j]) (sum_k f_b[k] f_a[k]^H)],
    ||f_d|| is the Frobenius norm over all L blocks.
  * r = d - 1 when the test of eq. (precision) fails (the sub-tolerance pair is dropped);
    r = L when every frequency has been used.
  * "sigma_3 = 0 for all (i, j)" is read as max sigma_3 <= PIVOT_RTOL_3D * scale, the scale
    being the largest 3x3 block norm of the slices C[k_1], ..., C[k_d] formed so far (the
    algorithm never sees the others; a smaller scale, e.g. the residual face's, lets
    rounding noise through as a pivot); in the H-matrix ACA variant the slice is never
    formed and the reconstructed residual face stands in for it.  The block is then kept
    dense (one face per frequency with a selector fibre), except
    when d > 1 and the residual face itself is below eps ||C^(d-1)||_F, which means the
    tensor is already reproduced (then r = d - 1).
  * Ties of an argmax go to the smallest index (row-major (i, j); smallest k).
  * H-matrix ACA variant (``aca3d(C, eps, eps_aca)``, Sec. 3.1): the residual face of step
    d is approximated by the matrix-valued ACA and recompressed (eq. (ACA)), both relative
    to eps_aca; the pivot block (i_d, j_d) is searched on the reconstruction of that
    approximation, and the approximation is the face H_d that enters C^(d).  The fibre
    line takes exact entries minus C^(d-1), as Algorithm 1 states.
  * Matrix-valued ACA (the paper defers to its references): steps of rank 3.  Step k takes
    the residual block row i, its block j of largest sigma_3 as pivot, the residual block
    column j times the pivot inverse as the new U columns and the residual row (conjugate
    transposed) as the new V columns.  The first row is 0; the next row is the unused row
    whose block of the new U columns has the largest sigma_3.  The stop test is that of
    ACA with a relative tolerance, ||U_k||_F ||V_k||_F <= eps_aca ||S_k||_F with S_k the
    approximation after step k (or an absolute tol).  A residual row without a regular
    block is skipped (next unused row); when every row has been used the ACA ends, and
    it has resolved the matrix unless a skipped row's residual is still above the
    threshold.
  * Recompression (eq. (ACA)): U = Q_U R_U, V = Q_V R_V (Householder QR), the SVD of
    R_U R_V^H, truncated to the smallest k whose dropped singular values satisfy
    sqrt(sum_{t>=k} s_t^2) <= eps_aca ||Sigma||_F (or <= an absolute tol).
"""
from __future__ import annotations

import numpy as np

PIVOT_RTOL = 1e-14     # matrix-valued ACA: a residual row without a regular block
# Algorithm 1: a residual face whose 3x3 blocks are all singular still shows sigma_3 of a few
# eps times the largest face-fibre product subtracted from it (up to about 1e-14 of the
# scale on small clusters); the threshold stays two orders above that rounding level
PIVOT_RTOL_3D = 1e-12


def sigma3(B):
    """Smallest singular value of each 3x3 block of B[..., 3, 3]."""
    return np.linalg.svd(B, compute_uv=False)[..., -1]


def _blockmax(H):
    """Largest Frobenius norm of the 3x3 blocks of H[..., 3, 3]."""
    return float(np.sqrt(np.max(np.sum(np.abs(H) ** 2, axis=(-2, -1)))))


def _fro2(A):
    return float(np.sum(np.abs(A) ** 2))


class Approx3D:
    """Result of 3D-ACA on one block: faces H[d] (m, n, 3, 3) and fibres f[d] (L, 3, 3).
    ``factors[d]`` holds (Ubar, Vbar) of a face kept in low rank (H_d = Ubar Vbar^H), or None
    for a dense face; ``faces[d]`` always holds the face as 3x3 blocks."""

    def __init__(self, faces, fibres, pivots, ks, dense, norm2=0.0, factors=None):
        self.faces = faces
        self.fibres = fibres
        self.pivots = pivots
        self.ks = ks
        self.dense = dense
        self.norm2 = norm2          # recursive ||C^(r)||_F^2 of the last step
        self.factors = list(factors) if factors is not None else [None] * len(faces)

    @property
    def rank(self):
        return len(self.faces)

    def tensor(self):
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


def aca3d(C, eps, eps_aca=None):
    """Algorithm 1 on a block tensor C[L, m, n, 3, 3].

    eps_aca None: the faces are the exact residual faces.  eps_aca > 0: the H-matrix ACA
    variant of Sec. 3.1 (admissible blocks): every residual face is replaced by its ACA +
    recompression at relative tolerance eps_aca, and the pivot is searched on that
    reconstruction."""
    L, m, n = C.shape[:3]
    faces, fibres, pivots, ks, factors = [], [], [], [], []
    G = {}  # G[(a, b)] = sum_ij H_a^H H_b
    F = {}  # F[(b, a)] = sum_k f_b f_a^H
    norm2 = 0.0
    used = np.zeros(L, dtype=bool)
    k = 0
    d = 0
    scale = 0.0  # largest 3x3 block norm of the slices formed so far
    while True:
        d += 1
        # face at k_d: entries minus the current approximation C^(d-1)
        R = C[k].copy()
        if eps_aca is None:
            scale = max(scale, _blockmax(R))
        for Ha, fa in zip(faces, fibres):
            R -= np.einsum("ijab,bc->ijac", Ha, fa[k])
        uv = None
        if eps_aca is not None:
            A = blocks_to_matrix(R)
            if np.any(A):
                U, V, _ = aca_matrix(A, eps=eps_aca)
                uv = recompress(U, V, eps=eps_aca)
                Hd = matrix_to_blocks(uv[0] @ uv[1].conj().T)  # the reconstruction
            else:
                Hd = R
        else:
            Hd = R
        if eps_aca is not None:
            scale = max(scale, _blockmax(Hd))
        s3 = sigma3(Hd)
        flat = int(np.argmax(s3))
        i_d, j_d = divmod(flat, n)
        if not (s3[i_d, j_d] > PIVOT_RTOL_3D * scale):
            if not np.any(C):
                return Approx3D([], [], [], [], dense=False)
            if d > 1 and np.sqrt(_fro2(R)) <= eps * np.sqrt(max(norm2, 0.0)):
                # the residual face vanishes: the tensor is reproduced, stop with r = d - 1
                return Approx3D(faces, fibres, pivots, ks, dense=False, norm2=norm2, factors=factors)
            return dense_fallback(C)
        P = Hd[i_d, j_d]
        # fibre at (i_d, j_d) over all frequencies: entries minus C^(d-1), times the pivot inverse
        Fib = C[:, i_d, j_d].copy()
        for Ha, fa in zip(faces, fibres):
            Fib -= np.einsum("ab,kbc->kac", Ha[i_d, j_d], fa)
        fd = np.einsum("ab,kbc->kac", np.linalg.inv(P), Fib)
        used[k] = True
        faces.append(Hd)
        fibres.append(fd)
        pivots.append((i_d, j_d))
        ks.append(k)
        factors.append(uv)
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
            faces.pop(), fibres.pop(), pivots.pop(), ks.pop(), factors.pop()
            return Approx3D(faces, fibres, pivots, ks, dense=False, norm2=norm2, factors=factors)
        if used.all():
            return Approx3D(faces, fibres, pivots, ks, dense=False, norm2=norm2, factors=factors)
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


def aca_matrix(A, tol=0.0, eps=0.0):
    """Matrix-valued partial-pivot ACA of A (3m x 3n) with rank-3 steps and sigma_3 pivots.

    Rows and columns of the residual are read from A minus the current approximation
    U V^H.  The ACA stops after the step whose new columns satisfy
    ||U_k||_F ||V_k||_F <= max(tol, eps ||U V^H||_F) (the norm of the approximation so
    far, formed explicitly), or when every block row has been used.  Returns (U, V, ok)
    with A ~= U V^H; ok is False when a row skipped for want of a regular block still has a
    residual above the threshold at the end."""
    m, n = A.shape[0] // 3, A.shape[1] // 3
    Us, Vs = [], []
    used = np.zeros(m, dtype=bool)
    scale = np.abs(A).max() if A.size else 0.0
    skipped = []
    i = 0

    def approx():
        if not Us:
            return np.zeros((3 * m, 0), dtype=A.dtype), np.zeros((3 * n, 0), dtype=A.dtype)
        return np.concatenate(Us, axis=1), np.concatenate(Vs, axis=1)

    def threshold():
        U, V = approx()
        return max(tol, eps * np.linalg.norm(U @ V.conj().T))

    def residual_rows(rows):
        U, V = approx()
        Rr = np.concatenate([A[3 * q:3 * q + 3] for q in rows], axis=0)
        return Rr - np.concatenate([U[3 * q:3 * q + 3] for q in rows], axis=0) @ V.conj().T

    while True:
        U, V = approx()
        row = A[3 * i:3 * i + 3] - U[3 * i:3 * i + 3] @ V.conj().T
        used[i] = True
        s3 = sigma3(row.reshape(3, n, 3).transpose(1, 0, 2))
        j = int(np.argmax(s3))
        if not (s3[j] > PIVOT_RTOL * scale):
            skipped.append(i)
            free = np.flatnonzero(~used)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        P = row[:, 3 * j:3 * j + 3]
        col = A[:, 3 * j:3 * j + 3] - U @ V[3 * j:3 * j + 3].conj().T
        Un = col @ np.linalg.inv(P)
        Vn = row.conj().T
        Us.append(Un)
        Vs.append(Vn)
        if np.linalg.norm(Un) * np.linalg.norm(Vn) <= threshold():
            break
        if used.all():
            break
        s3u = sigma3(Un.reshape(m, 3, 3))
        s3u[used] = -1.0
        i = int(np.argmax(s3u))
    U, V = approx()
    ok = not skipped or np.linalg.norm(residual_rows(skipped)) <= threshold()
    return U, V, bool(ok)


def recompress(U, V, tol=0.0, eps=0.0):
    """eq. (ACA): U V^H = Q_U (R_U R_V^H) Q_V^H, R_U R_V^H = X S Y^H (SVD), truncated to
    the smallest k with sqrt(sum_{t>=k} s_t^2) <= max(tol, eps ||S||_F).
    Returns Ubar = Q_U X_k S_k (3m x k) and Vbar = Q_V Y_k (3n x k)."""
    if U.shape[1] == 0:
        return U, V
    QU, RU = np.linalg.qr(U)
    QV, RV = np.linalg.qr(V)
    X, S, Yh = np.linalg.svd(RU @ RV.conj().T)
    thr = max(tol, eps * np.sqrt(np.sum(S**2)))
    tail = np.sqrt(np.cumsum((S**2)[::-1])[::-1])  # tail[k] = sqrt(sum_{t>=k} s_t^2)
    k = next((q for q in range(len(S)) if tail[q] <= thr), len(S))
    return (QU @ X[:, :k]) * S[:k], QV @ Yh[:k].conj().T


def compress_face(H, tol=0.0, eps=0.0):
    """ACA + recompression of one face H (m, n, 3, 3).  Returns ((Ubar, Vbar), kc): the
    factors (None when the ACA did not resolve the face or the face is zero) and the ACA
    column count."""
    A = blocks_to_matrix(H)
    if not np.any(A):
        return None, 0
    U, V, ok = aca_matrix(A, tol=tol, eps=eps)
    if not ok:
        return None, U.shape[1]
    return recompress(U, V, tol=tol, eps=eps), U.shape[1]


def compress_faces(ap, eps_aca):
    """Per-slice ACA as a pass over the exact faces of a finished 3D-ACA (in place; returns
    ap): face d is compressed to the absolute tolerance tol_d = eps_aca ||C^(r)||_F / ||f_d||_F,
    so each face-fibre term moves by at most about eps_aca ||C^(r)||_F.  This is the order
    of work the GPU library takes; the paper's order is ``aca3d(C, eps, eps_aca)``."""
    if ap.dense:
        return ap
    cn = np.sqrt(max(ap.norm2, 0.0))
    for d, (H, f) in enumerate(zip(ap.faces, ap.fibres)):
        fn = np.sqrt(_fro2(f))
        tol = eps_aca * cn / fn if fn > 0 else 0.0
        ap.factors[d] = compress_face(H, tol=tol)[0]
    return ap
