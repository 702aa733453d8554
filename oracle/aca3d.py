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
"""
from __future__ import annotations

import numpy as np

PIVOT_RTOL = 1e-14
MAX_FAIL = 8


def sigma3(B):
    """Smallest singular value of each 3x3 block of B[..., 3, 3]."""
    return np.linalg.svd(B, compute_uv=False)[..., -1]


def _fro2(A):
    return float(np.sum(np.abs(A) ** 2))


class Approx3D:
    """Result of 3D-ACA on one block: faces H[d] (m, n, 3, 3) and fibres f[d] (L, 3, 3)."""

    def __init__(self, faces, fibres, pivots, ks, dense):
        self.faces = faces
        self.fibres = fibres
        self.pivots = pivots
        self.ks = ks
        self.dense = dense

    @property
    def rank(self):
        return len(self.faces)

    def tensor(self, L=None):
        if not self.faces:
            return None
        m, n = self.faces[0].shape[:2]
        L = self.fibres[0].shape[0]
        C = np.zeros((L, m, n, 3, 3), dtype=np.complex128)
        for H, f in zip(self.faces, self.fibres):
            C += np.einsum("ijab,kbc->kijac", H, f)
        return C


def aca3d(C, eps, face_approx=None):
    """Algorithm 1 on a dense block tensor C[L, m, n, 3, 3].

    face_approx(Hres) -> Hd optionally replaces the exact residual face by an approximation
    (the per-slice ACA of far-field blocks); the pivot is then searched on the reconstructed
    approximation, as Sec. 3.1 describes.
    """
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
        Hd = R if face_approx is None else face_approx(R)
        s3 = sigma3(Hd)
        flat = int(np.argmax(s3))
        i_d, j_d = divmod(flat, n)
        if not (s3[i_d, j_d] > PIVOT_RTOL * blocknorm):
            if blocknorm == 0.0:
                return Approx3D([], [], [], [], dense=False)
            if d > 1 and np.sqrt(_fro2(Hd)) <= eps * np.sqrt(max(norm2, 0.0)):
                # the residual face vanishes: the tensor is reproduced, stop with r = d - 1
                return Approx3D(faces, fibres, pivots, ks, dense=False)
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
            return Approx3D(faces, fibres, pivots, ks, dense=False)
        if used.all():
            return Approx3D(faces, fibres, pivots, ks, dense=False)
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


def aca_matrix(A, eps, max_steps=None):
    """Matrix-valued partial-pivot ACA of A (3m x 3n) with rank-3 steps and sigma_3 pivots.

    Rows and columns of the residual are read from A minus the current approximation.
    Returns U (3m x 3r), V (3n x 3r) with A ~= U V^H.  Stops when
    ||U_k||_F ||V_k||_F <= eps ||S_k||_F (the update norm against the approximation norm).
    A residual row without a regular 3x3 block is skipped (next unused row); the iteration
    also stops when such a row is itself below eps ||S_k||_F or after MAX_FAIL skips in a row.
    """
    m, n = A.shape[0] // 3, A.shape[1] // 3
    if max_steps is None:
        max_steps = min(m, n)
    Us, Vs = [], []
    used_rows = np.zeros(m, dtype=bool)
    i = 0
    norm2 = 0.0
    scale = np.abs(A).max() if A.size else 0.0
    steps = 0
    fails = 0
    while steps < max_steps:
        row = A[3 * i:3 * i + 3].copy()
        for Uk, Vk in zip(Us, Vs):
            row -= Uk[3 * i:3 * i + 3] @ Vk.conj().T
        used_rows[i] = True
        s3 = sigma3(row.reshape(3, n, 3).transpose(1, 0, 2))
        j = int(np.argmax(s3))
        if not (s3[j] > PIVOT_RTOL * max(scale, 1e-300)):
            if np.linalg.norm(row) <= eps * np.sqrt(max(norm2, 0.0)):
                break
            fails += 1
            free = np.flatnonzero(~used_rows)
            if free.size == 0 or fails >= MAX_FAIL:
                break
            i = int(free[0])
            continue
        fails = 0
        P = row[:, 3 * j:3 * j + 3]
        col = A[:, 3 * j:3 * j + 3].copy()
        for Uk, Vk in zip(Us, Vs):
            col -= Uk @ Vk[3 * j:3 * j + 3].conj().T
        Un = col @ np.linalg.inv(P)
        Vn = row.conj().T
        cross = sum(np.trace((Uk.conj().T @ Un) @ (Vn.conj().T @ Vk)) for Uk, Vk in zip(Us, Vs))
        norm2 += 2.0 * np.real(cross) + np.real(np.trace((Un.conj().T @ Un) @ (Vn.conj().T @ Vn)))
        Us.append(Un)
        Vs.append(Vn)
        steps += 1
        if np.linalg.norm(Un) * np.linalg.norm(Vn) <= eps * np.sqrt(max(norm2, 0.0)):
            break
        if used_rows.all():
            break
        s3u = sigma3(Un.reshape(m, 3, 3))
        s3u[used_rows] = -1.0
        i = int(np.argmax(s3u))
    if not Us:
        return np.zeros((3 * m, 0), dtype=A.dtype), np.zeros((3 * n, 0), dtype=A.dtype)
    return np.concatenate(Us, axis=1), np.concatenate(Vs, axis=1)


def recompress(U, V, eps):
    """eq. (ACA): U V^H = Q_U (R_U R_V^H) Q_V^H = Q_U (Uc S Vc^H) Q_V^H, truncated so that
    the dropped singular values satisfy sqrt(sum_{i>k} s_i^2) <= eps ||s||.
    Returns Ubar (3m x k, scaled by the singular values) and Vbar (3n x k)."""
    if U.shape[1] == 0:
        return U, V
    QU, RU = np.linalg.qr(U)
    QV, RV = np.linalg.qr(V)
    Uc, S, Vch = np.linalg.svd(RU @ RV.conj().T)
    tot = np.sqrt(np.sum(S**2))
    k = len(S)
    while k > 0 and np.sqrt(np.sum(S[k - 1:] ** 2)) <= eps * tot:
        k -= 1
    k = max(k, 1) if tot > 0 else 0
    return (QU @ Uc[:, :k]) * S[:k], QV @ Vch[:k].conj().T


def aca_face(eps_aca):
    """face_approx for aca3d: per-slice ACA + recompression, reconstructed densely."""
    def f(Hres):
        A = blocks_to_matrix(Hres)
        U, V = aca_matrix(A, eps_aca)
        Ub, Vb = recompress(U, V, eps_aca)
        return matrix_to_blocks(Ub @ Vb.conj().T)
    return f
