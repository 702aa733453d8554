"""FP64 CPU oracle of the Laplace-domain elastodynamic BEM hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the product library neither imports nor links it and
shares no code with it.

* ``bem_oracle.c`` (plain C99, FP64, optional OpenMP): kernel U and T of the paper's
  Appendix A / Sec. 2.1, collocation entries with the quadrature rules, dense products, and
  the gradients of single- and double-layer bilinear forms with respect to the node
  coordinates and the material (regular and near pairs by the chain rule, self pairs as the
  derivative of the integral, the double layer's as a principal value).
* ``aca3d.py`` (numpy): the matrix-valued 3D-ACA of Algorithm 1 (Sec. 3), the matrix-valued
  ACA with QR/SVD recompression of eq. (ACA), and the H-matrix variant of Sec. 3.1 (faces
  approximated inside the loop, pivot on the reconstruction), for small tensors.
* ``cq.py`` (numpy): convolution quadrature weights and marching on in time (Sec. 2.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile bem_oracle.c with gcc (-O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.oracle_entries.restype = ctypes.c_int
        L.oracle_entries.argtypes = [dp, ctypes.c_int64, ip, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int32,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int64, ip, ip, ip, dp]
        L.oracle_matvec_rows.restype = ctypes.c_int
        L.oracle_matvec_rows.argtypes = [dp, ctypes.c_int64, ip, ctypes.c_int64,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int32,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int64, ip, ctypes.c_int32, dp, dp]
        L.oracle_point_entries.restype = ctypes.c_int
        L.oracle_point_entries.argtypes = [dp, ctypes.c_int64, ip, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int32,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int64, dp, ctypes.c_int64, ip, ip, ip, dp]
        L.oracle_kernel_point.restype = ctypes.c_int
        L.oracle_kernel_point.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_tri7.restype = None
        L.oracle_tri7.argtypes = [dp, dp]
        L.oracle_gauss_legendre.restype = None
        L.oracle_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_adjoint_v.restype = ctypes.c_int
        L.oracle_adjoint_v.argtypes = [dp, ctypes.c_int64, ip, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int32,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int32, dp, dp, ctypes.c_double,
                                       dp, dp, dp]
        L.oracle_adjoint_k.restype = ctypes.c_int
        L.oracle_adjoint_k.argtypes = [dp, ctypes.c_int64, ip, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int32,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int32, dp, dp, ctypes.c_double,
                                       dp, dp, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


OP_V, OP_K, OP_HK = 0, 1, 2
OP_KL0, OP_KL1, OP_KL2 = 4, 5, 6  # double layer weighted by the barycentric coordinate of vertex 0, 1, 2


class Problem:
    """Mesh + material + frequencies + quadrature options of one oracle evaluation."""

    def __init__(self, nodes, tris, s, rho=1.0, cp=1.0, cs=0.5, near_on=False,
                 r1=1.5, r2=3.0, self_nt=8, self_nr=8):
        self.nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
        self.s = np.ascontiguousarray(np.stack([s.real, s.imag], axis=-1))
        self.L = int(s.shape[0])
        self.K = int(self.tris.shape[0])
        self.rho, self.cp, self.cs = float(rho), float(cp), float(cs)
        self.near_on = int(bool(near_on))
        self.r1, self.r2 = float(r1), float(r2)
        self.self_nt, self.self_nr = int(self_nt), int(self_nr)

    def _common(self):
        return (_d(self.nodes), self.nodes.shape[0], _i(self.tris), self.K,
                self.rho, self.cp, self.cs, _d(self.s), self.L)

    def _quad(self, op):
        return (int(op), self.near_on, self.r1, self.r2, self.self_nt, self.self_nr)

    def entries(self, op, i, j, l):
        """ENTRY(op, i, j, l) for index arrays -> complex128 [n, 3, 3]."""
        i, j, l = (np.ascontiguousarray(np.ravel(a), dtype=np.int32) for a in np.broadcast_arrays(i, j, l))
        n = i.size
        out = np.zeros((n, 9, 2), dtype=np.float64)
        rc = lib().oracle_entries(*self._common(), *self._quad(op), n, _i(i), _i(j), _i(l), _d(out))
        if rc != 0:
            raise RuntimeError("oracle_entries failed with code %d" % rc)
        return (out[..., 0] + 1j * out[..., 1]).reshape(n, 3, 3)

    def dense(self, op):
        """All entries as a complex128 array [L, 3K, 3K] (small meshes only)."""
        K, L = self.K, self.L
        ii, jj, ll = np.meshgrid(np.arange(K), np.arange(K), np.arange(L), indexing="ij")
        E = self.entries(op, ii.ravel(), jj.ravel(), ll.ravel()).reshape(K, K, L, 3, 3)
        return np.ascontiguousarray(E.transpose(2, 0, 3, 1, 4).reshape(L, 3 * K, 3 * K))

    def dense_linear_dl(self, free_term=True):
        """Double layer against the continuous piecewise-linear shape functions of the nodes
        (Sec. 2.3, eqs. (subspace), (basis); K of eq. (discrVK) with phi_l), collocated at the
        centroids: complex128 [L, 3K, 3N], column block n = node n.  Entry (i, n) is the sum
        over the elements j sharing node n of int_{gamma_j} T(x_i, y) lambda_v(y) dy with v the
        position of n in element j.  free_term adds C phi_n(x_i) = I/2 * 1/3 for the three
        nodes of element i (eq. (discreteCollo) with C = I/2 at the centroids)."""
        K, L, N = self.K, self.L, self.nodes.shape[0]
        out = np.zeros((L, 3 * K, N, 3), dtype=np.complex128)
        for v in range(3):
            D = self.dense(OP_KL0 + v).reshape(L, 3 * K, K, 3)
            np.add.at(out, (slice(None), slice(None), self.tris[:, v]), D)
        if free_term:
            for v in range(3):
                for a in range(3):
                    out[:, 3 * np.arange(K) + a, self.tris[:, v], a] += 0.5 / 3.0
        return out.reshape(L, 3 * K, 3 * N)

    def solve(self, op, b, rhs_op=None):
        """x[r, l] = A_l^{-1} c[r, l] with A_l the dense operator op at s_l (the collocation
        system of Sec. 2.3 at each contour point), c = b, or c = B_l b with B the dense
        operator rhs_op (V t = (I/2 + K) g: op = OP_V, rhs_op = OP_HK).  LU solve per
        frequency (numpy).  b: [nrhs, L, 3K] -> [nrhs, L, 3K]."""
        b = np.asarray(b, dtype=np.complex128)
        A = self.dense(op)
        c = b if rhs_op is None else np.einsum("lij,rlj->rli", self.dense(rhs_op), b)
        x = np.empty_like(c)
        for l in range(self.L):
            x[:, l, :] = np.linalg.solve(A[l], c[:, l, :].T).T
        return x

    def point_entries(self, op, pts, p, j, l):
        """int_{gamma_j} kernel(pts[p], y) dy for field points off the boundary -> [n, 3, 3]."""
        pts = np.ascontiguousarray(np.reshape(pts, (-1, 3)), dtype=np.float64)
        p, j, l = (np.ascontiguousarray(np.ravel(a), dtype=np.int32) for a in np.broadcast_arrays(p, j, l))
        n = p.size
        out = np.zeros((n, 9, 2), dtype=np.float64)
        rc = lib().oracle_point_entries(*self._common(), int(op), self.near_on, self.r1, self.r2,
                                        pts.shape[0], _d(pts), n, _i(p), _i(j), _i(l), _d(out))
        if rc != 0:
            raise RuntimeError("oracle_point_entries failed with code %d" % rc)
        return (out[..., 0] + 1j * out[..., 1]).reshape(n, 3, 3)

    def adjoint_v(self, w, x, fd_h=0.0):
        """Value S = sum_{r, l} w[r, l]^T V(s_l) x[r, l] of the single layer and the gradient
        of Re S: (S, grad_nodes [n_nodes, 3], grad_mat [rho, c_p, c_s]), pair classes held
        fixed.  Regular and near pairs by the chain rule; self pairs as the derivative of the
        integral (the polar rule applied to grad U (lambda_a - 1/3) and to dU/dc, plus the area
        term), or with fd_h > 0 by central differences of the polar rule (step fd_h relative).
        w, x: [nrhs, L, 3K] complex."""
        w = np.ascontiguousarray(np.asarray(w, dtype=np.complex128).reshape(-1, self.L, 3 * self.K))
        x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(-1, self.L, 3 * self.K))
        assert w.shape == x.shape
        wr = np.ascontiguousarray(np.stack([w.real, w.imag], axis=-1))
        xr = np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1))
        val = np.zeros(2)
        gn = np.zeros((self.nodes.shape[0], 3))
        gm = np.zeros(3)
        rc = lib().oracle_adjoint_v(*self._common(), *self._quad(0)[1:], w.shape[0], _d(wr), _d(xr),
                                    float(fd_h), _d(val), _d(gn), _d(gm))
        if rc != 0:
            raise RuntimeError("oracle_adjoint_v failed with code %d" % rc)
        return complex(val[0], val[1]), gn, gm

    def adjoint_k(self, w, x, op=OP_K, fd_h=0.0):
        """Value S = sum_{r, l} w[r, l]^T A(s_l) x[r, l] of the double layer (op OP_K, or OP_HK
        with the free term) and the gradient of Re S: (S, grad_nodes [n_nodes, 3], grad_mat
        [rho, c_p, c_s]; the rho entry is 0, T not depending on rho), pair classes held fixed.
        Regular and near pairs by the chain rule through the Gauss points, the normal, the
        area and the collocation point, with the pointwise derivatives of T by central
        differences of the kernel (relative step fd_h, 1e-5 when fd_h <= 0).  Self pairs: the
        derivative of the principal-value integral by the polar rule (fd_h <= 0), or central
        differences of the rule itself (fd_h > 0, the derivative of the discrete operator).
        w, x: [nrhs, L, 3K] complex."""
        w = np.ascontiguousarray(np.asarray(w, dtype=np.complex128).reshape(-1, self.L, 3 * self.K))
        x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(-1, self.L, 3 * self.K))
        assert w.shape == x.shape and op in (OP_K, OP_HK)
        wr = np.ascontiguousarray(np.stack([w.real, w.imag], axis=-1))
        xr = np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1))
        val = np.zeros(2)
        gn = np.zeros((self.nodes.shape[0], 3))
        gm = np.zeros(3)
        rc = lib().oracle_adjoint_k(*self._common(), int(op), *self._quad(0)[1:], w.shape[0], _d(wr), _d(xr),
                                    float(fd_h), _d(val), _d(gn), _d(gm))
        if rc != 0:
            raise RuntimeError("oracle_adjoint_k failed with code %d" % rc)
        return complex(val[0], val[1]), gn, gm

    def matvec_rows(self, op, rows, x):
        """y[r, l, 3q + a] = (A_l x[r, l])[3 rows[q] + a] without storing A; x: [nrhs, L, 3K]."""
        x = np.asarray(x, dtype=np.complex128)
        if x.ndim == 2:
            x = x[None]
        nrhs = x.shape[0]
        assert x.shape == (nrhs, self.L, 3 * self.K)
        rows = np.ascontiguousarray(np.ravel(rows), dtype=np.int32)
        xr = np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1))
        y = np.zeros((nrhs, self.L, 3 * rows.size, 2), dtype=np.float64)
        rc = lib().oracle_matvec_rows(*self._common(), *self._quad(op), rows.size, _i(rows), nrhs, _d(xr), _d(y))
        if rc != 0:
            raise RuntimeError("oracle_matvec_rows failed with code %d" % rc)
        return y[..., 0] + 1j * y[..., 1]


def kernel_point(which, x, y, n, s, rho=1.0, cp=1.0, cs=0.5):
    """U (which=0) or T (which=1) at one point pair -> complex128 [3, 3]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = np.ascontiguousarray(n if n is not None else [0.0, 0.0, 1.0], dtype=np.float64)
    out = np.zeros((9, 2))
    rc = lib().oracle_kernel_point(int(which), _d(x), _d(y), _d(n), float(np.real(s)), float(np.imag(s)),
                                   float(rho), float(cp), float(cs), _d(out))
    if rc != 0:
        raise RuntimeError("oracle_kernel_point failed")
    return (out[:, 0] + 1j * out[:, 1]).reshape(3, 3)


def tri7():
    b = np.zeros(21)
    w = np.zeros(7)
    lib().oracle_tri7(_d(b), _d(w))
    return b.reshape(7, 3), w


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().oracle_gauss_legendre(int(n), _d(x), _d(w))
    return x, w


def num_threads():
    return int(lib().oracle_num_threads())
