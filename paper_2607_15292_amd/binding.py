"""ctypes binding of libbem.so (argument marshalling only; every step of the path runs in
the library's HIP kernels).  Names follow include/bem.h.

Buffers: numpy arrays are passed as host pointers; torch CUDA tensors as device pointers
(BEM_DEVICE_PTR), with the context's stream set to torch's current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BEM_LIBRARY", os.path.join(_HERE, "libbem.so"))

BEM_OK = 0
WARN_NOCONV = 2
ERR_NAMES = {-1: "BEM_ERR_ARG", -2: "BEM_ERR_MESH", -3: "BEM_ERR_MATERIAL", -4: "BEM_ERR_FREQ",
             -5: "BEM_ERR_STATE", -6: "BEM_ERR_HIP", -7: "BEM_ERR_NOMEM", -8: "BEM_ERR_NODEVICE"}
OP_V, OP_K, OP_HK, OP_TABLE = 0, 1, 2, 3
PREC_F64, PREC_MIXED = 0, 1
FACES_AFTER, FACES_IN_LOOP = 0, 1
DEVICE_PTR, SHARED_X, TRANSPOSE, FREE_TERM = 1, 2, 4, 8
OP_KL0, OP_KL1, OP_KL2 = 4, 5, 6

_lib = None


class BemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERR_NAMES.get(code, "error"), code, msg))
        self.code = code


class bem_quad(ctypes.Structure):
    _fields_ = [("near_on", ctypes.c_int32), ("near_r1", ctypes.c_double), ("near_r2", ctypes.c_double),
                ("self_nt", ctypes.c_int32), ("self_nr", ctypes.c_int32)]


class bem_aca_opts(ctypes.Structure):
    _fields_ = [("eps3d", ctypes.c_double), ("eps_aca", ctypes.c_double), ("eta", ctypes.c_double),
                ("leaf", ctypes.c_int32), ("prec", ctypes.c_int32), ("mixed_eps_floor", ctypes.c_double),
                ("pool_bytes", ctypes.c_int64), ("far_dense_max", ctypes.c_int32), ("aca_rounds", ctypes.c_int32),
                ("face_order", ctypes.c_int32)]


class bem_stats(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int64), ("n_near", ctypes.c_int64), ("n_far", ctypes.c_int64),
                ("n_dense_fallback", ctypes.c_int64), ("rank_min", ctypes.c_int32), ("rank_max", ctypes.c_int32),
                ("rank_mean", ctypes.c_double), ("aca_rank_max", ctypes.c_int32), ("aca_rank_mean", ctypes.c_double),
                ("bytes", ctypes.c_int64), ("compression_rate", ctypes.c_double),
                ("entries_generated", ctypes.c_int64), ("n_far_faces", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("n_aca_dense", ctypes.c_int64), ("aca_cols_mean", ctypes.c_double), ("aca_ms", ctypes.c_double),
                ("face_ms", ctypes.c_double), ("face_launches", ctypes.c_int64), ("face_pairs", ctypes.c_int64),
                ("face_flop", ctypes.c_double), ("recomp_ms", ctypes.c_double), ("recomp_launches", ctypes.c_int64),
                ("recomp_flop", ctypes.c_double), ("entries_regular", ctypes.c_int64),
                ("entries_near", ctypes.c_int64), ("entries_self", ctypes.c_int64), ("entries_other", ctypes.c_int64),
                ("face_bytes", ctypes.c_double), ("block_groups", ctypes.c_int64),
                ("apply_macs_c64", ctypes.c_double), ("apply_macs_c128", ctypes.c_double),
                ("apply_macs_sel", ctypes.c_double), ("apply_macs_fibre", ctypes.c_double),
                ("aca_kernel_ms", ctypes.c_double), ("aca_launches", ctypes.c_int64),
                ("aca_flop", ctypes.c_double), ("aca_bytes", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bem_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("max_refine", ctypes.c_int32), ("pad", ctypes.c_int32)]


class bem_solve_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("refinements", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class bem_batch_info(ctypes.Structure):
    _fields_ = [("nops", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("L", ctypes.c_int32), ("K_total", ctypes.c_int32),
                ("n_groups", ctypes.c_int32), ("n_segments", ctypes.c_int32), ("n_far_faces", ctypes.c_int32),
                ("seg_target", ctypes.c_int32), ("persistent", ctypes.c_int32), ("persistent_wgs", ctypes.c_int32),
                ("far_sorted", ctypes.c_int32), ("graph", ctypes.c_int32), ("graph_builds", ctypes.c_int32),
                ("graph_launches", ctypes.c_int32), ("n_tuned", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("tune_ms", ctypes.c_double * 8), ("tune_segments", ctypes.c_int32 * 8),
                ("workspace_bytes", ctypes.c_double), ("flop", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("pad", "tune_ms", "tune_segments")}
        d["tune_ms"] = list(self.tune_ms)[:self.n_tuned]
        d["tune_segments"] = list(self.tune_segments)[:self.n_tuned]
        return d


# exported symbols and their signatures (also checked by the CPU tests)
_P = ctypes.c_void_p
_SIGS = {
    "bem_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32]),
    "bem_destroy": (ctypes.c_int, [_P]),
    "bem_last_error": (ctypes.c_char_p, [_P]),
    "bem_set_stream": (ctypes.c_int, [_P, _P]),
    "bem_set_mesh": (ctypes.c_int, [_P, _P, ctypes.c_int64, _P, ctypes.c_int64]),
    "bem_set_components": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "bem_set_material": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "bem_set_frequencies": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "bem_freq_pairs": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "bem_set_quadrature": (ctypes.c_int, [_P, ctypes.POINTER(bem_quad)]),
    "bem_set_entry_table": (ctypes.c_int, [_P, _P]),
    "bem_entries": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, _P, _P, _P, ctypes.c_int32]),
    "bem_assemble_dense": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "bem_op_dense_copy": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "bem_compress": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(bem_aca_opts), ctypes.POINTER(ctypes.c_void_p)]),
    "bem_aca_matrix": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_double,
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      _P, _P]),
    "bem_aca_matrix_noalloc": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_double,
                                              ctypes.c_int32, _P, _P, _P]),
    "bem_op_stats": (ctypes.c_int, [_P, ctypes.POINTER(bem_stats)]),
    "bem_apply": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32]),
    "bem_apply_weighted": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "bem_solve": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.POINTER(bem_solve_opts),
                                 ctypes.POINTER(bem_solve_stats)]),
    "bem_cq_dirichlet": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _P, _P,
                                        ctypes.c_int32, ctypes.POINTER(bem_solve_opts),
                                        ctypes.POINTER(bem_solve_stats)]),
    "bem_apply_mf": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int32]),
    "bem_apply_linear_dl": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32]),
    "bem_matrix_free": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "bem_adjoint_v": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P, _P]),
    "bem_adjoint_k": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P, _P]),
    "bem_batch_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "bem_batch_apply": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "bem_batch_info_get": (ctypes.c_int, [_P, ctypes.POINTER(bem_batch_info)]),
    "bem_batch_destroy": (ctypes.c_int, [_P]),
    "bem_op_blocks": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), _P, _P]),
    "bem_partition": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), _P, _P]),
    "bem_op_freq_hist": (ctypes.c_int, [_P, _P]),
    "bem_op_destroy": (ctypes.c_int, [_P]),
    "bem_version": (ctypes.c_char_p, []),
}


def lib():
    """Loads libbem.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbem.so is not built (run __graft_entry__.build() or "
                              "python paper_2607_15292_amd/build.py); no fallback path exists")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, shape=None):
    """(pointer, flags) of a numpy array (host) or torch CUDA tensor (device).  With shape, the
    buffer must be complex128 of exactly that shape: the library reads and writes that many
    elements through the pointer."""
    if shape is not None:
        dt = str(a.dtype)
        if dt not in ("complex128", "torch.complex128"):
            raise ValueError("expected a complex128 buffer, got %s" % dt)
        if tuple(a.shape) != tuple(shape):
            raise ValueError("expected shape %s, got %s" % (tuple(shape), tuple(a.shape)))
    if _is_torch(a):
        if not a.is_cuda:
            raise ValueError("torch tensors must live on the GPU; use numpy for host buffers")
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if a.is_conj() or a.is_neg():
            raise ValueError("tensor is a lazy conjugate or negative view; call resolve_conj() / resolve_neg()")
        return ctypes.c_void_p(a.data_ptr()), DEVICE_PTR
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return ctypes.c_void_p(a.ctypes.data), 0


class Context:
    """Owns a bem_ctx (one device)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        rc = lib().bem_create(ctypes.byref(h), int(device))
        if rc != BEM_OK:
            raise BemError(rc, "bem_create(device=%d) failed" % device)
        self.h = h
        self.device = device
        self._keep = []

    def _check(self, rc):
        if rc < 0:
            raise BemError(rc, lib().bem_last_error(self.h).decode())
        return rc

    def close(self):
        if self.h:
            self._check(lib().bem_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().bem_destroy(self.h)
        except Exception:
            pass

    def set_stream(self, stream):
        """stream: torch.cuda.Stream, a raw hipStream_t as int, or None (null stream)."""
        raw = 0 if stream is None else (stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        self._check(lib().bem_set_stream(self.h, ctypes.c_void_p(raw)))

    def _sync_torch_stream(self):
        import torch
        self.set_stream(torch.cuda.current_stream())

    def set_mesh(self, nodes, tris):
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.K = int(tris.shape[0])
        self.n_nodes = int(nodes.shape[0])
        return self._check(lib().bem_set_mesh(self.h, nodes.ctypes.data, nodes.shape[0], tris.ctypes.data, tris.shape[0]))

    def set_meshes(self, meshes):
        """Several meshes [(nodes, tris), ...] in one context as components (a batch sharing
        material and contour): nodes and triangles concatenated in order, element offsets
        returned; the compressed operator is block diagonal over the meshes."""
        nodes, tris, comp, offs, noff = [], [], [], [0], 0
        for c, (X, T) in enumerate(meshes):
            nodes.append(np.asarray(X, dtype=np.float64))
            tris.append(np.asarray(T, dtype=np.int32) + noff)
            comp.append(np.full(len(T), c, dtype=np.int32))
            noff += len(X)
            offs.append(offs[-1] + len(T))
        self.set_mesh(np.concatenate(nodes), np.concatenate(tris))
        comp = np.ascontiguousarray(np.concatenate(comp))
        self._check(lib().bem_set_components(self.h, comp.ctypes.data, len(meshes)))
        return offs

    def set_material(self, rho, cp, cs):
        return self._check(lib().bem_set_material(self.h, float(rho), float(cp), float(cs)))

    def set_frequencies(self, s):
        s = np.atleast_1d(np.asarray(s, dtype=np.complex128))
        a = np.ascontiguousarray(np.stack([s.real, s.imag], axis=-1))
        self.L = int(s.shape[0])
        return self._check(lib().bem_set_frequencies(self.h, a.ctypes.data, self.L))

    def freq_pairs(self):
        n = ctypes.c_int32()
        self._check(lib().bem_freq_pairs(self.h, ctypes.byref(n)))
        return n.value

    def set_quadrature(self, near_on=False, near_r1=1.5, near_r2=3.0, self_nt=8, self_nr=8):
        q = bem_quad(int(bool(near_on)), float(near_r1), float(near_r2), int(self_nt), int(self_nr))
        return self._check(lib().bem_set_quadrature(self.h, ctypes.byref(q)))

    def set_entry_table(self, table):
        """table: torch complex128 CUDA tensor [L, K, K, 3, 3] (kept alive by the context)."""
        p, fl = _ptr(table)
        if not fl & DEVICE_PTR:
            raise ValueError("the entry table must be a device tensor")
        self._keep.append(table)
        return self._check(lib().bem_set_entry_table(self.h, p))

    def entries(self, op, i, j, l, prec=PREC_F64, out=None):
        """ENTRY(op, i, j, l) -> complex128 [n, 3, 3] (numpy for numpy indices, torch for torch)."""
        if _is_torch(i):
            import torch
            n = i.numel()
            if out is None:
                out = torch.empty((n, 3, 3), dtype=torch.complex128, device=i.device)
            self._sync_torch_stream()
        else:
            i, j, l = (np.ascontiguousarray(np.ravel(a), dtype=np.int32) for a in np.broadcast_arrays(i, j, l))
            n = i.size
            if out is None:
                out = np.empty((n, 3, 3), dtype=np.complex128)
        pi, fl = _ptr(i)
        pj, _ = _ptr(j)
        pl, _ = _ptr(l)
        po, _ = _ptr(out)
        self._check(lib().bem_entries(self.h, int(op), int(prec), int(n), pi, pj, pl, po, fl))
        return out

    def assemble_dense(self, op, prec=PREC_F64):
        h = ctypes.c_void_p()
        self._check(lib().bem_assemble_dense(self.h, int(op), int(prec), ctypes.byref(h)))
        return Operator(self, h)

    def compress(self, op, eps3d=1e-6, eps_aca=0.0, eta=1.5, leaf=64, prec=PREC_F64, mixed_eps_floor=1e-5,
                 pool_bytes=0, far_dense_max=48, aca_rounds=0, face_order=0):
        o = bem_aca_opts(float(eps3d), float(eps_aca), float(eta), int(leaf), int(prec), float(mixed_eps_floor),
                         int(pool_bytes), int(far_dense_max), int(aca_rounds), int(face_order))
        h = ctypes.c_void_p()
        self._check(lib().bem_compress(self.h, int(op), ctypes.byref(o), ctypes.byref(h)))
        return Operator(self, h)

    def matrix_free(self, op):
        """Matrix-free FP64 operator (V, K or HK): every product recomputes the entries with
        the context's current mesh, material, contour points and quadrature."""
        h = ctypes.c_void_p()
        self._check(lib().bem_matrix_free(self.h, int(op), ctypes.byref(h)))
        return Operator(self, h)

    def aca_matrix(self, A, tol, max_cols=0, prec=PREC_F64):
        """Per-slice ACA + recompression of one [3m][3n] host matrix; returns
        (kc, kk, Ubar, Vbar) with Ubar/Vbar None unless kk > 0."""
        dt = np.complex64 if prec == PREC_MIXED else np.complex128
        A = np.ascontiguousarray(A, dtype=dt)
        m, n = A.shape[0] // 3, A.shape[1] // 3
        cap = 3 * min(m, n)
        U = np.zeros(3 * m * cap, dtype=dt)
        V = np.zeros(3 * n * cap, dtype=dt)
        kc, kk = ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().bem_aca_matrix(self.h, int(prec), m, n, A.ctypes.data, float(tol), int(max_cols),
                                         ctypes.byref(kc), ctypes.byref(kk), U.ctypes.data, V.ctypes.data))
        k = kk.value
        if k <= 0:
            return kc.value, k, None, None
        return kc.value, k, U[:3 * m * k].reshape(3 * m, k), V[:3 * n * k].reshape(3 * n, k)

    def aca_matrix_noalloc(self, A, tol, max_cols=0, U=None, V=None, kc_kk=None):
        """bem_aca_matrix_noalloc on torch CUDA tensors: A [3m, 3n] complex128 or complex64
        (the precision follows A).  U, V, kc_kk (int32 [2]) are allocated here by torch unless
        given (the library itself allocates nothing).  Returns (kc, kk, U[:, :kk], V[:, :kk])
        after synchronising the stream; U, V are None unless kk > 0."""
        import torch
        assert _is_torch(A) and A.is_cuda and A.dim() == 2
        A = A.contiguous()
        prec = PREC_MIXED if A.dtype == torch.complex64 else PREC_F64
        m, n = A.shape[0] // 3, A.shape[1] // 3
        cap = 3 * min(m, n)
        if U is None:
            U = torch.zeros(3 * m * cap, dtype=A.dtype, device=A.device)
        if V is None:
            V = torch.zeros(3 * n * cap, dtype=A.dtype, device=A.device)
        if kc_kk is None:
            kc_kk = torch.zeros(2, dtype=torch.int32, device=A.device)
        self._sync_torch_stream()
        self._check(lib().bem_aca_matrix_noalloc(self.h, int(prec), m, n, A.data_ptr(), float(tol), int(max_cols),
                                                 kc_kk.data_ptr(), U.data_ptr(), V.data_ptr()))
        torch.cuda.current_stream().synchronize()
        kc, kk = (int(v) for v in kc_kk.cpu())
        if kk <= 0:
            return kc, kk, None, None
        return kc, kk, U[:3 * m * kk].reshape(3 * m, kk), V[:3 * n * kk].reshape(3 * n, kk)

    def apply_mf(self, op, x, y=None, transpose=False):
        """y[r, l] = A(s_l) x[r, l] (or A(s_l)^T x[r, l]) with entries recomputed (no storage);
        x: [nrhs, L, 3K] numpy or torch CUDA complex128."""
        nrhs = x.shape[0]
        if _is_torch(x):
            import torch
            if y is None:
                y = torch.empty_like(x)
            self._sync_torch_stream()
        elif y is None:
            y = np.empty_like(x)
        shp = (nrhs, self.L, 3 * self.K)
        px, fl = _ptr(x, shp)
        py, _ = _ptr(y, shp)
        self._check(lib().bem_apply_mf(self.h, int(op), int(bool(transpose)), int(nrhs), px, py, fl))
        return y

    def apply_linear_dl(self, g, y=None, free_term=True):
        """y[r, l] = (C +) K_lin(s_l) g[r, l]: the double layer against the nodal hat functions
        (entries recomputed); g: [nrhs, L, 3 n_nodes] numpy or torch CUDA complex128, y:
        [nrhs, L, 3K]."""
        nrhs = g.shape[0]
        shp_y = (nrhs, self.L, 3 * self.K)
        if _is_torch(g):
            import torch
            if y is None:
                y = torch.empty(shp_y, dtype=g.dtype, device=g.device)
            self._sync_torch_stream()
        elif y is None:
            y = np.empty(shp_y, dtype=np.complex128)
        pg, fl = _ptr(g, (nrhs, self.L, 3 * self.n_nodes))
        py, _ = _ptr(y, shp_y)
        self._check(lib().bem_apply_linear_dl(self.h, int(nrhs), pg, py, fl | (FREE_TERM if free_term else 0)))
        return y

    def adjoint_v(self, w, x):
        """(S, grad_nodes [n_nodes, 3], grad_mat [rho, c_p, c_s]) of S = sum w^T V(s_l) x
        (gradient of Re S); w, x: [nrhs, L, 3K] numpy or torch CUDA complex128."""
        nrhs = x.shape[0]
        if _is_torch(x):
            self._sync_torch_stream()
        shp = (nrhs, self.L, 3 * self.K)
        pw, fl = _ptr(w, shp)
        px, fl2 = _ptr(x, shp)
        if fl != fl2:
            raise ValueError("w and x must both be host arrays or both device tensors")
        val = np.zeros(2)
        gn = np.zeros((self.n_nodes, 3))
        gm = np.zeros(3)
        self._check(lib().bem_adjoint_v(self.h, int(nrhs), pw, px, fl, val.ctypes.data, gn.ctypes.data,
                                        gm.ctypes.data))
        return complex(val[0], val[1]), gn, gm

    def adjoint_k(self, w, x, op=OP_K):
        """(S, grad_nodes [n_nodes, 3], grad_mat [rho, c_p, c_s]) of S = sum w^T A(s_l) x with
        A = K (op OP_K) or I/2 + K (OP_HK), gradient of Re S; w, x as adjoint_v."""
        nrhs = x.shape[0]
        if _is_torch(x):
            self._sync_torch_stream()
        shp = (nrhs, self.L, 3 * self.K)
        pw, fl = _ptr(w, shp)
        px, fl2 = _ptr(x, shp)
        if fl != fl2:
            raise ValueError("w and x must both be host arrays or both device tensors")
        val = np.zeros(2)
        gn = np.zeros((self.n_nodes, 3))
        gm = np.zeros(3)
        self._check(lib().bem_adjoint_k(self.h, int(op), int(nrhs), pw, px, fl, val.ctypes.data, gn.ctypes.data,
                                        gm.ctypes.data))
        return complex(val[0], val[1]), gn, gm

    def partition(self, eta=1.5, leaf=64):
        n = ctypes.c_int64()
        self._check(lib().bem_partition(self.h, float(eta), int(leaf), ctypes.byref(n), None, None))
        rows = np.zeros((n.value, 8), dtype=np.int64)
        perm = np.zeros(self.K, dtype=np.int32)
        self._check(lib().bem_partition(self.h, float(eta), int(leaf), ctypes.byref(n), rows.ctypes.data,
                                        perm.ctypes.data))
        return rows, perm


class Operator:
    """Owns a bem_op (dense or compressed)."""

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h

    def destroy(self):
        if self.h:
            self.ctx._check(lib().bem_op_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().bem_op_destroy(self.h)
        except Exception:
            pass

    def stats(self):
        st = bem_stats()
        self.ctx._check(lib().bem_op_stats(self.h, ctypes.byref(st)))
        return st.as_dict()

    def dense(self, out=None):
        K, L = self.ctx.K, self.ctx.L
        if out is None:
            out = np.empty((L, 3 * K, 3 * K), dtype=np.complex128)
        p, fl = _ptr(out)
        if fl & DEVICE_PTR:
            self.ctx._sync_torch_stream()
        self.ctx._check(lib().bem_op_dense_copy(self.h, p, fl))
        return out

    def apply(self, x, y=None, shared_x=False, transpose=False):
        """y[r, l] = A(s_l) x[r, l] (A(s_l)^T with transpose); x: [nrhs, L, 3K] (or [nrhs, 3K]
        with shared_x)."""
        K, L = self.ctx.K, self.ctx.L
        nrhs = x.shape[0]
        if _is_torch(x):
            import torch
            if y is None:
                y = torch.empty((nrhs, L, 3 * K), dtype=torch.complex128, device=x.device)
            self.ctx._sync_torch_stream()
        elif y is None:
            y = np.empty((nrhs, L, 3 * K), dtype=np.complex128)
        px, fl = _ptr(x, (nrhs, 3 * K) if shared_x else (nrhs, L, 3 * K))
        py, _ = _ptr(y, (nrhs, L, 3 * K))
        self.ctx._check(lib().bem_apply(self.h, int(nrhs), px, py,
                                        fl | (SHARED_X if shared_x else 0) | (TRANSPOSE if transpose else 0)))
        return y

    def solve(self, b, x=None, inner=None, tol=1e-8, inner_tol=1e-3, restart=30, max_iter=500, max_refine=10,
              transpose=False):
        """x[r, l] = A(s_l)^{-1} b[r, l] by GMRES with iterative refinement (bem_solve);
        inner: a cheaper operator (same device, K and L; possibly of another context) for the
        inner GMRES runs.
        Returns (x, stats dict)."""
        K, L = self.ctx.K, self.ctx.L
        nrhs = b.shape[0]
        if _is_torch(b):
            import torch
            if x is None:
                x = torch.empty((nrhs, L, 3 * K), dtype=torch.complex128, device=b.device)
            self.ctx._sync_torch_stream()
        elif x is None:
            x = np.empty((nrhs, L, 3 * K), dtype=np.complex128)
        pb, fl = _ptr(b, (nrhs, L, 3 * K))
        px, _ = _ptr(x, (nrhs, L, 3 * K))
        o = bem_solve_opts(float(tol), float(inner_tol), int(restart), int(max_iter), int(max_refine), 0)
        st = bem_solve_stats()
        fl |= TRANSPOSE if transpose else 0
        rc = self.ctx._check(lib().bem_solve(self.h, inner.h if inner is not None else None, int(nrhs), pb, px, fl,
                                             ctypes.byref(o), ctypes.byref(st)))
        d = st.as_dict()
        d["rc"] = rc
        return x, d

    def cq_dirichlet(self, g, dt, R, H=None, t=None, tol=1e-8, restart=30, max_iter=500, max_refine=10):
        """Tractions t[n] of the Dirichlet problem in time by BDF2 convolution quadrature
        (marching on in time with weighted-sum histories); g: [N, 3K] samples at t_n = n dt.
        Returns (t, stats dict)."""
        N = g.shape[0]
        if _is_torch(g):
            import torch
            if t is None:
                t = torch.empty_like(g)
            self.ctx._sync_torch_stream()
        elif t is None:
            t = np.empty_like(g)
        pg, fl = _ptr(g, (N, 3 * self.ctx.K))
        pt, _ = _ptr(t, (N, 3 * self.ctx.K))
        o = bem_solve_opts(float(tol), 1e-3, int(restart), int(max_iter), int(max_refine), 0)
        st = bem_solve_stats()
        rc = self.ctx._check(lib().bem_cq_dirichlet(self.h, H.h if H is not None else None, int(N), float(dt),
                                                    float(R), pg, pt, fl, ctypes.byref(o), ctypes.byref(st)))
        d = st.as_dict()
        d["rc"] = rc
        return t, d

    def apply_weighted(self, W, y=None):
        K = self.ctx.K
        if _is_torch(W):
            import torch
            if y is None:
                y = torch.empty((3 * K,), dtype=torch.complex128, device=W.device)
            self.ctx._sync_torch_stream()
        elif y is None:
            y = np.empty((3 * K,), dtype=np.complex128)
        pw, fl = _ptr(W, (self.ctx.L, 3 * K))
        py, _ = _ptr(y, (3 * K,))
        self.ctx._check(lib().bem_apply_weighted(self.h, pw, py, fl))
        return y

    def blocks(self):
        n = ctypes.c_int64()
        self.ctx._check(lib().bem_op_blocks(self.h, ctypes.byref(n), None, None))
        rows = np.zeros((n.value, 8), dtype=np.int64)
        perm = np.zeros(self.ctx.K, dtype=np.int32)
        self.ctx._check(lib().bem_op_blocks(self.h, ctypes.byref(n), rows.ctypes.data, perm.ctypes.data))
        return rows, perm

    def freq_hist(self):
        h = np.zeros(self.ctx.L, dtype=np.int64)
        self.ctx._check(lib().bem_op_freq_hist(self.h, h.ctypes.data))
        return h


def version():
    return lib().bem_version().decode()


BATCH_GRAPH = 1
BATCH_TUNE = 2


class Batch:
    """Owns a bem_batch: the products of several compressed operators (same L) in one set of
    launches.  Keeps the operators alive while it lives."""

    def __init__(self, ops, nrhs=1, graph=False, tune=False):
        self.ops = list(ops)
        self.ctx = self.ops[0].ctx
        self.nrhs = int(nrhs)
        arr = (ctypes.c_void_p * len(self.ops))(*[o.h for o in self.ops])
        h = ctypes.c_void_p()
        self.ctx._sync_torch_stream()
        fl = (BATCH_GRAPH if graph else 0) | (BATCH_TUNE if tune else 0)
        self.ctx._check(lib().bem_batch_create(arr, len(self.ops), self.nrhs, fl, ctypes.byref(h)))
        self.h = h

    def apply(self, xs, ys=None):
        """ys[o][r, l] = A_o(s_l) xs[o][r, l]; xs: list of [nrhs, L, 3 K_o] arrays, all numpy or
        all torch CUDA tensors."""
        if len(xs) != len(self.ops):
            raise ValueError("one input per operator")
        dev = _is_torch(xs[0])
        if ys is None:
            if dev:
                import torch
                ys = [torch.empty_like(x) for x in xs]
            else:
                ys = [np.empty_like(x) for x in xs]
        if dev:
            self.ctx._sync_torch_stream()
        shp = [(self.nrhs, op.ctx.L, 3 * op.ctx.K) for op in self.ops]
        px, fl = zip(*[_ptr(x, sh) for x, sh in zip(xs, shp)])
        py, fly = zip(*[_ptr(y, sh) for y, sh in zip(ys, shp)])
        if len(set(fl) | set(fly)) != 1:
            raise ValueError("inputs and outputs must all be host arrays or all device tensors")
        ax = (ctypes.c_void_p * len(xs))(*[p.value for p in px])
        ay = (ctypes.c_void_p * len(ys))(*[p.value for p in py])
        self.ctx._check(lib().bem_batch_apply(self.h, ax, ay, fl[0]))
        return ys

    def info(self):
        i = bem_batch_info()
        self.ctx._check(lib().bem_batch_info_get(self.h, ctypes.byref(i)))
        return i.as_dict()

    def destroy(self):
        if self.h:
            self.ctx._check(lib().bem_batch_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().bem_batch_destroy(self.h)
        except Exception:
            pass
