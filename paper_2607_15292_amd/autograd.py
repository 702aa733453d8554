"""Differentiable single- and double-layer products and single-layer solutions:
torch.autograd.Function over the library's matrix-free product, transposed solves and
adjoints (bem_apply_mf, bem_solve with BEM_TRANSPOSE, bem_adjoint_v, bem_adjoint_k).  The gradients recompute the entries; nothing of the
operator is stored for them.

    y = single_layer(bem_ctx, nodes, material, x)

y[r, l] = V(s_l) x[r, l] for the mesh with node coordinates `nodes` (float64 [n_nodes, 3],
any device; the triangles and contour points are those set on `bem_ctx`), material
(rho, c_p, c_s) as a float64 tensor [3], and x complex128 [nrhs, L, 3K] on the GPU.  The
gradients are those of the discrete operator with the context's quadrature (pair classes of
the near rule held fixed): the node coordinates and the speeds by the adjoint kernel, x by the
transposed product.  double_layer(bem_ctx, nodes, material, x, tris, free_term=True) is the
same for (I/2 + K(s_l)) x or K(s_l) x.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def _load(ctx, tris, nodes, material):
    nodes_np = nodes.detach().to("cpu", torch.float64).numpy()
    mat = material.detach().to("cpu", torch.float64).numpy()
    ctx.set_mesh(nodes_np, tris)
    ctx.set_material(float(mat[0]), float(mat[1]), float(mat[2]))


class SingleLayer(torch.autograd.Function):
    @staticmethod
    def forward(fctx, bem_ctx, tris, nodes, material, x):
        _load(bem_ctx, tris, nodes, material)
        y = bem_ctx.apply_mf(B.OP_V, x.contiguous())
        fctx.bem = bem_ctx
        fctx.tris = tris
        fctx.save_for_backward(nodes, material, x)
        return y

    @staticmethod
    def backward(fctx, gy):
        nodes, material, x = fctx.saved_tensors
        bem = fctx.bem
        _load(bem, fctx.tris, nodes, material)
        # real loss: dL = Re sum conj(gy) dy, so the node and material gradients are those of
        # Re S with S = sum conj(gy)^T V x, and the input gradient is V^H gy
        w = gy.conj().resolve_conj().contiguous()
        g_nodes = g_mat = g_x = None
        if fctx.needs_input_grad[2] or fctx.needs_input_grad[3]:
            _, gn, gm = bem.adjoint_v(w, x.contiguous())
            g_nodes = torch.as_tensor(gn, dtype=nodes.dtype, device=nodes.device)
            g_mat = torch.as_tensor(gm, dtype=material.dtype, device=material.device)
        if fctx.needs_input_grad[4]:
            g_x = bem.apply_mf(B.OP_V, w, transpose=True).conj()
        return None, None, g_nodes, g_mat, g_x


def single_layer(bem_ctx, nodes, material, x, tris):
    """y[r, l] = V(s_l) x[r, l], differentiable in nodes, material and x."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    return SingleLayer.apply(bem_ctx, tris, nodes, material, x)


class DoubleLayer(torch.autograd.Function):
    """y[r, l] = A(s_l) x[r, l] with A = K or I/2 + K (matrix-free); backward as SingleLayer
    with the double layer's adjoint kernel (bem_adjoint_k) and its transposed product."""

    @staticmethod
    def forward(fctx, bem_ctx, tris, nodes, material, x, op):
        _load(bem_ctx, tris, nodes, material)
        y = bem_ctx.apply_mf(op, x.contiguous())
        fctx.bem = bem_ctx
        fctx.tris = tris
        fctx.op = op
        fctx.save_for_backward(nodes, material, x)
        return y

    @staticmethod
    def backward(fctx, gy):
        nodes, material, x = fctx.saved_tensors
        bem = fctx.bem
        _load(bem, fctx.tris, nodes, material)
        w = gy.conj().resolve_conj().contiguous()
        g_nodes = g_mat = g_x = None
        if fctx.needs_input_grad[2] or fctx.needs_input_grad[3]:
            _, gn, gm = bem.adjoint_k(w, x.contiguous(), op=fctx.op)
            g_nodes = torch.as_tensor(gn, dtype=nodes.dtype, device=nodes.device)
            g_mat = torch.as_tensor(gm, dtype=material.dtype, device=material.device)
        if fctx.needs_input_grad[4]:
            g_x = bem.apply_mf(fctx.op, w, transpose=True).conj()
        return None, None, g_nodes, g_mat, g_x, None


def double_layer(bem_ctx, nodes, material, x, tris, free_term=True):
    """y[r, l] = (I/2 + K(s_l)) x[r, l] (free_term) or K(s_l) x[r, l], differentiable in nodes,
    material and x."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    return DoubleLayer.apply(bem_ctx, tris, nodes, material, x, B.OP_HK if free_term else B.OP_K)


class SingleLayerSolve(torch.autograd.Function):
    """t[r, l] = V(s_l)^{-1} b[r, l] by GMRES (bem_solve) with V assembled dense, compressed
    in FP64 at eps, or matrix-free (entries recomputed at every product), optionally with a
    compressed inner operator carrying the GMRES iterations of the iterative refinement;
    backward: one transposed solve V^T nu = conj(g_t) per call with the same operators, then
    g_b = conj(nu) and the node and material gradients are minus those of
    Re sum nu^T V t (the adjoint kernel)."""

    @staticmethod
    def forward(fctx, bem_ctx, tris, nodes, material, b, tol, eps, matrix_free, inner):
        _load(bem_ctx, tris, nodes, material)
        if matrix_free:
            V = bem_ctx.matrix_free(B.OP_V)
        elif eps is None:
            V = bem_ctx.assemble_dense(B.OP_V)
        else:
            V = bem_ctx.compress(B.OP_V, eps3d=eps, prec=B.PREC_F64)
        own_inner = isinstance(inner, dict)
        Vi = bem_ctx.compress(B.OP_V, **inner) if own_inner else inner
        t, st = V.solve(b.contiguous(), inner=Vi, tol=tol)
        fctx.bem, fctx.tris, fctx.V, fctx.tol = bem_ctx, tris, V, tol
        fctx.Vi, fctx.own_inner = Vi, own_inner
        fctx.stats = [st]
        fctx.save_for_backward(nodes, material, t)
        return t

    @staticmethod
    def backward(fctx, gt):
        nodes, material, t = fctx.saved_tensors
        bem, V, Vi = fctx.bem, fctx.V, fctx.Vi
        _load(bem, fctx.tris, nodes, material)
        nu, st = V.solve(gt.conj().resolve_conj().contiguous(), inner=Vi, tol=fctx.tol, transpose=True)
        fctx.stats.append(st)
        V.destroy()
        if fctx.own_inner:
            Vi.destroy()
        fctx.V = fctx.Vi = None
        g_nodes = g_mat = None
        if fctx.needs_input_grad[2] or fctx.needs_input_grad[3]:
            _, gn, gm = bem.adjoint_v(nu, t.contiguous())
            g_nodes = -torch.as_tensor(gn, dtype=nodes.dtype, device=nodes.device)
            g_mat = -torch.as_tensor(gm, dtype=material.dtype, device=material.device)
        g_b = nu.conj() if fctx.needs_input_grad[4] else None
        return None, None, g_nodes, g_mat, g_b, None, None, None, None


def single_layer_solve(bem_ctx, nodes, material, b, tris, tol=1e-10, eps=None, matrix_free=False, inner=None):
    """t[r, l] = V(s_l)^{-1} b[r, l], differentiable in nodes, material and b.  V is dense
    (eps None), compressed in FP64 at eps, or matrix-free (matrix_free=True: FP64 entries
    recomputed at every product, nothing stored); inner: an operator for the inner GMRES runs
    of the iterative refinement (same device, K and L; kept by the caller), or a dict of
    Context.compress keywords for one compressed here and released after the backward pass."""
    tris = np.ascontiguousarray(tris, dtype=np.int32)
    return SingleLayerSolve.apply(bem_ctx, tris, nodes, material, b, tol, eps, bool(matrix_free), inner)
