"""Batched compression: several meshes as components of one context (one material, one
contour) are compressed in one set of launches and applied by one product.  The operator is
block diagonal over the meshes, and each diagonal block is the operator of that mesh compressed
alone: the same blocks, ranks and bytes, the same products (FP64 to rounding; mixed precision to
the FP32 accumulation of the far field, whose segments are cut differently), and the oracle's
rows on samples of every mesh."""
import numpy as np
import pytest

import oracle
from paper_2607_15292_amd import binding as B
from paper_2607_15292_amd import workloads as W

pytestmark = pytest.mark.gpu


def _meshes():
    X1, T1 = W.cube_grid(4, 1.0)                       # 192 triangles
    X2, T2 = W.icosphere(3)                            # 1280
    X3, T3 = W.cube_grid(2, 0.5)                       # 48
    return [(X1, T1), (X2 + np.array([4.0, 0.0, 0.0]), T2), (X3 + np.array([0.0, 3.0, 0.0]), T3)]


def _ctx(s):
    c = B.Context(0)
    c.set_material(1.0, 1.0, 0.5)
    c.set_frequencies(s)
    c.set_quadrature(near_on=True)
    return c


@pytest.mark.parametrize("prec,eps,tol_same,bound", [(B.PREC_F64, 1e-8, 1e-12, 1e-6), (B.PREC_MIXED, 1e-6, 1e-5, 1e-4)])
@pytest.mark.parametrize("opk", [B.OP_V, B.OP_HK])
def test_batched_compression_equals_each_mesh(prec, eps, tol_same, bound, opk):
    import torch
    assert torch.cuda.is_available()
    L = 16
    s = W.bdf2_contour(L, 0.1)
    meshes = _meshes()
    cu = _ctx(s)
    offs = cu.set_meshes(meshes)
    Kt = offs[-1]
    opu = cu.compress(opk, eps3d=eps, leaf=32, prec=prec)
    stu = opu.stats()
    x = W.random_rhs(21, (2, L, 3 * Kt))
    yu = opu.apply(x)
    nbytes, dense = 0, 0.0
    rng = np.random.default_rng(3)
    for q, (X, T) in enumerate(meshes):
        c = _ctx(s)
        c.set_mesh(X, T)
        op = c.compress(opk, eps3d=eps, leaf=32, prec=prec)
        st = op.stats()
        nbytes += st["bytes"]
        dense += L * (3 * len(T)) ** 2 * 16.0
        sl = slice(3 * offs[q], 3 * offs[q + 1])
        yq = op.apply(np.ascontiguousarray(x[:, :, sl]))
        diff = np.abs(yu[:, :, sl] - yq).max() / np.abs(yq).max()
        assert diff <= tol_same, (q, diff)
        rows = np.sort(rng.choice(len(T), size=min(12, len(T)), replace=False))
        yo = oracle.Problem(X, T, s, near_on=True).matvec_rows(opk, rows, np.ascontiguousarray(x[:, :, sl]))
        yg = yu[:, :, sl].reshape(2, L, len(T), 3)[:, :, rows, :].reshape(2, L, -1)
        err = float((np.linalg.norm(yg - yo, axis=-1) / np.linalg.norm(yo, axis=-1)).max())
        assert err < bound, (q, err)
        op.destroy()
        c.close()
    assert stu["bytes"] == nbytes
    assert abs(stu["compression_rate"] - nbytes / dense) < 1e-12
    opu.destroy()


def test_components_refuse_dense_and_matrix_free():
    L = 4
    c = _ctx(W.bdf2_contour(L, 0.1))
    c.set_meshes(_meshes()[:2])
    with pytest.raises(B.BemError):
        c.assemble_dense(B.OP_V)
    x = W.random_rhs(1, (1, L, 3 * (192 + 1280)))
    with pytest.raises(B.BemError):
        c.apply_mf(B.OP_V, x)
