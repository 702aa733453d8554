"""GPU parity of the raw entry generator and the dense all-frequency products against the
FP64 oracle, through the C-ABI.

Tolerances: FP64 entries agree elementwise to 1e-13 * max|entry| + 1e-10 * |entry| (same
rules, different but equivalent formulas and summation order; the principal-value self term
of K loses ~1e-11 of itself to cancellation).  Mixed entries (regular pairs in FP32, 7-point
sums of unit-roundoff 6e-8 terms) agree to 3e-6 of the largest entry of their block row.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15292_amd import binding as B
from paper_2607_15292_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def make(X, T, s, near_on=False, mat=(1.0, 1.0, 0.5)):
    c = B.Context(0)
    c.set_mesh(X, T)
    c.set_material(*mat)
    c.set_frequencies(s)
    c.set_quadrature(near_on=near_on)
    P = oracle.Problem(X, T, s, *mat, near_on=near_on)
    return c, P


def close64(g, o, atol=1e-13):
    """atol: 1e-13 of the largest entry for V; 1e-11 for K, whose principal-value self
    entries lose ~1e-11 of the largest entry to cancellation (order-dependent rounding)."""
    g, o = np.asarray(g), np.asarray(o)
    tol = atol * np.abs(o).max() + 1e-10 * np.abs(o)
    bad = np.abs(g - o) > tol
    return not bad.any(), float((np.abs(g - o) / (np.abs(o).max())).max())


def test_c1_dense_single_layer_all_entries(torch):
    # configuration 1: cube [-1,1]^3, 192 triangles, L = 16 BDF2 points, 7-point + Duffy
    X, T = W.cube_grid(4, 1.0)
    s = W.bdf2_contour(16, 0.1)
    c, P = make(X, T, s)
    op = c.assemble_dense(B.OP_V)
    G = op.dense()
    O = P.dense(oracle.OP_V)
    ok, err = close64(G, O)
    assert ok, err
    st = op.stats()
    assert st["entries_generated"] == 192 * 192 * 16


@pytest.mark.parametrize("opk", [B.OP_K, B.OP_HK])
def test_dense_double_layer_entries(torch, opk):
    X, T = W.cube_grid(3, 1.0)
    s = W.bdf2_contour(4, 0.1)
    c, P = make(X, T, s)
    G = c.assemble_dense(opk).dense()
    O = P.dense(opk)
    ok, err = close64(G, O, atol=1e-11)
    assert ok, err


@pytest.mark.parametrize("opk", [B.OP_V, B.OP_K])
def test_near_rule_entries_sphere(torch, opk):
    X, T = W.icosphere(2)
    s = W.bdf2_contour(8, 0.1)
    c, P = make(X, T, s, near_on=True, mat=(2.0, 1.0, 0.55))
    rng = np.random.default_rng(5)
    K = len(T)
    i = rng.integers(0, K, 3000)
    j = np.where(rng.random(3000) < 0.3, (i + rng.integers(0, 4, 3000)) % K, rng.integers(0, K, 3000))
    l = rng.integers(0, len(s), 3000)
    g = c.entries(opk, i, j, l)
    o = P.entries(opk, i, j, l)
    ok, err = close64(g, o, atol=1e-13 if opk == B.OP_V else 1e-11)
    assert ok, err


def test_mixed_precision_entries(torch):
    X, T = W.icosphere(2)
    s = W.bdf2_contour(16, 0.1)
    c, P = make(X, T, s, near_on=True)
    K = len(T)
    for opk in (B.OP_V, B.OP_K):
        i = np.repeat(np.arange(0, K, 7), K)
        j = np.tile(np.arange(K), len(np.arange(0, K, 7)))
        l = (i + j) % len(s)
        g = c.entries(opk, i, j, l, prec=B.PREC_MIXED).reshape(-1, K, 3, 3)
        o = P.entries(opk, i, j, l).reshape(-1, K, 3, 3)
        rowscale = np.abs(o).max(axis=(1, 2, 3))
        err = (np.abs(g - o).max(axis=(2, 3)) / rowscale[:, None]).max()
        assert err < 3e-6, err


def test_entries_device_pointers_match_host(torch):
    X, T = W.cube_grid(2, 1.0)
    s = W.bdf2_contour(6, 0.1)
    c, _ = make(X, T, s)
    rng = np.random.default_rng(1)
    i, j, l = rng.integers(0, len(T), 500), rng.integers(0, len(T), 500), rng.integers(0, 6, 500)
    h = c.entries(B.OP_V, i, j, l)
    ti, tj, tl = (torch.tensor(a, dtype=torch.int32, device="cuda") for a in (i, j, l))
    d = c.entries(B.OP_V, ti, tj, tl)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy(), h)


def test_entries_edge_cases(torch):
    X, T = W.cube_grid(2, 1.0)
    s = W.bdf2_contour(4, 0.1)
    c, P = make(X, T, s)
    # empty request
    assert c.entries(B.OP_V, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32)).shape == (0, 3, 3)
    # out-of-range index: host buffers are checked on the host
    with pytest.raises(B.BemError):
        c.entries(B.OP_V, [0], [len(T)], [0])
    # device buffers: the offending entry is NaN, the others are computed
    ti = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    tj = torch.tensor([1, len(T) + 5], dtype=torch.int32, device="cuda")
    tl = torch.tensor([0, 0], dtype=torch.int32, device="cuda")
    d = c.entries(B.OP_V, ti, tj, tl)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    assert np.isnan(d[1]).all() and np.isfinite(d[0]).all()
    ok, _ = close64(d[0], P.entries(0, 0, 1, 0)[0])
    assert ok


def test_single_element_and_single_frequency(torch):
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.2, 0.9, 0.0]])
    T = np.array([[0, 1, 2]], dtype=np.int32)
    c, P = make(X, T, [3.0 - 1.0j])
    for opk in (B.OP_V, B.OP_K, B.OP_HK):
        g = c.assemble_dense(opk).dense()
        ok, err = close64(g, P.dense(opk), atol=1e-13 if opk == B.OP_V else 1e-11)
        assert ok, (opk, err)


def test_conjugate_frequency_symmetry(torch):
    X, T = W.cube_grid(2, 1.0)
    s = np.array([4.0 + 3.0j, 4.0 - 3.0j])
    c, _ = make(X, T, s)
    G = c.assemble_dense(B.OP_K).dense()
    assert np.abs(G[1] - np.conj(G[0])).max() <= 1e-14 * np.abs(G[0]).max()


def test_dense_apply_and_weighted_sum(torch):
    X, T = W.cube_grid(4, 1.0)
    s = W.bdf2_contour(16, 0.1)
    c, P = make(X, T, s)
    op = c.assemble_dense(B.OP_V)
    O = P.dense(oracle.OP_V)
    M = 3 * len(T)
    x = W.random_rhs(0, (2, M))
    y = op.apply(x, shared_x=True)
    yo = np.einsum("lij,rj->rli", O, x)
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
    xs = W.random_rhs(3, (3, 16, M))
    y = op.apply(torch.tensor(xs, device="cuda")).cpu().numpy()
    yo = np.einsum("lij,rlj->rli", O, xs)
    assert np.abs(y - yo).max() <= 1e-12 * np.abs(yo).max()
    Wt = W.random_rhs(4, (16, M))
    yw = op.apply_weighted(Wt)
    ywo = np.einsum("lij,lj->i", O, Wt)
    assert np.abs(yw - ywo).max() <= 1e-12 * np.abs(ywo).max()
