"""Host logic of the H-matrix partition (Sec. 3.1, eqs. (cluster), (adm)), on a host-only
context: the blocks tile the index set exactly once, far blocks satisfy
min(diam) <= eta * dist with vertex boxes, near blocks are pairs of leaves that do not, and
the cluster order is a permutation."""
import numpy as np
import pytest

from paper_2607_15292_amd import binding as B
from paper_2607_15292_amd import workloads as W


def _boxes(X, T, perm, b, s):
    P = X[T[perm[b:b + s]]].reshape(-1, 3)
    return P.min(0), P.max(0)


def _diam(bx):
    return np.linalg.norm(bx[1] - bx[0])


def _dist(a, b):
    return np.linalg.norm(np.maximum(0, np.maximum(a[0] - b[1], b[0] - a[1])))


@pytest.mark.parametrize("mesh,leaf,eta", [("ico3", 64, 1.5), ("cube8", 32, 1.5), ("cube4", 16, 0.8),
                                           ("ico2", 1, 1.5), ("ico2", 1000, 1.5)])
def test_partition_properties(mesh, leaf, eta):
    X, T = {"ico3": lambda: W.icosphere(3), "ico2": lambda: W.icosphere(2), "cube8": lambda: W.cube_grid(8, 1.0),
            "cube4": lambda: W.cube_grid(4, 1.0)}[mesh]()
    c = B.Context(device=-1)
    c.set_mesh(X, T)
    rows, perm = c.partition(eta=eta, leaf=leaf)
    K = len(T)
    assert sorted(perm.tolist()) == list(range(K))
    cover = np.zeros((K, K), dtype=np.int32)
    for rb, rs, cb, cs, far, *_ in rows:
        cover[rb:rb + rs, cb:cb + cs] += 1
        A, Bx = _boxes(X, T, perm, rb, rs), _boxes(X, T, perm, cb, cs)
        adm = min(_diam(A), _diam(Bx)) <= eta * _dist(A, Bx)
        if far:
            assert adm
        else:
            assert not adm and rs <= leaf and cs <= leaf
    assert np.all(cover == 1)
    if K <= leaf:
        assert len(rows) == 1 and rows[0][4] == 0


def test_cluster_split_is_balanced():
    X, T = W.icosphere(3)
    c = B.Context(device=-1)
    c.set_mesh(X, T)
    rows, _ = c.partition(eta=1.5, leaf=64)
    sizes = set(int(r[1]) for r in rows) | set(int(r[3]) for r in rows)
    # 1280 = 2^8 * 5 halves down to 40-element leaves: every cluster size is 40 * 2^k
    assert all(s % 40 == 0 and ((s // 40) & (s // 40 - 1)) == 0 for s in sizes)


def _batch_meshes():
    X1, T1 = W.cube_grid(4, 1.0)
    X2, T2 = W.icosphere(3)
    X3, T3 = W.cube_grid(2, 0.5)
    return [(X1, T1), (X2 + np.array([4.0, 0.0, 0.0]), T2), (X3 + np.array([0.0, 3.0, 0.0]), T3)]


def test_components_partition_each_mesh_apart():
    """Several meshes as components of one context: no block couples two components, and the
    blocks and cluster order of each component are those of the mesh partitioned alone."""
    meshes = _batch_meshes()
    c = B.Context(device=-1)
    offs = c.set_meshes(meshes)
    rows, perm = c.partition(eta=1.5, leaf=32)
    comp = np.repeat(np.arange(len(meshes)), np.diff(offs))
    # cluster positions of each component are contiguous, in component order
    cpos = comp[perm]
    assert np.all(np.diff(cpos) >= 0)
    covered = np.zeros((offs[-1], offs[-1]), dtype=np.int32)
    for rb, rs, cb, cs, far, *_ in rows:
        assert len(set(cpos[rb:rb + rs]) | set(cpos[cb:cb + cs])) == 1
        covered[rb:rb + rs, cb:cb + cs] += 1
    for q, (X, T) in enumerate(meshes):
        b0 = offs[q]
        cq = B.Context(device=-1)
        cq.set_mesh(X, T)
        rq, pq = cq.partition(eta=1.5, leaf=32)
        assert np.array_equal(perm[b0:b0 + len(T)] - b0, pq)
        mine = sorted(tuple(r[:5]) for r in rows if cpos[r[0]] == q)
        theirs = sorted((r[0] + b0, r[1], r[2] + b0, r[3], r[4]) for r in rq)
        assert mine == theirs
        assert np.all(covered[b0:b0 + len(T), b0:b0 + len(T)] == 1)
    assert covered.sum() == sum(len(T) ** 2 for _, T in meshes)


def test_components_argument_errors():
    c = B.Context(device=-1)
    X, T = W.cube_grid(2, 1.0)
    z = np.zeros(len(T), np.int32)
    assert B.lib().bem_set_components(c.h, z.ctypes.data, 2) == -5  # before the mesh: BEM_ERR_STATE
    c.set_mesh(X, T)
    bad = np.zeros(len(T), np.int32)
    with pytest.raises(B.BemError):  # component 1 empty
        c._check(B.lib().bem_set_components(c.h, bad.ctypes.data, 2))
    bad[0] = 5
    with pytest.raises(B.BemError):  # out of range
        c._check(B.lib().bem_set_components(c.h, bad.ctypes.data, 2))
