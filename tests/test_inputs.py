"""Seeded input generators: the mesh families and contour points the workloads are built from.

Pins: node/element counts of the paper's unit-cube family (Table 1: 50/96, 194/384, 770/1536,
3074/6144), the icosphere and cube-grid counts, closed surfaces (Euler characteristic 2 and
enclosed volume by the divergence theorem), outward orientation, and the BDF2 contour points
(conjugate pairs, Re s > 0, min/max modulus).
"""
import os

import numpy as np
import pytest

from paper_2607_15292_amd import workloads as W


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_cube_meshes.txt")
TABLE1 = [tuple(float(v) for v in ln.split()) for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]


@pytest.mark.parametrize("level,nodes,elems,h", TABLE1)
def test_paper_cube_table1_counts(level, nodes, elems, h):
    X, T = W.paper_cube(int(level))
    s = W.mesh_summary(X, T)
    assert (s["nodes"], s["elements"]) == (int(nodes), int(elems))
    assert s["nodes"] - s["edges"] + s["elements"] == 2
    # h of Table 1 is the longest edge of the triangles of the unit cube
    P = X[T]
    assert np.allclose(np.linalg.norm(P[:, [1, 2, 0]] - P, axis=-1).max(axis=1), h)


def _volume(X, T):
    v0, v1, v2 = X[T[:, 0]], X[T[:, 1]], X[T[:, 2]]
    return np.einsum("ij,ij->i", v0, np.cross(v1, v2)).sum() / 6.0


def test_cube_grid_counts_and_orientation():
    X, T = W.cube_grid(4, 1.0)
    assert X.shape == (98, 3) and T.shape == (192, 3)
    assert abs(_volume(X, T) - 8.0) < 1e-12
    for n in (1, 2, 8):
        X, T = W.cube_grid(n, 0.5)
        assert T.shape[0] == 12 * n * n and abs(_volume(X, T) - 1.0) < 1e-12


@pytest.mark.parametrize("level,nodes,elems", [(3, 642, 1280), (4, 2562, 5120), (5, 10242, 20480)])
def test_icosphere_counts(level, nodes, elems):
    X, T = W.icosphere(level)
    assert X.shape[0] == nodes and T.shape[0] == elems
    assert np.allclose(np.linalg.norm(X, axis=1), 1.0)
    vol = _volume(X, T)
    assert 0.98 * 4 * np.pi / 3 < vol < 4 * np.pi / 3


@pytest.mark.parametrize("L,smin,smax", [(16, 6.446, 25.93), (64, 1.782, 35.20), (128, 0.897, 37.46)])
def test_bdf2_contour(L, smin, smax):
    s = W.bdf2_contour(L, 0.1)
    assert s.shape == (L,)
    assert np.all(s.real > 0)
    assert abs(abs(s).min() - smin) < 1e-3 and abs(abs(s).max() - smax) < 1e-2
    for l in range(1, L):
        assert s[L - l] == np.conj(s[l])
    R = 1e-10 ** (1.0 / (2 * L))
    z = R * np.exp(2j * np.pi * np.arange(L) / L)
    assert np.allclose(s, (3 - 4 * z + z * z) / 0.2, rtol=1e-14, atol=1e-14)


def test_random_rhs_seeded():
    a = W.random_rhs(0, (2, 5))
    b = W.random_rhs(0, (2, 5))
    assert a.dtype == np.complex128 and np.array_equal(a, b)
    assert not np.array_equal(a, W.random_rhs(1, (2, 5)))


@pytest.mark.parametrize("h", [0.1, 0.05])
def test_stator_shell_is_a_closed_oriented_surface(h):
    X, T = W.stator_shell(h)
    v0, v1, v2 = X[T[:, 0]], X[T[:, 1]], X[T[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(v1 - v0, v2 - v0), axis=1)
    assert area.min() > 0.1 * h * h
    # every edge in two triangles, traversed once in each direction (consistent orientation)
    D = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    _, dcount = np.unique(D, axis=0, return_counts=True)
    assert dcount.max() == 1
    E = np.sort(D, axis=1)
    _, ecount = np.unique(E, axis=0, return_counts=True)
    assert np.all(ecount == 2)
    # outward normals: the divergence theorem gives the solid's volume (annulus minus slots),
    # up to the chords of the circles
    vol = np.einsum("ij,ij->i", v0, np.cross(v1, v2)).sum() / 6.0
    exact = 1.5 * (np.pi * (1.0 - 0.49) - 36 * (0.05 / 0.7) * (0.8**2 - 0.7**2) / 2.0)
    assert abs(vol - exact) < 2e-3 * exact
    assert np.all(X[:, 2] >= 0.0) and np.all(X[:, 2] <= 1.5)
    assert np.abs(np.hypot(X[:, 0], X[:, 1])).max() <= 1.0 + 1e-12


def test_stator_shell_full_size():
    # the configuration's ~100k triangles at h = 0.0225
    X, T = W.stator_shell(0.0225)
    assert 90000 < len(T) < 115000
