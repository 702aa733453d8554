"""Pins of the oracle's quadrature rules.

* 7-point rule: exact for all monomials of degree <= 5 on a triangle, not for degree 6.
* Gauss-Legendre n points: exact to degree 2n - 1, not 2n.
* Self element, single layer, static limit: trace and normal-normal component equal the
  closed form of int_triangle 1/r dA from the centroid (sum over edges of
  d_e ln((R_b + s_b) / (R_a + s_a))).
* Self element, dynamic: the 8 x 8 polar rule converges to a 24 x 24 rule.
* Near-singular rule: the subdivided rule on an edge-adjacent pair agrees with brute force
  (7-point rule on 4^5 sub-triangles, summed in numpy from point evaluations).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2607_15292_amd import workloads


def test_tri7_degree5_exact():
    B, w = oracle.tri7()
    # reference triangle (0,0), (1,0), (0,1): point = B1 * (1,0) + B2 * (0,1)
    x, y = B[:, 1], B[:, 2]
    area = 0.5
    worst5, worst6 = 0.0, 0.0
    for a in range(7):
        for b in range(7 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = area * np.sum(w * x**a * y**b)
            err = abs(got - exact) / exact
            if a + b <= 5:
                worst5 = max(worst5, err)
            else:
                worst6 = max(worst6, err)
    assert worst5 < 1e-14
    assert worst6 > 1e-6  # degree 6 is not integrated exactly
    assert abs(w.sum() - 1.0) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 5, 8, 12])
def test_gauss_legendre_exactness(n):
    x, w = oracle.gauss_legendre(n)
    for k in range(2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x**k) - exact) < 1e-13
    k = 2 * n
    assert abs(np.sum(w * x**k) - 2.0 / (k + 1)) > 1e-8


def _inv_r_closed_form(tri, x):
    total = 0.0
    for a in range(3):
        va, vb = tri[a], tri[(a + 1) % 3]
        t = (vb - va) / np.linalg.norm(vb - va)
        foot = va + np.dot(x - va, t) * t
        d = np.linalg.norm(foot - x)
        sa, sb = np.dot(va - foot, t), np.dot(vb - foot, t)
        Ra, Rb = np.linalg.norm(va - x), np.linalg.norm(vb - x)
        total += d * math.log((Rb + sb) / (Ra + sa))
    return total


@pytest.mark.parametrize("tri", [
    [[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]],
    [[0.1, -0.2, 0.3], [0.9, 0.1, 0.2], [0.3, 0.8, -0.4]],
    [[0.0, 0.0, 0.0], [1.5, 0.0, 0.0], [0.2, 0.7, 0.0]],  # skewed
])
def test_self_single_layer_static_closed_form(tri):
    nodes = np.array(tri, dtype=np.float64)
    tris = np.array([[0, 1, 2]], dtype=np.int32)
    c1, c2, rho = 1.0, 0.5, 1.0
    x = nodes.mean(axis=0)
    J = _inv_r_closed_form(nodes, x)
    n = np.cross(nodes[1] - nodes[0], nodes[2] - nodes[0])
    n /= np.linalg.norm(n)
    tr_exact = (2 / c1**2 + 4 / c2**2) / (8 * np.pi * rho) * J
    nn_exact = (1 / c1**2 + 1 / c2**2) / (8 * np.pi * rho) * J
    # the 8 x 8 rule of the build resolves sec(theta) to ~1e-5; 24 x 24 to ~1e-10
    for nq, tol in ((8, 5e-5), (24, 1e-9)):
        P = oracle.Problem(nodes, tris, [1e-13], rho, c1, c2, self_nt=nq, self_nr=nq)
        E = P.entries(oracle.OP_V, 0, 0, 0)[0]
        assert abs(np.trace(E) - tr_exact) <= tol * abs(tr_exact)
        assert abs(n @ E @ n - nn_exact) <= tol * abs(nn_exact)


@pytest.mark.parametrize("s", [6.45, 13.8 - 9.7j, 35.2])
@pytest.mark.parametrize("op", [oracle.OP_V, oracle.OP_K])
def test_self_rule_converges(s, op):
    nodes, tris = workloads.cube_grid(4, 1.0)
    P8 = oracle.Problem(nodes, tris, [s], self_nt=8, self_nr=8)
    P24 = oracle.Problem(nodes, tris, [s], self_nt=24, self_nr=24)
    for e in (0, 17, 101):
        a = P8.entries(op, e, e, 0)[0]
        b = P24.entries(op, e, e, 0)[0]
        scale = np.abs(b).max() if op == oracle.OP_V else np.abs(P24.entries(oracle.OP_V, e, e, 0)[0]).max()
        assert np.abs(a - b).max() <= 5e-5 * scale


def _brute_force_entry(which, x, tri, n, s, levels=5):
    B, w = oracle.tri7()
    tris = [np.array(tri)]
    for _ in range(levels):
        nxt = []
        for p in tris:
            m01, m12, m20 = 0.5 * (p[0] + p[1]), 0.5 * (p[1] + p[2]), 0.5 * (p[2] + p[0])
            nxt += [np.array([p[0], m01, m20]), np.array([m01, p[1], m12]),
                    np.array([m20, m12, p[2]]), np.array([m01, m12, m20])]
        tris = nxt
    acc = np.zeros((3, 3), dtype=np.complex128)
    for p in tris:
        A = 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0]))
        for q in range(7):
            y = B[q] @ p
            acc += w[q] * A * oracle.kernel_point(which, x, y, n, s)
    return acc


@pytest.mark.slow
@pytest.mark.parametrize("op", [oracle.OP_V, oracle.OP_K])
def test_near_rule_matches_brute_force(op):
    nodes, tris = workloads.cube_grid(4, 1.0)
    s = 6.45 + 2.0j
    P = oracle.Problem(nodes, tris, [s], near_on=True)
    Poff = oracle.Problem(nodes, tris, [s], near_on=False)
    i, j = 0, 1  # the two halves of one square: edge-adjacent
    x = nodes[tris[i]].mean(axis=0)
    tri = nodes[tris[j]]
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    ref = _brute_force_entry(0 if op == oracle.OP_V else 1, x, tri, n, s)
    near = P.entries(op, i, j, 0)[0]
    plain = Poff.entries(op, i, j, 0)[0]
    scale = np.abs(ref).max()
    err_near = np.abs(near - ref).max() / scale
    err_plain = np.abs(plain - ref).max() / scale
    assert err_near < 2e-3
    assert err_near < 0.1 * err_plain
