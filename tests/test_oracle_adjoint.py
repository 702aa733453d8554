"""Pins of the oracle's adjoint of the single layer (oracle.Problem.adjoint_v): the gradient
of Re S, S = sum_{r, l} w[r, l]^T V(s_l) x[r, l], with respect to the node coordinates and
rho, c_p, c_s against central differences of the oracle's own dense operator (the plain
definition of the derivative of the discrete operator), translation invariance, and the value
against the dense product; with the near rule on, on a jittered mesh whose pairs keep their
classes under the difference steps."""
import numpy as np
import pytest

import oracle
from paper_2607_15292_amd import workloads as W


def _setup(level=1, L=3, nrhs=2):
    X, T = W.icosphere(level)
    s = W.bdf2_contour(8, 0.1)[[0, 2, 5]][:L]
    w = W.random_rhs(40, (nrhs, L, 3 * len(T)))
    x = W.random_rhs(41, (nrhs, L, 3 * len(T)))
    return X, T, s, w, x


def _S(X, T, s, w, x, rho=1.0, cp=1.0, cs=0.5):
    D = oracle.Problem(X, T, s, rho, cp, cs, near_on=False).dense(oracle.OP_V)
    return complex(np.einsum("rli,lij,rlj->", w, D, x))


def test_value_is_the_dense_bilinear_form():
    X, T, s, w, x = _setup()
    val, _, _ = oracle.Problem(X, T, s, near_on=False).adjoint_v(w, x)
    ref = _S(X, T, s, w, x)
    assert abs(val - ref) <= 1e-12 * abs(ref)


def test_node_gradient_matches_central_differences():
    X, T, s, w, x = _setup()
    _, g, _ = oracle.Problem(X, T, s, near_on=False).adjoint_v(w, x)
    rng = np.random.default_rng(5)
    h = 1e-5
    for _ in range(10):
        D = rng.standard_normal(X.shape)
        fd = (_S(X + h * D, T, s, w, x).real - _S(X - h * D, T, s, w, x).real) / (2 * h)
        an = float(np.sum(g * D))
        assert abs(an - fd) <= 1e-6 * np.linalg.norm(g) * np.linalg.norm(D), (an, fd)


def test_material_gradient_matches_central_differences():
    X, T, s, w, x = _setup()
    _, _, gm = oracle.Problem(X, T, s, 1.3, 1.1, 0.6, near_on=False).adjoint_v(w, x)
    base = dict(rho=1.3, cp=1.1, cs=0.6)
    for k, name in enumerate(("rho", "cp", "cs")):
        h = 1e-6 * base[name]
        p, m = dict(base), dict(base)
        p[name] += h
        m[name] -= h
        fd = (_S(X, T, s, w, x, **p).real - _S(X, T, s, w, x, **m).real) / (2 * h)
        assert abs(gm[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gm).max()), (name, gm[k], fd)


def test_translation_invariance():
    # S does not change when every node moves by the same vector
    X, T, s, w, x = _setup()
    _, g, _ = oracle.Problem(X, T, s, near_on=False).adjoint_v(w, x)
    assert np.abs(g.sum(axis=0)).max() <= 1e-7 * np.abs(g).max()  # central differences of the self rule


def _near_setup():
    # jittered mesh so that no pair sits on a class boundary of the near rule
    X, T, s, w, x = _setup()
    X = X + 0.02 * np.random.default_rng(9).standard_normal(X.shape)
    return X, T, s, w, x


def _class_margin(X, T, r1=1.5, r2=3.0):
    # smallest |d^2 / lmax_j^2 - r^2| over the pairs: how far the mesh is from a class switch
    P = X[T]
    c = P.mean(axis=1)
    e = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 1], P[:, 0] - P[:, 2]], axis=1)
    l2 = (e ** 2).sum(-1).max(-1)
    d2 = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1) / l2[None, :]
    return min(np.abs(d2 - r1 * r1).min(), np.abs(d2 - r2 * r2).min())


def _S_near(X, T, s, w, x, rho=1.0, cp=1.0, cs=0.5):
    D = oracle.Problem(X, T, s, rho, cp, cs, near_on=True).dense(oracle.OP_V)
    return complex(np.einsum("rli,lij,rlj->", w, D, x))


def test_near_rule_value_is_the_dense_bilinear_form():
    X, T, s, w, x = _near_setup()
    val, _, _ = oracle.Problem(X, T, s, near_on=True).adjoint_v(w, x)
    ref = _S_near(X, T, s, w, x)
    assert abs(val - ref) <= 1e-12 * abs(ref)
    # the near rule changes the form: the level-1 sphere has pairs of both near levels
    assert abs(val - _S(X, T, s, w, x)) > 1e-6 * abs(ref)


def test_near_rule_node_gradient_matches_central_differences():
    X, T, s, w, x = _near_setup()
    h = 1e-6
    assert _class_margin(X, T) > 1e2 * h
    _, g, _ = oracle.Problem(X, T, s, near_on=True).adjoint_v(w, x)
    _, g0, _ = oracle.Problem(X, T, s, near_on=False).adjoint_v(w, x)
    assert np.abs(g - g0).max() > 1e-6 * np.abs(g).max()
    rng = np.random.default_rng(6)
    for _ in range(8):
        D = rng.standard_normal(X.shape)
        fd = (_S_near(X + h * D, T, s, w, x).real - _S_near(X - h * D, T, s, w, x).real) / (2 * h)
        an = float(np.sum(g * D))
        assert abs(an - fd) <= 1e-6 * np.linalg.norm(g) * np.linalg.norm(D), (an, fd)


def test_near_rule_material_gradient_matches_central_differences():
    X, T, s, w, x = _near_setup()
    _, _, gm = oracle.Problem(X, T, s, 1.3, 1.1, 0.6, near_on=True).adjoint_v(w, x)
    base = dict(rho=1.3, cp=1.1, cs=0.6)
    for k, name in enumerate(("rho", "cp", "cs")):
        h = 1e-6 * base[name]
        p, m = dict(base), dict(base)
        p[name] += h
        m[name] -= h
        fd = (_S_near(X, T, s, w, x, **p).real - _S_near(X, T, s, w, x, **m).real) / (2 * h)
        assert abs(gm[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gm).max()), (name, gm[k], fd)


def test_near_rule_translation_invariance():
    X, T, s, w, x = _near_setup()
    _, g, _ = oracle.Problem(X, T, s, near_on=True).adjoint_v(w, x)
    assert np.abs(g.sum(axis=0)).max() <= 1e-7 * np.abs(g).max()  # central differences of the self rule


@pytest.mark.parametrize("near_on", [False, True])
def test_self_derivative_of_the_integral_against_the_rule(near_on):
    # the self pairs differentiated as integrals (polar rule of grad U (lambda_a - 1/3), area
    # term) against central differences of the polar rule itself: the same derivative up to the
    # rule's quadrature error (nodes), and identical for the material (the rule's points do not
    # move with the speeds)
    X, T, s, w, x = _setup()
    P = oracle.Problem(X, T, s, 1.3, 1.1, 0.6, near_on=near_on)
    v0, g0, m0 = P.adjoint_v(w, x)
    v1, g1, m1 = P.adjoint_v(w, x, fd_h=1e-5)
    assert abs(v0 - v1) <= 1e-13 * abs(v1)
    assert np.abs(g0 - g1).max() <= 3e-6 * np.abs(g1).max()
    assert np.abs(m0 - m1).max() <= 1e-9 * np.abs(m1).max()


# ---------------------------------------------------------------- double layer

def _SK(X, T, s, w, x, op=oracle.OP_K, rho=1.3, cp=1.1, cs=0.6, near_on=False):
    D = oracle.Problem(X, T, s, rho, cp, cs, near_on=near_on).dense(op)
    return complex(np.einsum("rli,lij,rlj->", w, D, x))


@pytest.mark.parametrize("op", [oracle.OP_K, oracle.OP_HK])
def test_double_layer_value_and_node_gradient(op):
    X, T, s, w, x = _setup()
    P = oracle.Problem(X, T, s, 1.3, 1.1, 0.6, near_on=False)
    val, g, gm = P.adjoint_k(w, x, op=op, fd_h=1e-5)  # self pairs: derivative of the rule
    assert abs(val - _SK(X, T, s, w, x, op)) <= 1e-12 * abs(val)
    assert gm[0] == 0.0  # T does not depend on rho
    rng = np.random.default_rng(7)
    h = 1e-5
    for _ in range(6):
        D = rng.standard_normal(X.shape)
        fd = (_SK(X + h * D, T, s, w, x, op).real - _SK(X - h * D, T, s, w, x, op).real) / (2 * h)
        assert abs(float(np.sum(g * D)) - fd) <= 1e-7 * np.linalg.norm(g) * np.linalg.norm(D)


def test_double_layer_material_gradient_and_translation():
    X, T, s, w, x = _setup()
    _, g, gm = oracle.Problem(X, T, s, 1.3, 1.1, 0.6, near_on=False).adjoint_k(w, x, fd_h=1e-5)
    for k, (cp, cs) in ((1, (1.1, 0.6)), (2, (1.1, 0.6))):
        h = 1e-6
        if k == 1:
            fd = (_SK(X, T, s, w, x, cp=cp + h * cp).real - _SK(X, T, s, w, x, cp=cp - h * cp).real) / (2 * h * cp)
        else:
            fd = (_SK(X, T, s, w, x, cs=cs + h * cs).real - _SK(X, T, s, w, x, cs=cs - h * cs).real) / (2 * h * cs)
        assert abs(gm[k] - fd) <= 1e-6 * abs(fd)
    # a rigid translation changes nothing
    assert np.abs(g.sum(axis=0)).max() <= 1e-7 * np.abs(g).max()  # central differences of the self rule


@pytest.mark.slow
def test_double_layer_near_rule_gradient():
    X, T, s, w, x = _setup()
    # jittered so that the difference steps switch no pair class of the near rule
    X = X + 0.01 * np.random.default_rng(3).standard_normal(X.shape)
    _, g, _ = oracle.Problem(X, T, s, 1.3, 1.1, 0.6, near_on=True).adjoint_k(w, x, fd_h=1e-5)
    rng = np.random.default_rng(8)
    h = 1e-6
    for _ in range(4):
        D = rng.standard_normal(X.shape)
        fd = (_SK(X + h * D, T, s, w, x, near_on=True).real - _SK(X - h * D, T, s, w, x, near_on=True).real) / (2 * h)
        assert abs(float(np.sum(g * D)) - fd) <= 1e-6 * np.linalg.norm(g) * np.linalg.norm(D)


@pytest.mark.parametrize("near_on", [False, True])
@pytest.mark.parametrize("op", [oracle.OP_K, oracle.OP_HK])
def test_double_layer_self_derivative_of_the_integral(near_on, op):
    # the self pairs differentiated as principal-value integrals (polar rule of d_r T (lambda_a -
    # 1/3) and of T with the normal's derivative, leading parts from the static kernel) against
    # central differences of the polar rule itself: the same derivative up to the rule's
    # quadrature error; the material derivative identical (the rule's points do not move with
    # the speeds); and each element's vertex derivatives sum to zero (sum_a (lambda_a - 1/3) = 0,
    # the normal and the area do not change under a translation)
    X, T, s, w, x = _setup()
    P = oracle.Problem(X, T, s, 1.3, 1.1, 0.6, near_on=near_on)
    v0, g0, m0 = P.adjoint_k(w, x, op=op)
    v1, g1, m1 = P.adjoint_k(w, x, op=op, fd_h=1e-5)
    assert abs(v0 - v1) <= 1e-13 * abs(v1)
    assert np.abs(g0 - g1).max() <= 5e-6 * np.abs(g1).max()
    assert np.abs(m0 - m1).max() <= 1e-8 * np.abs(m1).max()
    assert np.abs(g0.sum(axis=0)).max() <= 1e-10 * np.abs(g0).max()


def test_double_layer_self_derivative_converges_with_the_rule():
    # with a finer polar rule (16 x 16 points per sub-triangle) the quadrature error between the
    # derivative of the integral and the derivative of the rule falls from about 1e-6 to the
    # level of the difference quotients
    X, T, s, w, x = _setup(L=2, nrhs=1)
    P = oracle.Problem(X, T, s, 1.3, 1.1, 0.6, near_on=False, self_nt=16, self_nr=16)
    _, g0, _ = P.adjoint_k(w, x)
    _, g1, _ = P.adjoint_k(w, x, fd_h=1e-5)
    assert np.abs(g0 - g1).max() <= 2e-7 * np.abs(g1).max()
