"""C-ABI checks that need no GPU: the library loads, exports every function include/bem.h
declares, and validates its inputs on a host-only context (device = -1)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2607_15292_amd import binding as B
from paper_2607_15292_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bem.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bem_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert n in B._SIGS, "binding lacks " + n
    assert B.version().startswith("libbem")


def _host_ctx():
    return B.Context(device=-1)


def test_mesh_validation():
    c = _host_ctx()
    X, T = W.cube_grid(2, 1.0)
    assert c.set_mesh(X, T) == 0
    bad = T.copy()
    bad[3, 1] = X.shape[0]
    with pytest.raises(B.BemError) as e:
        c.set_mesh(X, bad)
    assert e.value.code == -2
    deg = T.copy()
    deg[0] = [0, 0, 1]
    with pytest.raises(B.BemError) as e:
        c.set_mesh(X, deg)
    assert e.value.code == -2
    with pytest.raises(B.BemError):
        c.set_mesh(X, T[:0])


def test_material_and_frequency_validation():
    c = _host_ctx()
    assert c.set_material(1.0, 1.0, 0.5) == 0
    assert c.set_material(1.0, 1.0, 0.9) == 1  # negative bulk modulus warning
    for args in [(0.0, 1.0, 0.5), (1.0, 0.5, 0.5), (1.0, 1.0, -0.1), (1.0, float("nan"), 0.5)]:
        with pytest.raises(B.BemError) as e:
            c.set_material(*args)
        assert e.value.code == -3
    assert c.set_frequencies(W.bdf2_contour(16)) == 0
    assert c.freq_pairs() == 14  # 7 conjugate pairs + 2 real points
    for s in ([1.0 + 0j, -0.5 + 1j], [0.0 + 2j], [float("inf")]):
        with pytest.raises(B.BemError) as e:
            c.set_frequencies(s)
        assert e.value.code == -4


def test_gpu_calls_refused_on_host_context():
    c = _host_ctx()
    X, T = W.cube_grid(2, 1.0)
    c.set_mesh(X, T)
    c.set_material(1.0, 1.0, 0.5)
    c.set_frequencies([6.0])
    with pytest.raises(B.BemError) as e:
        c.entries(0, [0], [1], [0])
    assert e.value.code == -8
    with pytest.raises(B.BemError) as e:
        c.assemble_dense(0)
    assert e.value.code == -8


def test_quadrature_option_validation():
    c = _host_ctx()
    assert c.set_quadrature(True, 1.5, 3.0, 8, 8) == 0
    with pytest.raises(B.BemError):
        c.set_quadrature(True, 1.5, 3.0, 0, 8)
    with pytest.raises(B.BemError):
        c.set_quadrature(True, 3.0, 1.5, 8, 8)


def test_binding_checks_buffer_shapes():
    # the binding refuses buffers whose shape or dtype differ from what the library will read
    a = np.zeros((2, 3, 12), dtype=np.complex128)
    assert B._ptr(a, (2, 3, 12))[1] == 0
    with pytest.raises(ValueError):
        B._ptr(a, (2, 4, 12))
    with pytest.raises(ValueError):
        B._ptr(a.astype(np.complex64), (2, 3, 12))
    with pytest.raises(ValueError):
        B._ptr(a[:, :, ::2], (2, 3, 6))
