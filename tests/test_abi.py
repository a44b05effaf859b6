"""The C ABI: the shared library loads, exports every entry point that
include/feasthip.h declares, and its host-only routines (contour nodes and the
rational filter, eq:rational) agree with the oracle.  No GPU needed."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1506_04463_amd as fh
from oracle import contour as ct

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "feasthip.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fh_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(fh.LIB_PATH), "build the library first"
    L = C.CDLL(fh.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    L = fh.lib()
    for n in _declared():
        assert getattr(L, n).argtypes is not None or getattr(L, n).restype is None, n


@pytest.mark.parametrize("center,a,ratio,angle,ne", [(0.1 + 0.1j, 0.25, 1.0, 0.0, 8),
                                                     (437.9, 308.2, 0.3, 0.0, 16),
                                                     (-1 - 2j, 3.0, 0.4, 0.7, 24),
                                                     (0.0, 1.0, 1.0, 0.0, 1)])
def test_contour_nodes_match_oracle(center, a, ratio, angle, ne):
    z, w = fh.contour_nodes(center, a, ratio, angle, ne)
    zo, wo = ct.ellipse_nodes(center, a, ratio, angle, ne)
    np.testing.assert_allclose(z, zo, rtol=1e-14, atol=1e-14 * abs(a))
    np.testing.assert_allclose(w, wo, rtol=1e-14, atol=1e-14 * abs(a))
    lam = np.array([center, center + 0.5 * a, center + 2 * a + 1j * a])
    np.testing.assert_allclose(fh.rational(z, w, lam), ct.rational(zo, wo, lam), rtol=1e-12, atol=1e-15)


def test_bad_arguments_are_rejected():
    L = fh.lib()
    c = fh.fh_contour(0.0, 0.0, -1.0, 1.0, 0.0, 8)
    z = np.zeros(8, np.complex128)
    assert L.fh_contour_nodes(C.byref(c), z.ctypes.data_as(C.POINTER(C.c_double)),
                              z.ctypes.data_as(C.POINTER(C.c_double))) < 0
    assert L.fh_contour_nodes(None, None, None) == -1
    assert L.fh_rational(0, None, None, 0, None, None) == -1
    assert L.fh_filter(None, None, 8, None, None, 4, None, None, None, None, None, None) == -1
    assert L.fh_feast(None, None, None, None, None, None, None, None, None, None, None) == -1
    o = fh.fh_opts()
    L.fh_default_opts(C.byref(o))
    assert o.max_iter > 0 and o.eps > 0 and o.restart == 30


def test_net_and_solve_arguments_are_rejected():
    L = fh.lib()
    assert L.fh_shifted_solve(None, None, 1, None, None, 1, None, None, None, None) == -1
    assert L.fh_ilu0_apply_c64(None, None, 0.0, 0.0, 0, 1, None, None) == -1
    assert L.fh_count_estimate(None, None, 8, None, None, 4, None, None, None, None) == -1
    assert L.fh_net_create(None, 1, 4, 4, 0, None, 1.0, 1.0, 0, None) == -1
    assert L.fh_net_destroy(None) == -1
    assert L.fh_net_param_count(None) == -1
    assert L.fh_net_get_params(None, None, None) == -1
    assert L.fh_net_set_params(None, None, None) == -1
    assert L.fh_net_forward(None, None, 1, 1, None, None, None, None) == -1
    assert L.fh_net_train_step(None, None, None, 1, 1, None, None, None, None, 1e-3, 1, None, None) == -1
    assert L.fh_problem_set_net(None, None) == -1


@pytest.mark.parametrize("verts,ne", [(np.array([-1 - 1j, 1 - 1j, 1 + 1j, -1 + 1j]), 16),
                                      (np.array([0, 2, 2 + 1j, 1 + 1j, 1 + 2j, 2j]), 18)])
def test_polygon_nodes_match_oracle(verts, ne):
    """Polygon contours (both orientations): the library's nodes and weights
    equal the oracle's; a node count that is not a multiple of the vertex
    count is rejected."""
    for v in (verts, verts[::-1]):
        z, w = fh.contour_nodes(0.0, 1.0, 1.0, 0.0, ne, polygon=v)
        zo, wo = ct.polygon_nodes(v, ne)
        np.testing.assert_allclose(z, zo, atol=1e-15)
        np.testing.assert_allclose(w, wo, atol=1e-16)
    with pytest.raises(fh.FeastError):
        fh.contour_nodes(0.0, 1.0, 1.0, 0.0, ne + 1, polygon=verts)
