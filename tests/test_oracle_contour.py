"""Pins of the oracle's quadrature nodes, weights and rational filter.

Paper: eq:cauchy and eq:rational (Section 1), contour options (Section 2.1),
trapezoidal rule (Section 2.3).
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import contour as ct


def test_circle_closed_form():
    # Nodes at the ne-th roots of -1 scaled by r: the trapezoidal filter is
    # exactly 1 / (1 + ((lam - c)/r)^ne)  (geometric-series identity).
    rng = np.random.default_rng(0)
    for ne in (4, 8, 16, 24):
        c, r = 0.1 + 0.1j, 0.25
        z, w = ct.ellipse_nodes(c, r, 1.0, 0.0, ne)
        lam = c + r * 2.0 * (rng.random(500) - 0.5 + 1j * (rng.random(500) - 0.5))
        u = (lam - c) / r
        far = np.abs(np.abs(u) - 1.0) > 1e-3          # stay away from the poles
        exact = 1.0 / (1.0 + u ** ne)
        got = ct.rational(z, w, lam)
        assert np.max(np.abs(got[far] - exact[far]) / np.abs(exact[far])) < 1e-11


def test_rotated_circle_closed_form():
    c, r, phi, ne = -0.3 + 0.2j, 0.7, 0.4, 8
    z, w = ct.ellipse_nodes(c, r, 1.0, phi, ne)
    lam = np.array([c, c + 0.3, c + 0.9j, c - 1.5 + 0.2j])
    u = np.exp(-1j * phi) * (lam - c) / r
    np.testing.assert_allclose(ct.rational(z, w, lam), 1.0 / (1.0 + u ** ne), rtol=1e-12)


def test_nodes_on_ellipse_and_weights_are_derivative():
    c, a, ratio, phi, ne = 2.0 - 1.0j, 3.0, 0.3, 0.9, 12
    b = ratio * a
    z, w = ct.ellipse_nodes(c, a, ratio, phi, ne)
    u = (z - c) * np.exp(-1j * phi)
    np.testing.assert_allclose((u.real / a) ** 2 + (u.imag / b) ** 2, 1.0, rtol=1e-13)
    # w_j = z'(t_j)/(i ne), z'(t) by central finite differences of the
    # parametrisation (not the closed-form derivative).
    t = 2 * math.pi * (np.arange(1, ne + 1) - 0.5) / ne
    zf = lambda s: c + np.exp(1j * phi) * (a * np.cos(s) + 1j * b * np.sin(s))
    d = 1e-6
    dz = (zf(t + d) - zf(t - d)) / (2 * d)
    np.testing.assert_allclose(w, dz / (1j * ne), rtol=1e-8, atol=1e-9)
    # counter-clockwise: argument of (z_j - c) increases with j
    ang = np.unwrap(np.angle(z - c))
    assert np.all(np.diff(ang) > 0)


def test_matches_exact_cauchy_integral():
    # (1/2 pi i) \oint dz/(z - lam) evaluated by adaptive quadrature along the
    # parametrisation; trapezoid converges exponentially to it.
    c, a, ratio, phi = 0.3 - 0.2j, 1.5, 0.4, 0.7
    b = ratio * a
    zf = lambda s: c + np.exp(1j * phi) * (a * np.cos(s) + 1j * b * np.sin(s))
    dzf = lambda s: np.exp(1j * phi) * (-a * np.sin(s) + 1j * b * np.cos(s))
    z, w = ct.ellipse_nodes(c, a, ratio, phi, 256)
    for lam in (0.3 - 0.2j, 0.5 + 0.1j, 2.5 + 0.0j, -1.5 + 0.9j):
        f = lambda s: dzf(s) / (zf(s) - lam) / (2j * math.pi)
        re = integrate.quad(lambda s: f(s).real, 0, 2 * math.pi, limit=400)[0]
        im = integrate.quad(lambda s: f(s).imag, 0, 2 * math.pi, limit=400)[0]
        assert abs(ct.rational(z, w, lam) - (re + 1j * im)) < 1e-10
        assert ct.inside_ellipse(lam, c, a, ratio, phi) == (abs(re - 1.0) < 1e-6)


def test_weights_sum_zero_and_conjugate_symmetry():
    # sum_j w_j = (1/2 pi i) \oint dz = 0 ; real-centred unrotated contour is
    # symmetric under conjugation, so rho_a(conj lam) = conj(rho_a(lam)).
    for ne in (2, 8, 16, 24):
        z, w = ct.ellipse_nodes(437.9, 308.2, 0.3, 0.0, ne)
        assert abs(w.sum()) < 1e-13 * np.abs(w).sum()
        dist = np.abs(z[:, None] - np.conj(z)[None, :]).min(axis=1)
        assert dist.max() < 1e-12 * np.abs(z).max()
        lam = np.array([300 + 20j, 700 - 5j, 10 + 1j])
        np.testing.assert_allclose(ct.rational(z, w, np.conj(lam)), np.conj(ct.rational(z, w, lam)),
                                   rtol=1e-12, atol=1e-15)


def test_filter_tends_to_indicator():
    z, w = ct.ellipse_nodes(0.0, 2.0, 0.5, 0.3, 4096)
    assert abs(ct.rational(z, w, 0.0) - 1.0) < 1e-12
    assert abs(ct.rational(z, w, 0.5 + 0.2j) - 1.0) < 1e-10
    assert abs(ct.rational(z, w, 10.0 + 3.0j)) < 1e-12


def test_inside_and_alpha():
    assert ct.inside_ellipse(0.0, 0.0, 1.0) and not ct.inside_ellipse(1.0, 0.0, 1.0)
    assert not ct.inside_ellipse(np.inf, 0.0, 1.0) and not ct.inside_ellipse(np.nan, 0.0, 1.0)
    # ellipse rotated by 90 degrees: long axis vertical
    assert ct.inside_ellipse(0.9j, 0.0, 1.0, 0.3, math.pi / 2)
    assert not ct.inside_ellipse(0.9, 0.0, 1.0, 0.3, math.pi / 2)
    assert ct.alpha(0.1 + 0.1j, 0.25) == pytest.approx(abs(0.1 + 0.1j) + 0.25)
    assert ct.alpha(3.0, 2.0, 2.0) == pytest.approx(3.0 + 4.0)


SQUARE = np.array([-1 - 1j, 1 - 1j, 1 + 1j, -1 + 1j])
LSHAPE = np.array([0, 2, 2 + 1j, 1 + 1j, 1 + 2j, 2j])          # non-convex, counterclockwise


@pytest.mark.parametrize("verts,per", [(SQUARE, 4), (LSHAPE, 5), (np.exp(2j * np.pi * np.arange(5) / 5), 3)])
def test_polygon_trapezoid_exact_for_linear_integrands(verts, per):
    """The trapezoid rule is exact for z^0 and z^1 on every side, so the
    closed-contour integrals of 1 and z vanish to rounding."""
    z, w = ct.polygon_nodes(verts, per * len(verts))
    assert abs(np.sum(w)) < 1e-15 * len(z)
    assert abs(np.sum(w * z)) < 1e-15 * len(z)


def test_polygon_filter_converges_second_order():
    """rho_a at an interior point tends to 1, at an exterior one to 0, with
    the trapezoid rule's O(h^2) error (the paper's square has 4 intervals per
    side: 16 nodes)."""
    errs = []
    for per in (4, 8, 16, 32):
        z, w = ct.polygon_nodes(SQUARE, 4 * per)
        errs.append(abs(ct.rational(z, w, np.array([0.2 + 0.1j]))[0] - 1.0))
        assert abs(ct.rational(z, w, np.array([2.5 - 0.3j]))[0]) < 0.1
    assert errs[0] < 0.1
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.0 < e0 / e1 < 5.0


def test_polygon_orientation_and_inside():
    """Clockwise vertices give the same rule; the inside test agrees with the
    filter of a fine rule (|rho| > 1/2 inside) on random points away from the
    boundary, for a convex and a non-convex polygon."""
    z1, w1 = ct.polygon_nodes(LSHAPE, 30)
    z2, w2 = ct.polygon_nodes(LSHAPE[::-1], 30)
    lam = np.array([0.5 + 0.5j, 1.5 + 1.5j, 3.0 + 0j])
    np.testing.assert_allclose(ct.rational(z1, w1, lam), ct.rational(z2, w2, lam), atol=1e-14)
    rng = np.random.default_rng(4)
    for verts in (SQUARE, LSHAPE):
        zf, wf = ct.polygon_nodes(verts, 400 * len(verts))
        pts = (rng.uniform(-1.5, 2.5, 400) + 1j * rng.uniform(-1.5, 2.5, 400))
        v = np.asarray(verts)
        # distance to the boundary: keep points at least 0.05 from every side
        def dist(x):
            a, b = v, np.roll(v, -1)
            t = np.clip(((x - a) * np.conj(b - a)).real / np.abs(b - a) ** 2, 0, 1)
            return np.min(np.abs(a + t * (b - a) - x))
        pts = np.array([x for x in pts if dist(x) > 0.05])
        inside = ct.inside_polygon(pts, verts)
        assert np.array_equal(inside, np.abs(ct.rational(zf, wf, pts)) > 0.5)
        assert 0 < inside.sum() < len(pts)
