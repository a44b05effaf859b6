"""Quadrature nodes/weights and the rational filter (oracle).

Paper: Section 1 (eq:cauchy, eq:rational), Section 2.1 (circle/ellipse defined
by a complex midpoint, a radius, an axis ratio and a rotation angle) and
Section 2.3 (the trapezoidal rule is the recommended rule for the
non-Hermitian problem).

Readings (the paper prints no formula for the nodes):
* nodes at t_j = 2 pi (j - 1/2)/ne, j = 1..ne, counter-clockwise;
* ellipse z(t) = c + e^{i phi} (a cos t + i b sin t), b = ratio * a;
* weights w_j = z'(t_j) / (i ne), so that sum_j w_j/(z_j - lam) is the
  trapezoidal approximation of (1/(2 pi i)) \\oint dz/(z - lam).

Pins: tests/test_oracle_contour.py (closed form of the circle filter,
finite-difference derivative of the parametrisation, an adaptive-quadrature
evaluation of the exact Cauchy integral, conjugate symmetry, sum of weights).
"""
from __future__ import annotations

import numpy as np


def ellipse_nodes(center, a, ratio=1.0, angle=0.0, ne=8):
    """Return (z, w), complex128 arrays of length ne."""
    j = np.arange(1, ne + 1, dtype=np.float64)
    t = 2.0 * np.pi * (j - 0.5) / ne
    b = ratio * a
    rot = np.exp(1j * angle)
    z = complex(center) + rot * (a * np.cos(t) + 1j * b * np.sin(t))
    # z'(t) = rot * (-a sin t + i b cos t);  w = z'(t) / (i ne)
    dz = rot * (-a * np.sin(t) + 1j * b * np.cos(t))
    w = dz / (1j * ne)
    return z.astype(np.complex128), w.astype(np.complex128)


def rational(z, w, lam):
    """rho_a(lam) = sum_j w_j / (z_j - lam)   (eq:rational)."""
    lam = np.asarray(lam, dtype=np.complex128)
    out = np.zeros(lam.shape, dtype=np.complex128)
    for zj, wj in zip(z, w):
        out = out + wj / (zj - lam)
    return out


def inside_ellipse(lam, center, a, ratio=1.0, angle=0.0):
    """Strict inside test of the ellipse (step 5.a); non-finite values are outside."""
    lam = np.asarray(lam, dtype=np.complex128)
    b = ratio * a
    with np.errstate(invalid="ignore", over="ignore"):
        u = (lam - complex(center)) * np.exp(-1j * angle)
        q = (u.real / a) ** 2 + (u.imag / b) ** 2
        ok = np.isfinite(lam.real) & np.isfinite(lam.imag) & (q < 1.0)
    return ok


def alpha(center, a, ratio=1.0):
    """Scale of eq:res: |lambda_mid| + r for a circle; |c| + max semi-axis here."""
    return abs(complex(center)) + max(a, ratio * a)


# --------------------------------------------------------------------------
# Polygon contours (the paper's custom contours, e.g. the squares of its
# multi-contour experiment with 4 trapezoidal intervals per side)
# --------------------------------------------------------------------------
def _ccw(verts):
    """Vertices in counterclockwise order (shoelace signed area)."""
    v = np.asarray(verts, dtype=np.complex128).reshape(-1)
    area2 = np.sum(v.real * np.roll(v, -1).imag - np.roll(v, -1).real * v.imag)
    return v if area2 >= 0 else v[::-1].copy()


def polygon_nodes(verts, ne):
    """Composite trapezoid rule for (1/2 pi i) times the closed integral of
    f(z) dz along the polygon, ne / nv intervals per side, nodes at the
    interval ends.  On side k from
    v_k to v_{k+1} with step h_k = (v_{k+1} - v_k) / p the interval ends are
    v_k + q h_k (q = 0 .. p-1; q = p is the next side's first node); an
    interior end gets h_k / (2 pi i), a vertex (h_{k-1} + h_k) / (2 (2 pi i))."""
    v = _ccw(verts)
    nv = len(v)
    assert ne % nv == 0 and ne >= nv
    per = ne // nv
    z, w = [], []
    for k in range(nv):
        h = (v[(k + 1) % nv] - v[k]) / per
        hprev = (v[k] - v[k - 1]) / per
        for q in range(per):
            z.append(v[k] + q * h)
            w.append(((hprev + h) / 2 if q == 0 else h) / (2j * np.pi))
    return np.array(z, dtype=np.complex128), np.array(w, dtype=np.complex128)


def inside_polygon(lam, verts):
    """Strict inside test by the winding number of the closed polygon around
    lam (sum of the signed angles its sides subtend); non-finite: outside."""
    lam = np.atleast_1d(np.asarray(lam, dtype=np.complex128))
    v = np.asarray(verts, dtype=np.complex128).reshape(-1)
    out = np.zeros(lam.shape, dtype=bool)
    for i, x in enumerate(lam):
        if not (np.isfinite(x.real) and np.isfinite(x.imag)):
            continue
        a = v - x
        b = np.roll(v, -1) - x
        wind = np.sum(np.angle(b / a)) / (2 * np.pi)
        out[i] = abs(round(wind)) == 1
    return out


def polygon_alpha(verts):
    """Scale of eq:res for a polygon: |g| + max_k |v_k - g|, g the mean vertex."""
    v = np.asarray(verts, dtype=np.complex128).reshape(-1)
    g = v.mean()
    return abs(g) + np.max(np.abs(v - g))
