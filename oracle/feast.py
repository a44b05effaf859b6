"""Non-Hermitian FEAST, step by step (oracle).

Follows the paper's complete algorithm figure (steps 0-5) and Sections 2.2-2.7.
complex128 throughout.  ``A`` is a dense ndarray or a scipy.sparse matrix; ``B``
is None (identity), a dense ndarray or a scipy.sparse matrix.

Readings where the paper is silent:
* V are the right eigenvectors of B_Q and Vh = V^{-H}, so B_Q = V Gamma Vh^H.
* Gamma^{-1/2} is the principal square root; Gamma^{-H/2} = conj(Gamma^{-1/2}).
* Sorting by decreasing |gamma| is stable (ties keep the original order).
* The resize threshold is |gamma_i| < eta max|gamma| with eta = 1e-16.
* The spurious test compares rho_a(lambda_i)^2 from the previous iteration with
  the current [B_Q]_ii (column i of Y is Ritz vector i), from iteration 2 on,
  with mu = 0.1.
* The reduced pencil is solved by QZ (scipy.linalg.eig with both sides); LAPACK's
  right vectors are kept and each left vector is divided by conj(wh_i^H B_U w_i)
  so that Wh^H B_U W = I.  Infinite or NaN Ritz values count as outside.
* Convergence (step 5.c): with m_r Ritz values inside the contour and m_s of
  them flagged spurious, m = m_r - m_s; the run has converged when the m
  smallest residuals among the inside pairs are all below eps.  Step 5.d then
  returns exactly those m pairs (ties in the residual keep the Ritz order).

Parity status: every function below is pinned in tests/test_oracle_feast.py
(residuals on a hand-computed 3 x 3 case and through alpha, the exit test on
synthetic residual/flag histories, the gauge by its three defining
properties, the filter and the whole iteration by prescribed spectra).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import contour as ct
from .linsolve import Counters, DirectFactor, shifted

ETA = 1e-16
MU = 0.1


def _mul(M, X):
    return M @ X


def _bmul(B, X):
    return X if B is None else B @ X


def _bhmul(B, X):
    return X if B is None else B.conj().T @ X


# --------------------------------------------------------------------------
# Step 1: contour integration (eq:qr, eq:ql)
# --------------------------------------------------------------------------
def factorize_nodes(A, B, z, counters=None):
    """One factorization of (z_j B - A) per node (Section 2.4)."""
    return [DirectFactor(shifted(A, B, zj), counters) for zj in z]


def contour_filter(A, B, z, w, Y, Yh, factors=None, counters=None):
    """Q = sum_j w_j (z_j B - A)^{-1} B Y ;  Qh = sum_j conj(w_j) (z_j B - A)^{-H} B^H Yh."""
    if factors is None:
        factors = factorize_nodes(A, B, z, counters)
    R = _bmul(B, Y).astype(np.complex128)
    Rh = _bhmul(B, Yh).astype(np.complex128)
    Q = np.zeros_like(R)
    Qh = np.zeros_like(Rh)
    for wj, F in zip(w, factors):
        Qj = F.solve(R, "N")
        Qhj = F.solve(Rh, "H")
        Q = Q + wj * Qj
        Qh = Qh + np.conj(wj) * Qhj
    return Q, Qh


def count_estimate(A, B, z, w, V):
    """Stochastic estimate of the number of eigenvalues inside the contour
    (the estimator FEAST v3.0 ships, cited in the paper's section on the
    software): the trace of the filter rho_a(B^{-1}A) = sum_j w_j (z_j B - A)^{-1} B,
    whose eigenvalues are rho_a(lambda_i) (about 1 inside, 0 outside),
    estimated with the probe block V (n x p): (1/p) trace(V^H rho_a V).
    Returns a complex number."""
    Q, _ = contour_filter(A, B, z, w, V, V)
    return np.trace(V.conj().T @ Q) / V.shape[1]


# --------------------------------------------------------------------------
# Steps 2-5 for one iteration
# --------------------------------------------------------------------------
def spurious_flags(BQ_diag, rho_prev):
    """Step 2.b: |rho_a^2 - [B_Q]_ii| / |rho_a^2| >= mu  (Section 2.7)."""
    r2 = np.asarray(rho_prev, dtype=np.complex128) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.abs(r2 - BQ_diag) / np.abs(r2)
    return ~(rel < MU)


def resize_biortho(Q, Qh, BQ, eta=ETA):
    """Steps 3.a-3.d: B_Q = V Gamma Vh^H, sort by |gamma| (descending, stable),
    drop |gamma| < eta max|gamma|, U = Q V G^{-1/2}, Uh = Qh Vh conj(G^{-1/2})."""
    gam, V = sla.eig(BQ)
    Vh = np.linalg.inv(V).conj().T
    order = np.argsort(-np.abs(gam), kind="stable")
    gam, V, Vh = gam[order], V[:, order], Vh[:, order]
    amax = np.max(np.abs(gam))
    mt = int(np.count_nonzero(np.abs(gam) >= eta * amax))
    g = gam[:mt]
    s = 1.0 / np.sqrt(g)
    U = Q @ (V[:, :mt] * s[None, :])
    Uh = Qh @ (Vh[:, :mt] * np.conj(s)[None, :])
    return dict(gamma=gam, V=V, Vh=Vh, m0t=mt, U=U, Uh=Uh)


def rayleigh_ritz(A, B, U, Uh):
    """Steps 4.a-4.b: A_U = Uh^H A U, B_U = Uh^H B U, QZ, Wh^H B_U W = I."""
    AU = Uh.conj().T @ _mul(A, U)
    BU = Uh.conj().T @ _bmul(B, U)
    lam, Wh, W = sla.eig(AU, BU, left=True, right=True)
    s = np.einsum("ij,ik,kj->j", Wh.conj(), BU, W)
    Wh = Wh / np.conj(s)[None, :]
    return dict(AU=AU, BU=BU, lam=lam, W=W, Wh=Wh)


def residuals(A, B, Y, Yh, lam, alpha):
    """eq:res with 1-norms, per column."""
    BY = _bmul(B, Y)
    BhYh = _bhmul(B, Yh)
    AY = _mul(A, Y)
    AhYh = A.conj().T @ Yh
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        r1 = np.abs(AY - BY * lam[None, :]).sum(axis=0) / (alpha * np.abs(BY).sum(axis=0))
        r2 = np.abs(AhYh - BhYh * np.conj(lam)[None, :]).sum(axis=0) / (alpha * np.abs(BhYh).sum(axis=0))
    r = np.maximum(r1, r2)
    r[~np.isfinite(r)] = np.inf
    return r


def exit_test(res, inside, m_s, eps):
    """Steps 5.c and 5.d: m = m_r - m_s, where m_r counts the inside Ritz pairs;
    converged when the m smallest residuals among the inside pairs are all
    below eps.  Returns (converged, m, sel) with sel the indices of those m
    pairs (stable order of increasing residual), which step 5.d places in the
    first m columns."""
    res = np.asarray(res, dtype=np.float64)
    idx_in = np.nonzero(np.asarray(inside, dtype=bool))[0]
    m = len(idx_in) - int(m_s)
    if m <= 0:
        return False, m, np.empty(0, dtype=np.int64)
    order = idx_in[np.argsort(res[idx_in], kind="stable")]
    sel = order[:m]
    return bool(np.all(res[sel] < eps)), m, sel


@dataclass
class Contour:
    center: complex
    a: float
    ratio: float = 1.0
    angle: float = 0.0
    ne: int = 8

    def nodes(self):
        return ct.ellipse_nodes(self.center, self.a, self.ratio, self.angle, self.ne)

    def inside(self, lam):
        return ct.inside_ellipse(lam, self.center, self.a, self.ratio, self.angle)

    def alpha(self):
        return ct.alpha(self.center, self.a, self.ratio)


@dataclass
class PolygonContour:
    """A polygon search contour (custom contour): vertices, ne nodes (ne / nv
    trapezoid intervals per side)."""
    verts: np.ndarray
    ne: int = 16

    def nodes(self):
        return ct.polygon_nodes(self.verts, self.ne)

    def inside(self, lam):
        return ct.inside_polygon(lam, self.verts)

    def alpha(self):
        return ct.polygon_alpha(self.verts)


def feast_iteration(A, B, z, w, cont: Contour, Y, Yh, rho_prev=None, factors=None, eps=1e-12,
                    counters=None, it=1):
    """One pass of steps 1-5 from the current subspaces (Y, Yh)."""
    rec = {}
    Q, Qh = contour_filter(A, B, z, w, Y, Yh, factors, counters)                 # step 1
    rec["Q"], rec["Qh"] = Q, Qh
    BQ = Qh.conj().T @ _bmul(B, Q)                                              # step 2.a
    rec["BQ"] = BQ
    m0 = Y.shape[1]
    if rho_prev is not None and it >= 2:                                        # step 2.b
        flags = spurious_flags(np.diag(BQ), rho_prev)
    else:
        flags = np.zeros(m0, dtype=bool)
    rb = resize_biortho(Q, Qh, BQ)                                              # step 3
    rec.update(gamma=rb["gamma"], m0t=rb["m0t"], U=rb["U"], Uh=rb["Uh"])
    rr = rayleigh_ritz(A, B, rb["U"], rb["Uh"])                                 # step 4.a-b
    rec.update(AU=rr["AU"], BU=rr["BU"])
    lam = rr["lam"]
    rho = ct.rational(z, w, lam)                                                # step 4.c
    Ynew = rb["U"] @ rr["W"]                                                    # step 4.d
    Yhnew = rb["Uh"] @ rr["Wh"]
    inside = cont.inside(lam)                                                   # step 5.a
    res = residuals(A, B, Ynew, Yhnew, lam, cont.alpha())                       # step 5.b
    rec.update(lam=lam, rho=rho, Y=Ynew, Yh=Yhnew, inside=inside, res=res, spurious=flags)
    return rec


@dataclass
class FeastResult:
    info: int
    lam: np.ndarray
    X: np.ndarray
    Xh: np.ndarray
    res: np.ndarray
    iters: int
    m0_final: int
    history: list = field(default_factory=list)
    counters: Counters | None = None


def gauge_normalize(X, Xh, B=None):
    """Output gauge: ||x||_2 = 1, largest-modulus entry (lowest index on ties)
    real positive, then xh <- xh / conj(xh^H B x) so that xh^H B x = 1."""
    X = X.copy()
    Xh = Xh.copy()
    for i in range(X.shape[1]):
        x = X[:, i] / np.linalg.norm(X[:, i])
        k = int(np.argmax(np.abs(x)))
        x = x * (np.abs(x[k]) / x[k])
        X[:, i] = x
        s = np.vdot(Xh[:, i], _bmul(B, x[:, None])[:, 0])
        Xh[:, i] = Xh[:, i] / np.conj(s)
    return X, Xh


def feast(A, B, cont: Contour, Y0, Yh0, eps=1e-12, max_iter=50, keep_history=False,
          z=None, w=None):
    """Non-Hermitian FEAST (complete algorithm figure).

    info: 0 converged, 1 no eigenvalue inside after max_iter, 2 max_iter reached,
    3 max_iter reached with every one of the m0 Ritz values inside the contour
    (m0 is then probably not above the number of eigenvalues inside, which the
    method requires: m0 >= m in step 0 of the complete algorithm figure; Section
    2.3 on the slow convergence of too small an m0).
    """
    if z is None:
        z, w = cont.nodes()
    counters = Counters()
    factors = factorize_nodes(A, B, z, counters)     # saved across iterations
    Y, Yh = np.array(Y0, dtype=np.complex128), np.array(Yh0, dtype=np.complex128)
    rho_prev = None
    prev_inside = None
    hist = []
    for it in range(1, max_iter + 1):
        rec = feast_iteration(A, B, z, w, cont, Y, Yh, rho_prev, factors, eps, counters, it)
        # m_s: flagged previous Ritz values that were inside the contour
        if prev_inside is not None:
            m_s = int(np.count_nonzero(rec["spurious"] & prev_inside))
        else:
            m_s = 0
        ok, m, sel = exit_test(rec["res"], rec["inside"], m_s, eps)             # step 5.c
        rec["m_s"], rec["m"] = m_s, m
        if keep_history:
            hist.append(rec)
        else:
            hist.append({k: rec[k] for k in ("lam", "res", "inside", "m0t", "gamma", "spurious")}
                        | {"m_s": m_s, "m": m})
        if ok:
            # step 5.d: the m converged pairs, gauge-normalized, sorted by (Re, Im)
            lam = rec["lam"][sel]
            X, Xh = gauge_normalize(rec["Y"][:, sel], rec["Yh"][:, sel], B)
            order = np.lexsort((lam.imag, lam.real))
            return FeastResult(0, lam[order], X[:, order], Xh[:, order], rec["res"][sel][order],
                               it, rec["m0t"], hist, counters)
        Y, Yh = rec["Y"], rec["Yh"]
        rho_prev = rec["rho"]
        prev_inside = rec["inside"]
    n_inside = int(np.count_nonzero(rec["inside"]))
    info = 1 if n_inside == 0 else (3 if n_inside >= Y0.shape[1] else 2)
    return FeastResult(info, rec["lam"], rec["Y"], rec["Yh"], rec["res"], max_iter, rec["m0t"],
                       hist, counters)
