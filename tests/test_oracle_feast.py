"""Pins of the oracle's contour filter and FEAST iteration.

Every check compares the oracle with something other than itself: matrices with
prescribed spectra (the filter then has the closed form X rho_a(Lambda) Xh^H B Y
of eq:q00 / eq:qhat0), brute-force QZ eigendecompositions, the closed-form
spectrum of the 2D convection-diffusion operator, and the invariants the paper
states (Xh^H B X = I, Uh^H B U = I, B_Q = (Yh^H B X) rho_a^2 (Xh^H B Y)).
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import contour as ct
from oracle import feast as F
from oracle import linsolve as L


def _prescribed(n=60, n_in=6, seed=11):
    return W.dense_prescribed(n=n, n_in=n_in, center=0.1 + 0.1j, radius=0.25, ne=8, m0=10, seed=seed)


def test_filter_prescribed_spectrum_standard():
    p = _prescribed()
    V, lam = p.info["V"], p.info["lam"]
    z, w = ct.ellipse_nodes(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    Q, Qh = F.contour_filter(p.A, None, z, w, p.Y0, p.Yh0)
    rho = ct.rational(z, w, lam)
    Vi = np.linalg.inv(V)
    Qx = V @ (rho[:, None] * (Vi @ p.Y0))                       # eq:q00
    Qhx = Vi.conj().T @ (np.conj(rho)[:, None] * (V.conj().T @ p.Yh0))   # eq:qhat0
    assert np.linalg.norm(Q - Qx) / np.linalg.norm(Qx) < 1e-11
    assert np.linalg.norm(Qh - Qhx) / np.linalg.norm(Qhx) < 1e-11
    # the same through the sparse (SuperLU) path on the dense pattern
    n = p.n
    As = L.csr_matrix({"n": n, "rowptr": np.arange(0, n * n + 1, n), "colind": np.tile(np.arange(n), n),
                       "val": p.A.ravel()})
    Q2, Qh2 = F.contour_filter(As, None, z, w, p.Y0, p.Yh0)
    assert np.linalg.norm(Q2 - Qx) / np.linalg.norm(Qx) < 1e-11
    assert np.linalg.norm(Qh2 - Qhx) / np.linalg.norm(Qhx) < 1e-11


def test_filter_prescribed_spectrum_generalized():
    # B^{-1} A = V Lambda V^{-1} with a general B: Xh^H = V^{-1} B^{-1}
    rng = np.random.default_rng(4)
    n = 50
    V = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = 0.9 * (rng.random(n) - 0.5 + 1j * (rng.random(n) - 0.5)) * 2
    B = np.eye(n) + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    A = B @ V @ np.diag(lam) @ np.linalg.inv(V)
    z, w = ct.ellipse_nodes(0.05 - 0.1j, 0.4, 0.6, 0.3, 12)
    Y = W.subspace(n, 7, 1)
    Yh = W.subspace(n, 7, 2)
    Q, Qh = F.contour_filter(A, B, z, w, Y, Yh)
    rho = ct.rational(z, w, lam)
    Vi = np.linalg.inv(V)
    Bi = np.linalg.inv(B)
    Qx = V @ (rho[:, None] * (Vi @ Y))
    Xh_H = Vi @ Bi
    Qhx = (Yh.conj().T @ B @ V @ np.diag(rho) @ Xh_H).conj().T
    assert np.linalg.norm(Q - Qx) / np.linalg.norm(Qx) < 1e-10
    assert np.linalg.norm(Qh - Qhx) / np.linalg.norm(Qhx) < 1e-10
    # B_Q closed form (eq:bdiag1)
    BQ = Qh.conj().T @ B @ Q
    BQx = Yh.conj().T @ B @ V @ np.diag(rho ** 2) @ Xh_H @ B @ Y
    assert np.linalg.norm(BQ - BQx) / np.linalg.norm(BQx) < 1e-10


def test_per_node_backward_error():
    p = _prescribed(n=80)
    z, w = ct.ellipse_nodes(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    for zj in z:
        Fj = L.DirectFactor(L.shifted(p.A, None, zj))
        M = zj * np.eye(p.n) - p.A
        X = Fj.solve(p.Y0, "N")
        be = np.linalg.norm(p.Y0 - M @ X) / (np.linalg.norm(M) * np.linalg.norm(X) + np.linalg.norm(p.Y0))
        assert be < 1e-14
        Xh = Fj.solve(p.Yh0, "H")
        be = np.linalg.norm(p.Yh0 - M.conj().T @ Xh) / (np.linalg.norm(M) * np.linalg.norm(Xh) + np.linalg.norm(p.Yh0))
        assert be < 1e-14


def test_biorthonormalization_and_resize():
    p = _prescribed()
    z, w = ct.ellipse_nodes(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    Q, Qh = F.contour_filter(p.A, None, z, w, p.Y0, p.Yh0)
    BQ = Qh.conj().T @ Q
    rb = F.resize_biortho(Q, Qh, BQ)
    m = rb["m0t"]
    assert m == p.m0
    assert np.max(np.abs(rb["Uh"].conj().T @ rb["U"] - np.eye(m))) < 1e-10
    assert np.all(np.diff(np.abs(rb["gamma"])) <= 0)
    # B_Q = V Gamma Vh^H
    np.testing.assert_allclose(rb["V"] @ np.diag(rb["gamma"]) @ rb["Vh"].conj().T, BQ, atol=1e-12)
    # duplicated start columns -> rank-deficient B_Q -> subspace shrinks
    Y = p.Y0.copy(); Yh = p.Yh0.copy()
    Y[:, 7:] = Y[:, :3]
    Yh[:, 7:] = Yh[:, :3]
    Q, Qh = F.contour_filter(p.A, None, z, w, Y, Yh)
    rb = F.resize_biortho(Q, Qh, Qh.conj().T @ Q)
    assert rb["m0t"] < p.m0
    # the rank-7 well-resolved part stays bi-orthonormal; directions kept at the
    # eta = 1e-16 edge are rounding noise and are not checked
    k = 7
    assert np.max(np.abs(rb["Uh"][:, :k].conj().T @ rb["U"][:, :k] - np.eye(k))) < 1e-6


def test_spurious_criterion():
    rho_prev = np.array([1.0, 0.9, 0.5, 1e-3 + 1e-3j])
    bq = np.array([1.0, 0.81 * 1.05, 0.25 * 2.0, ((1e-3 + 1e-3j) ** 2) * 1.2])
    flags = F.spurious_flags(bq, rho_prev)
    assert flags.tolist() == [False, False, True, True]
    # around the threshold mu = 0.1 (flagged when the relative gap is >= mu)
    assert F.spurious_flags(np.array([1.1 + 0j, 1.0999 + 0j]), np.array([1.0 + 0j, 1.0 + 0j])).tolist() == [True, False]


def test_rayleigh_ritz_normalization():
    rng = np.random.default_rng(8)
    m = 9
    AU = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    BU = np.eye(m) + 0.05 * (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    U = np.eye(m, dtype=complex)
    rr = F.rayleigh_ritz(AU, BU, U, U)
    W_, Wh, lam = rr["W"], rr["Wh"], rr["lam"]
    np.testing.assert_allclose(Wh.conj().T @ BU @ W_, np.eye(m), atol=1e-12)
    np.testing.assert_allclose(AU @ W_, BU @ W_ * lam[None, :], atol=1e-12)
    np.testing.assert_allclose(AU.conj().T @ Wh, BU.conj().T @ Wh * np.conj(lam)[None, :], atol=1e-12)
    ref = sla.eigvals(np.linalg.solve(BU, AU))
    np.testing.assert_allclose(np.sort_complex(lam), np.sort_complex(ref), atol=1e-12)


def test_feast_dense_prescribed_against_truth():
    p = W.dense_prescribed(n=150, n_in=8, center=0.1 + 0.1j, radius=0.25, ne=8, m0=16, seed=21)
    cont = F.Contour(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    r = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=60)
    assert r.info == 0
    lam_true = p.info["lam"][: p.info["n_in"]]
    lam_true = lam_true[np.lexsort((lam_true.imag, lam_true.real))]
    assert len(r.lam) == len(lam_true)
    assert np.max(np.abs(r.lam - lam_true)) < 1e-10 * cont.alpha()
    assert np.max(np.abs(r.Xh.conj().T @ r.X - np.eye(len(r.lam)))) < 1e-10
    # brute force with both sides (LAPACK QZ on the full matrix)
    ev = sla.eigvals(p.A)
    ev = ev[cont.inside(ev)]
    ev = ev[np.lexsort((ev.imag, ev.real))]
    assert np.max(np.abs(ev - r.lam)) < 1e-10 * cont.alpha()
    # eigen-residual ||Ax - lam x||_1 / (||A||_1 ||x||_1), right and left
    nA = np.abs(p.A).sum(axis=0).max()
    rr = np.abs(p.A @ r.X - r.X * r.lam).sum(axis=0) / (nA * np.abs(r.X).sum(axis=0))
    rl = np.abs(p.A.conj().T @ r.Xh - r.Xh * np.conj(r.lam)).sum(axis=0) / (nA * np.abs(r.Xh).sum(axis=0))
    assert rr.max() < 1e-10 and rl.max() < 1e-10
    # one factorization per node, two solves per node per iteration
    assert r.counters.factorizations == 8 and r.counters.solves == 2 * 8 * r.iters


def test_feast_generalized_brute_force():
    rng = np.random.default_rng(31)
    n = 90
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    B = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    ev = sla.eigvals(A, B)
    c = 0.2 - 0.1j
    d = np.sort(np.abs(ev - c))
    r = 0.5 * (d[5] + d[6])                     # exactly 6 inside, radius in the gap
    cont = F.Contour(c, r, 1.0, 0.0, 16)
    res = F.feast(A, B, cont, W.subspace(n, 12, 5), W.subspace(n, 12, 6), eps=1e-12, max_iter=40)
    assert res.info == 0 and len(res.lam) == 6
    evi = ev[cont.inside(ev)]
    evi = evi[np.lexsort((evi.imag, evi.real))]
    assert np.max(np.abs(evi - res.lam)) < 1e-10 * cont.alpha()
    np.testing.assert_allclose(res.Xh.conj().T @ B @ res.X, np.eye(6), atol=1e-10)
    np.testing.assert_allclose(A @ res.X, B @ res.X * res.lam, atol=1e-10)
    np.testing.assert_allclose(A.conj().T @ res.Xh, B.conj().T @ res.Xh * np.conj(res.lam), atol=1e-10)


def test_feast_convdiff_closed_form():
    # closed-form spectrum of T(bx) (x) I + I (x) T(by)
    p = W.convdiff2d(N=24, m_in=10, m0=20)
    A = L.csr_matrix(p.A)
    cont = F.Contour(p.contour.center, p.contour.a, p.contour.ratio, 0.0, 16)
    res = F.feast(A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=30)
    assert res.info == 0 and len(res.lam) == 10
    ref = p.info["lam_sorted"][:10]
    assert np.max(np.abs(np.sort(res.lam.real) - ref)) < 1e-10 * cont.alpha()
    assert np.max(np.abs(res.lam.imag)) < 1e-10 * cont.alpha()
    np.testing.assert_allclose(res.Xh.conj().T @ res.X, np.eye(10), atol=1e-10)


def test_hermitian_special_case_left_equals_right():
    rng = np.random.default_rng(41)
    n = 70
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.linspace(-3, 3, n) + 0.01 * rng.standard_normal(n)
    A = Qm @ np.diag(lam) @ Qm.conj().T
    A = 0.5 * (A + A.conj().T)
    ls = np.sort(lam)
    c = 0.5 * (ls[30] + ls[35])
    r = 0.5 * ((ls[36] - ls[29])) - 0.5 * min(ls[36] - ls[35], ls[30] - ls[29])
    cont = F.Contour(complex(c), r, 1.0, 0.0, 16)
    res = F.feast(A, None, cont, W.subspace(n, 12, 1), W.subspace(n, 12, 2), eps=1e-12, max_iter=40)
    assert res.info == 0 and len(res.lam) == 6
    np.testing.assert_allclose(res.Xh, res.X, atol=1e-9)          # Xh = X
    assert np.max(np.abs(res.lam.imag)) < 1e-12


def test_complex_symmetric_left_is_conjugate_right():
    rng = np.random.default_rng(42)
    n = 70
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = (G + G.T) / np.sqrt(8 * n)
    ev = sla.eigvals(A)
    c = ev[np.argmin(np.abs(ev))]
    d = np.sort(np.abs(ev - c))
    cont = F.Contour(c, 0.5 * (d[4] + d[5]), 1.0, 0.0, 16)
    res = F.feast(A, None, cont, W.subspace(n, 10, 3), W.subspace(n, 10, 4), eps=1e-12, max_iter=40)
    assert res.info == 0 and len(res.lam) == 5
    for i in range(5):
        x, xh = res.X[:, i], res.Xh[:, i]
        cosang = abs(np.vdot(np.conj(x), xh)) / (np.linalg.norm(x) * np.linalg.norm(xh))
        assert cosang > 1 - 1e-10                                    # Xh = conj(X) up to scale


def test_convergence_rate_prediction():
    # Section 2.3: residuals fall by |rho_a(lam_{m0+1}) / rho_a(lam_i)| per iteration.
    rng = np.random.default_rng(3)
    n, n_in, m0 = 200, 6, 8
    u_in = np.sqrt(rng.uniform(0.04, 0.36, n_in)) * np.exp(2j * np.pi * rng.random(n_in))
    r_out = np.sqrt(rng.uniform(1.25 ** 2, 4.0 ** 2, n - n_in))
    u_out = r_out * np.exp(2j * np.pi * rng.random(n - n_in))
    lam = 0.5 * np.concatenate([u_in, u_out])
    V = W.subspace(n, n, 77)
    V /= np.linalg.norm(V, axis=0, keepdims=True)
    A = np.linalg.solve(V.T, (V * lam[None, :]).T).T
    cont = F.Contour(0.0, 0.5, 1.0, 0.0, 8)
    z, w = cont.nodes()
    rho = np.abs(ct.rational(z, w, lam))
    srt = np.sort(rho)[::-1]
    rate = srt[m0] / np.min(rho[:n_in])                     # slowest wanted pair
    assert 0.02 < rate < 0.5
    res = F.feast(A, None, cont, W.subspace(n, m0, 1), W.subspace(n, m0, 2), eps=1e-14, max_iter=30)
    worst = []
    for h in res.history:
        r = h["res"][h["inside"]]
        worst.append(np.sort(r)[n_in - 1] if len(r) >= n_in else np.nan)
    worst = np.array(worst)
    idx = np.nonzero(np.isfinite(worst) & (worst > 1e-12))[0]
    idx = idx[idx >= 2]
    assert len(idx) >= 3
    obs = np.exp(np.polyfit(idx, np.log(worst[idx]), 1)[0])
    assert abs(np.log(obs / rate)) < np.log(1.6), (obs, rate)


def test_complex_symmetric_left_filter_is_conjugate():
    """Complex symmetric A (A = A^T): the left eigenvectors are the conjugates
    of the right ones, and with Yh = conj(Y) the left filter equals the
    conjugate of the right filter (the reduced-workload case of the paper
    that lets the left solves be skipped).  Checked with the oracle's own left
    solves, against scipy's left eigenvectors."""
    A = W.schrodinger2d_csr(8, L=8.0, nwells=3, seed=1)
    Asp = L.csr_matrix(A)
    assert abs(Asp - Asp.T).max() == 0
    Ad = W.csr_to_dense(A)
    lam, vl, vr = sla.eig(Ad, left=True, right=True)
    for i in range(0, A["n"], 7):
        x, xh = vr[:, i], vl[:, i]
        assert abs(np.vdot(np.conj(x), xh)) / (np.linalg.norm(x) * np.linalg.norm(xh)) > 1 - 1e-10
    c = lam[np.argsort(np.abs(lam - np.median(lam)))[0]]
    r = 0.5 * np.sort(np.abs(lam - c))[5:7].sum()
    z, w = ct.ellipse_nodes(c, r, 1.0, 0.0, 8)
    Y = W.subspace(A["n"], 8, 3)
    Q, Qh = F.contour_filter(Asp, None, z, w, Y, np.conj(Y))
    assert np.linalg.norm(Qh - np.conj(Q)) <= 1e-12 * np.linalg.norm(Q)
    # a general left block breaks the identity (the check has teeth)
    Q2, Qh2 = F.contour_filter(Asp, None, z, w, Y, W.subspace(A["n"], 8, 4))
    assert np.linalg.norm(Qh2 - np.conj(Q2)) > 1e-3 * np.linalg.norm(Q2)


def _real_3d_problem(N=6):
    """Real non-symmetric 3D convection-diffusion-reaction operator and an
    ellipse centred on the real axis around its lowest eigenvalues, among
    which are complex-conjugate pairs."""
    v = W.smooth_field3d(N, 4000)
    A = W.convdiff3d_csr(N, v)
    lam = np.linalg.eigvals(W.csr_to_dense(A))
    cont, inside = W.lowest_contour(lam, 10)
    return A, lam, cont, inside


def test_filter_of_conjugation_closed_blocks_is_conjugation_closed():
    """Real A and nodes symmetric about the real axis (each lower node the
    conjugate of an upper one, with the conjugate weight): for real blocks the
    filter is real, and when column k of the block is the conjugate of column
    i, column k of the filter is the conjugate of column i, on both sides
    (the reduced-workload case of the paper, real non-symmetric with a
    contour symmetric about the real axis: a lower node's solutions are the
    conjugates of its partner's, so n_e solves give both subspaces).  The
    oracle solves every node directly."""
    A, lam, cont, inside = _real_3d_problem()
    assert np.count_nonzero(np.abs(lam.imag) > 1e-6) > 0
    z, w = ct.ellipse_nodes(cont.center, cont.a, cont.ratio, 0.0, 16)
    assert np.abs(z[:, None] - np.conj(z)[None, :]).min(axis=1).max() < 1e-12 * cont.a
    Asp = L.csr_matrix(A)
    n = A["n"]
    Yr, Yhr = W.subspace(n, 6, 7).real, W.subspace(n, 6, 8).real
    Q, Qh = F.contour_filter(Asp, None, z, w, Yr, Yhr)
    assert np.abs(Q.imag).max() <= 1e-13 * np.abs(Q).max()
    assert np.abs(Qh.imag).max() <= 1e-13 * np.abs(Qh).max()
    # columns (0, 3) and (1, 4) conjugate pairs, 2 and 5 real
    Y, Yh = W.subspace(n, 6, 9), W.subspace(n, 6, 10)
    for Z in (Y, Yh):
        Z[:, 3], Z[:, 4] = np.conj(Z[:, 0]), np.conj(Z[:, 1])
        Z[:, 2], Z[:, 5] = Z[:, 2].real, Z[:, 5].real
    Q, Qh = F.contour_filter(Asp, None, z, w, Y, Yh)
    for M in (Q, Qh):
        sc = np.abs(M).max()
        assert np.abs(M[:, 3] - np.conj(M[:, 0])).max() <= 1e-13 * sc
        assert np.abs(M[:, 4] - np.conj(M[:, 1])).max() <= 1e-13 * sc
        assert np.abs(M[:, [2, 5]].imag).max() <= 1e-13 * sc
    # a contour off the real axis breaks the identity (the check has teeth)
    z2, w2 = ct.ellipse_nodes(cont.center + 0.2j * cont.a, cont.a, cont.ratio, 0.0, 16)
    Q2, _ = F.contour_filter(Asp, None, z2, w2, Yr, Yhr)
    assert np.abs(Q2.imag).max() > 1e-3 * np.abs(Q2).max()


def test_feast_from_real_start_keeps_conjugate_ritz_pairs():
    """From real start blocks every FEAST iterate of a real pencil under a
    contour symmetric about the real axis spans a subspace closed under
    conjugation, so at every iteration the m0 Ritz values (inside and
    outside) come in conjugate pairs or are real, and the converged pairs are
    the operator's eigenvalues inside the ellipse."""
    A, lam, cont, inside = _real_3d_problem()
    n = A["n"]
    c = F.Contour(cont.center, cont.a, cont.ratio, 0.0, 16)
    res = F.feast(L.csr_matrix(A), None, c, W.subspace(n, 16, 3).real, W.subspace(n, 16, 4).real, eps=1e-12,
                  max_iter=30, keep_history=True)
    assert res.info == 0 and len(res.lam) == inside
    alpha = c.alpha()
    truth = lam[c.inside(lam)]
    assert np.max(np.abs(res.lam[:, None] - truth[None, :]).min(axis=1)) < 1e-10 * alpha
    for rec in res.history:
        rl = rec["lam"]
        fin = rl[np.isfinite(rl)]
        gap = np.abs(fin[:, None] - np.conj(fin)[None, :]).min(axis=1)
        assert gap.max() <= 1e-8 * alpha, gap.max()
    # a complex start block has no such pairing in its first iterate
    res2 = F.feast(L.csr_matrix(A), None, c, W.subspace(n, 16, 3), W.subspace(n, 16, 4), eps=1e-12, max_iter=1,
                   keep_history=True)
    rl = res2.history[0]["lam"]
    assert np.abs(rl[:, None] - np.conj(rl)[None, :]).min(axis=1).max() > 1e-6 * alpha


def test_count_estimate_exact_trace_and_probes():
    """The eigenvalue-count estimator: with the identity as probe block (p = n)
    it is exactly trace(rho_a) / n, and for the trapezoid circle rho_a has the
    closed form 1 / (1 + ((lambda - c) / r)^Ne), summed over the prescribed
    eigenvalues; with 400 Rademacher probes it lands near that trace (the
    estimator's spread here is well below 1)."""
    p = W.dense_prescribed(n=160, n_in=9, center=0.1 + 0.1j, radius=0.25, m0=12, seed=3)
    c, r, ne = p.contour.center, p.contour.a, 16
    z, w = ct.ellipse_nodes(c, r, 1.0, 0.0, ne)
    lam = p.info["lam"]
    exact = np.sum(1.0 / (1.0 + ((lam - c) / r) ** ne))
    assert 6.0 < exact.real < 12.0          # 9 inside, partly weighted near the circle
    est = F.count_estimate(p.A, None, z, w, np.eye(p.n, dtype=np.complex128)) * p.n
    assert abs(est - exact) < 1e-9 * p.n
    rng = np.random.default_rng(11)
    V = rng.choice([-1.0, 1.0], size=(p.n, 400)).astype(np.complex128)
    est_r = F.count_estimate(p.A, None, z, w, V)
    assert abs(est_r - exact) < 1.5


# --------------------------------------------------------------------------
# eq:res, alpha, the output gauge and the exit test of steps 5.c / 5.d
# --------------------------------------------------------------------------
def test_residuals_hand_computed_3x3():
    """eq:res on a 3 x 3 generalized pencil worked out by hand.  A has one
    complex entry so that A vs A^H and lambda vs conj(lambda) give different
    numbers; B = diag(1, 2, 1); alpha = 2 (circle centre 1, radius 1).
    Column 0: y = yh = (1, 1, 0), lambda = 1 + i:
      A y - lambda B y = (1, 1 - 2i, 0)          -> (1 + sqrt 5) / (2 * 3)
      A^H yh - conj(lambda) B^H yh = (1 + i, 1 + i, 0) -> 2 sqrt 2 / (2 * 3)
    Column 1: y = (0, 0, 1), yh = (1, 1, 0), lambda = 1:
      right residual 0, left (1, 1 - i, 0)        -> (1 + sqrt 2) / (2 * 3)
    The max of the two sides is eq:res (both sides must be converged)."""
    A = np.array([[2, 1j, 0], [0, 3, 0], [0, 0, 1]], dtype=np.complex128)
    B = np.diag([1.0, 2.0, 1.0]).astype(np.complex128)
    Y = np.array([[1, 0], [1, 0], [0, 1]], dtype=np.complex128)
    Yh = np.array([[1, 1], [1, 1], [0, 0]], dtype=np.complex128)
    lam = np.array([1 + 1j, 1.0 + 0j])
    alpha = ct.alpha(1.0, 1.0, 1.0)
    assert alpha == 2.0
    res = F.residuals(A, B, Y, Yh, lam, alpha)
    r0 = max((1 + np.sqrt(5)) / 6, 2 * np.sqrt(2) / 6)
    r1 = (1 + np.sqrt(2)) / 6
    np.testing.assert_allclose(res, [r0, r1], rtol=1e-14)
    # alpha divides: another alpha scales eq:res by its inverse
    np.testing.assert_allclose(F.residuals(A, B, Y, Yh, lam, 7.0), [r0 * 2 / 7, r1 * 2 / 7], rtol=1e-14)


def test_alpha_circle_and_ellipse():
    """alpha of eq:res is |lambda_mid| + r for a circle; for an ellipse the
    larger semi-axis takes the place of r (either one may be the larger)."""
    assert ct.alpha(3 + 4j, 1.0, 1.0) == 6.0
    assert ct.alpha(3 + 4j, 1.0, 2.0) == 7.0        # vertical semi-axis 2
    assert ct.alpha(3 + 4j, 2.0, 0.5) == 7.0        # horizontal semi-axis 2
    assert ct.alpha(-2.0, 0.5, 0.3) == 2.5


def test_polygon_alpha_square_and_rectangle():
    """Polygon alpha = |g| + max_k |v_k - g|, g the mean vertex: for the
    square of half-side s centred at g the farthest vertex is at s sqrt 2."""
    g, s = 0.5 + 0.3j, 0.13
    sq = g + s * np.array([-1 - 1j, 1 - 1j, 1 + 1j, -1 + 1j])
    assert abs(ct.polygon_alpha(sq) - (abs(g) + s * np.sqrt(2))) < 1e-15
    assert abs(ct.polygon_alpha(sq[::-1]) - (abs(g) + s * np.sqrt(2))) < 1e-15
    rect = np.array([0, 4, 4 + 2j, 2j])               # g = 2 + i, corners at sqrt 5
    assert abs(ct.polygon_alpha(rect) - 2 * np.sqrt(5)) < 1e-15


def test_gauge_normalize_defining_properties():
    """Output gauge of step 5.d: unit 2-norm, the largest-modulus entry (lowest
    index on ties) real positive, xh^H B x = 1, each vector a multiple of the
    input one."""
    rng = np.random.default_rng(5)
    n, m = 12, 4
    X = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    Xh = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    X[3, 2] = X[7, 2] = 9.0 * np.exp(0.7j)          # a tie: index 3 wins
    B = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    Xn, Xhn = F.gauge_normalize(X, Xh, B)
    for i in range(m):
        x, xh = Xn[:, i], Xhn[:, i]
        assert abs(np.linalg.norm(x) - 1) < 1e-14
        k = int(np.argmax(np.abs(x)))
        assert abs(x[k].imag) < 1e-15 and x[k].real > 0
        assert abs(np.vdot(xh, B @ x) - 1) < 1e-13
        # the same directions
        assert abs(abs(np.vdot(X[:, i], x)) - np.linalg.norm(X[:, i])) < 1e-12
        assert abs(abs(np.vdot(Xh[:, i], xh)) - np.linalg.norm(Xh[:, i]) * np.linalg.norm(xh)) < 1e-10
    assert int(np.argmax(np.abs(Xn[:, 2]))) == 3 and abs(Xn[3, 2].imag) < 1e-15


def test_exit_test_synthetic_histories():
    """Steps 5.c / 5.d on synthetic residuals and flags: m = m_r - m_s, the m
    smallest inside residuals decide, exactly those m pairs are returned."""
    inside = np.array([True, True, True, False, True])
    res = np.array([1e-13, 1e-5, 1e-14, 1e-20, 3e-13])
    # no spurious flag: the m = 4 inside residuals include 1e-5 -> not converged
    ok, m, sel = F.exit_test(res, inside, 0, 1e-12)
    assert (ok, m) == (False, 4) and sel.tolist() == [2, 0, 4, 1]
    # one flagged pair: the m = 3 smallest (1e-14, 1e-13, 3e-13) decide
    ok, m, sel = F.exit_test(res, inside, 1, 1e-12)
    assert (ok, m) == (True, 3) and sel.tolist() == [2, 0, 4]
    # an outside pair never counts, however small its residual
    assert 3 not in sel
    # a tighter eps fails on the third of them
    assert F.exit_test(res, inside, 1, 2e-13)[0] is False
    # m_s >= m_r: nothing to converge
    ok, m, sel = F.exit_test(res, inside, 4, 1.0)
    assert ok is False and m == 0 and len(sel) == 0
    # no pair inside
    assert F.exit_test(res, np.zeros(5, bool), 0, 1.0)[:2] == (False, 0)
    # ties keep the Ritz order
    ok, m, sel = F.exit_test(np.array([1e-14, 1e-14, 1e-14]), np.ones(3, bool), 1, 1e-12)
    assert ok and sel.tolist() == [0, 1]


def test_feast_returns_exactly_the_exit_pairs():
    """The whole loop wires step 5.c to 5.d: the pairs returned are exactly the
    m of the last history record, i.e. the m smallest inside residuals, all
    below eps, and m = m_r - m_s."""
    p = W.dense_prescribed(n=120, n_in=7, center=0.1 + 0.1j, radius=0.25, ne=8, m0=14, seed=23)
    cont = F.Contour(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    r = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=60)
    assert r.info == 0
    h = r.history[-1]
    m_r = int(np.count_nonzero(h["inside"]))
    assert h["m"] == m_r - h["m_s"] == len(r.lam)
    want = np.sort(h["res"][h["inside"]])[: h["m"]]
    np.testing.assert_array_equal(np.sort(r.res), want)
    assert np.all(r.res < 1e-12)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_feast_degenerate_contours(seed):
    """Degenerate cases of the method.  A contour around no eigenvalue: no
    pair is ever returned as converged (the Ritz values that wander inside
    are filter noise, flagged spurious or above eps), and the status says
    whether any Ritz value was inside at the end (1: none, 2: some).  m0
    below the number of eigenvalues inside (10 inside, m0 = 6; the method
    needs m0 >= m): no convergence, and at the iteration limit every Ritz
    value is inside, status 3."""
    cont = F.Contour(0.1 + 0.1j, 0.25, 1.0, 0.0, 8)
    p = W.dense_prescribed(n=120, n_in=0, center=0.1 + 0.1j, radius=0.25, ne=8, m0=8, seed=seed)
    assert not np.any(np.abs(p.info["lam"] - (0.1 + 0.1j)) < 0.25)
    r = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=8)
    n_in = int(np.count_nonzero(r.history[-1]["inside"]))
    assert r.info == (1 if n_in == 0 else 2)
    assert all(h["m"] <= 0 or not np.all(np.sort(h["res"][h["inside"]])[: h["m"]] < 1e-12) for h in r.history)
    p = W.dense_prescribed(n=120, n_in=10, center=0.1 + 0.1j, radius=0.25, ne=8, m0=6, seed=seed)
    r = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=8)
    assert r.info == 3 and int(np.count_nonzero(r.history[-1]["inside"])) == 6
