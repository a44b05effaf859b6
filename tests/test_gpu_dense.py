"""GPU parity of the dense path (LU filter, Rayleigh-Ritz steps, full FEAST)
against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import contour as ct
from oracle import feast as F

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fh = pytest.importorskip("paper_1506_04463_amd")


@pytest.fixture(scope="module")
def handle():
    return fh.Handle(0)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _kappa_max(A, B, z):
    n = A.shape[0]
    Bm = np.eye(n) if B is None else B
    return max(np.linalg.cond(zj * Bm - A) for zj in z)


@pytest.mark.parametrize("n,m0,ne,gen", [(150, 16, 8, False), (97, 13, 5, False), (33, 7, 3, True),
                                         (64, 64, 8, True), (1, 1, 4, False), (200, 40, 16, True)])
def test_filter_dense_parity(handle, n, m0, ne, gen):
    rng = np.random.default_rng(n + m0)
    if n == 1:
        A = np.array([[0.05 + 0.02j]])
    else:
        A = W.dense_prescribed(n=n, n_in=min(6, n // 2), m0=m0, ne=ne, seed=n).A
    B = None
    if gen:
        B = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    z, w = ct.ellipse_nodes(0.1 + 0.1j, 0.25, 0.7, 0.3, ne)
    Y = W.subspace(n, m0, 1)
    Yh = W.subspace(n, m0, 2)
    Qo, Qho = F.contour_filter(A, B, z, w, Y, Yh)
    prob = fh.Problem(handle, _cuda(A), None if B is None else _cuda(B))
    Q, Qh, rep = fh.contour_filter(prob, z, w, _cuda(Y), _cuda(Yh))
    Q, Qh = Q.cpu().numpy(), Qh.cpu().numpy()
    tol = 100 * _kappa_max(A, B, z) * np.finfo(float).eps
    assert np.linalg.norm(Q - Qo) / np.linalg.norm(Qo) < tol
    assert np.linalg.norm(Qh - Qho) / np.linalg.norm(Qho) < tol
    assert rep["n_factor"] == ne and rep["n_solve"] == 2 * ne


def test_filter_reuses_saved_factorizations(handle):
    p = W.dense_prescribed(n=80, n_in=5, m0=8, seed=3)
    z, w = ct.ellipse_nodes(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    prob = fh.Problem(handle, _cuda(p.A))
    _, _, r1 = fh.contour_filter(prob, z, w, _cuda(p.Y0), _cuda(p.Yh0))
    Q, Qh, r2 = fh.contour_filter(prob, z, w, _cuda(p.Y0), _cuda(p.Yh0))
    assert r1["n_factor"] == 8 and r2["n_factor"] == 0
    Qo, Qho = F.contour_filter(p.A, None, z, w, p.Y0, p.Yh0)
    assert np.linalg.norm(Q.cpu().numpy() - Qo) / np.linalg.norm(Qo) < 1e-10


def test_reduced_steps_match_oracle(handle):
    p = W.dense_prescribed(n=120, n_in=6, m0=12, seed=5)
    z, w = ct.ellipse_nodes(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    Qo, Qho = F.contour_filter(p.A, None, z, w, p.Y0, p.Yh0)
    prob = fh.Problem(handle, _cuda(p.A))
    BQ = fh.reduced_matrix(prob, _cuda(Qho), _cuda(Qo)).cpu().numpy()
    BQo = Qho.conj().T @ Qo
    np.testing.assert_allclose(BQ, BQo, rtol=0, atol=1e-13 * np.abs(BQo).max())
    # steps 3.a-3.c
    gam, S, Sh, mt = fh.biortho_factors(handle, _cuda(BQo))
    rb = F.resize_biortho(Qo, Qho, BQo)
    assert mt == rb["m0t"]
    gam = gam.cpu().numpy()
    np.testing.assert_allclose(np.abs(gam), np.abs(rb["gamma"]), rtol=1e-9)
    np.testing.assert_allclose(gam, rb["gamma"], rtol=1e-8)
    S, Sh = S.cpu().numpy()[:, :mt], Sh.cpu().numpy()[:, :mt]
    np.testing.assert_allclose(Sh.conj().T @ BQo @ S, np.eye(mt), atol=1e-10)
    # U columns span the same directions as the oracle's (gauge: column phase)
    U = Qo @ S
    for k in range(mt):
        u, uo = U[:, k], rb["U"][:, k]
        c = abs(np.vdot(u, uo)) / (np.linalg.norm(u) * np.linalg.norm(uo))
        assert c > 1 - 1e-9
    # step 4.b on the oracle's U
    rr = F.rayleigh_ritz(p.A, None, rb["U"], rb["Uh"])
    lam, Wm, Whm = fh.reduced_eig(handle, _cuda(rr["AU"]), _cuda(rr["BU"]))
    lam, Wm, Whm = lam.cpu().numpy(), Wm.cpu().numpy(), Whm.cpu().numpy()
    AU, BU = rr["AU"], rr["BU"]
    np.testing.assert_allclose(np.sort_complex(lam), np.sort_complex(rr["lam"]), atol=1e-11)
    np.testing.assert_allclose(AU @ Wm, BU @ Wm * lam[None, :], atol=1e-10)
    np.testing.assert_allclose(AU.conj().T @ Whm, BU.conj().T @ Whm * np.conj(lam)[None, :], atol=1e-10)
    np.testing.assert_allclose(Whm.conj().T @ BU @ Wm, np.eye(len(lam)), atol=1e-10)


@pytest.mark.parametrize("m", [1, 2, 5, 36, 64, 100])
def test_reduced_eig_random(handle, m):
    rng = np.random.default_rng(m)
    AU = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    BU = np.eye(m) + 0.05 * (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
    lam, Wm, Whm = [t.cpu().numpy() for t in fh.reduced_eig(handle, _cuda(AU), _cuda(BU))]
    ref = sla.eigvals(AU, BU)
    d = np.abs(lam[:, None] - ref[None, :]).min(axis=1)
    assert d.max() < 1e-10 * np.abs(ref).max()
    assert np.max(np.abs(AU @ Wm - BU @ Wm * lam[None, :])) < 1e-10 * np.abs(AU).max()
    np.testing.assert_allclose(Whm.conj().T @ BU @ Wm, np.eye(m), atol=1e-9)


def _gauge(X, Xh):
    return F.gauge_normalize(X, Xh)


def _compare_feast(p, A, B, out, ref, cont):
    assert out["info"] == 0 and ref.info == 0
    assert len(out["lam"]) == len(ref.lam)
    alpha = cont.alpha()
    assert np.max(np.abs(out["lam"] - ref.lam)) < 1e-10 * alpha
    X, Xh = out["X"].cpu().numpy(), out["Xh"].cpu().numpy()
    Bm = np.eye(A.shape[0]) if B is None else B
    m = len(out["lam"])
    assert np.max(np.abs(Xh.conj().T @ Bm @ X - np.eye(m))) < 1e-10
    nA = np.abs(A).sum(axis=0).max()
    lam = out["lam"]
    rr = np.abs(A @ X - Bm @ X * lam).sum(axis=0) / (nA * np.abs(X).sum(axis=0))
    rl = np.abs(A.conj().T @ Xh - Bm.conj().T @ Xh * np.conj(lam)).sum(axis=0) / (nA * np.abs(Xh).sum(axis=0))
    assert rr.max() <= 1e-10 and rl.max() <= 1e-10
    assert out["res"].max() < 1e-12 * 10
    # vectors: gauge-normalized right vectors agree with the oracle's
    Xg, _ = _gauge(X, Xh)
    for k in range(m):
        assert abs(abs(np.vdot(Xg[:, k], ref.X[:, k])) - 1) < 1e-8


def test_feast_dense_first_config(handle):
    """Dense n=400, 24 eigenvalues in the circle (0.1+0.1i, 0.25), Ne=8, m0=36."""
    p = W.dense_prescribed()
    cont = F.Contour(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    ref = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=60)
    prob = fh.Problem(handle, _cuda(p.A))
    out = fh.feast(prob, p.contour.center, p.contour.a, 1.0, 0.0, 8, _cuda(p.Y0), _cuda(p.Yh0),
                   fh.default_opts(36, eps=1e-12, max_iter=60))
    _compare_feast(p, p.A, None, out, ref, cont)
    assert len(out["lam"]) == 24
    lam_true = p.info["lam"][:24]
    lam_true = lam_true[np.lexsort((lam_true.imag, lam_true.real))]
    assert np.max(np.abs(out["lam"] - lam_true)) < 1e-10 * cont.alpha()
    assert out["report"]["n_factor"] == 8


def test_feast_dense_generalized(handle):
    rng = np.random.default_rng(31)
    n = 90
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    B = np.eye(n) + 0.1 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
    ev = sla.eigvals(A, B)
    c = 0.2 - 0.1j
    d = np.sort(np.abs(ev - c))
    r = 0.5 * (d[5] + d[6])
    cont = F.Contour(c, r, 1.0, 0.0, 16)
    Y0, Yh0 = W.subspace(n, 12, 5), W.subspace(n, 12, 6)
    ref = F.feast(A, B, cont, Y0, Yh0, eps=1e-12, max_iter=40)
    prob = fh.Problem(handle, _cuda(A), _cuda(B))
    out = fh.feast(prob, c, r, 1.0, 0.0, 16, _cuda(Y0), _cuda(Yh0), fh.default_opts(12, max_iter=40))
    _compare_feast(None, A, B, out, ref, cont)


def test_singular_shift_reported(handle):
    n = 40
    lam = np.linspace(-1, 1, n) + 0.3j
    z, w = ct.ellipse_nodes(0.0, 0.5, 1.0, 0.0, 4)
    lam[7] = z[2]                                     # a node exactly on an eigenvalue
    A = np.diag(lam)
    prob = fh.Problem(handle, _cuda(A))
    Y = _cuda(W.subspace(n, 4, 1))
    with pytest.raises(fh.FeastError) as e:
        fh.contour_filter(prob, z, w, Y, Y.clone())
    assert e.value.code == 4


def test_bad_shapes_rejected(handle):
    p = W.dense_prescribed(n=40, n_in=4, m0=4, seed=2)
    prob = fh.Problem(handle, _cuda(p.A))
    z, w = ct.ellipse_nodes(0.1, 0.2, 1.0, 0.0, 4)
    with pytest.raises(ValueError):
        fh.contour_filter(prob, z, w, _cuda(p.Y0[:10]), _cuda(p.Yh0))
    import ctypes as C
    rc = fh.lib().fh_filter(handle._h, prob._p, 4, None, None, 0, None, None, None, None, None, None)
    assert rc == -4


def test_biortho_factors_graded_bq(handle):
    """B_Q of a subspace whose last 24 of 64 directions are suppressed to
    1e-9..1e-14 of the others (what the contour filter does to the directions
    beyond m when m0 is much larger): 40 eigenvalues of order one and 24 at
    or below rounding level.  The eigendecomposition succeeds, the resize
    keeps the 40, and the kept factors bi-orthonormalize B_Q."""
    rng = np.random.default_rng(5)
    n, m, k = 400, 64, 40
    scale = np.ones(m)
    scale[k:] = 10.0 ** -rng.uniform(9.0, 14.0, m - k)
    Q = W.subspace(n, m, 31) * scale
    Qh = W.subspace(n, m, 32) * scale
    BQ = Qh.conj().T @ Q
    g = np.sort(np.abs(np.linalg.eigvals(BQ)))[::-1]
    assert g[k - 1] > 1e-3 * g[0] and g[k] < 1e-14 * g[0]
    gam, S, Sh, mt = fh.biortho_factors(handle, _cuda(BQ), 1e-12)
    assert mt == k
    gam = gam.cpu().numpy()
    np.testing.assert_allclose(np.abs(gam[:k]), g[:k], rtol=1e-9)
    S, Sh = S.cpu().numpy()[:, :mt], Sh.cpu().numpy()[:, :mt]
    np.testing.assert_allclose(Sh.conj().T @ BQ @ S, np.eye(mt), atol=1e-9)


def test_count_estimate_dense_exact_trace(handle):
    """Dense problem, identity probes (p = n): the estimate is trace(rho_a) / n,
    the closed-form filter summed over the prescribed eigenvalues."""
    p = W.dense_prescribed(n=96, n_in=7, center=0.1 + 0.1j, radius=0.25, m0=12, seed=4)
    c, r, ne = p.contour.center, p.contour.a, 16
    z, w = ct.ellipse_nodes(c, r, 1.0, 0.0, ne)
    exact = np.sum(1.0 / (1.0 + ((p.info["lam"] - c) / r) ** ne))
    prob = fh.Problem(handle, _cuda(p.A))
    est, rep = fh.count_estimate(prob, z, w, _cuda(np.eye(p.n, dtype=np.complex128)))
    assert abs(est * p.n - exact) < 1e-9 * p.n


def test_feast_polygon_contour_matches_oracle(handle):
    """FEAST with a square contour (4 trapezoid intervals per side, 16 nodes,
    as in the paper's multi-contour experiment): the polygon's nodes, inside
    test and alpha, against the oracle with the same polygon."""
    p = W.dense_prescribed(n=200, n_in=12, center=0.1 + 0.1j, radius=0.25, m0=24, seed=7)
    # half-side in the widest gap of the eigenvalues' max-norm distance from the
    # centre (ratio 1.17): 7 inside, none within a few percent of the edges
    c, h = 0.1 + 0.1j, 0.1832
    sq = np.array([c - h - 1j * h, c + h - 1j * h, c + h + 1j * h, c - h + 1j * h])
    cont = F.PolygonContour(sq, 16)
    ref = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=40)
    prob = fh.Problem(handle, _cuda(p.A))
    opts = fh.default_opts(24, eps=1e-12, max_iter=40)
    out = fh.feast(prob, 0.0, 1.0, 1.0, 0.0, 16, _cuda(p.Y0), _cuda(p.Yh0), opts, polygon=sq)
    assert out["info"] == 0 and ref.info == 0
    inside = ct.inside_polygon(p.info["lam"], sq)
    truth = np.sort_complex(p.info["lam"][inside])
    # the paper's exit (steps 5.c / 5.d): the same iteration and pairs as the oracle
    assert out["report"]["iters"] == ref.iters
    assert 0 < len(out["lam"]) == len(ref.lam) <= len(truth)
    lam = np.sort_complex(out["lam"])
    np.testing.assert_allclose(lam, np.sort_complex(ref.lam), atol=1e-10 * cont.alpha())
    assert np.max(np.abs(lam[:, None] - truth[None, :]).min(axis=1)) < 1e-9 * cont.alpha()
    # the confirmed exit (opts.confirm) returns every prescribed eigenvalue inside
    out = fh.feast(prob, 0.0, 1.0, 1.0, 0.0, 16, _cuda(p.Y0), _cuda(p.Yh0),
                   fh.default_opts(24, eps=1e-12, max_iter=40, confirm=1), polygon=sq)
    assert out["info"] == 0 and len(out["lam"]) == len(truth) > 0
    np.testing.assert_allclose(np.sort_complex(out["lam"]), truth, atol=1e-9 * cont.alpha())


def _gap(d, lo, hi):
    """Size in the widest relative gap of the sorted distances d within [lo, hi]."""
    d = np.sort(d)
    best = None
    for a, b in zip(d[:-1], d[1:]):
        if lo <= a and b <= hi and (best is None or b / a > best[0]):
            best = (b / a, np.sqrt(a * b))
    return best[1]


@pytest.mark.parametrize("prec", [0, 1])
def test_feast_batched_multi_contour_one_matrix(handle, prec):
    """Multi-contour partition of one matrix (the paper's contour-grid
    experiment in small): two squares (16 nodes, 4 per side) and two circles
    (16 nodes) over one 600 x 600 matrix with eigenvalues in the unit disk,
    all in one batched call, with FP64 solves (eps 1e-12) or complex-FP32
    solves with FP64 refinement (eps 1e-10); each contour returns exactly
    the prescribed eigenvalues it contains (confirmed exit, opts.confirm)."""
    p = W.dense_prescribed(n=600, n_in=20, center=0.0, radius=0.3, m0=32, seed=9)
    lam = p.info["lam"]
    conts, truth = [], []
    for c in (-0.1j, 0.6 + 0.1j):                                  # squares
        h = _gap(np.maximum(np.abs((lam - c).real), np.abs((lam - c).imag)), 0.08, 0.16)
        sq = np.array([c - h - 1j * h, c + h - 1j * h, c + h + 1j * h, c - h + 1j * h])
        conts.append((0.0, 1.0, 1.0, 0.0, 16, sq))
        truth.append(lam[ct.inside_polygon(lam, sq)])
    for c in (-0.45 + 0.4j, 0.4 - 0.45j):                         # circles
        r = _gap(np.abs(lam - c), 0.08, 0.18)
        conts.append((c, r, 1.0, 0.0, 16))
        truth.append(lam[np.abs(lam - c) < r])
    assert all(0 < len(t) <= 16 for t in truth)
    prob = fh.Problem(handle, _cuda(p.A))
    if prec == 0:
        opts = fh.default_opts(32, eps=1e-12, max_iter=40, confirm=1)
    else:
        opts = fh.default_opts(32, eps=1e-10, max_iter=40, precision=fh.FH_PREC_MIXED, inner_tol=1e-12,
                               max_refine=10, confirm=1)
    Y0s = [_cuda(W.subspace(p.n, 32, 700 + i)) for i in range(4)]
    Yh0s = [_cuda(W.subspace(p.n, 32, 710 + i)) for i in range(4)]
    rc, outs = fh.feast_batched([prob] * 4, conts, Y0s, Yh0s, opts)
    assert rc == 0
    for out, t in zip(outs, truth):
        assert out["info"] == 0 and len(out["lam"]) == len(t)
        np.testing.assert_allclose(np.sort_complex(out["lam"]), np.sort_complex(t), atol=1e-9)


def test_feast_fp64_bq_qr_retry_unit_disk_circle(handle):
    """A case whose B_Q made the shifted QR iteration exhaust its budget at
    iteration 6 (status 7) when the iteration had neither the reversed-order
    retry nor the stall deflation for clusters: the 4000 x 4000 matrix with
    eigenvalues area-uniform in the unit disk, the circle at 0.5 - 0.3i with
    its radius in the widest eigenvalue gap near 0.17 (156 eigenvalues
    inside), m0 = 200, Ne = 16, FP64 direct solves.  FEAST meets eps = 1e-7
    and returns exactly the prescribed eigenvalues (confirmed exit,
    opts.confirm).  With the stall deflation the first attempt converges; the
    retry itself is covered by the forced-retry test below."""
    n, m0 = 4000, 200
    A, lam = W.dense_unit_disk(n, 12)
    c = 0.5 - 0.3j
    d = np.sort(np.abs(lam - c))
    best = None
    for a, b in zip(d[:-1], d[1:]):
        if 0.9 * 0.17 <= a and b <= 1.1 * 0.17 and (best is None or b / a > best[0]):
            best = (b / a, np.sqrt(a * b))
    r = best[1]
    truth = np.sort_complex(lam[np.abs(lam - c) < r])
    assert len(truth) == 156
    prob = fh.Problem(handle, _cuda(A))
    o = fh.default_opts(m0, precision=fh.FH_PREC_FP64, eps=1e-7, max_iter=40, confirm=1)
    out = fh.feast(prob, c, r, 1.0, 0.0, 16, _cuda(W.subspace(n, m0, 911)), _cuda(W.subspace(n, m0, 961)), o)
    assert out["info"] == 0
    got = np.sort_complex(out["lam"])
    assert len(got) == len(truth)
    np.testing.assert_allclose(got, truth, rtol=0, atol=1e-9)
    # the returned vectors are bi-orthonormal to the accuracy the reduced
    # eigenvectors allow: 156 clustered eigenvalues of a non-normal matrix
    # (measured 8e-7; a wrong pairing of left and right vectors gives O(1))
    X, Xh = out["X"], out["Xh"]
    G = (Xh.conj().T @ X).cpu().numpy()
    assert np.max(np.abs(G - np.eye(len(got)))) < 1e-5


def test_feast_forced_bq_retry_gives_the_same_pairs(handle, monkeypatch):
    """The reversed-order retry of the B_Q eigendecomposition (J B_Q J, then
    the rows of S and Sh reversed) forced at every iteration through the
    library's test switch FH_TEST_BQ_REVERSED: same exit, same eigenvalues,
    bi-orthonormal vectors, and the report counts one retry per iteration."""
    p = W.dense_prescribed(n=300, n_in=12, center=0.1 + 0.1j, radius=0.25, ne=8, m0=24, seed=5)
    prob = fh.Problem(handle, _cuda(p.A))
    o = fh.default_opts(24, precision=fh.FH_PREC_FP64, eps=1e-12, max_iter=40)
    c = p.contour
    args = (prob, c.center, c.a, 1.0, 0.0, 8)
    plain = fh.feast(*args, _cuda(p.Y0), _cuda(p.Yh0), o)
    monkeypatch.setenv("FH_TEST_BQ_REVERSED", "1")
    forced = fh.feast(*args, _cuda(p.Y0), _cuda(p.Yh0), o)
    monkeypatch.delenv("FH_TEST_BQ_REVERSED")
    assert plain["info"] == 0 and forced["info"] == 0
    assert plain["report"]["n_bq_retry"] == 0
    assert forced["report"]["n_bq_retry"] == forced["report"]["iters"]
    a, b = np.sort_complex(plain["lam"]), np.sort_complex(forced["lam"])
    assert len(a) == len(b) == 12
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-10)
    np.testing.assert_allclose(b, np.sort_complex(p.info["lam"][:12]), rtol=0, atol=1e-10)
    G = (forced["Xh"].conj().T @ forced["X"]).cpu().numpy()
    assert np.max(np.abs(G - np.eye(12))) < 1e-10


@pytest.mark.parametrize("seed,n,n_in,m0", [(1, 120, 6, 24), (9, 150, 8, 30)])
def test_feast_exit_with_spurious_flags_matches_oracle(handle, seed, n, n_in, m0):
    """Steps 5.c / 5.d with m_s > 0 at the exit iteration (the subspace is
    four times the eigenvalue count, so spurious Ritz values sit inside the
    circle): the library takes the same exit as the oracle -- same iteration,
    same m_s, the same m = m_r - m_s pairs."""
    p = W.dense_prescribed(n=n, n_in=n_in, center=0.1 + 0.1j, radius=0.25, ne=8, m0=m0, seed=seed)
    cont = F.Contour(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    ref = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=60)
    assert ref.info == 0 and ref.history[-1]["m_s"] > 0
    prob = fh.Problem(handle, _cuda(p.A))
    out = fh.feast(prob, p.contour.center, p.contour.a, 1.0, 0.0, 8, _cuda(p.Y0), _cuda(p.Yh0),
                   fh.default_opts(m0, eps=1e-12, max_iter=60))
    rep = out["report"]
    assert rep["iters"] == ref.iters
    assert rep["m_s"] == ref.history[-1]["m_s"]
    _compare_feast(p, p.A, None, out, ref, cont)


def test_feast_confirm_option_returns_every_converged_pair(handle):
    """opts.confirm = 1 (not the paper's rule): on this start the paper's exit
    passes over one true eigenpair flagged as spurious and returns 5 of the 6
    eigenvalues inside; the confirmed exit returns all 6 (the prescribed
    ones), and the literal exit's 5 are among them."""
    p = W.dense_prescribed(n=120, n_in=6, center=0.1 + 0.1j, radius=0.25, ne=8, m0=24, seed=13)
    cont = F.Contour(p.contour.center, p.contour.a, 1.0, 0.0, 8)
    ref = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=60)
    assert ref.info == 0 and len(ref.lam) == 5
    prob = fh.Problem(handle, _cuda(p.A))
    lit = fh.feast(prob, p.contour.center, p.contour.a, 1.0, 0.0, 8, _cuda(p.Y0), _cuda(p.Yh0),
                   fh.default_opts(24, eps=1e-12, max_iter=60))
    assert lit["info"] == 0 and len(lit["lam"]) == 5
    assert np.max(np.abs(lit["lam"] - ref.lam)) < 1e-10 * cont.alpha()
    con = fh.feast(prob, p.contour.center, p.contour.a, 1.0, 0.0, 8, _cuda(p.Y0), _cuda(p.Yh0),
                   fh.default_opts(24, eps=1e-12, max_iter=60, confirm=1))
    assert con["info"] == 0 and len(con["lam"]) == 6
    assert con["report"]["iters"] >= lit["report"]["iters"]
    lam_true = p.info["lam"][:6]
    lam_true = lam_true[np.lexsort((lam_true.imag, lam_true.real))]
    assert np.max(np.abs(con["lam"] - lam_true)) < 1e-10 * cont.alpha()
    assert np.max(np.abs(lit["lam"][:, None] - con["lam"][None, :]).min(axis=1)) < 1e-10 * cont.alpha()
    X, Xh = con["X"].cpu().numpy(), con["Xh"].cpu().numpy()
    assert np.max(np.abs(Xh.conj().T @ X - np.eye(6))) < 1e-10
    # confirm = 2: the paper's exit iteration, every converged inside pair
    # returned -- as many as the oracle's iterate has inside pairs below eps
    rec = ref.history[-1]
    n_conv = int(np.count_nonzero(rec["inside"] & (rec["res"] < 1e-12)))
    assert n_conv >= 5
    c2 = fh.feast(prob, p.contour.center, p.contour.a, 1.0, 0.0, 8, _cuda(p.Y0), _cuda(p.Yh0),
                  fh.default_opts(24, eps=1e-12, max_iter=60, confirm=2))
    assert c2["info"] == 0 and c2["report"]["iters"] == lit["report"]["iters"] == ref.iters
    assert len(c2["lam"]) == n_conv
    d = np.abs(c2["lam"][:, None] - lam_true[None, :]).min(axis=1)
    assert d.max() < 1e-10 * cont.alpha()
    assert np.max(np.abs(lit["lam"][:, None] - c2["lam"][None, :]).min(axis=1)) < 1e-10 * cont.alpha()


def test_biortho_factors_clustered_bq_regression(handle):
    """Regression: a B_Q recorded when the 64^3 convection-diffusion-reaction
    workload (no preconditioner) failed with status 7 at its 12th iteration:
    72 eigenvalues rho_a^2 = 1 within about 1e-8 (the converged pairs), on
    which the shifted QR iteration's local deflation test stalled at a
    trailing subdiagonal entry of 1e-11 for its whole budget, on both basis
    orders.  The decomposition now succeeds: the eigenvalues equal LAPACK's
    (to the cluster's conditioning) and the factors bi-orthonormalize B_Q."""
    import os
    BQ = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bq_cluster_convdiff3d64.npy"))
    m = BQ.shape[0]
    gam, S, Sh, mt = fh.biortho_factors(handle, _cuda(BQ))
    gam, S, Sh = gam.cpu().numpy(), S.cpu().numpy(), Sh.cpu().numpy()
    ref = sla.eigvals(BQ)
    assert np.max(np.abs(gam[:, None] - ref[None, :]).min(axis=1)) < 1e-7
    assert mt == m
    G = Sh[:, :mt].conj().T @ BQ @ S[:, :mt]
    assert np.max(np.abs(G - np.eye(mt))) < 1e-6


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_feast_degenerate_contours(handle, seed):
    """A contour around no eigenvalue returns no converged pair, with status 1
    (no Ritz value inside at the end) or 2 (some, all unconverged filter
    noise), as the oracle does; m0 = 6 under a contour with 10 eigenvalues
    inside ends with every Ritz value inside and status 3, the oracle's."""
    cont = F.Contour(0.1 + 0.1j, 0.25, 1.0, 0.0, 8)
    p = W.dense_prescribed(n=120, n_in=0, center=0.1 + 0.1j, radius=0.25, ne=8, m0=8, seed=seed)
    ref = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=8)
    prob = fh.Problem(handle, _cuda(p.A))
    out = fh.feast(prob, cont.center, cont.a, 1.0, 0.0, 8, _cuda(p.Y0), _cuda(p.Yh0),
                   fh.default_opts(8, eps=1e-12, max_iter=8))
    ritz = out["ritz"].cpu().numpy()
    n_in = int(np.count_nonzero(np.abs(ritz - cont.center) < cont.a))
    assert ref.info in (fh.FH_NO_EIG_INSIDE, fh.FH_NOT_CONVERGED)
    assert out["info"] == (fh.FH_NO_EIG_INSIDE if n_in == 0 else fh.FH_NOT_CONVERGED)
    assert out["report"]["iters"] == 8
    p = W.dense_prescribed(n=120, n_in=10, center=0.1 + 0.1j, radius=0.25, ne=8, m0=6, seed=seed)
    ref = F.feast(p.A, None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=8)
    prob = fh.Problem(handle, _cuda(p.A))
    out = fh.feast(prob, cont.center, cont.a, 1.0, 0.0, 8, _cuda(p.Y0), _cuda(p.Yh0),
                   fh.default_opts(6, eps=1e-12, max_iter=8))
    assert ref.info == out["info"] == fh.FH_M0_TOO_SMALL
