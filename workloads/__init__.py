"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module builds problem instances only: matrices, contours (centre, semi-axes,
rotation) and start subspaces.  It holds none of the eigensolver's arithmetic
(no quadrature, no shifted solves, no Rayleigh-Ritz); both the CPU oracle and
the HIP path receive exactly these arrays.

Recipes (the paper measures on the NEP collection and on CSH4, neither of which
is available here; these synthetic problems stand in for them, shaped like the
paper's own dense "eigenvalues inside the unit disk" matrix of the parallelism
experiments in Section 4.1 and like the sparse operators FEAST is aimed at):

* ``dense_prescribed``  -- A = V diag(lam) V^{-1}, V complex Gaussian with unit
  2-norm columns; ``n_in`` eigenvalues area-uniform inside a circle, the rest
  area-uniform in the unit disk outside that circle.
* ``convdiff2d``        -- -Laplace(u) + b.grad(u) on the unit square, Dirichlet,
  5-point central differences scaled by 1/h^2, lexicographic order (x fastest),
  real CSR.
* ``gen_dense_batch``   -- A = G/sqrt(n), B = I + 0.1 G'/sqrt(n), G complex
  Gaussian with E|g|^2 = 1.
* ``subspace``          -- complex Gaussian (N(0,1) + i N(0,1))/sqrt(2) block.

All random draws use numpy's PCG64 (``numpy.random.default_rng``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _cgauss(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def subspace(n: int, m0: int, seed: int) -> np.ndarray:
    """Complex Gaussian n x m0 start block (row i holds the m0 entries of row i)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_cgauss(rng, (n, m0)))


@dataclass
class Contour:
    """Ellipse z(t) = c + e^{i angle} (a cos t + i b sin t), b = ratio * a."""
    center: complex
    a: float
    ratio: float = 1.0
    angle: float = 0.0
    ne: int = 8


@dataclass
class Problem:
    name: str
    n: int
    A: object                      # dense ndarray (n x n, complex128) or CSR dict
    B: object | None               # None means B = I
    contour: Contour
    m0: int
    Y0: np.ndarray
    Yh0: np.ndarray
    info: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# Dense problem with prescribed spectrum (first configuration and its minis)
# --------------------------------------------------------------------------
def _area_uniform_disk(rng, count, center, radius):
    u = rng.random(count)
    v = rng.random(count)
    return center + radius * np.sqrt(u) * np.exp(2j * math.pi * v)


def dense_prescribed(n=400, n_in=24, center=0.1 + 0.1j, radius=0.25, ne=8, m0=36,
                     seed=1) -> Problem:
    rng = np.random.default_rng(seed)
    V = _cgauss(rng, (n, n))
    V /= np.linalg.norm(V, axis=0, keepdims=True)
    lam_in = _area_uniform_disk(rng, n_in, center, radius)
    out = []
    while len(out) < n - n_in:
        cand = _area_uniform_disk(rng, 2 * (n - n_in), 0.0, 1.0)
        cand = cand[np.abs(cand - center) >= radius]
        out.extend(cand.tolist())
    lam = np.concatenate([lam_in, np.array(out[: n - n_in])])
    # A = V diag(lam) V^{-1}  ->  A^T = V^{-T} (V diag(lam))^T
    A = np.linalg.solve(V.T, (V * lam[None, :]).T).T
    Y0 = subspace(n, m0, seed * 100 + 1)
    Yh0 = subspace(n, m0, seed * 100 + 2)
    return Problem(name=f"dense_prescribed_n{n}", n=n, A=np.ascontiguousarray(A), B=None,
                   contour=Contour(center=center, a=radius, ratio=1.0, angle=0.0, ne=ne),
                   m0=m0, Y0=Y0, Yh0=Yh0,
                   info={"lam": lam, "V": V, "n_in": n_in})


def dense_unit_disk(n=4000, seed=12):
    """A = V diag(lam) V^{-1}, lam area-uniform in the unit disk, V Gaussian with
    unit columns (the matrix of the paper's multi-contour experiment: a dense
    matrix whose eigenvalues all lie in the unit disk).  Returns (A, lam)."""
    rng = np.random.default_rng(seed)
    V = _cgauss(rng, (n, n))
    V /= np.linalg.norm(V, axis=0, keepdims=True)
    lam = _area_uniform_disk(rng, n, 0.0, 1.0)
    A = np.linalg.solve(V.T, (V * lam[None, :]).T).T
    return np.ascontiguousarray(A), lam


# --------------------------------------------------------------------------
# 2D convection-diffusion, 5-point central differences (second configuration)
# --------------------------------------------------------------------------
def convdiff2d_csr(N: int, bx: float, by: float):
    """CSR (0-based, sorted columns) of -Lap(u) + (bx, by).grad(u) on an N x N
    interior grid of the unit square, h = 1/(N+1), index = ix + N*iy."""
    h = 1.0 / (N + 1)
    inv_h2 = 1.0 / (h * h)
    n = N * N
    rowptr = np.zeros(n + 1, dtype=np.int32)
    cols = []
    vals = []
    # coefficients: u_{p-1}: -1/h^2 - b/(2h); u_{p+1}: -1/h^2 + b/(2h)
    wx, ex = -inv_h2 - bx / (2 * h), -inv_h2 + bx / (2 * h)
    sy, ny = -inv_h2 - by / (2 * h), -inv_h2 + by / (2 * h)
    diag = 4.0 * inv_h2
    idx = 0
    for iy in range(N):
        for ix in range(N):
            r = ix + N * iy
            if iy > 0:
                cols.append(r - N); vals.append(sy)
            if ix > 0:
                cols.append(r - 1); vals.append(wx)
            cols.append(r); vals.append(diag)
            if ix < N - 1:
                cols.append(r + 1); vals.append(ex)
            if iy < N - 1:
                cols.append(r + N); vals.append(ny)
            idx = len(cols)
            rowptr[r + 1] = idx
    return {"n": n, "rowptr": rowptr, "colind": np.asarray(cols, dtype=np.int32),
            "val": np.asarray(vals, dtype=np.float64)}


def convdiff1d_eigs(N: int, b: float) -> np.ndarray:
    """Eigenvalues of tridiag(-1/h^2 - b/2h, 2/h^2, -1/h^2 + b/2h) (N x N): the
    Toeplitz closed form 2/h^2 - 2 sqrt(beta*gamma) cos(j pi h), j = 1..N.
    Used only to place the second configuration's contour in spectral gaps."""
    h = 1.0 / (N + 1)
    beta = -1.0 / h**2 - b / (2 * h)
    gamma = -1.0 / h**2 + b / (2 * h)
    j = np.arange(1, N + 1)
    return 2.0 / h**2 - 2.0 * np.sqrt(beta * gamma) * np.cos(j * math.pi * h)


def convdiff2d(N=256, bx=20.0, by=10.0, m_in=41, ne=16, m0=64, ratio=0.3, seed=2,
               left_margin=15.0) -> Problem:
    """Ellipse on the real axis from lam_1 - left_margin to the midpoint of the
    gap between eigenvalues m_in and m_in + 1 (sorted, closed form)."""
    ex = convdiff1d_eigs(N, bx)
    ey = convdiff1d_eigs(N, by)
    lam = np.sort((ex[:, None] + ey[None, :]).ravel())
    left = lam[0] - left_margin
    right = 0.5 * (lam[m_in - 1] + lam[m_in])
    c = 0.5 * (left + right)
    a = 0.5 * (right - left)
    A = convdiff2d_csr(N, bx, by)
    n = N * N
    Y0 = subspace(n, m0, seed * 100 + 1)
    Yh0 = subspace(n, m0, seed * 100 + 2)
    return Problem(name=f"convdiff2d_N{N}", n=n, A=A, B=None,
                   contour=Contour(center=complex(c, 0.0), a=a, ratio=ratio, angle=0.0, ne=ne),
                   m0=m0, Y0=Y0, Yh0=Yh0,
                   info={"lam_sorted": lam, "m_in": m_in, "N": N, "b": (bx, by)})


# --------------------------------------------------------------------------
# Batch of dense generalized problems (third configuration)
# --------------------------------------------------------------------------
def gen_dense_batch(count=64, nmin=256, nmax=2048, ne=8, m0=32, radius=0.3, seed=3,
                    scaled_radius=False):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    probs = []
    for i, n in enumerate(sizes):
        n = int(n)
        A = _cgauss(rng, (n, n)) / math.sqrt(n)
        B = np.eye(n) + 0.1 * _cgauss(rng, (n, n)) / math.sqrt(n)
        c = complex(_area_uniform_disk(rng, 1, 0.0, 1.0)[0])
        r = radius * math.sqrt(nmin / n) if scaled_radius else radius
        Y0 = subspace(n, m0, seed * 100000 + 2 * i + 1)
        Yh0 = subspace(n, m0, seed * 100000 + 2 * i + 2)
        probs.append(Problem(name=f"gen_dense_{i}_n{n}", n=n, A=np.ascontiguousarray(A),
                             B=np.ascontiguousarray(B),
                             contour=Contour(center=c, a=r, ratio=1.0, angle=0.0, ne=ne),
                             m0=m0, Y0=Y0, Yh0=Yh0))
    return probs


# --------------------------------------------------------------------------
# Small helpers for tests
# --------------------------------------------------------------------------
# --------------------------------------------------------------------------
# 3D convection-diffusion-reaction with a smooth random convection field
# (fourth configuration)
# --------------------------------------------------------------------------
def smooth_field3d(N: int, seed: int, vmax: float = 30.0, modes: int = 3) -> np.ndarray:
    """Three components [3, N, N, N] (axes z, y, x) of a sum of low Fourier
    modes with Gaussian amplitudes and random phases, scaled to max |v| = vmax."""
    rng = np.random.default_rng(seed)
    g = (np.arange(N) + 1.0) / (N + 1)
    Z, Yg, X = np.meshgrid(g, g, g, indexing="ij")
    v = np.zeros((3, N, N, N))
    for d in range(3):
        for kz in range(1, modes + 1):
            for ky in range(1, modes + 1):
                for kx in range(1, modes + 1):
                    a = rng.standard_normal() / (kz * kz + ky * ky + kx * kx)
                    pz, py, px = rng.uniform(0, 2 * math.pi, 3)
                    v[d] += a * np.sin(kz * math.pi * Z + pz) * np.sin(ky * math.pi * Yg + py) * \
                        np.sin(kx * math.pi * X + px)
    mag = np.sqrt((v ** 2).sum(axis=0)).max()
    return v * (vmax / mag)


def convdiff3d_csr(N: int, v: np.ndarray, c: float = 5.0):
    """CSR of -Lap(u) + v(x).grad(u) + c u, 7-point central differences on the
    N^3 interior grid of the unit cube (Dirichlet), h = 1/(N+1),
    index = x + N*(y + N*z); v: [3, N, N, N] as from smooth_field3d (z, y, x)."""
    import scipy.sparse as sp
    h = 1.0 / (N + 1)
    n = N ** 3
    idx = np.arange(n).reshape(N, N, N)          # [z, y, x]
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [np.full(n, 6.0 / h ** 2 + c)]
    # component d of v acts along axis d of [z, y, x]
    for axis, comp in ((2, 2), (1, 1), (0, 0)):   # x, y, z
        vd = v[comp]
        for sgn in (-1, 1):
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            if sgn < 0:
                src[axis], dst[axis] = slice(1, None), slice(0, -1)
            else:
                src[axis], dst[axis] = slice(0, -1), slice(1, None)
            r = idx[tuple(src)].ravel()
            cc = idx[tuple(dst)].ravel()
            coef = -1.0 / h ** 2 + sgn * vd[tuple(src)].ravel() / (2 * h)
            rows.append(r)
            cols.append(cc)
            vals.append(coef)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sort_indices()
    return {"n": n, "rowptr": A.indptr.astype(np.int32), "colind": A.indices.astype(np.int32),
            "val": A.data.astype(np.float64)}


def csr_to_dense(A) -> np.ndarray:
    n = A["n"]
    D = np.zeros((n, n), dtype=np.result_type(A["val"].dtype, np.float64))
    rp, ci, v = A["rowptr"], A["colind"], A["val"]
    for i in range(n):
        D[i, ci[rp[i]:rp[i + 1]]] = v[rp[i]:rp[i + 1]]
    return D


def random_sparse_csr(n, density, seed, complex_vals=True, diag_shift=0.0):
    """Random sparse matrix with a full diagonal (for ILU(0)/SpMM edge cases)."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        k = rng.random(n) < density
        k[i] = True
        rows.append(np.nonzero(k)[0].astype(np.int32))
    rowptr = np.zeros(n + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum([len(r) for r in rows])
    colind = np.concatenate(rows).astype(np.int32)
    nnz = len(colind)
    if complex_vals:
        val = _cgauss(rng, nnz)
    else:
        val = rng.standard_normal(nnz)
    # make it diagonally heavy so ILU(0) exists
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            if colind[p] == i:
                val[p] = val[p] + diag_shift
    return {"n": n, "rowptr": rowptr, "colind": colind, "val": val}


# --------------------------------------------------------------------------
# Complex-symmetric 2D operator (fifth configuration and its small variants)
# --------------------------------------------------------------------------
def schrodinger2d_fields(N: int, L: float = 40.0, nwells: int = 50, depth: float = 20.0, sigma: float = 1.0,
                         seed: int = 5):
    """Potential V and absorbing profile W on the N x N interior grid of
    (0, L)^2 (h = L/(N+1), row iy holds x1 = (ix+1) h): V = -depth * sum of
    Gaussian wells (width sigma, centres area-uniform in [0.1L, 0.9L]^2),
    W = w(x1) + w(x2) with w(t) = max(0, (|t - L/2| - 0.4L)/(0.1L))^2."""
    rng = np.random.default_rng(seed)
    h = L / (N + 1)
    x = (np.arange(N) + 1) * h
    cen = 0.1 * L + 0.8 * L * rng.random((nwells, 2))
    V = np.zeros((N, N))
    for c1, c2 in cen:
        g1 = np.exp(-((x - c1) ** 2) / (2 * sigma ** 2))
        g2 = np.exp(-((x - c2) ** 2) / (2 * sigma ** 2))
        V -= depth * np.outer(g2, g1)                  # [iy, ix]
    ramp = np.maximum(0.0, (np.abs(x - L / 2) - 0.4 * L) / (0.1 * L)) ** 2
    Wf = ramp[None, :] + ramp[:, None]
    return V, Wf, h


def schrodinger2d_csr(N: int, L: float = 40.0, nwells: int = 50, depth: float = 20.0, sigma: float = 1.0,
                      eta: float = 5.0, seed: int = 5):
    """A = -Lap_h + diag(V) - i eta diag(W) on (0, L)^2, Dirichlet, 5-point,
    h = L/(N+1), index = ix + N*iy, columns sorted within each row
    (r - N, r - 1, r, r + 1, r + N).  V, W as in schrodinger2d_fields.
    A is complex symmetric (A = A^T)."""
    V, Wf, h = schrodinger2d_fields(N, L, nwells, depth, sigma, seed)
    n = N * N
    diag = 4.0 / h ** 2 + V.ravel() - 1j * eta * Wf.ravel()
    off = -1.0 / h ** 2
    idx = np.arange(n, dtype=np.int64).reshape(N, N)        # [iy, ix]
    ix = np.tile(np.arange(N), N)
    iy = np.repeat(np.arange(N), N)
    # per-row entry slots in column order: south, west, centre, east, north
    has = np.stack([iy > 0, ix > 0, np.ones(n, bool), ix < N - 1, iy < N - 1], axis=1)
    colv = np.stack([np.arange(n) - N, np.arange(n) - 1, np.arange(n), np.arange(n) + 1, np.arange(n) + N], axis=1)
    valv = np.empty((n, 5), dtype=np.complex128)
    valv[:, :] = off
    valv[:, 2] = diag
    cnt = has.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(cnt)
    colind = colv[has].astype(np.int32)
    val = valv[has]
    del idx
    return {"n": n, "rowptr": rowptr.astype(np.int32), "colind": colind, "val": val, "V": V, "W": Wf}


def schrodinger2d_contour(eigs, m_target=120, ratio=0.5, window=12, left_margin=1.0):
    """Ellipse of the complex-symmetric workload from its lowest eigenvalues
    (eigs: the eigenvalues nearest a shift below the spectrum, any order; all
    lie in Im <= 0 because W >= 0).  The ellipse holds the j lowest
    eigenvalues (by real part), j within m_target +- window where the gap
    Re(lam_{j+1}) - Re(lam_j) is widest; it crosses the real axis at
    Re(lam_1) - left_margin and at the middle of that gap, has axis ratio
    `ratio`, and its centre lies in the lower half-plane at a quarter of the
    vertical semi-axis below the real axis.  Returns (Contour, j)."""
    ev = np.asarray(eigs, dtype=np.complex128)
    re = np.sort(ev.real)
    lo, hi = max(1, m_target - window), min(len(re) - 1, m_target + window)
    j = max(range(lo, hi + 1), key=lambda q: re[q] - re[q - 1])
    left = re[0] - left_margin
    right = 0.5 * (re[j - 1] + re[j])
    hw = 0.5 * (right - left)
    delta = 0.25 * ratio * hw
    a = math.sqrt(hw * hw + (delta / ratio) ** 2)
    return Contour(center=complex(0.5 * (left + right), -delta), a=a, ratio=ratio, angle=0.0), j


def schrodinger2d(N=1024, eigs=None, m_target=120, ne=24, m0=160, ratio=0.5, seed=5, **op) -> Problem:
    """Complex-symmetric 2D workload (fifth configuration): the operator of
    schrodinger2d_csr(N, seed=seed, **op), the ellipse of
    schrodinger2d_contour around about m_target of its lowest eigenvalues
    (eigs: reference eigenvalues nearest a shift below the spectrum), Ne
    nodes, m0 columns; Y0 complex Gaussian, Yh0 = conj(Y0) (the left
    eigenvectors of a complex symmetric matrix are the conjugates of the
    right ones)."""
    A = schrodinger2d_csr(N, seed=seed, **op)
    cont, j = schrodinger2d_contour(eigs, m_target=m_target, ratio=ratio)
    cont.ne = ne
    n = A["n"]
    Y0 = subspace(n, m0, seed * 100 + 1)
    return Problem(name=f"schrodinger2d_N{N}", n=n, A=A, B=None, contour=cont, m0=m0, Y0=Y0,
                   Yh0=np.ascontiguousarray(np.conj(Y0)),
                   info={"m_in": j, "eigs": np.asarray(eigs), "N": N})


def lowest_contour(eigs, m_target, ratio=0.3, window=8, left_margin_frac=0.02):
    """Ellipse around the eigenvalues of smallest real part (eigs: the
    eigenvalues nearest a shift below the spectrum).  Sorted by real part,
    the j lowest (j within m_target +- window where the gap
    Re(lam_{j+1}) - Re(lam_j) is widest) fix the ellipse: centred on the real
    axis, crossing it just left of Re(lam_1) (by left_margin_frac of the
    span) and at the middle of that gap; the vertical semi-axis is `ratio`
    times the horizontal one, widened where one of those j eigenvalues would
    fall outside.  Returns (Contour, number of the given eigenvalues inside);
    raises if the ellipse reaches beyond the disc the given eigenvalues cover
    (the count would then be incomplete)."""
    ev = np.asarray(eigs, dtype=np.complex128)
    ev = ev[np.argsort(ev.real, kind="stable")]
    re = ev.real
    lo, hi = max(1, m_target - window), min(len(re) - 1, m_target + window)
    j = max(range(lo, hi + 1), key=lambda q: re[q] - re[q - 1])
    right = 0.5 * (re[j - 1] + re[j])
    left = re[0] - left_margin_frac * (right - re[0])
    c = 0.5 * (left + right)
    a = 0.5 * (right - left)
    b = ratio * a
    for x in ev[:j]:
        u = (x.real - c) / a
        if abs(u) < 1:
            b = max(b, 1.1 * abs(x.imag) / math.sqrt(1 - u * u))
    inside = int(np.count_nonzero(((ev.real - c) / a) ** 2 + (ev.imag / b) ** 2 < 1.0))
    covered = np.abs(ev).max()
    reach = max(abs(c - a), abs(c + a), math.hypot(c, b))
    if reach >= covered:
        raise ValueError(f"the ellipse reaches |z| = {reach:.4g}, beyond the {covered:.4g} the reference covers")
    return Contour(center=complex(c, 0.0), a=float(a), ratio=float(b / a), angle=0.0), inside


def convdiff3d(N=64, field_seed=4000, eigs=None, m_target=64, ne=16, m0=96, seed=4) -> Problem:
    """3D convection-diffusion-reaction workload (fourth configuration):
    -Lap u + v.grad u + 5 u on the N^3 interior grid of the unit cube, 7-point
    central differences, v = smooth_field3d(N, field_seed) (|v| <= 30); the
    ellipse of lowest_contour around about m_target of its lowest eigenvalues
    (eigs: reference eigenvalues nearest a shift below the spectrum); Ne
    nodes, m0 columns, complex Gaussian start blocks."""
    v = smooth_field3d(N, field_seed)
    A = convdiff3d_csr(N, v)
    cont, j = lowest_contour(eigs, m_target)
    cont.ne = ne
    n = A["n"]
    return Problem(name=f"convdiff3d_N{N}", n=n, A=A, B=None, contour=cont, m0=m0,
                   Y0=subspace(n, m0, seed * 100 + 1), Yh0=subspace(n, m0, seed * 100 + 2),
                   info={"m_in": j, "eigs": np.asarray(eigs), "N": N, "field": v})
