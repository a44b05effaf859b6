"""Pins of the oracle's ILU(0) and direct shifted solves.

ILU(0) is defined by two facts: L unit lower and U upper on the pattern of M,
and (LU)_ij = M_ij for every (i, j) in that pattern.  Without fill (a
tridiagonal matrix) it is the exact LU factorization.
"""
import numpy as np
import scipy.linalg as sla

import workloads as W
from oracle import linsolve as L


def _shift_csr(A, z):
    val = -np.asarray(A["val"], dtype=np.complex128)
    for i in range(A["n"]):
        for p in range(A["rowptr"][i], A["rowptr"][i + 1]):
            if A["colind"][p] == i:
                val[p] += z
    return val


def test_ilu0_matches_pattern_convdiff():
    A = W.convdiff2d_csr(9, 20.0, 10.0)
    val = _shift_csr(A, 300 + 40j)
    lu = L.ilu0(A["rowptr"], A["colind"], val)
    Lm, Um = L.ilu0_split(A["rowptr"], A["colind"], lu)
    P = Lm @ Um
    M = W.csr_to_dense({**A, "val": val})
    mask = M != 0
    assert np.max(np.abs((P - M)[mask])) < 1e-10 * np.max(np.abs(M))
    # outside the pattern the product has genuine fill (ILU(0) drops it)
    assert np.max(np.abs(P[~mask])) > 1e-6


def test_ilu0_random_pattern():
    A = W.random_sparse_csr(40, 0.12, seed=5, complex_vals=True, diag_shift=6.0)
    lu = L.ilu0(A["rowptr"], A["colind"], A["val"])
    Lm, Um = L.ilu0_split(A["rowptr"], A["colind"], lu)
    M = W.csr_to_dense(A)
    mask = M != 0
    assert np.max(np.abs((Lm @ Um - M)[mask])) < 1e-12 * np.max(np.abs(M))


def test_ilu0_exact_without_fill():
    n = 30
    rng = np.random.default_rng(3)
    d = 4 + rng.random(n) + 1j * rng.random(n)
    lo = rng.random(n - 1) + 0.3j
    up = rng.random(n - 1) - 0.2j
    M = np.diag(d) + np.diag(lo, -1) + np.diag(up, 1)
    rowptr = [0]
    cols, vals = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                cols.append(j)
                vals.append(M[i, j])
        rowptr.append(len(cols))
    rowptr, cols = np.array(rowptr), np.array(cols)
    lu = L.ilu0(rowptr, cols, np.array(vals))
    Lm, Um = L.ilu0_split(rowptr, cols, lu)
    np.testing.assert_allclose(Lm @ Um, M, atol=1e-13)
    x = rng.standard_normal((n, 3)) + 0j
    np.testing.assert_allclose(L.ilu0_apply(rowptr, cols, lu, M @ x), x, atol=1e-12)
    np.testing.assert_allclose(L.ilu0_apply(rowptr, cols, lu, M.conj().T @ x, "H"), x, atol=1e-12)


def test_direct_solves_both_sides():
    rng = np.random.default_rng(1)
    n = 50
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    z = 0.3 + 0.7j
    M = z * B - A
    X = rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4))
    cnt = L.Counters()
    F = L.DirectFactor(L.shifted(A, B, z), cnt)
    np.testing.assert_allclose(M @ F.solve(X, "N"), X, atol=1e-11)
    np.testing.assert_allclose(M.conj().T @ F.solve(X, "H"), X, atol=1e-11)
    As = L.csr_matrix({"n": n, "rowptr": np.arange(0, n * n + 1, n), "colind": np.tile(np.arange(n), n),
                       "val": A.ravel()})
    Fs = L.DirectFactor(L.shifted(As, None, z), cnt)
    Ms = z * np.eye(n) - A
    np.testing.assert_allclose(Ms @ Fs.solve(X, "N"), X, atol=1e-11)
    np.testing.assert_allclose(Ms.conj().T @ Fs.solve(X, "H"), X, atol=1e-11)
    assert cnt.factorizations == 2 and cnt.solves == 4
