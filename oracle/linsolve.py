"""Shifted linear systems of the contour filter (oracle).

Paper: Section 2.4 -- one factorization of (z_j B - A) per node serves both the
right system (eq:qr) and, through a conjugate-transpose solve, the left system
(eq:ql): ne factorizations and 2 ne solves for a complex general problem
(Table tab:solve, first row).

Dense: LAPACK LU with partial pivoting (scipy.linalg.lu_factor / lu_solve with
trans=0 and trans=2).  Sparse: SuperLU (scipy.sparse.linalg.splu, trans 'N' and
'H').  These are library primitives used as single steps.

ILU(0): incomplete LU on the sparsity pattern of the matrix, natural ordering,
written out from its definition (IKJ form): for each row i and each k < i in
the pattern of row i, l_ik = a_ik / u_kk and a_ij -= l_ik u_kj for every j > k
in the pattern of row i.  Pins: tests/test_oracle_ilu.py ((LU)_ij = M_ij on the
pattern; exact LU when the pattern has no fill).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class Counters:
    """Factorization / solve counts (Table tab:solve)."""

    def __init__(self):
        self.factorizations = 0
        self.solves = 0


def csr_matrix(A):
    """workloads CSR dict -> scipy.sparse.csr_matrix."""
    n = A["n"]
    return sp.csr_matrix((A["val"], A["colind"], A["rowptr"]), shape=(n, n))


def shifted(A, B, z):
    """z B - A for dense ndarray or scipy sparse A; B None means identity."""
    if sp.issparse(A):
        n = A.shape[0]
        Bm = sp.identity(n, dtype=np.complex128, format="csr") if B is None else B
        return (z * Bm - A.astype(np.complex128)).tocsc()
    n = A.shape[0]
    Bm = np.eye(n, dtype=np.complex128) if B is None else B
    return z * Bm - A


class DirectFactor:
    """One factorization of M = z B - A; solve() with trans 'N' or 'H'."""

    def __init__(self, M, counters=None):
        self.sparse = sp.issparse(M)
        if self.sparse:
            self.lu = spla.splu(sp.csc_matrix(M))
        else:
            self.lu = sla.lu_factor(M, check_finite=True)
        if counters is not None:
            counters.factorizations += 1
        self.counters = counters

    def solve(self, R, trans="N"):
        if self.counters is not None:
            self.counters.solves += 1
        if self.sparse:
            return self.lu.solve(np.asarray(R, dtype=np.complex128), trans=trans)
        return sla.lu_solve(self.lu, R, trans={"N": 0, "T": 1, "H": 2}[trans])


def ilu0(rowptr, colind, val):
    """ILU(0) of a CSR matrix with sorted column indices and a full diagonal.

    Returns the factor values aligned with the CSR pattern: entries left of the
    diagonal hold L (unit diagonal implied), the diagonal and entries right of
    it hold U.  Plain Python loops: intended for modest n.
    """
    n = len(rowptr) - 1
    a = np.array(val, dtype=np.complex128, copy=True)
    diag_pos = np.empty(n, dtype=np.int64)
    for i in range(n):
        cols = colind[rowptr[i]:rowptr[i + 1]]
        hit = np.nonzero(cols == i)[0]
        if len(hit) != 1:
            raise ValueError(f"row {i} has no diagonal entry")
        diag_pos[i] = rowptr[i] + hit[0]
    for i in range(n):
        lo, hi = rowptr[i], rowptr[i + 1]
        pos_of = {int(colind[p]): p for p in range(lo, hi)}
        for p in range(lo, hi):
            k = int(colind[p])
            if k >= i:
                break
            a[p] = a[p] / a[diag_pos[k]]
            lik = a[p]
            # subtract lik * u_kj for j > k present in row i
            for q in range(diag_pos[k] + 1, rowptr[k + 1]):
                j = int(colind[q])
                pij = pos_of.get(j)
                if pij is not None:
                    a[pij] = a[pij] - lik * a[q]
    return a


def ilu0_split(rowptr, colind, lu):
    """Dense L (unit lower) and U from ILU(0) values (small n, for tests)."""
    n = len(rowptr) - 1
    L = np.eye(n, dtype=np.complex128)
    U = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for p in range(rowptr[i], rowptr[i + 1]):
            j = colind[p]
            if j < i:
                L[i, j] = lu[p]
            else:
                U[i, j] = lu[p]
    return L, U


def ilu0_apply(rowptr, colind, lu, R, trans="N"):
    """(LU)^{-1} R (trans 'N') or (LU)^{-H} R (trans 'H') by dense triangular
    solves of the split factors (tests only; small n)."""
    L, U = ilu0_split(rowptr, colind, lu)
    if trans == "N":
        y = sla.solve_triangular(L, R, lower=True, unit_diagonal=True)
        return sla.solve_triangular(U, y, lower=False)
    # (LU)^H x = r  ->  U^H y = r, then L^H x = y
    y = sla.solve_triangular(U.conj().T, R, lower=True)
    return sla.solve_triangular(L.conj().T, y, lower=False, unit_diagonal=True)
