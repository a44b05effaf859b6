"""Reference eigenvalues of large sparse operators (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of this package.  For operators too
large for a dense eigendecomposition (the 1024 x 1024 complex-symmetric
workload, n = 1,048,576), the eigenvalues nearest a shift sigma come from
ARPACK's implicitly restarted Arnoldi method in shift-invert mode
(scipy.sparse.linalg.eigs): Arnoldi on (A - sigma I)^{-1}, applied through
one sparse LU factorization, whose largest eigenvalues 1/(lambda - sigma)
belong to the lambda nearest sigma.  This is an independent library method
(no contour integral, no subspace filter), so it can certify what FEAST
finds inside a contour.

Pin: tests/test_oracle_reference.py compares it with LAPACK's dense
eigenvalues on a small operator of the same family.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def nearest_eigenvalues(A, k, sigma, tol=1e-12, ordering="MMD_AT_PLUS_A"):
    """The k eigenvalues of the CSR operator A (dict with n, rowptr, colind,
    val) nearest sigma, sorted by (Re, Im).  A real matrix with a real shift
    is factorized in real arithmetic (the real and imaginary parts of each
    right-hand side are solved separately).  ordering: SuperLU's column
    ordering (minimum degree on A^T + A suits 2D grids; COLAMD 3D ones)."""
    n = A["n"]
    val = np.asarray(A["val"])
    real = not np.iscomplexobj(val) and complex(sigma).imag == 0.0
    dt = np.float64 if real else np.complex128
    Mf = sp.csr_matrix((val.astype(dt), A["colind"], A["rowptr"]), shape=(n, n)).tocsc()
    shifted = (Mf - (complex(sigma).real if real else sigma) * sp.identity(n, format="csc", dtype=dt)).tocsc()
    lu = spla.splu(shifted, permc_spec=ordering)

    def solve(x):
        x = np.asarray(x, dtype=np.complex128)
        if real:
            return lu.solve(np.ascontiguousarray(x.real)) + 1j * lu.solve(np.ascontiguousarray(x.imag))
        return lu.solve(x)

    op = spla.LinearOperator((n, n), matvec=solve, dtype=np.complex128)
    M = Mf.astype(np.complex128)
    vals = spla.eigs(M, k=k, sigma=sigma, OPinv=op, which="LM", return_eigenvectors=False, tol=tol)
    return vals[np.lexsort((vals.imag, vals.real))]


def dense_generalized_eigenvalues(A, B=None):
    """All eigenvalues of the dense pencil (A, B) (B None: identity) by LAPACK's
    QZ (scipy.linalg.eigvals), the brute-force reference for dense problems."""
    import scipy.linalg as sla
    return sla.eigvals(A, B) if B is not None else sla.eigvals(A)
