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


def nearest_eigenvalues(A, k, sigma, tol=1e-12):
    """The k eigenvalues of the CSR operator A (dict with n, rowptr, colind,
    val) nearest sigma, sorted by (Re, Im)."""
    n = A["n"]
    M = sp.csr_matrix((A["val"], A["colind"], A["rowptr"]), shape=(n, n)).tocsc()
    shifted = (M - sigma * sp.identity(n, format="csc", dtype=M.dtype)).tocsc()
    lu = spla.splu(shifted, permc_spec="MMD_AT_PLUS_A")
    dtype = np.result_type(M.dtype, np.complex128)
    op = spla.LinearOperator((n, n), matvec=lambda x: lu.solve(np.asarray(x, dtype=dtype)), dtype=dtype)
    vals = spla.eigs(M.astype(dtype), k=k, sigma=sigma, OPinv=op, which="LM", return_eigenvectors=False, tol=tol)
    return vals[np.lexsort((vals.imag, vals.real))]
