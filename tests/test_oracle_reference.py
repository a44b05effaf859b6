"""Pin of oracle/reference.py: ARPACK shift-invert eigenvalues equal LAPACK's
dense eigenvalues nearest the shift, on a small operator of the
complex-symmetric Schroedinger-type family."""
import numpy as np
import scipy.linalg as sla

import workloads as W
from oracle import reference as R


def test_nearest_eigenvalues_equal_dense_eigenvalues():
    A = W.schrodinger2d_csr(24, L=12.0, nwells=6, seed=2)
    ev = sla.eigvals(W.csr_to_dense(A))
    sigma = ev.real.min() - 1.0
    k = 20
    got = R.nearest_eigenvalues(A, k, sigma)
    want = ev[np.argsort(np.abs(ev - sigma))[:k]]
    want = want[np.lexsort((want.imag, want.real))]
    assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))
    # the k nearest a shift below the spectrum are (here) the k of smallest real part
    low = np.sort(ev.real)[:k]
    np.testing.assert_allclose(np.sort(got.real), low, rtol=0, atol=1e-9)
