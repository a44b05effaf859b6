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


def test_nearest_eigenvalues_real_matrix_real_shift():
    """The real-arithmetic factorization path (real matrix, real shift): the
    3D convection-diffusion-reaction operator on an 8^3 grid, against LAPACK."""
    N = 8
    A = W.convdiff3d_csr(N, W.smooth_field3d(N, 4000))
    ev = sla.eigvals(W.csr_to_dense(A))
    k = 30
    got = R.nearest_eigenvalues(A, k, 0.0, ordering="COLAMD")
    scale = np.abs(ev).max()
    # each one is an eigenvalue, and they are the nearest the shift (a
    # conjugate pair may straddle the k-th distance, so compare as sets)
    assert np.max(np.abs(got[:, None] - ev[None, :]).min(axis=1)) < 1e-10 * scale
    d = np.sort(np.abs(ev))
    inner = ev[np.abs(ev) < d[k - 1] * (1 - 1e-9)]
    assert np.max(np.abs(inner[:, None] - got[None, :]).min(axis=1)) < 1e-10 * scale
    assert len(got) == k
