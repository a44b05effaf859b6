"""Pins of the seeded workload generators that carry prescribed eigenvalues."""
import numpy as np
from scipy.optimize import linear_sum_assignment

import workloads as W


def test_dense_unit_disk_has_the_prescribed_eigenvalues():
    """A = V diag(lam) V^{-1}: LAPACK's eigenvalues of A are the prescribed
    ones (optimal one-to-one matching), and LAPACK's eigenpairs satisfy
    A x = lambda x to rounding level."""
    A, lam = W.dense_unit_disk(200, 5)
    ev = np.linalg.eigvals(A)
    r, c = linear_sum_assignment(np.abs(ev[:, None] - lam[None, :]))
    assert np.max(np.abs(ev[r] - lam[c])) < 1e-8
    w, X = np.linalg.eig(A)
    assert np.max(np.linalg.norm(A @ X - X * w[None, :], axis=0)) < 1e-9 * np.linalg.norm(A, 2)


def test_dense_unit_disk_eigenvalues_area_uniform_in_unit_disk():
    """Every prescribed eigenvalue lies in the closed unit disk, and the share
    inside radius r is r^2 (area-uniform) within four standard deviations."""
    _, lam = W.dense_unit_disk(1000, 12)
    assert np.all(np.abs(lam) <= 1.0)
    for r in (0.3, 0.5, 0.8):
        p = r * r
        share = np.mean(np.abs(lam) < r)
        assert abs(share - p) < 4 * np.sqrt(p * (1 - p) / len(lam))
    assert abs(np.mean(lam)) < 4 * np.sqrt(0.5 / len(lam))
