"""Writes tests/golden/schrodinger2d_N1024_lowest.json: the 180 eigenvalues
nearest sigma = -45 (below the whole spectrum, whose lowest eigenvalue is
near -40) of the complex-symmetric Schroedinger-type operator on the
1024 x 1024 grid (workloads.schrodinger2d_csr(1024): domain (0, 40)^2, 50
Gaussian wells of depth 20, absorbing ramp on the outer 10 %, eta = 5),
computed by the oracle's ARPACK shift-invert reference (oracle/reference.py).
They place the contour of that workload (its 116 lowest lie inside) and
certify the eigenvalues FEAST finds there.  About half an hour of CPU.

    python tests/golden/make_schrodinger_reference.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import reference as R  # noqa: E402

N, K, SIGMA = 1024, 180, -45.0


def main():
    t0 = time.time()
    A = W.schrodinger2d_csr(N)
    ev = R.nearest_eigenvalues(A, K, SIGMA)
    out = {"operator": f"workloads.schrodinger2d_csr({N})", "n": A["n"], "k": K, "sigma": SIGMA,
           "method": "oracle.reference.nearest_eigenvalues (ARPACK shift-invert, tol 1e-12)",
           "seconds": time.time() - t0,
           "eigenvalues": [[float(x.real), float(x.imag)] for x in ev]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"schrodinger2d_N{N}_lowest.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["seconds"])


if __name__ == "__main__":
    main()
