"""Writes tests/golden/convdiff3d_N64_lowest.json: the 100 eigenvalues nearest
sigma = 0 (below the whole spectrum) of the 3D convection-diffusion-reaction
operator -Lap u + v.grad u + 5 u on the 64^3 grid with the held-out
convection field (workloads.convdiff3d_csr(64, workloads.smooth_field3d(64,
4000))), computed by the oracle's ARPACK shift-invert reference
(oracle/reference.py; real LU, COLAMD ordering).  They place the contour of that workload and certify
the eigenvalues FEAST finds there.

    python tests/golden/make_convdiff3d_reference.py [N]
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import reference as R  # noqa: E402

K, SIGMA, FIELD = 100, 0.0, 4000


def main():
    N = int(sys.argv[1]) if len(sys.argv) > 1 else 64
    t0 = time.time()
    A = W.convdiff3d_csr(N, W.smooth_field3d(N, FIELD))
    ev = R.nearest_eigenvalues(A, K, SIGMA, ordering="COLAMD")
    out = {"operator": f"workloads.convdiff3d_csr({N}, workloads.smooth_field3d({N}, {FIELD}))", "n": A["n"], "k": K,
           "sigma": SIGMA, "method": "oracle.reference.nearest_eigenvalues (ARPACK shift-invert, real LU with COLAMD, tol 1e-12)",
           "seconds": time.time() - t0, "eigenvalues": [[float(x.real), float(x.imag)] for x in ev]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"convdiff3d_N{N}_lowest.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["seconds"])


if __name__ == "__main__":
    main()
