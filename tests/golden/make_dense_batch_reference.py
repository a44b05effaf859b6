"""Writes tests/golden/dense_batch64_inside.json: for each of the 64 dense
generalized problems of the third configuration (workloads.gen_dense_batch
with the radius scaled as 0.3 sqrt(256 / n_i)), the eigenvalues of (A_i, B_i)
inside its circle, from LAPACK's QZ on the whole pencil
(oracle.reference.dense_generalized_eigenvalues), and the distance of the
nearest eigenvalue outside (a measure of the convergence rate).  About an hour
of CPU on one core.

    python tests/golden/make_dense_batch_reference.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import reference as R  # noqa: E402


def main():
    t0 = time.time()
    probs = W.gen_dense_batch(count=64, nmin=256, nmax=2048, ne=8, m0=32, seed=3, scaled_radius=True)
    out = []
    for p in probs:
        ev = R.dense_generalized_eigenvalues(p.A, p.B)
        c, r = p.contour.center, p.contour.a
        d = np.abs(ev - c)
        ins = ev[d < r]
        ins = ins[np.lexsort((ins.imag, ins.real))]
        out.append({"n": p.n, "center": [c.real, c.imag], "radius": r,
                    "inside": [[float(x.real), float(x.imag)] for x in ins],
                    "nearest_outside_over_radius": float(d[d >= r].min() / r)})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dense_batch64_inside.json")
    with open(path, "w") as f:
        json.dump({"workload": "workloads.gen_dense_batch(count=64, seed=3, scaled_radius=True)",
                   "method": "oracle.reference.dense_generalized_eigenvalues (LAPACK QZ)",
                   "seconds": time.time() - t0, "problems": out}, f, indent=1)
    print(path, time.time() - t0)


if __name__ == "__main__":
    main()
