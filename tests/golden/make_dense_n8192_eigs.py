"""Write the reference eigenvalues of the N = 8192 dense generalized workload.

Calls only the oracle: Rayleigh-Ritz on the whole space (Y = I) is the plain
definition of the pencil's eigenpairs; only the lowest `keep` values are
stored.  Inputs come from the seeded generator (seed 1001), exactly as the
benchmark builds them.

    python tests/golden/make_dense_n8192_eigs.py   # a few minutes on 8 cores
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import rr  # noqa: E402


def main(n=8192, n_low=256, keep=320, seed=1001):
    t0 = time.time()
    p = wl.dense_generalized(n=n, n_low=n_low, block=keep, degree=20, seed=seed)
    lam = rr.pencil_eigenvalues(p.A, p.B, keep)
    out = {"source": "oracle.rr.pencil_eigenvalues on workloads.dense_generalized "
                     f"(n={n}, n_low={n_low}, seed={seed}); lowest {keep} eigenvalues of (A, B)",
           "n": n, "n_low": n_low, "seed": seed, "sigma_max": p.meta["sigma_max"],
           "eps": p.eps, "eigenvalues": [float(v) for v in lam],
           "negative_count_A": int(np.count_nonzero(p.lam_A < 0)),
           "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, f"dense_generalized_n{n}_eigs.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", keep, "eigenvalues in", out["seconds"], "s")


if __name__ == "__main__":
    main()
