"""Write normx_gmm_n1000_p1e5_d3.json: ||X||^2 of the large benchmark data set
by the oracle, and the scale its parity is measured against.

The data set is the large Gaussian mixture of the benchmark (d = 3, n = 1000,
r = 100 means, p = 100000 observations, sigma = 1e-2, synth key 3) stored in
fp32 (the values as fp32 holds them, widened exactly).  The value is
oracle.normx.normx_implicit on those values; the scale is the same
expression on |V|, which bounds the sum of the absolute terms.  Calls only
the oracle and the seeded generators.

Usage (from the repository root, a few minutes on 8 host cores):
    python tests/golden/make_normx_full.py
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle.normx import normx_implicit  # noqa: E402

D, N, R, P, SIGMA, KEY = 3, 1000, 100, 100000, 1e-2, 3


def main():
    t0 = time.time()
    V, nu, _ = synth.gmm(N, R, P, SIGMA, KEY)
    V32 = V.astype(np.float32).astype(np.float64)
    value = normx_implicit(V32, nu, D)
    scale = normx_implicit(np.abs(V32), nu, D)
    out = {"what": "||X||^2 = nu' [V'V]^d nu of the large Gaussian mixture, fp32-stored V, by the oracle",
           "workload": {"d": D, "n": N, "r": R, "p": P, "sigma": SIGMA, "synth_key": KEY, "storage": "fp32"},
           "value": value, "scale_abs": scale,
           "made_by": "python tests/golden/make_normx_full.py (oracle.normx.normx_implicit)"}
    with open(os.path.join(HERE, "normx_gmm_n1000_p1e5_d3.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
