"""Writes tiny_fp64.json: the oracle's Ritz values along the warm-started
chain of the tiny planted workload (n=512, p=16, degree 8, interval
[-1, 0.5], 12 eigenvalues in [2, 10], 500 in [-1, 0.5], one cold step and
ten warm steps on X_k = X_{k-1} + 1e-3 sym(N(0,1))/sqrt(n)).

The paper prints no worked example of the extraction step, so this file is
a regression fixture of the oracle itself, plus the dense eigenvalues of
the final X (numpy.linalg.eigvalsh) that the chain must reach.  Calls only
oracle/ and the seeded generators.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1904_10585_amd import workloads as wl  # noqa: E402


def main():
    w = wl.WORKLOADS["tiny_fp64"]
    X, _, _ = wl.workload_matrices(w)
    U = wl.start_block(w.n, w.p, w.config)
    thetas = []
    for k in range(w.steps):
        if k:
            X = X + wl.perturbation(w.n, w.config, k)
        out = oracle.extract(X, X, U, w.degree, w.a, w.b)
        U = out["V"]
        thetas.append([float(v) for v in out["theta"]])
    dense = np.sort(np.linalg.eigvalsh(X))[::-1][: w.p]
    doc = {
        "workload": "tiny_fp64",
        "source": "oracle.extract along the warm chain; dense = numpy.linalg.eigvalsh(X_10)",
        "n": w.n, "p": w.p, "degree": w.degree, "interval": [w.a, w.b],
        "theta_per_step": thetas,
        "dense_top_p_final": [float(v) for v in dense],
    }
    with open(os.path.join(HERE, "tiny_fp64.json"), "w") as f:
        json.dump(doc, f, indent=1)


if __name__ == "__main__":
    main()
