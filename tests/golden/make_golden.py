"""Write the stored expected values under tests/golden/ by calling only the oracle.

    python tests/golden/make_golden.py [config ...]

For each named workload it records the leading eigenvalues of the dense
alpha = 1 normalised Gaussian operator (Alg. 1; Eq. (2)), computed by the
oracle's float64 Lanczos (Sec. 2.2) over the oracle's exact dense product, and
the same for the oracle's compressed operator K~ (Eq. (3)).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import diffusion as DF  # noqa: E402
from oracle import hmatrix as HM  # noqa: E402


DENSE_MAX = 40000   # largest n whose dense eigenvalues are computed


def golden(name: str) -> dict:
    cfg = synth.get_config(name)
    X, eps = synth.configs.make_inputs(cfg)
    n, r = X.shape[0], cfg["r"]
    t0 = time.time()
    if n <= DENSE_MAX:
        lam_d, _, info_d = DF.eigs(lambda v: HM.dense_kmatvec(X, eps, v), n, r, tol=1e-11, seed=cfg["seed"])
    else:   # matrix-free dense products of 1e10 kernel values each are out of reach here
        lam_d, info_d = None, {"iters": 0}
    t1 = time.time()
    H = HM.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"])
    lam_h, _, info_h = DF.eigs(H.matvec, n, r, tol=1e-11, seed=cfg["seed"])
    t2 = time.time()
    return {
        "config": name,
        "n": n,
        "eps": eps,
        "source": "oracle: dense float64 Lanczos (Alg. 1 + Sec. 2.2) and the oracle's compressed K~ (Eq. (3))",
        "dense_eigenvalues": None if lam_d is None else [float(x) for x in lam_d],
        "dense_iters": int(info_d["iters"]),
        "hmatrix_eigenvalues": [float(x) for x in lam_h],
        "hmatrix_iters": int(info_h["iters"]),
        "seconds": {"dense": t1 - t0, "hmatrix": t2 - t1},
    }


def main(names):
    for name in names:
        g = golden(name)
        path = os.path.join(HERE, f"eigs_{name}.json")
        with open(path, "w") as f:
            json.dump(g, f, indent=1)
        print(path, g["seconds"], g["dense_eigenvalues"], g["hmatrix_eigenvalues"])


if __name__ == "__main__":
    main(sys.argv[1:] or ["scurve-2k", "scurve-32k"])
