"""Write the stored expected values under tests/golden/ by calling only the oracle.

    python tests/golden/make_golden.py [config ...]            eigenvalues
    python tests/golden/make_golden.py --structure [config ...] structure digests

For each named workload it records the leading eigenvalues of the dense
alpha = 1 normalised Gaussian operator (Alg. 1; Eq. (2)), computed by the
oracle's float64 Lanczos (Sec. 2.2) over the oracle's exact dense product, and
the same for the oracle's compressed operator K~ (Eq. (3)).

With --structure it records SHA-256 digests of the oracle's compressed
structure at full size (tree permutation, neighbour lists, near and far lists,
ranks and skeletons; Sec. 2.1 and Eq. (3)), for workloads whose arrays are too
large to store.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))   # tests/: the digest layout shared with the GPU tests

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
    H = HM.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"], budget=cfg.get("budget", 0.05))
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


def structure(name: str) -> dict:
    cfg = synth.get_config(name)
    X, eps = synth.configs.make_inputs(cfg)
    t0 = time.time()
    H = HM.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"], budget=cfg.get("budget", 0.05))
    from structure_check import structure_digests
    dig = structure_digests(H)
    r, _, _ = H.ranks()
    return {"config": name, "n": X.shape[0], "eps": eps,
            "source": "oracle: CPU build of the compression (Sec. 2.1, Eq. (3)), SHA-256 per array",
            "digests": dig, "max_rank": int(r[2:].max()), "seconds": time.time() - t0}


def main(names):
    for name in names:
        g = golden(name)
        path = os.path.join(HERE, f"eigs_{name}.json")
        with open(path, "w") as f:
            json.dump(g, f, indent=1)
        print(path, g["seconds"], g["dense_eigenvalues"], g["hmatrix_eigenvalues"])


def main_structure(names):
    for name in names:
        g = structure(name)
        path = os.path.join(HERE, f"structure_{name}.json")
        with open(path, "w") as f:
            json.dump(g, f, indent=1)
        print(path, g["seconds"])


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--structure":
        main_structure(args[1:] or ["scurve-32k", "mnist-64k", "scurve-100k"])
    else:
        main(args or ["scurve-2k", "scurve-32k"])
