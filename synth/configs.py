"""Named workloads.

Each entry fixes the data family, size, seed and the compression parameters
(leaf size m, max rank s, tolerance tau, neighbour count k) together with the
evaluation precision and the number of eigenpairs r.  ``make_inputs`` returns the
points and the bandwidth eps; everything else is a plain parameter.
"""
from __future__ import annotations

from . import generators as g

CONFIGS = {
    # 3-D S-curve, everything in float64
    "scurve-2k": dict(family="scurve", n=2048, dim=3, seed=0, m=128, s=64, tau=1e-5, k=32,
                      near_prec="f64", far_prec="f64", r=10, block=1),
    # 3-D S-curve, float32 evaluation tiles, float64 Lanczos
    "scurve-32k": dict(family="scurve", n=32768, dim=3, seed=1, m=256, s=128, tau=1e-5, k=32,
                       near_prec="f32", far_prec="f32", r=10, block=1),
    # MNIST-shaped u8 codes, mixed tiles: bf16 near field, f32 skeleton (far) field
    # (compared against the f32 path; bf16 far tiles alone cost 1.2e-4 in lambda_4)
    "mnist-64k": dict(family="mnist", n=65536, dim=784, seed=2, m=256, s=256, tau=1e-4, k=32,
                      near_prec="bf16", far_prec="f32", r=10, block=1),
    # the MNIST-shaped workload's parameters at a size whose dense float64 spectrum the
    # oracle computes (the golden eigenvalues of the mixed path)
    "mnist-8k": dict(family="mnist", n=8192, dim=784, seed=2, m=256, s=256, tau=1e-4, k=32,
                     near_prec="bf16", far_prec="f32", r=10, block=1),
    # 3-D S-curve, 100k points, f16 near tiles, block Lanczos with 16 start vectors
    "scurve-100k": dict(family="scurve", n=100000, dim=3, seed=3, m=512, s=256, tau=1e-5, k=32,
                        near_prec="f16", far_prec="f32", r=20, block=16),
    # local-bandwidth S-curve used by the geometry check of the oracle
    "scurve-2k-local": dict(family="scurve", n=2048, dim=3, seed=4, m=128, s=64, tau=1e-5, k=32,
                            near_prec="f64", far_prec="f64", r=10, block=1, eps=0.1),
    # 6-D Gaussian cloud of the scaling study
    "gauss6-100k": dict(family="gauss6", n=100000, dim=6, seed=5, m=768, s=768, tau=1e-3, k=64,
                        near_prec="f32", far_prec="f32", r=10, block=1),
}


def tree_depth(n: int, m: int) -> int:
    """Smallest depth d with ceil(n / 2^d) <= m (a perfect binary tree)."""
    d = 0
    while -(-n // (1 << d)) > m:
        d += 1
    return d


def get_config(name: str) -> dict:
    return dict(CONFIGS[name])


def make_points(family: str, n: int, seed: int, dim: int = 3):
    if family == "scurve":
        X, _ = g.s_curve(n, seed)
        return X
    if family == "mnist":
        X, _ = g.mnist_shaped(n, seed, dim=dim)
        return X
    if family == "gauss6":
        return g.gaussian_cloud(n, seed, dim=dim)
    raise ValueError(family)


def make_inputs(cfg: dict, n: int | None = None):
    """Points and eps for a config (optionally at a reduced size n)."""
    n = cfg["n"] if n is None else n
    X = make_points(cfg["family"], n, cfg["seed"], cfg["dim"])
    eps = cfg.get("eps")
    if eps is None:
        eps = g.median_sq_dist_eps(X, cfg["seed"])
    return X, float(eps)


# Serving stream: Poisson arrivals, each request an S-curve or MNIST-shaped
# instance with N log-uniform in [4096, 65536], 8 eigenpairs at relative
# residual 1e-6.  Per-family compression parameters:
# (MNIST-shaped: s = 128, below every leaf of m = 256; u8 requests with a rank
# above the smallest leaf are refused by the library)
SERVING_FAMILIES = {
    "scurve": dict(dim=3, m=256, s=128, tau=1e-5, k=32),
    "mnist": dict(dim=784, m=256, s=128, tau=1e-4, k=32),
}
SERVING = dict(rate=20.0, r=8, tol=1e-6, n_lo=4096, n_hi=65536, arrival_seed=7, request_seed0=1000)
# tile precisions (near, far) of the two paths the serving stream compares
SERVING_PATHS = {"mixed": ("bf16", "f32"), "plain_f32": ("f32", "f32")}


def serving_instance(i: int):
    """Request i of the serving stream: family, points and eps (seed 1000 + i)."""
    seed = SERVING["request_seed0"] + i
    rng = np_random(seed)
    fam = "scurve" if rng.random() < 0.5 else "mnist"
    n = int(round(2.0 ** rng.uniform(12.0, 16.0)))
    p = SERVING_FAMILIES[fam]
    X = make_points(fam, n, seed, p["dim"])
    eps = g.median_sq_dist_eps(X, seed)
    return dict(family=fam, n=n, seed=seed, X=X, eps=float(eps), **p)


def serving_arrivals(duration_s: float, rate: float | None = None):
    """Poisson arrival times in [0, duration_s)."""
    rate = SERVING["rate"] if rate is None else rate
    rng = np_random(SERVING["arrival_seed"])
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            return out
        out.append(t)


def np_random(seed: int):
    import numpy as np
    return np.random.default_rng(seed)


__all__ = ["CONFIGS", "get_config", "make_inputs", "make_points", "tree_depth", "SERVING", "SERVING_FAMILIES",
           "SERVING_PATHS",
           "serving_instance", "serving_arrivals"]
