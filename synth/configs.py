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
    # MNIST-shaped u8 codes, bf16 tiles (compared against the f32 path)
    "mnist-64k": dict(family="mnist", n=65536, dim=784, seed=2, m=256, s=256, tau=1e-4, k=32,
                      near_prec="bf16", far_prec="bf16", r=10, block=1),
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


__all__ = ["CONFIGS", "get_config", "make_inputs", "make_points", "tree_depth"]
