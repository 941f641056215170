"""Seeded point-cloud generators.

* ``s_curve`` stands in for the 3-D S-curve data set of the eigenpair experiments
  (Sec. 4.1.1): arc parameter t ~ U(-1.5 pi, 1.5 pi), height ~ U(0, 2), the curve
  (sin t, h, sign(t)(cos t - 1)) plus isotropic Gaussian noise of sd 0.01.
* ``mnist_shaped`` stands in for the MNIST experiment (Sec. 4.1.2).  No MNIST item
  is reproduced: it is a 10-component Gaussian mixture in a 16-dimensional latent
  space, mapped linearly to 784 pixels, clipped to [0, 1] and quantised to k/255.
  Points are returned as the u8 codes k (the value a pixel stands for is k/255).
* ``gaussian_cloud`` is the 6-D Gaussian point cloud of the scaling study (Sec. 4.2).

The bandwidth rule ``median_sq_dist_eps`` (median squared pair distance) is part of
the input recipe: the paper leaves sigma to the user (Eq. (2)).
"""
from __future__ import annotations

import numpy as np


def s_curve(n: int, seed: int, noise: float = 0.01):
    """Return (X float64 [n,3], t float64 [n]) for the noisy S-curve."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(-1.5 * np.pi, 1.5 * np.pi, n)
    h = rng.uniform(0.0, 2.0, n)
    X = np.stack([np.sin(t), h, np.sign(t) * (np.cos(t) - 1.0)], axis=1)
    X = X + noise * rng.standard_normal((n, 3))
    return np.ascontiguousarray(X, dtype=np.float64), t


def mnist_shaped(n: int, seed: int, dim: int = 784, latent: int = 16, comps: int = 10):
    """Return (codes uint8 [n,dim], labels int64 [n]).

    Draw order: component means, labels, latent points, linear map, bias.
    """
    rng = np.random.default_rng(seed)
    mu = 2.0 * rng.standard_normal((comps, latent))
    labels = rng.integers(0, comps, n)
    z = mu[labels] + rng.standard_normal((n, latent))
    A = 0.5 * rng.standard_normal((dim, latent)) / 4.0
    b = -1.0 + 0.3 * rng.standard_normal(dim)
    y = np.clip(z @ A.T + b, 0.0, 1.0)
    codes = np.rint(255.0 * y).astype(np.uint8)
    return np.ascontiguousarray(codes), labels


def gaussian_cloud(n: int, seed: int, dim: int = 6):
    """Standard normal points in R^dim (float64)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((n, dim)), dtype=np.float64)


def two_clusters(n_each: int, seed: int, gap: float = 100.0, dim: int = 3):
    """Two unit-variance blobs whose centres are ``gap`` apart (float64)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n_each, dim))
    b = rng.standard_normal((n_each, dim))
    b[:, 0] += gap
    return np.ascontiguousarray(np.concatenate([a, b]), dtype=np.float64)


def _pair_sq(X, i, j, chunk=1 << 14):
    out = np.empty(i.shape[0], np.float64)
    for s in range(0, i.shape[0], chunk):
        a, b = X[i[s:s + chunk]], X[j[s:s + chunk]]
        if X.dtype == np.uint8:
            d = a.astype(np.int32) - b.astype(np.int32)
            out[s:s + chunk] = np.einsum("ij,ij->i", d, d).astype(np.float64) / 65025.0
        else:
            d = a - b
            out[s:s + chunk] = (d * d).sum(axis=-1)
    return out


def median_sq_dist_eps(X: np.ndarray, seed: int, exact_max: int = 4096, pairs: int = 1 << 20):
    """Median squared distance over point pairs (i < j), computed in float64.

    Up to ``exact_max`` points every pair is used; above it ``pairs`` pairs
    (i != j) are drawn with replacement from ``default_rng(seed + 7)``.  For u8
    codes the distance is the one between the values k/255.
    """
    n = X.shape[0]
    if n <= exact_max:
        iu, ju = np.triu_indices(n, 1)
        vals = []
        step = 1 << 20
        for s in range(0, iu.size, step):
            vals.append(_pair_sq(X, iu[s:s + step], ju[s:s + step]))
        return float(np.median(np.concatenate(vals)))
    rng = np.random.default_rng(seed + 7)
    i = rng.integers(0, n, pairs)
    j = rng.integers(0, n - 1, pairs)
    j = j + (j >= i)
    return float(np.median(_pair_sq(X, i, j)))
