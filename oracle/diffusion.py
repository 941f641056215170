"""Diffusion-maps normalisation on top of any float64 kernel product (Alg. 1, alpha = 1).

Oracle -- test infrastructure only (tests/, smoke(), bench.py's cpu_baseline).

Given u = K w (dense, or the compressed K~ of Eq. (3)) the degree vectors are
q = K 1 and d = Q^-1 K Q^-1 1, and the symmetric conjugate of the Markov matrix
acts as S x = c * K (c * x) with c = 1 / (q sqrt(d)).  Eigenvectors phi of S map
to right eigenvectors psi = phi / sqrt(d) of P = D^-1 Q^-1 K Q^-1.
"""
from __future__ import annotations

import numpy as np

from . import lanczos as _lz
from .dense import sign_fix


def degrees(kmatvec, n: int):
    q = kmatvec(np.ones(n))
    d = kmatvec(1.0 / q) / q
    c = 1.0 / (q * np.sqrt(d))
    return q, d, c


def normalised_matvec(kmatvec, c):
    return lambda x: c * kmatvec(c * x)


def eigs(kmatvec, n: int, r: int, tol: float = 1e-10, max_basis: int = 300, seed: int = 0):
    """Leading r eigenpairs of S for the kernel product ``kmatvec`` (descending)."""
    q, d, c = degrees(kmatvec, n)
    v0 = _lz.start_vector(n, seed)
    theta, phi, info = _lz.lanczos(normalised_matvec(kmatvec, c), n, r, tol=tol, max_basis=max_basis, v0=v0)
    order = np.argsort(theta)[::-1]
    theta, phi = theta[order], sign_fix(phi[:, order] / np.linalg.norm(phi[:, order], axis=0))
    info.update(q=q, d=d, c=c)
    return theta, phi, info
