"""Float64 Lanczos with full reorthogonalisation (Sec. 2.2, Alg. 2 in its symmetric form).

Oracle -- test infrastructure only (tests/, smoke(), bench.py's cpu_baseline).

For a symmetric operator the Arnoldi factorisation of Alg. 2 / Eq. (5) has a
tridiagonal H (Sec. 2.2, "Implicitly restarted Lanczos method").  Each step here
computes z = A x_j, orthogonalises it against every basis vector twice
(classical Gram-Schmidt applied twice), and records alpha_j (diagonal) and
beta_j = ||r_j|| (off-diagonal).  Ritz values are the eigenvalues of the
tridiagonal matrix T_j; the Ritz pair (theta_i, y_i) has residual norm
|beta_j e_j^T y_i|, and the iteration stops when the leading r pairs satisfy
|beta_j y_{j,i}| <= tol |theta_i| (Sec. 2.2: a Ritz pair is exact when r_j = 0).
"""
from __future__ import annotations

import numpy as np

from .hmatrix import rand_u32

PURPOSE_LANCZOS = 4


def start_vector(n: int, seed: int, col: int = 0) -> np.ndarray:
    """Philox draws (purpose 4) mapped to (-1/2, 1/2), unit norm."""
    v = np.array([(rand_u32(seed, PURPOSE_LANCZOS, col, 0, i) + 0.5) / 4294967296.0 - 0.5 for i in range(n)])
    return v / np.linalg.norm(v)


def lanczos(matvec, n: int, r: int, tol: float = 1e-10, max_basis: int = 300, v0=None, check_every: int = 1):
    """Leading r eigenpairs (largest algebraic) of a symmetric operator.

    Returns (theta [r], Y [n, r], info dict).  ``matvec`` maps a float64 vector
    of length n to A times it.
    """
    v = np.ones(n) / np.sqrt(n) if v0 is None else np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    V = np.zeros((n, max_basis + 1))
    V[:, 0] = v
    alpha = np.zeros(max_basis)
    beta = np.zeros(max_basis)
    m = 0
    theta = Y = None
    converged = False
    for j in range(max_basis):
        z = matvec(V[:, j])
        h1 = V[:, : j + 1].T @ z
        z = z - V[:, : j + 1] @ h1
        h2 = V[:, : j + 1].T @ z
        z = z - V[:, : j + 1] @ h2
        alpha[j] = h1[j] + h2[j]
        beta[j] = np.linalg.norm(z)
        m = j + 1
        if m >= r and ((m % check_every) == 0 or j == max_basis - 1 or beta[j] == 0.0):
            T = np.diag(alpha[:m]) + np.diag(beta[: m - 1], 1) + np.diag(beta[: m - 1], -1)
            lam, S = np.linalg.eigh(T)
            order = np.argsort(lam)[::-1][:r]
            theta, Y = lam[order], S[:, order]
            bounds = np.abs(beta[j] * Y[-1, :])
            if np.all(bounds <= tol * np.abs(theta)) or beta[j] == 0.0:
                converged = True
                break
        if beta[j] == 0.0:
            break
        V[:, j + 1] = z / beta[j]
    X = V[:, :m] @ Y
    info = dict(iters=m, converged=converged, alpha=alpha[:m].copy(), beta=beta[:m].copy(),
                bounds=np.abs(beta[m - 1] * Y[-1, :]))
    return theta, X, info
