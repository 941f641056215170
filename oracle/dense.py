"""Dense float64 definitions of the diffusion-maps operator (Sec. 2.1, Alg. 1).

Oracle -- test infrastructure only (tests/, smoke(), bench.py's cpu_baseline).
Nothing here is blocked, fused or reordered: each function is the definition.

Readings of the paper used here (Alg. 1 as printed is ambiguous in places):
* Eq. (2) with sigma^2 = eps:  W_ij = exp(-||x_i - x_j||^2 / eps), W_ii = 1.
* Alg. 1, normalisation with alpha = 1:  W^a = Q^-1 W Q^-1, Q = diag(W 1).
* Alg. 1, Markov matrix:  P = D^-1 W^a with D = diag(W^a 1) (row-stochastic; the
  printed formula divides by Q^a again, which is not a transition matrix).
* P is never formed for the eigenproblem: the symmetric conjugate
  S = D^-1/2 W^a D^-1/2 has the same eigenvalues, and psi = D^-1/2 phi maps an
  eigenvector phi of S to one of P.  Written with c = 1 / (q sqrt(d)):
  S x = c * (W (c * x)).
"""
from __future__ import annotations

import numpy as np


def sq_dists(X: np.ndarray) -> np.ndarray:
    """Matrix of ||x_i - x_j||^2 (u8 codes stand for k/255)."""
    if X.dtype == np.uint8:
        A = X.astype(np.int64)
        out = np.empty((A.shape[0], A.shape[0]), np.float64)
        for i in range(A.shape[0]):
            d = A - A[i]
            out[i] = (d * d).sum(axis=1).astype(np.float64) / 65025.0
        return out
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((X.shape[0], X.shape[0]), np.float64)
    for d in range(X.shape[1]):
        t = X[:, d][:, None] - X[:, d][None, :]
        out = out + t * t
    return out


def kernel_matrix(X: np.ndarray, eps: float) -> np.ndarray:
    """Eq. (2): W_ij = exp(-||x_i - x_j||^2 / eps)."""
    return np.exp(-(sq_dists(X) / eps))


def alpha_normalise(W: np.ndarray, alpha: float = 1.0) -> np.ndarray:
    """Alg. 1: W^a_ij = W_ij / (Q_i^a Q_j^a) with Q the row sums (degrees) of W."""
    q = W.sum(axis=1)
    qa = q ** alpha
    return W / qa[:, None] / qa[None, :]


def markov(W: np.ndarray, alpha: float = 1.0) -> np.ndarray:
    """Alg. 1: row-stochastic transition matrix P = D^-1 W^a."""
    Wa = alpha_normalise(W, alpha)
    return Wa / Wa.sum(axis=1)[:, None]


def symmetric_conjugate(W: np.ndarray, alpha: float = 1.0):
    """S = D^-1/2 W^a D^-1/2 and the degree vectors (q of W, d of W^a)."""
    q = W.sum(axis=1)
    Wa = alpha_normalise(W, alpha)
    d = Wa.sum(axis=1)
    s = 1.0 / np.sqrt(d)
    S = Wa * s[:, None] * s[None, :]
    return S, q, d


def sign_fix(V: np.ndarray) -> np.ndarray:
    """Make the largest-magnitude entry of each column positive (first on ties)."""
    V = np.array(V, dtype=np.float64, copy=True)
    for c in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, c])))
        if V[i, c] < 0:
            V[:, c] = -V[:, c]
    return V


def leading_eigs(S: np.ndarray, r: int):
    """Alg. 1 eigendecomposition step: the r largest eigenpairs of symmetric S, descending."""
    lam, vec = np.linalg.eigh(S)
    order = np.argsort(lam)[::-1][:r]
    return lam[order], sign_fix(vec[:, order])


def diffusion_eigs(X: np.ndarray, eps: float, r: int, alpha: float = 1.0):
    """Leading r eigenvalues of P (via S), phi (eigenvectors of S) and psi = phi / sqrt(d)."""
    W = kernel_matrix(X, eps)
    S, q, d = symmetric_conjugate(W, alpha)
    lam, phi = leading_eigs(S, r)
    psi = phi / np.sqrt(d)[:, None]
    return lam, phi, psi, d


def intrinsic_dim(lam: np.ndarray, t: int, delta: float) -> int:
    """Alg. 1 last step, read as max{l : lambda_l^t > delta lambda_1^t} (1-based l)."""
    lt = np.abs(lam) ** t
    ok = np.nonzero(lt > delta * lt[0])[0]
    return int(ok[-1] + 1) if ok.size else 0
