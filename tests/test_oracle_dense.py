"""Pins of the oracle's dense definitions (Eq. (2), Alg. 1, Sec. 2.2) against closed forms.

Each test checks the oracle against a fact fixed by mathematics, not by
re-typing the oracle's own formula.
"""
import numpy as np
import pytest

import synth
from oracle import dense as D
from oracle import diffusion as DF
from oracle import lanczos as LZ


def _simplex(n, r):
    """n points with all pairwise squared distances r^2 (scaled unit vectors)."""
    return (r / np.sqrt(2.0)) * np.eye(n)


@pytest.mark.parametrize("n,r2,eps", [(2, 1.0, 1.0), (3, 2.5, 4.0), (7, 0.3, 0.7)])
def test_regular_simplex_closed_form(n, r2, eps):
    # All off-diagonal kernel values equal e = exp(-r^2/eps); with alpha = 1 the
    # conjugate S = K / (1 + (n-1) e) has eigenvalues 1 and (1-e)/(1+(n-1)e).
    X = _simplex(n, np.sqrt(r2))
    e = np.exp(-r2 / eps)
    lam, phi, psi, d = D.diffusion_eigs(X, eps, n)
    want = np.array([1.0] + [(1 - e) / (1 + (n - 1) * e)] * (n - 1))
    np.testing.assert_allclose(lam, want, rtol=0, atol=1e-14)


def test_kernel_scale_is_sigma_squared():
    # Eq. (2) with sigma^2 = eps: points at squared distance eps have W = 1/e.
    X = np.array([[0.0, 0.0], [3.0, 4.0]])
    W = D.kernel_matrix(X, 25.0)
    assert W[0, 1] == pytest.approx(np.exp(-1.0), rel=1e-15)
    assert W[0, 0] == 1.0


def test_u8_codes_stand_for_k_over_255():
    X = np.array([[0, 255], [255, 0]], dtype=np.uint8)
    W = D.kernel_matrix(X, 2.0)
    assert W[0, 1] == pytest.approx(np.exp(-1.0), rel=1e-15)


@pytest.fixture(scope="module")
def scurve512():
    X, _ = synth.s_curve(512, 11)
    eps = synth.median_sq_dist_eps(X, 11)
    return X, eps


def test_top_eigenpair_closed_form(scurve512):
    # P = D^-1 W^a is row-stochastic, so lambda_1 = 1; the matching eigenvector
    # of S is sqrt(d) / ||sqrt(d)||.
    X, eps = scurve512
    lam, phi, psi, d = D.diffusion_eigs(X, eps, 5)
    assert abs(lam[0] - 1.0) < 1e-13
    want = np.sqrt(d) / np.linalg.norm(np.sqrt(d))
    assert np.linalg.norm(np.abs(phi[:, 0]) - want) < 1e-12
    # psi_1 = phi_1 / sqrt(d) is constant
    assert np.ptp(psi[:, 0]) < 1e-12 * np.abs(psi[:, 0]).max()


def test_markov_and_conjugate_share_spectrum(scurve512):
    X, eps = scurve512
    W = D.kernel_matrix(X, eps)
    P = D.markov(W)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-14)
    lam, phi, psi, d = D.diffusion_eigs(X, eps, 6)
    # psi = D^-1/2 phi are right eigenvectors of P
    for c in range(6):
        np.testing.assert_allclose(P @ psi[:, c], lam[c] * psi[:, c], atol=1e-12 * np.abs(psi[:, c]).max())


def test_symmetric_and_psd(scurve512):
    X, eps = scurve512
    W = D.kernel_matrix(X, eps)
    S, q, d = D.symmetric_conjugate(W)
    assert np.array_equal(W, W.T)
    assert np.abs(S - S.T).max() <= 1e-16
    ev = np.linalg.eigvalsh(W)
    assert ev.min() >= -W.shape[0] * 1e-15 * ev.max()


def test_infinite_bandwidth_limit():
    # eps -> inf: W -> 1 1^T, the normalised operator has eigenvalues {1, 0, ..., 0}.
    X, _ = synth.s_curve(64, 3)
    lam, *_ = D.diffusion_eigs(X, 1e14, 4)
    np.testing.assert_allclose(lam, [1, 0, 0, 0], atol=1e-12)


def test_two_separated_clusters_have_double_unit_eigenvalue():
    # Disconnected components: S is block diagonal, each block has eigenvalue 1.
    X = synth.two_clusters(40, 5, gap=200.0)
    lam, *_ = D.diffusion_eigs(X, 2.0, 3)
    assert abs(lam[0] - 1) < 1e-13 and abs(lam[1] - 1) < 1e-13 and lam[2] < 1 - 1e-3


def test_lanczos_tridiagonal_toeplitz_closed_form():
    # Eigenvalues of tridiag(b, a, b) of order n are a + 2 b cos(k pi / (n + 1)).
    n, a, b = 400, 0.3, -0.45
    T = np.diag(np.full(n, a)) + np.diag(np.full(n - 1, b), 1) + np.diag(np.full(n - 1, b), -1)
    theta, X, info = LZ.lanczos(lambda v: T @ v, n, 4, tol=1e-12, max_basis=n, v0=LZ.start_vector(n, 9))
    k = np.arange(1, n + 1)
    exact = np.sort(a + 2 * b * np.cos(k * np.pi / (n + 1)))[::-1][:4]
    assert info["converged"]
    np.testing.assert_allclose(theta, exact, rtol=1e-10)
    for c in range(4):
        assert np.linalg.norm(T @ X[:, c] - theta[c] * X[:, c]) < 1e-7


def test_lanczos_matches_dense_eigh(scurve512):
    X, eps = scurve512
    lam, phi, psi, d = D.diffusion_eigs(X, eps, 8)
    W = D.kernel_matrix(X, eps)
    th, ph, info = DF.eigs(lambda v: W @ v, X.shape[0], 8, tol=1e-12)
    np.testing.assert_allclose(th, lam, rtol=1e-10, atol=1e-13)
    for c in range(8):
        assert abs(abs(ph[:, c] @ phi[:, c]) - 1) < 1e-8


def test_first_nontrivial_eigenvector_monotone_at_local_bandwidth():
    # Sec. 4.1.1 compares embeddings through the first non-trivial eigenvector;
    # at a local bandwidth it parametrises the S-curve's arc.
    cfg = synth.get_config("scurve-2k-local")
    X, t = synth.s_curve(cfg["n"], cfg["seed"])
    lam, phi, psi, d = D.diffusion_eigs(X, cfg["eps"], 2)
    v = psi[:, 1]
    rt = np.argsort(np.argsort(t))
    rv = np.argsort(np.argsort(v))
    rho = np.corrcoef(rt, rv)[0, 1]
    assert abs(rho) >= 0.99
    order = np.argsort(t)
    means = np.array([b.mean() for b in np.array_split(v[order], 32)])
    steps = np.diff(means) * np.sign(rho)
    assert np.all(steps > 0)


def test_intrinsic_dimension_reading():
    lam = np.array([1.0, 0.9, 0.5, 0.1])
    assert D.intrinsic_dim(lam, 1, 0.4) == 3
    assert D.intrinsic_dim(lam, 2, 0.4) == 2
