"""Diffusion-map outputs through the C ABI (Alg. 1, last steps) and the paper's
integration path (scipy's eigsh driving the compressed operator's matvec).

psi = phi / sqrt(d), lambda^t and d(t) = max{l : |lambda_l|^t > delta |lambda_1|^t}
are compared with the oracle's on the same compressed operator; the constant
first right eigenvector and the closed form d(0) pin the definitions.
"""
import numpy as np
import pytest

import synth
from oracle import dense as D
from oracle import diffusion as DF
from oracle import hmatrix as HM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    from paper_2311_06115_amd import hdm
    cfg = synth.get_config("scurve-2k")
    X, eps = synth.configs.make_inputs(cfg)
    op = hdm.Operator(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"], near_prec="f64")
    H = HM.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"])
    return cfg, X, eps, op, H


def test_psi_lambda_t_and_dimension_against_the_oracle(c1):
    from paper_2311_06115_amd import hdm
    cfg, X, eps, op, H = c1
    ev, vecs, info, st = op.eigs(cfg["r"], tol=1e-11)
    assert st == 0
    th, ph, oinfo = DF.eigs(H.matvec, X.shape[0], cfg["r"], tol=1e-12)
    opsi = ph / np.sqrt(oinfo["d"])[:, None]
    for t, delta in [(1, 0.1), (3, 0.05), (8, 0.01)]:
        psi, coords, lt, dim = hdm.diffusion_map(op, ev, vecs, t=t, delta=delta)
        psi, coords = psi.cpu().numpy(), coords.cpu().numpy()
        np.testing.assert_allclose(lt, th ** t, rtol=1e-9)
        assert dim == D.intrinsic_dim(th, t, delta)
        for k in range(6):   # well separated eigenvalues: vectors to the eigensolver's accuracy
            assert np.linalg.norm(psi[:, k] - opsi[:, k]) <= 1e-6 * np.linalg.norm(opsi[:, k]), k
            np.testing.assert_allclose(coords[:, k], lt[k] * psi[:, k], rtol=1e-15, atol=0)
    print(f"[gpu] d(t): {[hdm.diffusion_map(op, ev, vecs, t=t, delta=0.05)[3] for t in (1, 2, 4, 8, 16)]}")


def test_first_right_eigenvector_is_constant_and_d0_counts_all(c1):
    from paper_2311_06115_amd import hdm
    cfg, X, eps, op, H = c1
    ev, vecs, info, st = op.eigs(4, tol=1e-11)
    psi, coords, lt, dim = hdm.diffusion_map(op, ev, vecs, t=0, delta=0.5)
    p1 = psi[:, 0].cpu().numpy()
    assert np.ptp(p1) <= 1e-9 * np.abs(p1).mean()      # P 1 = 1: psi_1 is constant
    assert np.all(lt == 1.0) and dim == 4                # t = 0: every weight is 1
    dims = [hdm.diffusion_map(op, ev, vecs, t=t, delta=0.05)[3] for t in range(0, 12)]
    assert all(a >= b for a, b in zip(dims, dims[1:]))  # d(t) does not grow with t


def test_scipy_eigsh_drives_the_gpu_product(c1):
    # the paper's software path: ARPACK's implicitly restarted Lanczos over a
    # LinearOperator whose matvec is the compressed, normalised operator
    import scipy.sparse.linalg as spla
    from paper_2311_06115_amd import hdm
    cfg, X, eps, op, H = c1
    A = hdm.linear_operator(op, normalised=True)
    lam, _ = spla.eigsh(A, k=6, which="LA", tol=1e-12, v0=np.ones(X.shape[0]))
    lam = np.sort(lam)[::-1]
    ev, _, _, st = op.eigs(6, tol=1e-11, vectors=False)
    print(f"[gpu] eigsh over hdm_matvec vs hdm_eigs: {np.max(np.abs(lam - ev) / ev):.2e}")
    np.testing.assert_allclose(lam, ev, rtol=1e-9)
