"""Thick-restart Lanczos (Sec. 2.2: the implicitly restarted method with exact
shifts) on a basis smaller than the unrestarted solve needs: 10 eigenpairs with
at most 15 basis vectors.  The eigenvalues must still match the oracle's
(float64 Lanczos without restarts on the same compressed operator): 1e-10 with
float64 tiles at 2048 points, 1e-6 with float32 tiles at 32768 points against
the stored oracle values."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import diffusion as DF
from oracle import hmatrix as HM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _hdm():
    from paper_2311_06115_amd import hdm
    return hdm


def test_restarted_solve_2k_float64():
    cfg = synth.get_config("scurve-2k")
    X, eps = synth.configs.make_inputs(cfg)
    op = _hdm().Operator(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"], near_prec="f64")
    H = HM.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"])
    ev, vecs, info, st = op.eigs(10, tol=1e-10, max_basis=15)
    print(f"[gpu] scurve-2k restarted (basis 15): {info.iters} steps, status {st}")
    assert st == 0 and info.converged and info.iters > 15   # the basis was restarted
    th, ph, _ = DF.eigs(H.matvec, X.shape[0], 10, tol=1e-12)
    assert np.max(np.abs(ev - th) / np.abs(th)) <= 1e-10
    V = vecs.cpu().numpy()
    for c in range(6):
        assert abs(abs(V[:, c] @ ph[:, c]) - 1.0) <= 1e-8
    # the unrestarted solve of the same operator gives the same eigenvalues
    ev0, _, info0, _ = op.eigs(10, tol=1e-10, vectors=False)
    assert info0.iters <= 30 and np.max(np.abs(ev - ev0) / np.abs(ev0)) <= 1e-10
    op.close()


def test_restarted_solve_32k_float32_tiles():
    cfg = synth.get_config("scurve-32k")
    X, eps = synth.configs.make_inputs(cfg)
    op = _hdm().Operator(torch.from_numpy(X).cuda(), eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"],
                         near_prec="f32")
    ev, _, info, st = op.eigs(10, tol=1e-10, max_basis=15, seed=cfg["seed"], vectors=False)
    print(f"[gpu] scurve-32k restarted (basis 15): {info.iters} steps, status {st}")
    assert st == 0 and info.converged and info.iters > 15
    g = json.load(open(os.path.join(HERE, "golden", "eigs_scurve-32k.json")))
    hm = np.array(g["hmatrix_eigenvalues"])
    assert np.max(np.abs(ev - hm) / np.abs(hm)) <= 1e-6
    op.close()


def test_restarts_are_bounded():
    cfg = synth.get_config("scurve-2k")
    X, eps = synth.configs.make_inputs(cfg)
    op = _hdm().Operator(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"], near_prec="f64")
    ev, _, info, st = op.eigs(10, tol=1e-300, max_basis=15, vectors=False)   # never converges
    # 15 steps, then 100 restarts keeping 12 vectors (3 new steps each)
    assert st == 4 and not info.converged and info.iters == 15 + 100 * 3
    op.close()
