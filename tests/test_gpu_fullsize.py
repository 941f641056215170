"""Parity at the benchmarked size and launch configuration (S-curve, N = 32768, f32 tiles).

Structure is compared whole against the oracle's CPU build; the product against
the oracle's float64 H-matvec element by element and against the exact dense
operator on sampled rows (the oracle evaluates those rows one by one);
eigenvalues against the stored oracle values (tests/golden/make_golden.py).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import hmatrix as HM
from structure_check import check_product, check_skeletons, product_bound

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def c2():
    from paper_2311_06115_amd import hdm
    cfg = synth.get_config("scurve-32k")
    X, eps = synth.configs.make_inputs(cfg)
    print(f"[gpu] compress scurve-32k n={X.shape[0]}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    op = hdm.Operator(Xd, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"], near_prec=cfg["near_prec"],
                      far_prec=cfg["far_prec"])
    H = HM.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"])
    return cfg, X, eps, op, H


def test_structure_bit_exact(c2):
    cfg, X, eps, op, H = c2
    assert np.array_equal(op.perm(), H.perm())
    gi, gd = op.knn()
    oi, od = H.knn()
    assert np.array_equal(gi, oi) and np.array_equal(gd, od)
    for a, b in zip(op.near(), H.near()):
        assert np.array_equal(a, b)
    for a, b in zip(op.far(), H.far()):
        assert np.array_equal(a, b)
    compared, ties, pmax = check_skeletons(op, H, cfg["s"], cfg["tau"])
    print(f"[gpu] scurve-32k: {compared} nodes compared, {ties} near-tie pivots, max P deviation {pmax:.2e}")


def test_product_against_oracle_and_dense_rows(c2):
    cfg, X, eps, op, H = c2
    rng = np.random.default_rng(21)
    w = rng.standard_normal(X.shape[0])
    u = op.matvec(torch.from_numpy(w).cuda()).cpu().numpy()
    ref = H.matvec(w)
    rel = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    print(f"[gpu] f32 product vs oracle K~: {rel:.2e}")
    assert rel <= 2e-6
    worst = check_product(u, ref, product_bound(H, w, "f32"), "scurve-32k f32")
    print(f"[gpu] f32 product at full size: worst entry at {worst:.2e} of its bound")
    rows = np.sort(rng.choice(X.shape[0], 256, replace=False))
    dense = np.array([HM.dense_kmatvec(X, eps, w, (int(i), int(i) + 1))[0] for i in rows])
    rel_d = np.linalg.norm(u[rows] - dense) / np.linalg.norm(dense)
    print(f"[gpu] product vs dense K on 256 sampled rows: {rel_d:.2e}")
    assert rel_d <= 10 * cfg["tau"]


def test_eigenvalues_against_stored_oracle(c2):
    cfg, X, eps, op, H = c2
    ev, vecs, info, st = op.eigs(cfg["r"], tol=1e-10, seed=cfg["seed"])
    assert st == 0 and info.converged
    g = json.load(open(os.path.join(HERE, "golden", "eigs_scurve-32k.json")))
    hm = np.array(g["hmatrix_eigenvalues"])
    dense = np.array(g["dense_eigenvalues"])
    rel = np.abs(ev - hm) / np.abs(hm)
    rel_d = np.abs(ev - dense) / np.abs(dense)
    print(f"[gpu] eig rel err vs oracle K~ {rel.max():.2e}, vs dense {rel_d.max():.2e}, steps {info.iters}")
    assert rel.max() <= 1e-6
    assert abs(ev[0] - 1.0) <= 1e-6
    # unit-norm, sign-fixed Ritz vectors
    V = vecs.cpu().numpy()
    np.testing.assert_allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-12)
    for c in range(V.shape[1]):
        assert V[np.argmax(np.abs(V[:, c])), c] > 0
