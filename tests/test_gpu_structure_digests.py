"""Structure parity at full size for the workloads whose oracle compression takes
minutes: SHA-256 digests of the tree permutation, neighbour lists, near and far
lists, ranks and skeletons (Sec. 2.1, Eq. (3)), written by
tests/golden/make_golden.py --structure from the oracle alone, against the same
digests of the GPU operator.  The permutation, neighbours and lists are required
bit-exact; ranks and skeletons are equal at these sizes (a near-tie pivot, which
the small-size parity tests allow within the rounding bound of pivoted QR, would
show here as a differing digest).
"""
import json
import os

import pytest

import synth
from structure_check import structure_digests

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("name", ["scurve-32k", "mnist-64k", "scurve-100k"])
def test_structure_digests_at_full_size(name):
    from paper_2311_06115_amd import hdm
    g = json.load(open(os.path.join(HERE, "golden", f"structure_{name}.json")))
    cfg = synth.get_config(name)
    X, eps = synth.configs.make_inputs(cfg)
    assert abs(eps - g["eps"]) <= 1e-12 * g["eps"] and X.shape[0] == g["n"]
    print(f"[gpu] compress {name} n={X.shape[0]}", flush=True)
    op = hdm.Operator(torch.from_numpy(X).cuda(), eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"],
                      near_prec=cfg["near_prec"], far_prec=cfg["far_prec"], budget=cfg.get("budget", 0.05))
    got = structure_digests(op)
    op.close()
    want = g["digests"]
    for key in ("perm", "knn_idx", "knn_d2", "near", "far"):
        assert got[key] == want[key], f"{name}: {key} differs from the oracle"
    same = {k: got[k] == want[k] for k in ("ranks", "skeletons")}
    print(f"[gpu] {name}: permutation, neighbours and lists equal the oracle's; ranks/skeletons {same}")
    assert all(same.values()), f"{name}: ranks or skeletons differ from the oracle ({same})"
