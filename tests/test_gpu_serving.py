"""Serving loop: continuous batching of eigensolves (admission, shared launches, alone vs in the mix)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _hdm():
    from paper_2311_06115_amd import hdm
    return hdm


def _req(n, seed, prec="f32"):
    X, _ = synth.s_curve(n, seed)
    eps = synth.median_sq_dist_eps(X, seed)
    return dict(X=X, eps=eps, m=128, s=48, tau=1e-5, k=16, seed=seed, near_prec=prec)


REQS = [_req(2048, 101), _req(3000, 102), _req(4096, 103), _req(2500, 104, "bf16"), _req(1800, 105)]
# a first solve that runs to its basis limit, long enough for the others to join its launches
# (a basis above 512 vectors is not restarted: the solve ends there)
LONG = dict(_req(4096, 100), tol=1e-300, max_basis=600)


def _alone(q, r=6, tol=1e-8):
    hdm = _hdm()
    op = hdm.Operator(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], near_prec=q["near_prec"])
    ev, _, info, st = op.eigs(r, tol=q.get("tol", tol), seed=q["seed"], max_basis=q.get("max_basis", 0),
                              vectors=False)
    op.close()
    return ev, info.iters, st


def test_results_alone_equal_results_in_the_mix():
    hdm = _hdm()
    reqs = [LONG] + REQS
    alone = [_alone(q) for q in reqs]
    srv = hdm.Server(max_slots=8)
    tickets = [srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], 6, tol=q.get("tol", 1e-8),
                          near_prec=q["near_prec"], max_basis=q.get("max_basis", 0)) for q in reqs]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"[gpu] serving stats {st}")
    assert alone[0][2] == 4 and res[0]["status"] == 4   # the long solve stops at its basis limit
    for (ev, iters, s0), r in zip(alone, res):
        assert r["status"] == s0
        assert r["iters"] == iters
        # the solve's arithmetic does not depend on its neighbours in a batch
        assert np.array_equal(r["evals"], ev), (r["evals"], ev)
    assert st["completed"] == len(reqs) and st["shared_launches"] > 0


def test_memory_admission_and_accounting():
    hdm = _hdm()
    from paper_2311_06115_amd.hdm import lib  # noqa: F401
    q = REQS[0]
    # a budget that fits one request at a time
    srv0 = hdm.Server(max_slots=8)
    t = srv0.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], 4)
    srv0.wait(t)
    one = srv0.stats()["peak_resident_bytes"]
    srv0.close()
    budget = int(one * 1.5)
    srv = hdm.Server(max_slots=8, mem_budget_bytes=budget)
    ts = [srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"] + i, 4) for i in range(4)]
    out = [srv.wait(t) for t in ts]
    st = srv.stats()
    srv.close()
    assert all(o["status"] == 0 for o in out)
    assert st["peak_resident_bytes"] <= budget
    assert st["completed"] == 4


def test_rejections_and_cancellation():
    hdm = _hdm()
    q = REQS[1]
    srv = hdm.Server(max_slots=1, mem_budget_bytes=1 << 40)
    bad = q["X"].copy()
    bad[3, 0] = np.nan
    with pytest.raises(hdm.HdmError) as e:
        srv.submit(bad, q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], 4)
    assert e.value.status == 1
    t1 = srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], 4)
    t2 = srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], 4)
    srv.cancel(t2)          # queued behind t1 (one slot)
    r1, r2 = srv.wait(t1), srv.wait(t2)
    assert r1["status"] == 0 and r2["status"] == 6
    st = srv.stats()
    srv.close()
    assert st["cancelled"] == 1 and st["completed"] == 1
    tiny = hdm.Server(max_slots=2, mem_budget_bytes=1 << 20)
    with pytest.raises(hdm.HdmError) as e:
        tiny.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], 4)
    assert e.value.status == 2
    assert tiny.stats()["rejected"] == 1
    tiny.close()


def _mnist_req(n, seed, near="bf16", far="f32"):
    X, _ = synth.mnist_shaped(n, seed)
    return dict(X=X, eps=synth.median_sq_dist_eps(X, seed), m=256, s=64, tau=1e-4, k=16, seed=seed,
                near_prec=near, far_prec=far)


def test_u8_requests_alone_equal_in_the_mix():
    """u8 codes (matrix-core distance blocks), ragged leaves, compressed on the server's
    worker threads and solved in shared launches: each result equals the one alone."""
    hdm = _hdm()
    reqs = [_mnist_req(3001, 201), _mnist_req(2048, 202), _mnist_req(4096, 203), _mnist_req(2500, 204)]
    alone = []
    for q in reqs:
        op = hdm.Operator(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], near_prec=q["near_prec"],
                          far_prec=q["far_prec"])
        ev, _, info, st = op.eigs(6, tol=1e-8, seed=q["seed"], vectors=False)
        op.close()
        alone.append((ev, info.iters, st))
    srv = hdm.Server(max_slots=4, compressors=2)
    tickets = [srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], 6, tol=1e-8,
                          near_prec=q["near_prec"], far_prec=q["far_prec"]) for q in reqs]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"[gpu] u8 serving stats {st}")
    for (ev, iters, s0), r in zip(alone, res):
        assert r["status"] == s0 == 0
        assert r["iters"] == iters
        assert np.array_equal(r["evals"], ev), (r["evals"], ev)
    assert st["completed"] == len(reqs)


def test_u8_serving_parameters_of_the_stream_alone_equal_in_the_mix():
    """The MNIST-shaped serving parameters (m = 256, s = 128 below every leaf),
    ragged leaves, compressed on the worker threads: each result equals the one
    alone, and the server drops its host copy of X once the operator exists."""
    hdm = _hdm()
    reqs = []
    for n, seed in [(6000, 211), (9000, 212)]:
        q = _mnist_req(n, seed)
        q["s"] = 128
        reqs.append(q)
    alone = []
    for q in reqs:
        op = hdm.Operator(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], near_prec=q["near_prec"],
                          far_prec=q["far_prec"])
        ev, _, info, st = op.eigs(8, tol=1e-6, seed=q["seed"], vectors=False)
        op.close()
        alone.append((ev, info.iters, st))
    srv = hdm.Server(max_slots=4, compressors=2)
    tickets = [srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], 8, tol=1e-6,
                          near_prec=q["near_prec"], far_prec=q["far_prec"]) for q in reqs]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"[gpu] u8 s=128 serving stats {st}")
    for (ev, iters, s0), r in zip(alone, res):
        assert r["status"] == s0 == 0
        assert r["iters"] == iters
        assert np.array_equal(r["evals"], ev)
        assert r["x_released"] == 1


def test_u8_rank_above_the_smallest_leaf_is_refused():
    hdm = _hdm()
    q = _mnist_req(4278, 7)
    srv = hdm.Server(max_slots=2)
    with pytest.raises(hdm.HdmError) as e:
        srv.submit(q["X"], q["eps"], q["m"], 256, q["tau"], q["k"], q["seed"], 8)
    assert e.value.status == 1
    with pytest.raises(hdm.HdmError) as e:
        hdm.Operator(q["X"], q["eps"], q["m"], 256, q["tau"], q["k"], q["seed"])
    assert e.value.status == 1
    srv.close()


@pytest.mark.skip(reason="u8 requests with max_rank_s above the smallest leaf (MNIST-shaped N = 21850 and 4278, "
                         "s = 256, 170/171- and 133/134-point leaves) ended two GPU runs in a memory fault whose "
                         "cause is not found; the library refuses them (HDM_EINVAL) until it is")
def test_u8_rank_above_leaf_serving():
    hdm = _hdm()
    reqs = [_mnist_req(21850, 1000), _mnist_req(4278, 1001)]
    srv = hdm.Server(max_slots=4, compressors=2)
    ts = [srv.submit(q["X"], q["eps"], q["m"], 256, q["tau"], q["k"], q["seed"], 8, tol=1e-6,
                     near_prec=q["near_prec"], far_prec=q["far_prec"]) for q in reqs]
    assert all(srv.wait(t)["status"] == 0 for t in ts)
    srv.close()
