"""Products replayed as HIP graphs against the same products launched kernel by kernel.

A product on one operator is recorded once as a graph and replayed with new
vector arguments.  Every replay must equal the eager launches bit for bit
(the kernels and their order of sums are the same), across replays with other
eager work and synchronisations in between, for one and several right-hand
sides, raw and normalised, float64 and float16 tiles.  A profiling context
launches eagerly (each kernel timed by its own stamps) with the same results.
The eigensolver launches eagerly whatever the setting and gives the same
eigenvalues either way.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _hdm():
    from paper_2311_06115_amd import hdm
    return hdm


_ops = {}


def _op(near, far):
    key = (near, far)
    if key not in _ops:
        hdm = _hdm()
        ctx = hdm.Context(0)
        X, _ = synth.s_curve(1537, 9)
        eps = synth.median_sq_dist_eps(X, 9)
        print(f"[gpu] compress scurve-ragged-1537 near={near} far={far}", flush=True)
        op = hdm.Operator(X, eps, 100, 40, 1e-5, 16, 9, near_prec=near, far_prec=far, ctx=ctx)
        _ops[key] = (ctx, op, X.shape[0])
    return _ops[key]


def _products(ctx, op, W, normalised, graphs, reps):
    ctx.graphs(graphs)
    out = []
    for r in range(reps):
        U = op.matvec(W[r], normalised=normalised)
        # eager work of the program between replays
        junk = torch.randn(4096, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        out.append(U.cpu().numpy())
    return out


@pytest.mark.parametrize("near,far", [("f64", None), ("f32", None), ("f16", "f32")])
@pytest.mark.parametrize("nrhs", [1, 5, 16])
@pytest.mark.parametrize("normalised", [False, True])
def test_graph_replays_equal_eager(near, far, nrhs, normalised):
    ctx, op, n = _op(near, far)
    rng = np.random.default_rng(100 + nrhs)
    reps = 4
    shape = (n,) if nrhs == 1 else (n, nrhs)
    W = [torch.from_numpy(rng.standard_normal(shape)).cuda() for _ in range(reps)]
    eager = _products(ctx, op, W, normalised, False, reps)
    graph = _products(ctx, op, W, normalised, True, reps)
    again = _products(ctx, op, W, normalised, True, reps)   # cached graph, replayed again
    ctx.graphs(True)
    for r in range(reps):
        assert np.array_equal(graph[r], eager[r]), r
        assert np.array_equal(again[r], eager[r]), r


def test_graph_products_under_profiling():
    ctx, op, n = _op("f16", "f32")
    x = torch.from_numpy(np.random.default_rng(7).standard_normal(n)).cuda()
    ctx.graphs(False)
    want = op.matvec(x, normalised=True).cpu().numpy()
    ctx.graphs(True)
    ctx.profile(True)
    for _ in range(3):
        got = op.matvec(x, normalised=True).cpu().numpy()
        assert np.array_equal(got, want)
    ph = ctx.phase_times()
    ctx.profile(False)
    # every phase of the three products was timed (eager launches under profiling);
    # the upward pass runs as its own launches per level, or inside the near-field
    # launch where the tiles outlast it
    for name in ("prep", "l2l", "s2s", "combine"):
        launches, ms = ph[name]
        assert launches == 3, (name, launches)
        assert ms > 0.0, name
    assert ph["n2s"][0] % 3 == 0


def test_graph_eigs_equal_eager():
    ctx, op, n = _op("f32", None)
    ctx.graphs(False)
    ev0, v0, i0, s0 = op.eigs(8, tol=1e-10, seed=3)
    ctx.graphs(True)
    ev1, v1, i1, s1 = op.eigs(8, tol=1e-10, seed=3)
    assert s0 == 0 and s1 == 0
    assert np.array_equal(ev0, ev1)
    assert i0.iters == i1.iters
    assert torch.equal(v0, v1)
    ctx.graphs(False)
    evb0, _, _, _ = op.eigs(8, tol=1e-10, block=4, seed=3, vectors=False)
    ctx.graphs(True)
    evb1, _, _, _ = op.eigs(8, tol=1e-10, block=4, seed=3, vectors=False)
    assert np.array_equal(evb0, evb1)


def test_profiling_one_phase_only():
    ctx, op, n = _op("f32", None)
    x = torch.from_numpy(np.random.default_rng(8).standard_normal(n)).cuda()
    ctx.graphs(False)
    want = op.matvec(x, normalised=True).cpu().numpy()
    ctx.graphs(True)
    ctx.profile(True, phases=["l2l"])
    for _ in range(2):
        assert np.array_equal(op.matvec(x, normalised=True).cpu().numpy(), want)
    ph = ctx.phase_times()
    ctx.profile(False)
    assert ph["l2l"][0] == 2 and ph["l2l"][1] > 0.0
    for name in ("prep", "n2s", "s2s", "combine", "ortho", "compress"):
        assert ph[name][0] == 0, name
