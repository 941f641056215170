"""Benchmark: diffusion-map eigensolves per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload scurve-32k]

One step is one pass of the whole hot path over one batch of synthetic input:
compression of the points into the hierarchical operator (tree, neighbours,
lists, skeletons, tiles, alpha = 1 degrees) and the float64 Lanczos eigensolve
for the leading r eigenpairs, each iteration applying the compressed operator
once.  The points are resident in HBM before the timed region starts.

Printed: one JSON line with the throughput, per-step latency percentiles, the
H-matvec bandwidth, the roofline of the near-field kernel (HIP events recorded
around each of its launches inside the timed region), and the oracle timed on
the host cores on the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-matvec GB/s (%HBM roof) + eigensolves/sec, p50/p99 latency vs plain FP32"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pmc_traffic(workload: str, kernel_src: str):
    """HBM bytes per L2L launch from a committed counter summary, if it still matches the kernel source."""
    path = os.path.join(ROOT, "profiles", f"l2l_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("evaluate_hip_sha1") != kernel_src:
        return None
    return rec.get("traffic_bytes_per_launch")


def cpu_baseline(cfg, X, eps, r):
    """The oracle's full eigensolve of the same workload (compression + degrees + float64 Lanczos) on one core."""
    import threadpoolctl

    from oracle import diffusion as DF
    from oracle import hmatrix as HM
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        H = HM.HMatrix(X, eps, cfg["m"], cfg["s"], cfg["tau"], cfg["k"], cfg["seed"])
        th, _, info = DF.eigs(H.matvec, X.shape[0], r, tol=1e-10, seed=cfg["seed"])
        dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "eigensolves/s", "cores": 1, "kind": "oracle",
            "sample": f"one complete oracle eigensolve of the same workload ({X.shape[0]} points: float64 compression, "
                      f"degrees and Lanczos to 1e-10 over the oracle's float64 H-matvec, {info['iters']} steps), "
                      f"{dt:.1f} s on 1 host core"}


def serving_leg(hdm, pool, arrivals, near, far, max_slots=8):
    """Replay the arrival stream against the server; returns its statistics."""
    import synth
    srv = hdm.Server(max_slots=max_slots, mem_budget_bytes=200 << 30, compressors=2)
    S = synth.SERVING
    for q in pool[:2]:   # warm-up: allocations and first launches
        srv.wait(srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], S["r"], tol=S["tol"],
                            near_prec=near, far_prec=far))
    srv.close()
    srv = hdm.Server(max_slots=max_slots, mem_budget_bytes=200 << 30, compressors=2)
    t0 = time.monotonic()
    tickets = []
    for i, ta in enumerate(arrivals):
        q = pool[i % len(pool)]
        delay = t0 + ta - time.monotonic()
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"] + i, S["r"],
                                  tol=S["tol"], near_prec=near, far_prec=far, arrival_s=t0 + ta))
    res = [srv.wait(t, timeout=600) for t in tickets]
    st = srv.stats()
    srv.close()
    st["failed"] = sum(1 for r in res if r["status"] not in (0, 4))
    st["not_converged"] = sum(1 for r in res if r["status"] == 4)
    return st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scurve-32k")
    ap.add_argument("--matvec-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run one plain 1 GiB device copy (counter scale)")
    ap.add_argument("--serve-seconds", type=float, default=0.0,
                    help="length of the serving stream (disabled in this build: any value > 0 exits)")
    ap.add_argument("--serve-pool", type=int, default=8, help="distinct request instances the stream cycles through")
    args = ap.parse_args()
    if args.serve_seconds > 0:
        # two runs of this leg ended with a GPU memory fault whose cause is not yet found
        print("the serving leg is disabled in this build (a GPU fault under investigation); "
              "tests/test_gpu_serving.py covers the serving loop", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2311_06115_amd import hdm

    cfg = synth.get_config(args.workload)
    X, eps = synth.configs.make_inputs(cfg)
    r, block = cfg["r"], cfg["block"]
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev).contiguous()
    ctx = hdm.context(0)
    kw = dict(m=cfg["m"], s=cfg["s"], tau=cfg["tau"], k=cfg["k"], seed=cfg["seed"], near_prec=cfg["near_prec"],
              far_prec=cfg["far_prec"], ctx=ctx)
    tol = 1e-10

    def step():
        op = hdm.Operator(Xd, eps, **kw)
        ev, _, info, st = op.eigs(r, tol=tol, block=block, seed=cfg["seed"], vectors=True)
        steps = info.iters
        op.close()
        return ev, steps, st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    # inside the timed region only the near-field kernel is timed (HIP events on its
    # stream, for the roofline); the per-phase breakdown comes from one more step below
    ctx.profile(True, phases=["l2l"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        ev, lsteps, st = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = ctx.phase_times()
    ctx.profile(False)
    total = t1 - t0
    value = args.steps / total
    # one untimed step with every phase timed, for the breakdown
    ctx.profile(True)
    step()
    torch.cuda.synchronize()
    breakdown = ctx.phase_times()
    ctx.profile(False)

    # operator statistics and a standalone product timing on a resident operator
    op = hdm.Operator(Xd, eps, **kw)
    st_op = op.stats()
    x = torch.randn(X.shape[0], dtype=torch.float64, device=dev)
    for _ in range(5):
        op.matvec(x, normalised=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.matvec_reps):
        op.matvec(x, normalised=True)
    e1.record()
    torch.cuda.synchronize()
    mv_s = e0.elapsed_time(e1) / 1e3 / args.matvec_reps
    ev_acc = None
    gold = os.path.join(ROOT, "tests", "golden", f"eigs_{args.workload}.json")
    if os.path.exists(gold):
        g = json.load(open(gold))
        hm = np.array(g["hmatrix_eigenvalues"][:r])
        ev_acc = {"max_rel_err_vs_oracle_hmatrix_f64": float(np.max(np.abs(ev - hm) / np.abs(hm)))}
        if g["dense_eigenvalues"] is not None:   # not computed for the largest workloads
            dense = np.array(g["dense_eigenvalues"][:r])
            ev_acc["max_rel_err_vs_dense_f64"] = float(np.max(np.abs(ev - dense) / np.abs(dense)))
    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    op.close()

    l2l_n, l2l_ms = phases["l2l"]
    l2l_avg_s = l2l_ms / 1e3 / max(l2l_n, 1)
    achieved = st_op.algo_bytes_near / l2l_avg_s / 1e9
    src_sha = hashlib.sha1(open(os.path.join(ROOT, "paper_2311_06115_amd", "csrc", "evaluate.hip"), "rb").read()).hexdigest()
    traffic = pmc_traffic(args.workload, src_sha)
    serving = None
    if args.serve_seconds > 0:
        pool = [synth.configs.serving_instance(i) for i in range(args.serve_pool)]
        arrivals = synth.configs.serving_arrivals(args.serve_seconds)
        mixed = serving_leg(hdm, pool, arrivals, *synth.SERVING_PATHS["mixed"])
        plain = serving_leg(hdm, pool, arrivals, *synth.SERVING_PATHS["plain_f32"])
        keep = ("completed", "solves_per_s", "p50_latency_s", "p99_latency_s", "peak_resident_bytes",
                "shared_launches", "failed", "not_converged")
        serving = {"stream": f"Poisson {synth.SERVING['rate']}/s for {args.serve_seconds} s, "
                             f"{len(arrivals)} requests cycling {args.serve_pool} instances "
                             f"(S-curve / MNIST-shaped, N log-uniform in [4096, 65536]), "
                             f"r={synth.SERVING['r']}, rel. residual {synth.SERVING['tol']}",
                   "mixed": {k: mixed[k] for k in keep}, "plain_f32": {k: plain[k] for k in keep},
                   "mixed_tiles": "near %s, far %s" % synth.SERVING_PATHS["mixed"],
                   "pool_n": [q["n"] for q in pool], "pool_family": [q["family"] for q in pool]}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, X, eps, r)
    lat_ms = np.array(lat) * 1e3
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "eigensolves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{cfg['near_prec']} tiles, f64 Lanczos",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['family']} N={cfg['n']} D={cfg['dim']}, m={cfg['m']}, "
                               f"s={cfg['s']}, tau={cfg['tau']}, k={cfg['k']}, {cfg['near_prec']} tiles, "
                               f"r={r} eigenpairs, Lanczos rel. residual {tol}",
                   "n": cfg["n"], "eps": eps, "lanczos_steps": int(lsteps), "status": int(st)},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "hmatvec": {"us_per_call": mv_s * 1e6, "algo_bytes": st_op.algo_bytes_matvec,
                    "GBps": st_op.algo_bytes_matvec / mv_s / 1e9,
                    "frac_hbm": st_op.algo_bytes_matvec / mv_s / 1e9 / HBM_PEAK_GBS,
                    "near_bytes": st_op.algo_bytes_near, "resident_bytes": st_op.bytes_total,
                    "depth": st_op.depth, "mean_leaf_rank": st_op.mean_leaf_rank, "max_rank": st_op.max_rank,
                    "near_pairs": st_op.near_pairs, "far_pairs": st_op.far_pairs},
        "phase_ms_per_step": {k: v[1] for k, v in breakdown.items()},   # one extra step, every phase timed
        "phase_launches_per_step": {k: v[0] for k, v in breakdown.items()},
        "eigenvalue_accuracy": ev_acc,
        "roofline": {"kernel": "k_l2l (near field, with the leaf level of the upward pass)", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_us": l2l_avg_s * 1e6, "launches": int(l2l_n),
                     "algo_bytes_per_launch": st_op.algo_bytes_near},
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
