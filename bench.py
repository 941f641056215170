"""Benchmark: diffusion-map eigensolves per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload scurve-100k]
                    [--serve-seconds S] [--thrash-mib M] [--no-cpu-baseline]

One step is one pass of the whole hot path over one batch of synthetic input:
compression of the points into the hierarchical operator (tree, neighbours,
lists, skeletons, tiles, alpha = 1 degrees) and the float64 Lanczos eigensolve
for the leading r eigenpairs, each iteration applying the compressed operator.
The points are resident in HBM before the timed region starts.  The default
workload is the largest single-GPU configuration: the 100000-point S-curve with
float16 near tiles on the matrix cores, float32 far tiles and block Lanczos with
16 vectors per step (20 eigenpairs).

Printed: one JSON line with the throughput, per-step latency percentiles, the
H-matvec bandwidth, the roofline of the near-field kernel (HIP events recorded
around each of its launches inside the timed region), the serving stream (mixed
against plain float32 tiles, p50/p99 latency), and the oracle timed on the host
cores on a bounded sample of the same workload.
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
MFMA_F16_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pmc_traffic(workload: str, kernel_src: str):
    """HBM bytes per near-field launch from a committed counter summary, if it still matches the kernel source."""
    path = os.path.join(ROOT, "profiles", f"l2l_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("evaluate_hip_sha1") != kernel_src:
        return None
    return rec.get("traffic_bytes_per_launch")


def omp_threads() -> int:
    try:
        import ctypes
        return int(ctypes.CDLL("libgomp.so.1").omp_get_max_threads())
    except OSError:
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_baseline(X, eps, vector_products, target_s=10.0):
    """The oracle's dense float64 product (Eq. (2), kernel values evaluated on the fly) timed on a
    bounded sample (about target_s seconds of whole products), scaled to one eigensolve of the same
    workload: the same number of operator applications as the GPU solve used, each a dense product."""
    from oracle import hmatrix as HM
    import numpy as np
    n = X.shape[0]
    w = np.random.default_rng(0).standard_normal(n)
    t0 = time.perf_counter()
    HM.dense_kmatvec(X, eps, w, (0, min(n, 1024)))   # calibration (also loads the library)
    est = (time.perf_counter() - t0) * n / min(n, 1024)
    reps = max(1, min(vector_products, int(round(target_s / max(est, 1e-9)))))
    t0 = time.perf_counter()
    for _ in range(reps):
        HM.dense_kmatvec(X, eps, w)
    dt = time.perf_counter() - t0
    per_product = dt / reps
    solve = per_product * vector_products
    return {"value": 1.0 / solve, "unit": "eigensolves/s", "cores": omp_threads(), "kind": "oracle",
            "sample": f"{reps} whole dense float64 products of the oracle (kernel evaluated on the fly, {n} points) "
                      f"took {dt:.1f} s ({per_product:.2f} s each), scaled to the {vector_products} operator "
                      f"applications of the GPU eigensolve (degrees + Lanczos); the Lanczos orthogonalisation "
                      f"is not included"}


def serving_leg(hdm, pool, arrivals, near, far, max_slots=8):
    """Replay the arrival stream against the server; returns its statistics and results."""
    import synth
    srv = hdm.Server(max_slots=max_slots, mem_budget_bytes=200 << 30, compressors=2)
    S = synth.SERVING
    for q in pool[:2]:   # warm-up: allocations and first launches
        srv.wait(srv.submit(q["X"], q["eps"], q["m"], q["s"], q["tau"], q["k"], q["seed"], S["r"], tol=S["tol"],
                            near_prec=near, far_prec=far), timeout=600)
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
    st["mean_service_s"] = sum(r["service_s"] for r in res) / max(len(res), 1)
    st["offered_per_s"] = len(arrivals) / max(arrivals[-1], 1e-9) if arrivals else 0.0
    return st, res


def serving(hdm, seconds, pool_size):
    """The served stream: Poisson 20/s, S-curve or MNIST-shaped, N log-uniform in [4096, 65536], r = 8 at
    residual 1e-6, against mixed (bf16 near, f32 far) and plain float32 tiles on the same stream.  Where
    a path cannot keep up with the offered rate, it is replayed at 80% of its measured capacity."""
    import numpy as np
    import synth
    pool = [synth.configs.serving_instance(i) for i in range(pool_size)]
    arrivals = synth.configs.serving_arrivals(seconds)
    keep = ("completed", "solves_per_s", "p50_latency_s", "p99_latency_s", "mean_service_s", "offered_per_s",
            "peak_resident_bytes", "shared_launches", "failed", "not_converged")
    out = {"stream": f"Poisson {synth.SERVING['rate']}/s for {seconds} s, {len(arrivals)} requests cycling "
                     f"{pool_size} instances (S-curve m=256 s=128 tau=1e-5 / MNIST-shaped m=256 s=128 tau=1e-4, "
                     f"N log-uniform in [4096, 65536]), r={synth.SERVING['r']}, rel. residual {synth.SERVING['tol']}",
           "pool_n": [q["n"] for q in pool], "pool_family": [q["family"] for q in pool]}
    results = {}
    for name, (near, far) in synth.SERVING_PATHS.items():
        log(f"[bench] serving path {name} ({near} near, {far} far), {len(arrivals)} requests")
        st, res = serving_leg(hdm, pool, arrivals, near, far)
        entry = {k: st[k] for k in keep}
        entry["tiles"] = f"near {near}, far {far}"
        cap = st["solves_per_s"]
        if cap < 0.9 * synth.SERVING["rate"] or st["mean_service_s"] > 0.05:
            rate = 0.8 * cap
            low = synth.configs.serving_arrivals(seconds, rate=rate)
            log(f"[bench] serving path {name}: capacity {cap:.1f}/s below the offered rate; replay at {rate:.1f}/s")
            st2, res = serving_leg(hdm, pool, low, near, far)
            entry["at_80pct_capacity"] = dict({k: st2[k] for k in keep}, rate=rate)
        results[name] = res
        out[name] = entry
    # the same requests on both paths: eigenvalues of the mixed path against plain float32
    if len(results.get("mixed", [])) == len(results.get("plain_f32", [])):
        worst = 0.0
        for a, b in zip(results["mixed"], results["plain_f32"]):
            if a["status"] == 0 and b["status"] == 0:
                worst = max(worst, float(np.max(np.abs(a["evals"] - b["evals"]) / np.abs(b["evals"]))))
        out["mixed_vs_f32_max_rel_eig_diff"] = worst
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scurve-100k")
    ap.add_argument("--matvec-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run one plain 1 GiB device copy (counter scale)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="length of each serving stream (0: skip)")
    ap.add_argument("--serve-pool", type=int, default=8, help="distinct request instances the stream cycles through")
    ap.add_argument("--rhs", type=int, default=0,
                    help="also time one product of K~ with this many right-hand sides (16 per pass)")
    ap.add_argument("--thrash-mib", type=int, default=0,
                    help="also time the standalone product with this many MiB evicted from the caches between "
                         "products (once by a write, once by a read)")
    args = ap.parse_args()
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
              far_prec=cfg["far_prec"], ctx=ctx, budget=cfg.get("budget", 0.05))
    tol = 1e-10

    def step():
        op = hdm.Operator(Xd, eps, **kw)
        ev, _, info, st = op.eigs(r, tol=tol, block=block, seed=cfg["seed"], vectors=True)
        op.close()
        return ev, info, st

    log(f"[bench] {args.workload}: warm-up")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat = []
    # inside the timed region only the near-field kernel is timed (HIP events on its
    # stream, for the roofline); the per-phase breakdown comes from one more step below
    ctx.profile(True, phases=["l2l"])
    torch.cuda.synchronize()
    log(f"[bench] {args.workload}: {args.steps} timed steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        ev, info, st = step()
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
    thrash = None
    if args.thrash_mib > 0:
        # M MiB touched between products evict the last-level cache (256 MiB): by a
        # write (its dirty lines are written back while the product runs) and by a
        # read (clean eviction: the product starts from a cold cache)
        junk = torch.empty(args.thrash_mib << 17, dtype=torch.float64, device=dev)
        junk.fill_(1.0)
        thrash = {"mib_between_products": args.thrash_mib}
        for mode in ("write", "read"):
            times = []
            for i in range(args.matvec_reps):
                if mode == "write":
                    junk.fill_(float(i))
                else:
                    junk.sum()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                op.matvec(x, normalised=True)
                b.record()
                torch.cuda.synchronize()
                times.append(a.elapsed_time(b) / 1e3)
            t_med = float(np.median(times))
            thrash[mode] = {"us_per_call_median": t_med * 1e6, "GBps": st_op.algo_bytes_matvec / t_med / 1e9,
                            "frac_hbm": st_op.algo_bytes_matvec / t_med / 1e9 / HBM_PEAK_GBS}
        del junk
    multi = None
    if args.rhs > 0:
        # the scaling study's evaluation: K~ times args.rhs right-hand sides
        Wm = torch.randn(X.shape[0], args.rhs, dtype=torch.float64, device=dev)
        op.matvec(Wm)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            op.matvec(Wm)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) / 1e3)
        t_med = float(np.median(times))
        passes = (args.rhs + 15) // 16
        multi = {"rhs": args.rhs, "s_per_product": t_med, "ms_per_rhs": t_med * 1e3 / args.rhs,
                 "passes_of_16": passes,
                 "GBps_near_tiles": st_op.near_tile_bytes * passes / t_med / 1e9,
                 "what": "K~ times the right-hand sides (not normalised), median of 3"}
        del Wm
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

    # the near-field launches of the timed region: block products of `block` right-hand sides
    # (float16 tiles on the matrix cores) or single-column products with the leaf level of the
    # upward pass; algorithmic bytes = unpadded tiles once + the input and output vectors
    l2l_n, l2l_ms = phases["l2l"]
    l2l_avg_s = l2l_ms / 1e3 / max(l2l_n, 1)
    nrhs = block
    ev_bytes = 4 if cfg["near_prec"] != "f64" else 8
    if nrhs == 1:
        algo_near = st_op.algo_bytes_near
        kname = "near field (k_l2l, with the leaf level of the upward pass), one right-hand side"
    else:
        algo_near = st_op.near_tile_bytes + 2 * nrhs * X.shape[0] * ev_bytes
        kname = (f"near field ({'k_l2l_mma, float16 tiles on the matrix cores' if cfg['near_prec'] == 'f16' else 'k_l2l'}"
                 f"), {nrhs} right-hand sides")
    achieved = algo_near / l2l_avg_s / 1e9
    near_flops = 2.0 * st_op.near_elems * nrhs
    src_sha = hashlib.sha1(open(os.path.join(ROOT, "paper_2311_06115_amd", "csrc", "evaluate.hip"), "rb").read()).hexdigest()
    traffic = pmc_traffic(args.workload, src_sha)
    serve = None
    if args.serve_seconds > 0:
        serve = serving(hdm, args.serve_seconds, args.serve_pool)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] oracle sample on the host")
        cpu = cpu_baseline(X, eps, int(info.matvecs) + 2)
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
        "dtype": f"{cfg['near_prec']} near / {cfg['far_prec']} far tiles, f32 accumulation, f64 Lanczos",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['family']} N={cfg['n']} D={cfg['dim']}, m={cfg['m']}, "
                               f"s={cfg['s']}, tau={cfg['tau']}, k={cfg['k']}, {cfg['near_prec']} near / "
                               f"{cfg['far_prec']} far tiles, r={r} eigenpairs, "
                               f"{'block Lanczos b=%d' % block if block > 1 else 'Lanczos'}, rel. residual {tol}",
                   "n": cfg["n"], "eps": eps, "lanczos_steps": int(info.iters), "operator_applications":
                   int(info.matvecs), "status": int(st)},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "hmatvec": {"us_per_call": mv_s * 1e6, "algo_bytes": st_op.algo_bytes_matvec,
                    "GBps": st_op.algo_bytes_matvec / mv_s / 1e9,
                    "frac_hbm": st_op.algo_bytes_matvec / mv_s / 1e9 / HBM_PEAK_GBS,
                    "what": "one single-column normalised product, standalone, 50 back to back",
                    "near_bytes": st_op.algo_bytes_near, "resident_bytes": st_op.bytes_total,
                    "depth": st_op.depth, "mean_leaf_rank": st_op.mean_leaf_rank, "max_rank": st_op.max_rank,
                    "near_pairs": st_op.near_pairs, "far_pairs": st_op.far_pairs, "cache_thrash": thrash},
        "phase_ms_per_step": {k: v[1] for k, v in breakdown.items()},   # one extra step, every phase timed
        "phase_launches_per_step": {k: v[0] for k, v in breakdown.items()},
        "eigenvalue_accuracy": ev_acc,
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_us": l2l_avg_s * 1e6, "launches": int(l2l_n),
                     "algo_bytes_per_launch": algo_near,
                     "mfma_tflops": near_flops / l2l_avg_s / 1e12,
                     "mfma_frac_f16_peak": near_flops / l2l_avg_s / 1e12 / MFMA_F16_PEAK_TFLOPS},
        "multi_rhs": multi,
        "serving": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
