"""Benchmark: ms per low-rank Poisson solve at n = 65535 (rank-20 RHS, rank cap 64).

One step = one whole solve (DST of the factors, warm start, every Cross-DEIM pass until the
stopping test, final truncation and DST back) on seeded synthetic input already resident in
HBM. The headline `value` is the mixed-precision path (FP32 DSTs and fibers, FP64 QR, core and
stopping test); the FP64 path is timed beside it. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--served", type=int, default=2000, help="requests in the served stream (0: skip)")
    ap.add_argument("--served-active", type=int, default=8)
    ap.add_argument("--served-budget-gb", type=float, default=64.0)
    return ap.parse_args()


def time_solves(sol, args_dev, steps, warmup):
    import torch

    for _ in range(warmup):
        sol.solve(*args_dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        _, _, _, r, info = sol.solve(*args_dev)
        infos.append(info.as_dict())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall * 1e3 / steps, infos


def dst_roofline(sol, n, ncols, reps=20):
    """Live HIP-event timing of the batched DST-I (FP64) on an n x ncols matrix."""
    import torch

    from paper_2607_06021_amd import fortran

    X = fortran(torch.randn(n, ncols, dtype=torch.float64, device="cuda"))
    for _ in range(3):
        sol.dst1(X)
    stream = sol.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sol.dst1(X)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bytes_alg = 2.0 * n * ncols * 8
    gbs = bytes_alg / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "dst1 (pass1+pass2)",
            "ms_per_launch": round(ms, 4), "alg_bytes_per_launch": bytes_alg}


def served_leg(count, seed, budget_gb, max_active, rate=None):
    """Served stream: saturated throughput, then Poisson arrivals at 70% of it (p50/p99)."""
    import numpy as np
    import torch

    import workloads
    from paper_2607_06021_amd.lrp import Server

    dev = torch.device("cuda:0")
    probe = workloads.served_stream(count=count, rate_per_s=1.0, seed=seed)
    log(f"served: generating {count} right-hand sides on the device")
    inputs = [workloads.bump_rhs_device(r.n, r.seed, r.rank, 0.05, 0.2, dev) for r in probe]
    torch.cuda.synchronize()

    def run(reqs, rate_s):
        with Server(budget_bytes=int(budget_gb * (1 << 30)), max_active=max_active) as srv:
            t0 = time.perf_counter()
            tickets = []
            for r in reqs:
                if rate_s is not None:
                    due = t0 + r.arrival_s
                    while time.perf_counter() < due:
                        pass
                U, sg, V = inputs[r.idx]
                tickets.append(srv.submit(r.n, U, sg, V, 48, 1e-10, 20, r.precision, sync=False))
            res = [srv.wait(t) for t in tickets]
            wall = time.perf_counter() - t0
            st = srv.stats()
        lat = np.array([x[6] for x in res])
        bad = sum(1 for x in res if x[4] < 0)
        return wall, lat, bad, st

    # warm the contexts of every shape once, then measure the saturated rate
    nsat = min(count, 400)
    run(probe[: min(count, 40)], None)
    wall, lat, bad, _ = run(probe[:nsat], None)
    sat = nsat / wall
    use_rate = rate if rate is not None else 0.7 * sat
    reqs = workloads.served_stream(count=count, rate_per_s=use_rate, seed=seed)
    log(f"served: saturated {sat:.1f} solves/s; Poisson arrivals at {use_rate:.1f}/s")
    wall, lat, bad, st = run(reqs, use_rate)
    return {"requests": count, "arrival_rate_per_s": round(use_rate, 2), "saturated_solves_per_s": round(sat, 2),
            "solves_per_s": round(count / wall, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "failed": int(bad),
            "mix": "n in {1023,4095,16383,65535,262143} w.p. .3/.3/.2/.15/.05, rank U{2..20}, cap 48, "
                   "FP64 or mixed w.p. 0.5", "max_active": max_active, "contexts": st["contexts"]}


def cpu_baseline(w, U, s, V):
    import threadpoolctl

    from oracle import crossdeim as cd

    with threadpoolctl.threadpool_limits(limits=None):
        info = threadpoolctl.threadpool_info()
    threads = max([d.get("num_threads", 1) for d in info] + [1])
    t0 = time.perf_counter()
    o = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    sec = time.perf_counter() - t0
    return o, {"value": round(sec * 1e3, 1), "unit": "ms/solve", "cores": threads, "kind": "oracle",
               "sample": f"one full FP64 solve of the same workload (seed 0, {o.iters} passes)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads
    from paper_2607_06021_amd import Solver, fortran

    w64 = workloads.CONFIGS["n65535_r20_fp64"]
    wmx = workloads.CONFIGS["n65535_r20_mixed"]
    U, s, V = workloads.make(w64, args.seed)
    dev = torch.device("cuda:0")
    args_dev = (fortran(torch.from_numpy(U).to(dev)), torch.from_numpy(s).to(dev),
                fortran(torch.from_numpy(V).to(dev)))
    results = {}
    outs = {}
    for prec, w in (("mixed", wmx), ("fp64", w64)):
        if args.precision not in ("both", prec):
            continue
        log(f"timing {prec}: n={w.n} r_max={w.r_max} steps={args.steps} warmup={args.warmup}")
        sol = Solver(w.n, w.r_max, w.tol, maxiter=w.maxiter, precision=prec)
        ms, infos = time_solves(sol, args_dev, args.steps, args.warmup)
        Uo, So, Vo, r, info = sol.solve(*args_dev)
        outs[prec] = (Uo[:, :r].cpu().numpy(), So[:r].cpu().numpy(), Vo[:, :r].cpu().numpy())
        results[prec] = {"ms": ms, "info": info.as_dict(), "dev_ms": float(np.median([i["ms"] for i in infos]))}
        if prec == "fp64":
            results["roofline"] = dst_roofline(sol, w.n, w.r_max)
        sol.close()
        log(f"  {prec}: {ms:.3f} ms/solve (device {results[prec]['dev_ms']:.3f} ms) "
            f"iters {info.iters} rank {info.rank} status {info.status}")
    served = None
    if args.served > 0:
        served = served_leg(args.served, 2026, args.served_budget_gb, args.served_active)
        log(f"  served: p50 {served['p50_ms']} ms, p99 {served['p99_ms']} ms, {served['solves_per_s']} solves/s")
    cpu = None
    err = {}
    if not args.no_cpu_baseline:
        from oracle import crossdeim as cd

        log("cpu baseline: oracle solve")
        o, cpu = cpu_baseline(w64, U, s, V)
        for prec, f in outs.items():
            err[prec] = cd.rel_err(f, (o.U, o.S, o.V))
    if "mixed" in outs and "fp64" in outs:
        from oracle import crossdeim as cd

        err["mixed_vs_fp64_gpu"] = cd.rel_err(outs["mixed"], outs["fp64"])
    head = "mixed" if "mixed" in results else "fp64"
    line = {
        "metric": "ms/solve at n=65535 r<=64, FP64 vs mixed; HBM GB/s; served p50/p99 latency",
        "value": round(results[head]["ms"], 4),
        "unit": "ms/solve",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(results[head]["ms"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"Poisson n=65535 (h=1/65536), rank-20 Gaussian-bump RHS (seed {args.seed}), "
                               f"rank cap 64, tol 1e-10, {head} precision",
                   "precision": head},
        "fp64_ms_per_solve": round(results["fp64"]["ms"], 4) if "fp64" in results else None,
        "mixed_ms_per_solve": round(results["mixed"]["ms"], 4) if "mixed" in results else None,
        "mixed_speedup": (round(results["fp64"]["ms"] / results["mixed"]["ms"], 3)
                          if "fp64" in results and "mixed" in results else None),
        "passes": {p: results[p]["info"]["iters"] for p in ("mixed", "fp64") if p in results},
        "rank": {p: results[p]["info"]["rank"] for p in ("mixed", "fp64") if p in results},
        "rel_err_vs_oracle": {k: float(f"{v:.3e}") for k, v in err.items()},
        "served_p50_ms": served["p50_ms"] if served else None,
        "served_p99_ms": served["p99_ms"] if served else None,
        "served": served,
        "roofline": results.get("roofline"),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
