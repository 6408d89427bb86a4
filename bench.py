"""Benchmark: ms per low-rank Poisson solve at n = 65535 (rank-20 RHS, rank cap 64).

One step = one whole solve (DST of the factors, warm start, every Cross-DEIM pass until the
stopping test, final truncation and DST back) on seeded synthetic input already resident in
HBM. The headline `value` is the mixed-precision path (FP32 DSTs and fibers, FP64 QR, core and
stopping test); the FP64 path is timed beside it. Also reported: a measured device copy rate,
both precisions at n = 2^20 - 1 (rank-30 RHS) with the streaming kernels' rooflines and the
error against the oracle's stored sketches, and a served stream of mixed sizes (p50/p99 from
the scheduled arrival, by size, queue wait versus run). Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--large-steps L] [--served R]
                    [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import gc
import json
import math
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
    ap.add_argument("--large-steps", type=int, default=4,
                    help="timed solves per precision at n = 2^20 - 1 (0: skip that leg)")
    ap.add_argument("--served", type=int, default=2000, help="requests in the served stream (0: skip)")
    ap.add_argument("--served-active", type=int, default=32)
    ap.add_argument("--served-budget-gb", type=float, default=192.0)
    ap.add_argument("--served-compare-active", type=int, default=8,
                    help="also measure the saturated rate at this many active requests, grouping on and off "
                         "(0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="copy one 256 MiB device tensor and exit (calibrates the HBM byte counters)")
    return ap.parse_args()


def copy_probe():
    """A plain device copy of known size: 256 MiB read and 256 MiB written."""
    import torch

    a = torch.ones(2 ** 25, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: {a.numel() * 8} bytes copied")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from a committed rocprofv3 counter summary
    (profiles/*_traffic.md), or None if there is none or its kernel sources changed since the
    counters were taken."""
    import glob
    import hashlib

    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        fields = {}
        for line in open(path):
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                fields[k] = v
        if fields.get("kernel") != kernel or fields.get("workload") != workload:
            continue
        h = hashlib.sha256()
        for src in fields.get("sources", "").split():
            try:
                with open(os.path.join(ROOT, src), "rb") as f:
                    h.update(f.read())
            except OSError:
                return None
        if h.hexdigest() != fields.get("source_sha256"):
            return None
        return int(fields["hbm_bytes_per_launch"])
    return None


def time_solves(sol, args_dev, steps, warmup):
    import numpy as np
    import torch
    from paper_2607_06021_amd.lrp import empty_fortran

    # output buffers allocated once, as a caller solving many right-hand sides would
    dev = args_dev[0].device
    out = (empty_fortran(sol.n, sol.r_max, torch.float64, dev),
           torch.empty(sol.r_max, dtype=torch.float64, device=dev),
           empty_fortran(sol.n, sol.r_max, torch.float64, dev))
    # Python's cyclic garbage collector is paused over the warm-up and the timed loop (as timeit
    # does): a full collection with torch loaded takes tens of milliseconds and otherwise lands on
    # one solve. It runs before the warm-up, so the device is busy right up to the timed loop.
    gc.collect()
    gc.disable()
    try:
        for _ in range(warmup):
            sol.solve(*args_dev, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        marks = []
        for _ in range(steps):
            _, _, _, r, info = sol.solve(*args_dev, out=out)
            infos.append(info)
            marks.append(time.perf_counter())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gc.enable()
    infos = [i.as_dict() for i in infos]
    per = np.diff([t0] + marks) * 1e3  # each solve returns after its device work has finished
    log(f"  per-solve wall ms: min {per.min():.3f} median {np.median(per):.3f} max {per.max():.3f} "
        f"(slowest: solve {int(per.argmax())})")
    return wall * 1e3 / steps, infos


# MI355X published peaks
FP64_PEAK_TFLOPS = 78.6


def profile_solve(w, prec, args_dev):
    """One solve in profile mode: per-kernel device time from HIP events recorded around every
    launch on the solve's stream, plus the pass sizes needed for the algorithmic counts."""
    from paper_2607_06021_amd import Solver

    with Solver(w.n, w.r_max, w.tol, maxiter=w.maxiter, precision=prec, profile=True) as sol:
        sol.solve(*args_dev)  # warm
        _, _, _, r, info = sol.solve(*args_dev)
        prof = sol.profile()
        trace = sol.trace()
    return prof, trace, info


def kernel_model(w, prec, trace, info, rF):
    """Algorithmic bytes and flops of each kernel class over one solve (what the method must
    move or compute; counted from the pass sizes of the trace)."""
    n = w.n
    wb = 4 if prec == "mixed" else 8           # width of the spectral factors and fibers
    r = info.rank
    passes = trace                              # passes actually computed
    out = {}
    # DST: forward U_F, V_F (read FP64, write w); back: read and write the rank live columns
    # (the zero fill of the r_max - r unused output columns is not counted)
    out["dst"] = {"bytes": 2 * n * rF * (8 + wb) + 2 * (2 * n * r * 8)}
    fb = 0
    pb = 0
    pf = 0
    cf = 0.0
    for t in passes:
        pI, pJ = len(t["I_pre"]), len(t["J_pre"])
        rk = t["rank"]
        fb += 2 * n * rF * wb + n * (pI + pJ) * wb + 2 * n * wb
        pb += n * (pI + pJ) * 8 + 2 * n * rk * 8
        pf += 2 * n * (pI + pJ) * rk
        # core: Householder QR of the m0 x k0 interpolation rows, triangular inverse, the core
        # product, the SVD of the |J| x |I| core (Golub-Van Loan count 4m^2n + 8mn^2 + 9n^3) and,
        # when the indicator was evaluated, two singular-value-only SVDs (4mn^2 - 4n^3/3)
        m0, k0 = max(pI, pJ), min(pI, pJ)
        mm, kk = max(pI, pJ), min(pI, pJ)
        cf += 2 * m0 * k0 ** 2 - 2 * k0 ** 3 / 3 + k0 ** 3 / 3 + 2 * pI * pJ * k0
        cf += 4 * mm ** 2 * kk + 8 * mm * kk ** 2 + 9 * kk ** 3
        if math.isfinite(t["indicator"]):
            for a, b in ((t["nI"], rk), (t["nJ"], rk)):
                a, b = max(a, b), min(a, b)
                cf += 4 * a * b * b - 4 * b ** 3 / 3
    out["fiber"] = {"bytes": fb}
    pb += 2 * (n * rF * 8 + n * rF * 8)       # warm start: U_-1 = Q U^, V_-1 = Z V~ (rank <= r_F)
    pf += 2 * 2 * n * rF * rF
    out["prod"] = {"bytes": pb, "flops": pf}
    out["core"] = {"flops": cf}
    # thin QRs (Householder, LAPACK counts): factorization 2 n p^2 - 2 p^3 / 3 per side and the
    # same again to form the explicit Q; the warm start factors U^, V^ (p = r_F)
    qf = 2 * (2 * n * rF ** 2 - 2 * rF ** 3 / 3)
    for t in passes:
        for pp in (len(t["I_pre"]), len(t["J_pre"])):
            qf += 2 * n * pp ** 2 - 2 * pp ** 3 / 3
    out["tsqr"] = {"flops": qf}
    # rho (passes where it was evaluated): M = A^T B (pass a), then Y = B - A M and Y^T Y (pass b)
    ra = rb = 0.0
    prev = None
    for t in passes:
        rk = t["rank"]
        if prev is not None and math.isfinite(t["rho"]):
            ra += 2 * 2 * n * rk * prev
            rb += 2 * (2 * n * rk * prev + 2 * n * prev * prev)
        prev = rk
    out["rho_a"] = {"flops": ra}
    out["rho_b"] = {"flops": rb}
    return out


def rooflines(w, prec, prof, trace, info, rF):
    """Roofline per kernel class over one profiled solve: total algorithmic bytes (flops) of
    the class divided by its total device time (HIP events); launches that found the solve
    already finished count in the time, not in the work."""
    m = kernel_model(w, prec, trace, info, rF)

    def t(*names):
        return (sum(prof.get(nm, (0, 0.0))[1] for nm in names),
                max([prof.get(nm, (0, 0.0))[0] for nm in names]))

    def hbm(bytes_, ms, launches, kernel):
        gbs = bytes_ / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kernel,
                "ms_per_launch": round(ms / max(launches, 1), 5), "launches": launches,
                "alg_bytes_per_launch": round(bytes_ / max(launches, 1))}

    res = {"dst": hbm(m["dst"]["bytes"], *t("k_dst_pass1", "k_dst_pass2", "k_dst_single"),
                      "k_dst_pass1 + k_dst_pass2 (four-step), or k_dst_single"),
           "fiber": hbm(m["fiber"]["bytes"], *t("k_fiber"), "k_fiber"),
           "prod": hbm(m["prod"]["bytes"], *t("k_prod"), "k_prod (FP64 MFMA)")}
    def alu(flops, ms, launches, kernel):
        tf = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        return {"bound": "alu", "achieved": round(tf, 6), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tf / FP64_PEAK_TFLOPS, 7), "traffic": None, "kernel": kernel,
                "ms_per_launch": round(ms / max(launches, 1), 5), "launches": launches,
                "alg_flops_per_launch": round(flops / max(launches, 1))}

    res["core"] = alu(m["core"]["flops"], *t("k_core"), "k_core (one workgroup)")
    # the factorization and the formation of Q each carry the Householder count
    res["tsqr_factor"] = alu(m["tsqr"]["flops"], *t("k_tsqr_factor"), "k_tsqr_factor (all tree levels)")
    res["tsqr_apply"] = alu(m["tsqr"]["flops"], *t("k_tsqr_apply"), "k_tsqr_apply (all tree levels)")
    res["rho_a"] = alu(m["rho_a"]["flops"], *t("k_rho_a"), "k_rho_a")
    res["rho_b"] = alu(m["rho_b"]["flops"], *t("k_rho_b"), "k_rho_b")
    return res


def saturated_rates(inputs, probe, budget_gb, max_active):
    """Saturated solve rate of the first 400 requests of the stream (all submitted at once) with
    same-stage grouping on, off, and on again, every shape warmed first in each setting; the
    mean group size is request passes per pass launch."""
    import numpy as np

    from paper_2607_06021_amd.lrp import Server

    nsat = min(len(probe), 400)
    out = {}
    with Server(budget_bytes=int(budget_gb * (1 << 30)), max_active=max_active) as srv:
        def run(reqs):
            t0 = time.perf_counter()
            ts = [srv.submit(r.n, *inputs[r.idx], 48, 1e-10, 20, r.precision, sync=False) for r in reqs]
            res = [srv.wait(t) for t in ts]
            return time.perf_counter() - t0, res

        shapes = {}
        for r in probe:
            shapes.setdefault((r.n, r.precision), []).append(r)
        rates = {True: [], False: []}
        for grouping in (True, False, True):
            srv.set_grouping(grouping)
            for rs in shapes.values():
                run((rs * max_active)[:max_active])
            st0 = srv.stats()
            wall, res = run(probe[:nsat])
            st = srv.stats()
            rates[grouping].append(nsat / wall)
            if grouping:
                out["mean_group_size"] = round((st["passes"] - st0["passes"]) /
                                               max(1, st["pass_launches"] - st0["pass_launches"]), 2)
            out["run_p50_ms_grouping_" + ("on" if grouping else "off")] = round(
                float(np.median([x[8] for x in res])), 3)
    out["solves_per_s_grouping_on"] = round(float(np.mean(rates[True])), 1)
    out["solves_per_s_grouping_off"] = round(float(np.mean(rates[False])), 1)
    out["max_active"] = max_active
    return out


def served_leg(count, seed, budget_gb, max_active, rate=None, compare_active=0):
    """Served stream through one Server kept open throughout: first every shape of the stream
    is warmed (max_active requests of each at once, so the contexts the measurement needs
    exist), then the saturated rate is measured, then Poisson arrivals at 70% of it. Latency
    runs from each request's scheduled arrival time to its completion; it is reported overall,
    by grid size, and split into the wait for admission and the run after it. Then the saturated
    rate with same-stage grouping on and off, at max_active and at compare_active requests."""
    import numpy as np
    import torch

    import workloads
    from paper_2607_06021_amd.lrp import Server

    dev = torch.device("cuda:0")
    torch.cuda.empty_cache()  # the contexts are device allocations of their own
    probe = workloads.served_stream(count=count, rate_per_s=1.0, seed=seed)
    log(f"served: generating {count} right-hand sides on the device")
    inputs = [workloads.bump_rhs_device(r.n, r.seed, r.rank, 0.05, 0.2, dev) for r in probe]
    torch.cuda.synchronize()

    def pct(x, q):
        return round(float(np.percentile(x, q)), 3) if len(x) else None

    with Server(budget_bytes=int(budget_gb * (1 << 30)), max_active=max_active) as srv:
        def run(reqs, rate_s):
            t0 = time.perf_counter()
            tickets, late = [], []
            for r in reqs:
                due = t0 + (r.arrival_s if rate_s is not None else 0.0)
                if rate_s is not None:
                    while time.perf_counter() < due:
                        pass
                late.append(max(0.0, time.perf_counter() - due) * 1e3)
                U, sg, V = inputs[r.idx]
                tickets.append(srv.submit(r.n, U, sg, V, 48, 1e-10, 20, r.precision, sync=False))
            res = [srv.wait(t) for t in tickets]
            wall = time.perf_counter() - t0
            return wall, res, np.array(late)

        # warm every (n, precision) shape: max_active requests of it in flight together
        shapes = {}
        for r in probe:
            shapes.setdefault((r.n, r.precision), []).append(r)
        for rs in shapes.values():
            run((rs * max_active)[:max_active], None)
        ctx0 = srv.stats()["contexts"]
        nsat = min(count, 400)
        wall, _, _ = run(probe[:nsat], None)
        sat = nsat / wall
        use_rate = rate if rate is not None else 0.7 * sat
        reqs = workloads.served_stream(count=count, rate_per_s=use_rate, seed=seed)
        log(f"served: {ctx0} contexts warm; saturated {sat:.1f} solves/s; Poisson arrivals at {use_rate:.1f}/s")
        st0 = srv.stats()
        wall, res, late = run(reqs, use_rate)
        st = srv.stats()
    grouping = {"mean_group_size_poisson": round((st["passes"] - st0["passes"]) /
                                                 max(1, st["pass_launches"] - st0["pass_launches"]), 2),
                "saturated": [saturated_rates(inputs, probe, budget_gb, max_active)]}
    if compare_active:
        grouping["saturated"].append(saturated_rates(inputs, probe, budget_gb, compare_active))
    for g in grouping["saturated"]:
        log(f"served: saturated at {g['max_active']} active: {g['solves_per_s_grouping_on']} solves/s grouped "
            f"(mean group {g['mean_group_size']}), {g['solves_per_s_grouping_off']} ungrouped")
    lat = late + np.array([x[6] for x in res])           # from the scheduled arrival
    queue = late + np.array([x[7] for x in res])         # arrival to admission
    runms = np.array([x[8] for x in res])                # admission to completion
    bad = [(r.idx, r.n, r.rank, r.precision, int(x[4])) for r, x in zip(reqs, res) if x[4] < 0]
    by_n = {}
    for nn in sorted({r.n for r in reqs}):
        sel = np.array([r.n == nn for r in reqs])
        by_n[str(nn)] = {"requests": int(sel.sum()), "p50_ms": pct(lat[sel], 50), "p99_ms": pct(lat[sel], 99),
                         "run_p50_ms": pct(runms[sel], 50), "run_p99_ms": pct(runms[sel], 99),
                         "queue_p99_ms": pct(queue[sel], 99)}
    return {"requests": count, "arrival_rate_per_s": round(use_rate, 2), "saturated_solves_per_s": round(sat, 2),
            "solves_per_s": round(count / wall, 2), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
            "latency_from": "scheduled arrival",
            "queue_p50_ms": pct(queue, 50), "queue_p99_ms": pct(queue, 99),
            "run_p50_ms": pct(runms, 50), "run_p99_ms": pct(runms, 99),
            "submit_lateness_p99_ms": pct(late, 99), "by_n": by_n, "failed": len(bad),
            "failures": [{"request": i, "n": nn, "rank": rk, "precision": pr, "status": stt}
                         for i, nn, rk, pr, stt in bad[:10]],
            "mix": "n in {1023,4095,16383,65535,262143} w.p. .3/.3/.2/.15/.05, rank U{2..20}, cap 48, "
                   "FP64 or mixed w.p. 0.5", "max_active": max_active, "contexts_warm": ctx0,
            "contexts_after": st["contexts"], "grouping": grouping}


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


def dominant_roofline(res, workload):
    """Roofline of the kernel with the largest device time in the profiled solve; `traffic` is
    the kernel's measured HBM bytes per launch where a current counter summary exists."""
    key = {"k_core": "core", "k_dst_pass1": "dst", "k_dst_pass2": "dst", "k_dst_single": "dst",
           "k_fiber": "fiber", "k_prod": "prod", "k_tsqr_factor": "tsqr_factor",
           "k_tsqr_apply": "tsqr_apply", "k_rho_a": "rho_a", "k_rho_b": "rho_b"}.get(res["dominant"])
    if key is None:
        return {"bound": "alu", "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": None, "kernel": res["dominant"], "note": "no algorithmic model for this kernel"}
    r = dict(res["rooflines"][key])
    r["traffic"] = measured_traffic(res["dominant"], workload)
    r["share_of_solve"] = res["profile"][res["dominant"]]["share"]
    return r


def copy_bandwidth():
    """Measured device-to-device copy rate (read + write bytes per second) of a 2 GiB tensor:
    the practical HBM ceiling the streaming kernels are compared with."""
    import numpy as np
    import torch

    a = torch.ones(2 ** 28, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    times = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    gbs = 2 * a.numel() * 8 / (float(np.median(times)) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return round(gbs, 1)


def run_leg(w, prec, args_dev, steps, warmup, rF):
    """Time `steps` solves of workload `w` (after `warmup`), then profile one solve."""
    import numpy as np

    from paper_2607_06021_amd import Solver

    log(f"timing {w.name} {prec}: n={w.n} r_max={w.r_max} steps={steps} warmup={warmup}")
    sol = Solver(w.n, w.r_max, w.tol, maxiter=w.maxiter, precision=prec)
    ms, infos = time_solves(sol, args_dev, steps, warmup)
    Uo, So, Vo, r, info = sol.solve(*args_dev)
    out = (Uo[:, :r].cpu().numpy(), So[:r].cpu().numpy(), Vo[:, :r].cpu().numpy())
    res = {"ms": ms, "info": info.as_dict(), "dev_ms": float(np.median([i["ms"] for i in infos]))}
    sol.close()
    del Uo, So, Vo
    prof, trace, pinfo = profile_solve(w, prec, args_dev)
    # the profile opens with empty calibration launches (the floor of a dispatch's duration);
    # they are reported but are not part of the solve
    total = sum(v for k, (_, v) in prof.items() if k != "empty kernel")
    res["profile"] = {k: {"launches": v[0], "ms": round(v[1], 4),
                          "share": None if k == "empty kernel" else round(v[1] / total, 4)}
                      for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    res["rooflines"] = rooflines(w, prec, prof, trace, pinfo, rF)
    res["dominant"] = max(((k, v) for k, v in prof.items() if k != "empty kernel"), key=lambda kv: kv[1][1])[0]
    log(f"  {prec}: {ms:.3f} ms/solve (device {res['dev_ms']:.3f} ms) "
        f"iters {info.iters} rank {info.rank} status {info.status}")
    return res, out


def device_inputs(w, seed):
    import torch

    import workloads
    from paper_2607_06021_amd import fortran

    U, s, V = workloads.make(w, seed)
    dev = torch.device("cuda:0")
    return (U, s, V), (fortran(torch.from_numpy(U).to(dev)), torch.from_numpy(s).to(dev),
                       fortran(torch.from_numpy(V).to(dev)))


def large_leg(args):
    """n = 2^20 - 1, rank-30 RHS, both precisions: time per solve, the streaming kernels'
    rooflines, and the error against the oracle through its stored Gaussian sketches."""
    import numpy as np
    import torch

    import workloads

    gold_path = os.path.join(ROOT, "tests", "golden", "n1048575_r30_fp64_seed0.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else None
    w64 = workloads.CONFIGS["n1048575_r30_fp64"]
    wmx = workloads.CONFIGS["n1048575_r30_mixed"]
    (U, s, V), args_dev = device_inputs(w64, 0)
    rF = U.shape[1]
    del U, s, V
    out = {}
    outs = {}
    for prec, w in (("fp64", w64), ("mixed", wmx)):
        if args.precision not in ("both", prec):
            continue
        res, o = run_leg(w, prec, args_dev, args.large_steps, 1, rF)
        outs[prec] = o
        e = None
        if gold is not None:
            e = sketched_rel_err(w.n, o[0], o[1], o[2], gold)
        out[prec] = {"ms_per_solve": round(res["ms"], 3), "device_ms": round(res["dev_ms"], 3),
                     "passes": res["info"]["iters"], "rank": res["info"]["rank"], "status": res["info"]["status"],
                     "sketched_rel_err_vs_oracle": float(f"{e:.3e}") if e is not None else None,
                     "dominant": res["dominant"],
                     "rooflines": {k: res["rooflines"][k] for k in ("dst", "fiber", "prod")},
                     "profile": dict(list(res["profile"].items())[:8])}
    del args_dev
    torch.cuda.empty_cache()
    out["workload"] = ("Poisson n=1048575 (h=2^-20), rank-30 Gaussian-bump RHS (seed 0), rank cap 64, tol 1e-10")
    out["mixed_speedup"] = (round(out["fp64"]["ms_per_solve"] / out["mixed"]["ms_per_solve"], 3)
                            if "fp64" in out and "mixed" in out else None)
    return out


def sketched_rel_err(n, U, S, V, gold):
    """Relative Frobenius error of U diag(S) V^T against the oracle's solution, estimated through
    the Gaussian sketches stored with it (Om^T U_o diag(S_o), Om'^T V_o; the seeds give Om, Om')."""
    import numpy as np

    import workloads

    k = gold["sketch_k"]
    Om = workloads.sketch_matrix(n, k, gold["sketch_seeds"][0])
    A = Om.T @ (U * S[None, :])
    del Om
    Om = workloads.sketch_matrix(n, k, gold["sketch_seeds"][1])
    B = Om.T @ V
    del Om
    ref = np.array(gold["sketch_U"]) @ np.array(gold["sketch_V"]).T
    return float(np.linalg.norm(A @ B.T - ref) / np.linalg.norm(ref))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU per process; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    import workloads

    w64 = workloads.CONFIGS["n65535_r20_fp64"]
    wmx = workloads.CONFIGS["n65535_r20_mixed"]
    (U, s, V), args_dev = device_inputs(w64, args.seed)
    results = {}
    outs = {}
    for prec, w in (("mixed", wmx), ("fp64", w64)):
        if args.precision not in ("both", prec):
            continue
        results[prec], outs[prec] = run_leg(w, prec, args_dev, args.steps, args.warmup, U.shape[1])
    copy_gbs = copy_bandwidth()
    log(f"  device copy: {copy_gbs} GB/s")
    large = None
    if args.large_steps > 0:
        large = large_leg(args)
    served = None
    if args.served > 0:
        served = served_leg(args.served, 2026, args.served_budget_gb, args.served_active,
                            compare_active=args.served_compare_active)
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
        "copy_gbs": copy_gbs,
        "served_p50_ms": served["p50_ms"] if served else None,
        "served_p99_ms": served["p99_ms"] if served else None,
        "served": served,
        "roofline": dominant_roofline(results[head], (wmx if head == "mixed" else w64).name),
        "kernels": {p: {"rooflines": results[p]["rooflines"], "profile": results[p]["profile"]}
                    for p in ("mixed", "fp64") if p in results},
        "n1048575": large,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
