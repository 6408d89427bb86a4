"""Whole-solve parity of the HIP path (through the C-ABI) against the CPU oracle.

FP64: the ordered index sets handed to every cross approximation, the pruned sizes, the
ranks, the status and the pass count must be identical; the relative Frobenius error of the
solution against the oracle's must be <= 1e-10. Mixed precision: error <= 1e-5 against the
oracle (printed for every case)."""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import crossdeim as cd

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def dev(a):
    torch = _torch()
    from paper_2607_06021_amd import fortran

    a = np.asarray(a, dtype=np.float64)
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return fortran(t) if a.ndim == 2 else t


def gpu_solve(n, U, s, V, r_max, tol, maxiter, precision="fp64", prune_tau=0.0, guess=None, replay=None):
    """One solve through the C-ABI. guess: (U0, S0, V0) host arrays (S0 may be None);
    replay: list of (I, J) sets for the first passes."""
    from paper_2607_06021_amd import Solver

    with Solver(n, r_max, tol, maxiter=maxiter, precision=precision, prune_tau=prune_tau) as sol:
        if replay is not None:
            sol.set_index_sets(replay)
        g = None
        if guess is not None:
            g = (dev(guess[0]), None if guess[1] is None else dev(guess[1]), dev(guess[2]))
        Uo, So, Vo, r, info = sol.solve(dev(U), dev(s), dev(V), guess=g)
        res = {
            "U": Uo[:, :r].cpu().numpy(),
            "S": So.cpu().numpy(),
            "V": Vo[:, :r].cpu().numpy(),
            "rank": r,
            "info": info.as_dict(),
            "sets": sol.index_sets(),
            "trace": sol.trace(),
            "Ufull": Uo.cpu().numpy(),
            "Vfull": Vo.cpu().numpy(),
        }
    return res


# rho = ||X_k - X_{k-1}||_F / ||S_k||_F: two iterates that each agree with the oracle's to the
# FP64 result tolerance 1e-10 (relative Frobenius) move rho by at most 2e-10 (plus the
# relative error of the norm, far below 1e-8).
RHO_ABS, RHO_REL = 2e-10, 1e-8


def oracle_spread(n, U, s, V, r_max, tol, maxiter, reps=2, **kw):
    """Per-pass spread of the oracle's own rho and indicator when the right-hand side is
    perturbed by 1e-15 relative (rounding of the inputs): max |change| over `reps` seeded
    perturbations. Early passes of forced (replayed) index sets can be ill-conditioned, and
    their rho then moves far more than the final result does."""
    o = cd.solve(n, U, s, V, r_max, tol, maxiter, **kw)
    spread = [[0.0, 0.0] for _ in o.trace]
    for r in range(reps):
        Up = U * (1.0 + 1e-15 * np.random.default_rng(r).standard_normal(U.shape))
        p = cd.solve(n, Up, s, V, r_max, tol, maxiter, **kw)
        for k, (a, b) in enumerate(zip(o.trace, p.trace)):
            for q, (x, y) in enumerate(((a.rho, b.rho), (a.indicator, b.indicator))):
                if math.isfinite(x) and math.isfinite(y):
                    spread[k][q] = max(spread[k][q], abs(x - y))
    return spread


def compare_stop_values(g, o, label, spread=None):
    """rho and the indicator of every pass where the GPU computed them (it skips them where the
    stopping test cannot pass) against the oracle's values of the same pass.

    The indicator is min(eta1 (1 + eta2), eta2 (1 + eta1)) S_min / ||S||_F with
    eta = 1/sigma_min of the interpolation rows of the iterate's orthonormal basis. With both
    iterates within 1e-10 ||S||_F of each other (the FP64 result tolerance): S_min moves by at
    most 1e-10 ||S||_F (singular values are 1-Lipschitz in the Frobenius norm), a relative
    change d = 1e-10 ||S||_F / S_min; the basis spans the iterate's column space, which moves
    by an angle of about d, so sigma_min of its rows moves by about d and eta by a relative
    d eta. The bound is twice the sum of these relative changes.

    spread (optional, from oracle_spread): per pass, the oracle's own change under rounding of
    its inputs; ten times it is added to each bound."""
    for tg, to in zip(g["trace"], o.trace):
        sp = spread[to.k] if spread is not None and to.k < len(spread) else (0.0, 0.0)
        if math.isfinite(tg["rho"]):
            d = abs(tg["rho"] - to.rho)
            tol = RHO_ABS + RHO_REL * to.rho + 10.0 * sp[0]
            print(f"  {label} pass {to.k}: rho gpu {tg['rho']:.6e} oracle {to.rho:.6e} diff {d:.1e} bound {tol:.1e}",
                  flush=True)
            assert d <= tol, f"pass {to.k} rho"
        if math.isfinite(tg["indicator"]):
            smin_rel = float(to.S[-1]) / float(np.linalg.norm(to.S))
            d_rel = 1e-10 / smin_rel
            tol = to.indicator * (2.0 * d_rel * (1.0 + to.eta1 + to.eta2) + 1e-8) + 10.0 * sp[1]
            d = abs(tg["indicator"] - to.indicator)
            print(f"  {label} pass {to.k}: indicator gpu {tg['indicator']:.6e} oracle {to.indicator:.6e} "
                  f"diff {d:.1e} bound {tol:.1e}", flush=True)
            assert d <= tol, f"pass {to.k} indicator"


def compare_fp64(g, o, label, spread=None):
    info = g["info"]
    print(f"{label}: status {info['status']}/{o.status} iters {info['iters']}/{o.iters} rank {g['rank']}/{o.rank}",
          flush=True)
    for tg, to in zip(g["trace"], o.trace):
        same = tg["I_pre"] == to.I_pre and tg["J_pre"] == to.J_pre
        if not same:
            print(f"  pass {to.k}: sets differ; oracle cut margins gapI {to.gapI:.2e} gapJ {to.gapJ:.2e}")
            print("   gpu I", tg["I_pre"], "\n   orc I", to.I_pre, "\n   gpu J", tg["J_pre"], "\n   orc J", to.J_pre)
    assert len(g["trace"]) == len(o.trace)
    for tg, to in zip(g["trace"], o.trace):
        assert tg["I_pre"] == to.I_pre and tg["J_pre"] == to.J_pre, f"pass {to.k}"
        assert tg["nI"] == len(to.I) and tg["nJ"] == len(to.J), f"pass {to.k} pruning"
        assert tg["rank"] == to.rank, f"pass {to.k} rank"
        assert tg["branch"] == to.branch, f"pass {to.k} branch of Algorithm 1"
    assert info["status"] == o.status
    assert info["iters"] == o.iters
    assert g["rank"] == o.rank
    assert g["sets"] == (o.I, o.J)
    compare_stop_values(g, o, label, spread)
    e = cd.rel_err((g["U"], g["S"][: g["rank"]], g["V"]), (o.U, o.S, o.V))
    print(f"  rel err vs oracle {e:.3e}  gpu ms {info['ms']:.3f}")
    assert e <= 1e-10
    # output padding: zero columns and singular values beyond the rank
    assert np.all(g["S"][g["rank"]:] == 0.0)
    assert np.all(g["Ufull"][:, g["rank"]:] == 0.0) and np.all(g["Vfull"][:, g["rank"]:] == 0.0)
    return e


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_n255_fp64_parity(seed):
    w = workloads.CONFIGS["n255_r5_fp64"]
    U, s, V = workloads.make(w, seed)
    print(f"solve {w.name} seed {seed}", flush=True)
    o = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    g = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    compare_fp64(g, o, f"{w.name} seed {seed}")


@pytest.mark.parametrize("seed", [0, 1])
def test_n4095_fp64_parity(seed):
    w = workloads.CONFIGS["n4095_r10_fp64"]
    U, s, V = workloads.make(w, seed)
    print(f"solve {w.name} seed {seed}", flush=True)
    o = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    g = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    compare_fp64(g, o, f"{w.name} seed {seed}")


def test_n65535_fp64_parity():
    w = workloads.CONFIGS["n65535_r20_fp64"]
    U, s, V = workloads.make(w, 0)
    print(f"solve {w.name} seed 0", flush=True)
    o = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    g = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    compare_fp64(g, o, w.name)


def test_n65535_mixed_error():
    """Mixed precision against the FP64 oracle and against the GPU's own FP64 path (both at the
    1e-5 tolerance of the mixed path)."""
    w = workloads.CONFIGS["n65535_r20_mixed"]
    U, s, V = workloads.make(w, 0)
    print(f"solve {w.name} seed 0", flush=True)
    o = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    g = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, precision="mixed")
    g64 = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, precision="fp64")
    e = cd.rel_err((g["U"], g["S"][: g["rank"]], g["V"]), (o.U, o.S, o.V))
    e64 = cd.rel_err((g["U"], g["S"][: g["rank"]], g["V"]), (g64["U"], g64["S"][: g64["rank"]], g64["V"]))
    print(f"  mixed: status {g['info']['status']} iters {g['info']['iters']} rank {g['rank']} "
          f"rel err vs FP64 oracle {e:.3e}, vs GPU FP64 path {e64:.3e}")
    assert e <= 1e-5
    assert e64 <= 1e-5


# the paper's grid sizes n = 2^k (n + 1 not a power of two: the Bluestein DST), with the
# recipes of the n = 255, 4095 and 65535 workloads
@pytest.mark.parametrize("name,n,seed", [("n255_r5_fp64", 1024, 0), ("n4095_r10_fp64", 4096, 1),
                                         ("n65535_r20_fp64", 65536, 0)])
def test_paper_grid_sizes_fp64_parity(name, n, seed):
    w = workloads.CONFIGS[name]
    U, s, V = workloads.make(w, seed, n=n)
    print(f"solve {name} recipe at n={n} seed {seed}", flush=True)
    o = cd.solve(n, U, s, V, w.r_max, w.tol, w.maxiter)
    g = gpu_solve(n, U, s, V, w.r_max, w.tol, w.maxiter)
    compare_fp64(g, o, f"n={n}")


def test_paper_grid_size_mixed_error():
    w = workloads.CONFIGS["n65535_r20_mixed"]
    n = 65536
    U, s, V = workloads.make(w, 0, n=n)
    print(f"mixed at n={n}", flush=True)
    o = cd.solve(n, U, s, V, w.r_max, w.tol, w.maxiter)
    g = gpu_solve(n, U, s, V, w.r_max, w.tol, w.maxiter, precision="mixed")
    e = cd.rel_err((g["U"], g["S"][: g["rank"]], g["V"]), (o.U, o.S, o.V))
    print(f"  mixed n={n}: status {g['info']['status']} iters {g['info']['iters']} rank {g['rank']} "
          f"rel err vs FP64 oracle {e:.3e} ms {g['info']['ms']:.2f}", flush=True)
    assert e <= 1e-5


@pytest.mark.parametrize("n", [255, 1024, 65535])
def test_manufactured_sine_rank_one(n):
    k, l, a = 5, 9, 2.0
    U, s, V = workloads.sine_rhs(n, [(k, l, a)])
    print(f"sine n={n}", flush=True)
    g = gpu_solve(n, U, s, V, 8, 1e-10, 10)
    assert g["rank"] == 1
    h = 1.0 / (n + 1)
    den = (4.0 / h ** 2) * (math.sin(k * math.pi * h / 2) ** 2 + math.sin(l * math.pi * h / 2) ** 2)
    x = workloads.grid(n)
    e = cd.rel_err((g["U"], g["S"][:1], g["V"]), (np.sin(k * math.pi * x)[:, None], np.array([a / den]),
                                                  np.sin(l * math.pi * x)[:, None]))
    print(f"  rel err vs closed form {e:.2e}")
    assert e <= 1e-13
    assert g["sets"] == ([k - 1], [l - 1])


def test_edge_cases_status_and_zero_rhs():
    n = 255
    U, s, V = workloads.make("n255_r5_fp64", 0, n=n)
    print("edge: zero rhs", flush=True)
    z = gpu_solve(n, U, np.zeros_like(s), V, 16, 1e-10, 10)
    assert z["rank"] == 1 and z["info"]["status"] == 0 and np.all(z["S"] == 0.0) and np.all(z["U"] == 0.0)
    print("edge: maxiter 1", flush=True)
    o1 = cd.solve(n, U, s, V, 16, 1e-10, 1)
    g1 = gpu_solve(n, U, s, V, 16, 1e-10, 1)
    compare_fp64(g1, o1, "maxiter=1")
    print("edge: tiny cap", flush=True)
    o2 = cd.solve(n, U[:, :3], s[:3], V[:, :3], 4, 1e-14, 20)
    assert o2.status == cd.STATUS_STAGNATED
    g2 = gpu_solve(n, U[:, :3], s[:3], V[:, :3], 4, 1e-14, 20)
    compare_fp64(g2, o2, "r_max=4")
    print("edge: r_F > r_max is rejected", flush=True)
    from paper_2607_06021_amd import LrpError

    with pytest.raises(LrpError):
        gpu_solve(n, U, s, V, 3, 1e-10, 5)
    print("edge: rank-1 rhs of width 1 column", flush=True)
    o3 = cd.solve(n, U[:, :1], s[:1], V[:, :1], 16, 1e-10, 10)
    g3 = gpu_solve(n, U[:, :1], s[:1], V[:, :1], 16, 1e-10, 10)
    compare_fp64(g3, o3, "r_F=1")


def test_nonfinite_input_rejected():
    from paper_2607_06021_amd import LrpError

    n = 255
    U, s, V = workloads.make("n255_r5_fp64", 0, n=n)
    U[17, 2] = np.nan
    print("edge: NaN input", flush=True)
    with pytest.raises(LrpError) as ei:
        gpu_solve(n, U, s, V, 16, 1e-10, 10)
    assert ei.value.code == -4


def test_repeat_solves_are_bitwise_identical():
    w = workloads.CONFIGS["n4095_r10_fp64"]
    U, s, V = workloads.make(w, 3)
    from paper_2607_06021_amd import Solver

    print("determinism", flush=True)
    with Solver(w.n, w.r_max, w.tol, maxiter=w.maxiter) as sol:
        a = sol.solve(dev(U), dev(s), dev(V))
        A = [t.cpu().numpy().copy() for t in a[:3]]
        b = sol.solve(dev(U), dev(s), dev(V))
        B = [t.cpu().numpy() for t in b[:3]]
    for x, y in zip(A, B):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_context_serves_different_ranks_and_pass_counts(precision):
    """The passes are captured once per context (two graphs per iterate parity) and replayed:
    solves of different input rank, pass count and stop status on one context (the maxiter is
    fixed per context, so the cases are grouped by it) must each be bitwise equal to the same
    solve on a fresh context."""
    from paper_2607_06021_amd import Solver

    w = workloads.CONFIGS["n4095_r10_fp64"]
    cases = []
    for seed, rk, maxiter in ((5, 4, 20), (6, 12, 20), (7, 9, 2), (5, 4, 20)):
        U, s, V = workloads.make(w, seed)
        cases.append((U[:, :rk], s[:rk], V[:, :rk], maxiter))
    print(f"one context, {precision}", flush=True)

    def run(sol, case):
        U, s, V, _ = case
        Uo, So, Vo, r, info = sol.solve(dev(U), dev(s), dev(V))
        return [Uo.cpu().numpy().copy(), So.cpu().numpy().copy(), Vo.cpu().numpy().copy()], r, info.as_dict()

    fresh = []
    for case in cases:
        with Solver(w.n, w.r_max, w.tol, maxiter=case[3], precision=precision) as sol:
            fresh.append(run(sol, case))
    shared = {}
    for maxiter in sorted({c[3] for c in cases}):
        with Solver(w.n, w.r_max, w.tol, maxiter=maxiter, precision=precision) as sol:
            for i, case in enumerate(cases):
                if case[3] == maxiter:
                    shared[i] = run(sol, case)
    for i in range(len(cases)):
        (A, ra, ia), (B, rb, ib) = fresh[i], shared[i]
        print(f"  case {i}: rank {ra}/{rb} iters {ia['iters']}/{ib['iters']} status {ia['status']}/{ib['status']}",
              flush=True)
        assert ra == rb and ia["iters"] == ib["iters"] and ia["status"] == ib["status"]
        for x, y in zip(A, B):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("seed", [0, 2])
def test_rank_above_32_fp64_parity(seed):
    """Right-hand sides of rank 40 (the fiber build for ranks above 32), cap 64: identical sets
    and <= 1e-10 against the oracle (cases whose oracle sets are stable under 1e-15 noise)."""
    n = 4095
    U, s, V, _ = workloads.bump_rhs(n, 300 + seed, 40, 0.01, 0.1)
    print(f"solve n {n} rank 40 seed {seed}", flush=True)
    o = cd.solve(n, U, s, V, 64, 1e-10, 20)
    g = gpu_solve(n, U, s, V, 64, 1e-10, 20)
    compare_fp64(g, o, f"rank-40 seed {seed}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_context_switches_fiber_builds(precision):
    """Ranks above and below 32 alternate on one context (two fiber builds, each with its own
    captured passes): every solve bitwise equal to the same solve on a fresh context."""
    from paper_2607_06021_amd import Solver

    n = 4095
    cases = []
    for seed, rk in ((300, 40), (301, 12), (302, 40), (303, 32)):
        U, s, V, _ = workloads.bump_rhs(n, seed, rk, 0.01, 0.1)
        cases.append((dev(U), dev(s), dev(V)))
    print(f"fiber builds on one context, {precision}", flush=True)
    fresh = []
    for U, s, V in cases:
        with Solver(n, 64, 1e-10, maxiter=20, precision=precision) as sol:
            Uo, So, Vo, r, info = sol.solve(U, s, V)
            fresh.append((Uo.clone(), So.clone(), Vo.clone(), r, info.iters))
    with Solver(n, 64, 1e-10, maxiter=20, precision=precision) as sol:
        for (U, s, V), (Uf, Sf, Vf, rf, itf) in zip(cases, fresh):
            Uo, So, Vo, r, info = sol.solve(U, s, V)
            assert r == rf and info.iters == itf
            assert torch_equal(Uo, Uf) and torch_equal(So, Sf) and torch_equal(Vo, Vf)


def torch_equal(a, b):
    import torch

    return bool(torch.equal(a, b))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_profile_mode_same_result_and_kernel_times(precision):
    """A context with the profile flag launches the passes kernel by kernel (no graphs) with
    HIP events around every launch: the result must be bitwise the same as with graphs, and
    the per-kernel times must cover the solve."""
    w = workloads.CONFIGS["n65535_r20_fp64"]
    U, s, V = workloads.make(w, 0)
    from paper_2607_06021_amd import Solver

    print(f"profile mode {precision}", flush=True)
    args = (dev(U), dev(s), dev(V))
    with Solver(w.n, 64, w.tol, maxiter=w.maxiter, precision=precision) as sol:
        a = sol.solve(*args)
        A = [t.cpu().numpy().copy() for t in a[:3]]
    with Solver(w.n, 64, w.tol, maxiter=w.maxiter, precision=precision, profile=True) as sol:
        b = sol.solve(*args)
        B = [t.cpu().numpy() for t in b[:3]]
        prof = sol.profile()
        info = b[4]
    for x, y in zip(A, B):
        assert np.array_equal(x, y)
    assert a[3] == b[3] and a[4].iters == info.iters
    # every launch is timed by events attached to its own dispatch
    for name in ("k_select", "k_topk_block", "k_pi", "k_eta"):
        assert name in prof and prof[name][0] >= 1 and prof[name][1] >= 0.0, name
    for name in ("k_core", "k_core_warm", "k_tsqr_factor", "k_tsqr_apply", "k_fiber", "k_prod",
                 "k_dst_pass1", "k_dst_pass2"):
        assert name in prof and prof[name][0] >= 1 and prof[name][1] > 0.0, name
    assert 0.0 < prof["empty kernel"][1] / 16 < 0.05
    assert prof["k_core"][0] >= info.iters and prof["k_core_warm"][0] == 1
    total = sum(ms for _, ms in prof.values())
    print(f"  solve {info.ms:.3f} ms, kernels {total:.3f} ms", flush=True)
    assert 0.5 * info.ms < total < 1.05 * info.ms


def load_golden():
    path = os.path.join(GOLDEN, "n1048575_r30_fp64_seed0.json")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    with open(path) as f:
        return json.load(f)


def sketched_rel_err(n, U, S, V, gold):
    """||Om^T (W - W_o) Om'||_F / ||Om^T W_o Om'||_F with W = U diag(S) V^T and the oracle's
    sketches A_o = Om^T U_o diag(S_o), B_o = Om'^T V_o. For Gaussian Om, Om' (k columns) the
    squared sketched norm of a matrix is k^2 times its squared Frobenius norm in expectation,
    so the ratio estimates the relative Frobenius error."""
    k = gold["sketch_k"]
    Om = workloads.sketch_matrix(n, k, gold["sketch_seeds"][0])
    A = Om.T @ (U * S[None, :])
    del Om
    Om = workloads.sketch_matrix(n, k, gold["sketch_seeds"][1])
    B = Om.T @ V
    del Om
    Ao, Bo = np.array(gold["sketch_U"]), np.array(gold["sketch_V"])
    ref = Ao @ Bo.T
    return float(np.linalg.norm(A @ B.T - ref) / np.linalg.norm(ref))


def test_n1048575_fp64_against_golden():
    """Full-size n = 2^20 - 1: the oracle takes minutes, so its per-pass index sets, ranks, rho
    and indicator, its singular values, sampled rows and Gaussian sketches of its solution were
    stored by tests/golden/make_golden.py (oracle only)."""
    gold = load_golden()
    w = workloads.CONFIGS["n1048575_r30_fp64"]
    U, s, V = workloads.make(w, 0)
    print(f"solve {w.name} seed 0 (golden)", flush=True)
    g = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    info = g["info"]
    print(f"  status {info['status']}/{gold['status']} iters {info['iters']}/{gold['iters']} rank {g['rank']}/{gold['rank']} ms {info['ms']:.2f}")
    assert [t["I_pre"] for t in g["trace"]] == gold["I_pre"]
    assert [t["J_pre"] for t in g["trace"]] == gold["J_pre"]
    assert info["status"] == gold["status"] and info["iters"] == gold["iters"] and g["rank"] == gold["rank"]
    S = g["S"][: g["rank"]]
    assert np.max(np.abs(S - np.array(gold["S"]))) <= 1e-10 * gold["S"][0]
    rows = np.array(gold["rows"])
    # W(i, j) at sampled grid points, computed from the stored oracle rows
    Wg = (g["U"][rows] * S[None, :]) @ g["V"][rows].T
    Wo = (np.array(gold["U_rows"]) * np.array(gold["S"])[None, :]) @ np.array(gold["V_rows"]).T
    err = np.max(np.abs(Wg - Wo)) / np.max(np.abs(Wo))
    print(f"  sampled entries max rel err {err:.2e}")
    assert err <= 1e-9
    for k, tg in enumerate(g["trace"]):
        if math.isfinite(tg["rho"]):
            print(f"  pass {k}: rho gpu {tg['rho']:.6e} oracle {gold['rho'][k]:.6e}")
            assert abs(tg["rho"] - gold["rho"][k]) <= RHO_ABS + RHO_REL * gold["rho"][k]
    es = sketched_rel_err(w.n, g["U"], S, g["V"], gold)
    print(f"  sketched relative Frobenius error {es:.2e}")
    assert es <= 1e-10


def test_n1048575_mixed_against_golden_and_fp64():
    """The mixed path at n = 2^20 - 1: error against the oracle (through its stored sketches)
    and against the GPU's FP64 path (exact, in factored form), both <= 1e-5."""
    gold = load_golden()
    w = workloads.CONFIGS["n1048575_r30_mixed"]
    U, s, V = workloads.make(w, 0)
    print(f"solve {w.name} seed 0 (golden)", flush=True)
    gm = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, precision="mixed")
    g64 = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, precision="fp64")
    rm, r64 = gm["rank"], g64["rank"]
    es = sketched_rel_err(w.n, gm["U"], gm["S"][:rm], gm["V"], gold)
    e64 = cd.rel_err((gm["U"], gm["S"][:rm], gm["V"]), (g64["U"], g64["S"][:r64], g64["V"]))
    print(f"  mixed: status {gm['info']['status']} iters {gm['info']['iters']} rank {rm}; "
          f"sketched error vs oracle {es:.2e}, vs GPU FP64 {e64:.2e}; ms {gm['info']['ms']:.2f}")
    assert es <= 1e-5 and e64 <= 1e-5
