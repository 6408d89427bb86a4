"""Parity of the HIP path with the oracle on the rarer routes of a solve, through the C-ABI:

  * Algorithm 1's second branch (|J| > |I|: the core solves with Z(J,:));
  * the core's Jacobi pseudo-inverse (taken where a bound cannot show that the cutoff drops no
    singular value of the interpolation rows);
  * Algorithm 4's initial guess U0, V0 (a warm start from a previous solution);
  * replayed index sets (the diagnostic that separates rounding from set divergence).

FP64 cases must give identical ordered index sets at every pass, the same branch of
Algorithm 1, sizes, ranks, status and pass count, and a relative error <= 1e-10 against the
oracle. The right-hand sides are separable sine modes (whose spectral solution has exact zero
rows and columns, so pruning removes different numbers of rows and columns) plus weak seeded
bumps; they were chosen by running the oracle alone (see SECOND_BRANCH for the criterion)."""
import numpy as np
import pytest

import workloads
from oracle import crossdeim as cd
from test_gpu_solve import compare_fp64, gpu_solve, oracle_spread

pytestmark = pytest.mark.gpu


def sine_plus_bumps(n, modes, bump_seed, n_bumps, bump_scale=1e-2):
    U, s, V = workloads.sine_rhs(n, modes)
    if n_bumps:
        Ub, sb, Vb = workloads.make("n255_r5_fp64", bump_seed, n=n)
        U = np.hstack([U, Ub[:, :n_bumps]])
        V = np.hstack([V, Vb[:, :n_bumps]])
        s = np.concatenate([s, bump_scale * sb[:n_bumps]])
    return np.asfortranarray(U), s, np.asfortranarray(V)


# (n, modes, bump seed, bumps, r_max, maxiter): the oracle takes |J| > |I| at a later pass.
# Kept only where the oracle itself is insensitive to rounding: with the input perturbed by
# 1e-15 relative (four seeds) its index sets, ranks and pass count stay the same and its result
# moves by less than 1e-11 (many such right-hand sides are ill-conditioned enough that rounding
# alone changes a discrete decision or moves the result by more than the 1e-10 tolerance).
SECOND_BRANCH = [
    (255, [(15, 19, 0.947690609812321), (8, 15, -1.4828431443678827)], 228, 1, 32, 10),
    (255, [(7, 1, -2.6328702074086703), (7, 18, 2.287889768374534), (19, 10, 0.830165546635623),
           (5, 14, -0.32350473962469367)], 263, 1, 32, 10),
    (255, [(29, 9, -0.8655285237589894), (20, 7, -1.3729669358236254), (29, 16, -0.4752190689915521)],
     131, 1, 32, 10),
    (255, [(13, 8, 0.30027651841828845), (25, 23, 0.46757528576185525), (18, 9, 0.9490966814610048)],
     528, 2, 32, 10),
    (4095, [(11, 11, -0.7729722441509735), (20, 24, 0.8454613625332678), (6, 15, -0.489578954885817),
            (15, 8, -2.2022597702579945)], 140, 1, 32, 10),
    (4095, [(16, 27, 1.5129715529870995), (3, 29, -0.06137297530171238)], 941, 2, 32, 10),
]


@pytest.mark.parametrize("case", SECOND_BRANCH, ids=[f"n{c[0]}-{i}" for i, c in enumerate(SECOND_BRANCH)])
def test_second_branch_of_algorithm1(case):
    n, modes, bseed, nb, r_max, maxiter = case
    U, s, V = sine_plus_bumps(n, modes, bseed, nb)
    print(f"second branch: n={n} modes {modes} bumps {nb} (seed {bseed})", flush=True)
    o = cd.solve(n, U, s, V, r_max, 1e-10, maxiter)
    assert any(not t.branch for t in o.trace), "the case must reach |J| > |I| in the oracle"
    g = gpu_solve(n, U, s, V, r_max, 1e-10, maxiter)
    compare_fp64(g, o, f"n={n}")
    assert any(not t["branch"] for t in g["trace"])


# pure sine modes: C = W^(:, J) then has exactly zero columns, and the interpolation rows of
# the orthonormal basis can be singular to rounding
JACOBI = [
    (255, [(20, 24, 0.22461902534909414)]),
    (255, [(19, 3, -1.6082422850112825), (12, 6, -1.7564604476259789)]),
    (255, [(7, 23, 1.4560154985822233)]),
    (255, [(12, 23, -0.36233625364362343), (7, 26, 1.6989366631605227)]),
    (4095, [(7, 14, -0.3269543230964199)]),
    (4095, [(20, 10, 0.002782362028699419)]),
]


def test_jacobi_pseudo_inverse_route():
    routes = []
    for n, modes in JACOBI:
        U, s, V = sine_plus_bumps(n, modes, 0, 0)
        print(f"jacobi route: n={n} modes {modes}", flush=True)
        o = cd.solve(n, U, s, V, 32, 1e-10, 10)
        g = gpu_solve(n, U, s, V, 32, 1e-10, 10)
        routes.append([t["route"] for t in g["trace"]])
        print(f"  routes {routes[-1]}", flush=True)
        compare_fp64(g, o, f"n={n} {modes}")
    assert any("jacobi" in r for r in routes), "no case took the Jacobi route on the GPU"


@pytest.mark.parametrize("seed", [0, 1])
def test_warm_start_from_previous_solution(seed):
    """Algorithm 4's initial guess: solve a right-hand side, perturb its amplitudes by 1 %, and
    solve again from the previous solution (each side chains its own previous result)."""
    w = workloads.CONFIGS["n4095_r10_fp64"]
    U, s, V = workloads.make(w, seed)
    s2 = s * (1.0 + 0.01 * np.random.default_rng(100 + seed).standard_normal(s.size))
    print(f"warm start: {w.name} seed {seed}", flush=True)
    o1 = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    g1 = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    compare_fp64(g1, o1, "first solve")
    cold = cd.solve(w.n, U, s2, V, w.r_max, w.tol, w.maxiter)
    o2 = cd.solve(w.n, U, s2, V, w.r_max, w.tol, w.maxiter, warm=(o1.U, o1.S, o1.V))
    assert o2.iters < cold.iters
    r1 = g1["rank"]
    g2 = gpu_solve(w.n, U, s2, V, w.r_max, w.tol, w.maxiter, guess=(g1["U"], g1["S"][:r1], g1["V"]))
    compare_fp64(g2, o2, f"warm solve ({o2.iters} passes, cold {cold.iters})")


def test_zero_guess_leaves_the_start_from_the_rhs():
    w = workloads.CONFIGS["n255_r5_fp64"]
    U, s, V = workloads.make(w, 1)
    print("zero guess", flush=True)
    a = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    z = np.zeros((w.n, 3), order="F")
    b = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, guess=(z, np.ones(3), z))
    assert np.array_equal(a["Ufull"], b["Ufull"]) and np.array_equal(a["Vfull"], b["Vfull"])
    assert np.array_equal(a["S"], b["S"]) and a["info"]["iters"] == b["info"]["iters"]
    o = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, warm=(z, np.ones(3), z))
    compare_fp64(b, o, "zero guess")


def test_guess_with_unit_weights_and_nonfinite_guess():
    from paper_2607_06021_amd import LrpError

    w = workloads.CONFIGS["n255_r5_fp64"]
    U, s, V = workloads.make(w, 2)
    Ug, sg, Vg = workloads.make(w, 3)
    print("guess with unit weights", flush=True)
    o = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, warm=(Ug, None, Vg))
    g = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, guess=(Ug, None, Vg))
    compare_fp64(g, o, "guess from other bumps")
    Ug[3, 1] = np.inf
    with pytest.raises(LrpError) as ei:
        gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, guess=(Ug, sg, Vg))
    assert ei.value.code == -4


@pytest.mark.parametrize("n", [255, 4095])
def test_replayed_sets(n):
    """Pass 0 takes 6 rows and 9 columns (|J| > |I|), pass 1 the reverse shape; later passes
    select from the iterate these give."""
    w = workloads.CONFIGS["n4095_r10_fp64"]
    U, s, V = workloads.make(w, 0, n=n)
    replay = [(list(range(0, 12, 2)), list(range(1, 19, 2))),
              (list(range(0, 12, 2)) + [20, 21, 22, 23, 24, 25], list(range(1, 19, 2)) + [30])]
    print(f"replay n={n}", flush=True)
    o = cd.solve(n, U, s, V, 32, 1e-10, 20, replay=replay)
    g = gpu_solve(n, U, s, V, 32, 1e-10, 20, replay=replay)
    assert [t["I_pre"] for t in g["trace"][:2]] == [r[0] for r in replay]
    assert not g["trace"][0]["branch"]
    # the forced sets make the early iterates ill-conditioned: their rho moves under rounding
    # far more than the result does, so its bound includes the oracle's own spread
    compare_fp64(g, o, f"replay n={n}", spread=oracle_spread(n, U, s, V, 32, 1e-10, 20, replay=replay))


def test_mixed_replay_of_fp64_sets_reports_the_rounding_loss():
    """The mixed-precision path run on the index sets of the FP64 path: the difference of the
    two results is then the rounding of the FP32 stages alone (tolerance 1e-5 of the mixed path)."""
    w = workloads.CONFIGS["n65535_r20_mixed"]
    U, s, V = workloads.make(w, 0)
    print("mixed replay of FP64 sets, n=65535", flush=True)
    g64 = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, precision="fp64")
    sets = [(t["I_pre"], t["J_pre"]) for t in g64["trace"]]
    gm = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, precision="mixed")
    gr = gpu_solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, precision="mixed", replay=sets)
    used = min(len(gr["trace"]), len(sets))
    assert [t["I_pre"] for t in gr["trace"][:used]] == [x[0] for x in sets[:used]]
    ref = (g64["U"], g64["S"][: g64["rank"]], g64["V"])
    e_free = cd.rel_err((gm["U"], gm["S"][: gm["rank"]], gm["V"]), ref)
    e_replay = cd.rel_err((gr["U"], gr["S"][: gr["rank"]], gr["V"]), ref)
    print(f"  mixed vs FP64 GPU: own sets {e_free:.2e} ({gm['info']['iters']} passes), "
          f"FP64 sets {e_replay:.2e} ({gr['info']['iters']} passes)", flush=True)
    assert e_free <= 1e-5 and e_replay <= 1e-5
