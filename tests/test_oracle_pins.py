"""Pins of the oracle's Algorithm 4 parts against routes that share no code with it.

* the indicator of Algorithm 4 (eta_1, eta_2 on the pruned sets) against matrices whose
  interpolation rows have singular values known by construction;
* the warm start against the SVD of the dense F^ (and of a dense guess, the U0, V0 inputs
  of Algorithm 4);
* column-pivoted QR (QDEIM, Algorithm 2) against SciPy's LAPACK routine and Gram-Schmidt;
* the whole iteration against tests/brute_crossdeim.py, a dense re-implementation that runs
  Algorithm 1 as printed (the SVD of the |J| x n matrix W) on the explicit W^, on tiny grids:
  ordered index sets, pruned sizes, branch of Algorithm 1, significant rank, rho, eta and the
  indicator of every pass, status, pass count, final rank and product;
* mutation tests: each plausible mistake planted in a copy of the oracle's source must make
  one of these comparisons fail.
"""
import math
import os
import sys
import types

import numpy as np
import pytest

import brute_crossdeim as bf
import workloads
from oracle import crossdeim as cd

EPS = float(np.finfo(np.float64).eps)
ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "crossdeim.py")


# --------------------------------------------------------------------------------------
# cases for the dense comparison
# --------------------------------------------------------------------------------------
def sine_plus_bumps(n, modes, bump_seed, n_bumps, bump_scale):
    """Sine modes (exactly structured W^: zero rows and columns) plus weak seeded bumps."""
    U, s, V = workloads.sine_rhs(n, modes)
    if n_bumps:
        Ub, sb, Vb = workloads.make("n255_r5_fp64", bump_seed, n=n)
        U = np.hstack([U, Ub[:, :n_bumps]])
        V = np.hstack([V, Vb[:, :n_bumps]])
        s = np.concatenate([s, bump_scale * sb[:n_bumps]])
    return U, s, V


def _cases():
    out = []
    for n in (31, 63):
        for seed in range(5):
            out.append((f"bumps-n{n}-s{seed}", n, ("n255_r5_fp64", seed), 16, 10, {}))
    for seed in range(3):
        out.append((f"bumps+sines-n63-s{seed}", 63, ("n4095_r10_fp64", seed), 32, 20, {}))
    # a right-hand side whose pruning is uneven, so that a later pass has |J| > |I| (the
    # second branch of Algorithm 1)
    out.append(("else-branch-n63", 63, ("sine", [(1, 9, -0.5871942603400888), (8, 10, 0.967036908966546),
                                                  (4, 9, -0.8039005872403687)], 168, 1, 1e-2), 32, 10, {}))
    out.append(("else-branch-n63-b", 63, ("sine", [(7, 8, -1.210047387615151), (10, 7, 0.9686460234228775),
                                                    (6, 7, -0.4311181065019909), (4, 4, 0.7234757361001739)],
                                          359, 2, 1e-2), 32, 10, {}))
    for n in (31, 63):
        for seed in range(2):
            out.append((f"qdeim-bumps-n{n}-s{seed}", n, ("n255_r5_fp64", seed), 16, 10, {"selector": "qdeim"}))
            out.append((f"qdeim-bumps+sines-n{n}-s{seed}", n, ("n4095_r10_fp64", seed), 32, 20,
                        {"selector": "qdeim"}))
    for seed in (1, 2):
        out.append((f"warm-n63-s{seed}", 63, ("n4095_r10_fp64", seed), 32, 20, {"warm": "previous"}))
    out.append(("replay-else-n63", 63, ("n4095_r10_fp64", 0), 32, 20, {"replay": "uneven"}))
    return out


CASES = _cases()


def make_case(spec, n):
    if spec[0] == "sine":
        return sine_plus_bumps(n, *spec[1:])
    return workloads.make(spec[0], spec[1], n=n)


def case_inputs(case):
    name, n, spec, r_max, maxiter, kw = case
    U, s, V = make_case(spec, n)
    kw = dict(kw)
    if kw.get("warm") == "previous":
        # warm start from the solution of a slightly different right-hand side (its physical
        # factors and singular values, as a caller would pass them)
        prev = bf.solve(n, U, s, V, r_max, 1e-10, maxiter)
        s = s * (1.0 + 1e-3 * np.arange(1, s.size + 1))
        kw["warm"] = (prev["U"], prev["S"], prev["V"])
    if kw.get("replay") == "uneven":
        # forced sets: pass 0 takes 6 rows and 9 columns (|J| > |I|), pass 1 the reverse
        kw["replay"] = [(list(range(0, 12, 2)), list(range(1, 19, 2))),
                        (list(range(0, 12, 2)) + [20, 21, 22, 23, 24, 25], list(range(1, 19, 2)) + [30])]
    return n, U, s, V, r_max, 1e-10, maxiter, kw


def sig_rank(S):
    return int(np.count_nonzero(S > 1e-12 * S[0])) if S.size else 0


def disagreements(o, b):
    """Differences between an oracle Result and a brute-force result (empty: they agree)."""
    bad = []
    if len(o.trace) != len(b["passes"]):
        bad.append(f"passes {len(o.trace)} vs {len(b['passes'])}")
    for to, tb in zip(o.trace, b["passes"]):
        k = to.k
        if to.I_pre != tb.I_pre or to.J_pre != tb.J_pre:
            bad.append(f"pass {k}: index sets")
        if len(to.I) != len(tb.I) or len(to.J) != len(tb.J):
            bad.append(f"pass {k}: pruned sizes {len(to.I)},{len(to.J)} vs {len(tb.I)},{len(tb.J)}")
        if to.branch != tb.branch:
            bad.append(f"pass {k}: branch")
        if sig_rank(to.S) != sig_rank(tb.S):
            bad.append(f"pass {k}: rank {sig_rank(to.S)} vs {sig_rank(tb.S)}")
        if math.isinf(to.rho) != math.isinf(tb.rho) or (
                math.isfinite(to.rho) and abs(to.rho - tb.rho) > 1e-6 * to.rho + 1e-11):
            bad.append(f"pass {k}: rho {to.rho:.6e} vs {tb.rho:.6e}")
        # eta and the indicator are determined by the iterate only while its smallest singular
        # value is above the rounding level; below it, the directions of the smallest singular
        # values are rounding noise and only the stop decision (status, pass count) is compared
        well = to.S.size and to.S[-1] >= 1e-9 * np.linalg.norm(to.S)
        if well:
            for nm, a, c in (("eta1", to.eta1, tb.eta1), ("eta2", to.eta2, tb.eta2)):
                if abs(a - c) > 1e-6 * abs(a):
                    bad.append(f"pass {k}: {nm} {a:.6e} vs {c:.6e}")
            if abs(to.indicator - tb.indicator) > 1e-6 * to.indicator:
                bad.append(f"pass {k}: indicator {to.indicator:.6e} vs {tb.indicator:.6e}")
    if o.status != b["status"] or o.iters != b["iters"] or o.rank != b["rank"]:
        bad.append(f"status/iters/rank {o.status},{o.iters},{o.rank} vs {b['status']},{b['iters']},{b['rank']}")
    else:
        e = cd.rel_err((b["U"], b["S"], b["V"]), (o.U, o.S, o.V))
        if not e <= 1e-10:
            bad.append(f"solution rel err {e:.2e}")
    return bad


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_oracle_equals_dense_brute_force(case):
    n, U, s, V, r_max, tol, maxiter, kw = case_inputs(case)
    o = cd.solve(n, U, s, V, r_max, tol, maxiter, **kw)
    b = bf.solve(n, U, s, V, r_max, tol, maxiter, **kw)
    assert disagreements(o, b) == []
    if case[0].startswith("else-branch") or case[0].startswith("replay"):
        assert any(not t.branch for t in o.trace), "the case must reach |J| > |I|"
    if "warm" in kw:  # the guess is the previous solution: fewer passes than a cold start
        cold = cd.solve(n, U, s, V, r_max, tol, maxiter)
        assert o.iters < cold.iters


# --------------------------------------------------------------------------------------
# the indicator against matrices with known singular values
# --------------------------------------------------------------------------------------
def planted_basis(n, I, d, rng):
    """n x r orthonormal U whose rows I (|I| >= r) have singular values exactly d (all < 1):
    U(I,:) = P diag(d) W^T and U(rest,:) = P2 diag(sqrt(1 - d^2)) W^T, so U^T U = I."""
    r = len(d)
    rest = [i for i in range(n) if i not in I]
    P, _ = np.linalg.qr(rng.standard_normal((len(I), r)))
    P2, _ = np.linalg.qr(rng.standard_normal((len(rest), r)))
    W, _ = np.linalg.qr(rng.standard_normal((r, r)))
    U = np.zeros((n, r))
    U[I] = P @ np.diag(d) @ W.T
    U[rest] = P2 @ np.diag(np.sqrt(1.0 - np.asarray(d) ** 2)) @ W.T
    return U


def test_indicator_known_singular_values():
    rng = np.random.default_rng(21)
    n = 80
    I = [3, 17, 40, 41, 55, 70]
    J = [1, 2, 9, 33, 60]
    d1 = np.array([0.9, 0.6, 0.35, 0.2])
    d2 = np.array([0.8, 0.7, 0.5, 0.125])
    U = planted_basis(n, I, d1, rng)
    V = planted_basis(n, J, d2, rng)
    assert np.allclose(U.T @ U, np.eye(4), atol=1e-14)
    S = np.array([5.0, 2.0, 0.5, 1e-3])
    ind, eta1, eta2 = cd.indicator(U, S, V, I, J)
    e1, e2 = 1.0 / 0.2, 1.0 / 0.125  # eta = ||U(I,:)^+||_2 = 1 / smallest singular value
    want = min(e1 * (1 + e2), e2 * (1 + e1)) * 1e-3 / math.sqrt(25 + 4 + 0.25 + 1e-6)
    assert abs(eta1 - e1) <= 1e-12 * e1 and abs(eta2 - e2) <= 1e-12 * e2
    assert abs(ind - want) <= 1e-12 * want
    # fewer rows than columns: sigma_min is the smallest of min(|I|, r) values
    ind3, eta13, _ = cd.indicator(U, S, V, I[:3], J)
    assert eta13 == pytest.approx(1.0 / np.linalg.svd(U[I[:3]], compute_uv=False)[-1], rel=1e-12)


# --------------------------------------------------------------------------------------
# warm start (Algorithm 4 inputs)
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [63, 255])
def test_warm_start_is_the_truncated_svd_of_fhat(n):
    U, s, V = workloads.make("n4095_r10_fp64", 3, n=n)
    Uh, Vh = cd.spectral_factors(n, U, s, V)
    U1, S1, V1 = cd.warm_start(Uh, Vh)
    Fh = bf.sine_matrix(n) @ ((U * (s / (n + 1) ** 2)[None, :]) @ V.T) @ bf.sine_matrix(n)
    X = (U1 * S1[None, :]) @ V1.T
    assert np.linalg.norm(X - Fh) <= 1e-14 * np.linalg.norm(Fh)
    assert np.allclose(U1.T @ U1, np.eye(S1.size), atol=1e-14)
    assert np.allclose(V1.T @ V1, np.eye(S1.size), atol=1e-14)
    assert np.all(np.diff(S1) <= 0)
    sv = np.linalg.svd(Fh, compute_uv=False)
    assert np.allclose(S1, sv[: S1.size], rtol=1e-12)


def test_warm_start_truncates_a_rank_deficient_rhs():
    n = 127
    U, s, V = workloads.make("n255_r5_fp64", 0, n=n)
    U = np.hstack([U, U[:, :1]])  # a repeated column: F has rank 5 with 6 factors
    V = np.hstack([V, V[:, :1]])
    s = np.concatenate([s, [0.7]])
    Uh, Vh = cd.spectral_factors(n, U, s, V)
    U1, S1, V1 = cd.warm_start(Uh, Vh)
    assert S1.size == 5
    assert S1[-1] > 6 * EPS * S1[0] * 1e6


def test_warm_start_from_a_guess_is_its_dense_svd():
    n = 63
    rng = np.random.default_rng(2)
    U0 = rng.standard_normal((n, 4))
    V0 = rng.standard_normal((n, 4))
    S0 = np.array([3.0, 1.0, 0.25, 0.01])
    U1, S1, V1 = cd.warm_start_from(n, U0, S0, V0)
    Z = bf.sine_matrix(n)
    G = Z @ ((U0 * S0[None, :]) @ V0.T) @ Z
    assert np.linalg.norm((U1 * S1[None, :]) @ V1.T - G) <= 1e-14 * np.linalg.norm(G)
    assert np.allclose(S1, np.linalg.svd(G, compute_uv=False)[:4], rtol=1e-12)
    # unit weights when S0 is None
    U2, S2, V2 = cd.warm_start_from(n, U0, None, V0)
    G2 = Z @ (U0 @ V0.T) @ Z
    assert np.linalg.norm((U2 * S2[None, :]) @ V2.T - G2) <= 1e-14 * np.linalg.norm(G2)
    # a zero guess leaves the start from the right-hand side
    U, s, V = workloads.make("n255_r5_fp64", 0, n=n)
    a = cd.solve(n, U, s, V, 16, 1e-10, 10)
    b = cd.solve(n, U, s, V, 16, 1e-10, 10, warm=(np.zeros((n, 2)), None, np.zeros((n, 2))))
    assert np.array_equal(a.U, b.U) and a.iters == b.iters
    # the right-hand side's own spectral factors as the guess reproduce the default solve
    h2 = 1.0 / (n + 1) ** 2
    c = cd.solve(n, U, s, V, 16, 1e-10, 10, warm=(U, h2 * s, V))
    assert [t.I_pre for t in c.trace] == [t.I_pre for t in a.trace]
    assert cd.rel_err((c.U, c.S, c.V), (a.U, a.S, a.V)) <= 1e-12


# --------------------------------------------------------------------------------------
# column-pivoted QR (QDEIM)
# --------------------------------------------------------------------------------------
def test_pivoted_qr_matches_lapack_and_gram_schmidt():
    sl = pytest.importorskip("scipy.linalg")
    rng = np.random.default_rng(0)
    for trial in range(8):
        m, n = int(rng.integers(2, 9)), int(rng.integers(10, 80))
        A = rng.standard_normal((m, n)) * rng.uniform(0.1, 3.0, n)[None, :]
        piv, gaps = cd.pivoted_qr_order(A, m)
        ref = [int(p) for p in sl.qr(A, pivoting=True, mode="r")[1][:m]]
        assert piv == ref
        assert piv == bf.gram_schmidt_pivots(A, m)


def test_pivoted_qr_ties_go_to_the_smaller_index():
    A = np.zeros((3, 8))
    A[0, 5] = A[0, 2] = 1.0          # equal norms: column 2 first, then 5 is dependent
    A[1, 6] = 1.0 + 1e-15            # within the tie window of the unit columns
    A[2, 7] = 0.5
    piv, _ = cd.pivoted_qr_order(A, 3)
    assert piv == [2, 6, 7]
    # an all-zero matrix: pivots in index order
    assert cd.pivoted_qr_order(np.zeros((2, 5)), 2)[0] == [0, 1]


def test_qdeim_select_union_and_safeguard():
    rng = np.random.default_rng(5)
    n = 30
    U, _ = np.linalg.qr(rng.standard_normal((n, 3)))
    piv, _ = cd.pivoted_qr_order(U.T, 3)
    first = cd.qdeim_select(U, 3, [], 10, True)
    assert first.indices[:3] == piv and len(first.indices) == 4  # safeguard at k = 0
    again = cd.qdeim_select(U, 3, first.indices, 10, False)  # nothing new: one extra index
    assert again.indices[:4] == first.indices and len(again.indices) == 5
    pi = np.sum(U * U, axis=1)
    outside = [i for i in range(n) if i not in first.indices]
    assert again.indices[4] == max(outside, key=lambda i: (pi[i], -i))
    assert len(cd.qdeim_select(U, 3, [], 2, True).indices) == 2  # cap


# --------------------------------------------------------------------------------------
# planted mistakes
# --------------------------------------------------------------------------------------
MUTATIONS = [
    ("sigma_max instead of sigma_min", "compute_uv=False)[-1]", "compute_uv=False)[0]"),
    ("indicator on the pre-prune sets", "indicator(cr.U, cr.S, cr.V, I, J)",
     "indicator(cr.U, cr.S, cr.V, selI.indices, selJ.indices)"),
    ("largest instead of smallest singular value in the indicator", "* float(S[-1]) / nrm", "* float(S[0]) / nrm"),
    ("transposed right factor in the warm start", "return Qu @ A[:, :r], s[:r].copy(), Qv @ Bt[:r].T",
     "return Qu @ A[:, :r], s[:r].copy(), Qv @ Bt[:, :r]"),
    ("branches of Algorithm 1 exchanged", "    if len(J) <= len(I):\n        M = pinv", "    if len(J) > len(I):\n        M = pinv"),
    ("absolute prune threshold", "keep = a >= tau * a.max()", "keep = a >= tau"),
    ("top-k over all indices", "free[np.asarray(list(I_prev), dtype=np.int64)] = False", "pass"),
    ("leverage over all columns", "np.sum(U[:, :r_sig] ** 2, axis=1)", "np.sum(U ** 2, axis=1)"),
    ("final rank one too large", "            r_star = r\n", "            r_star = min(r + 1, S.size)\n"),
    ("rho of a sum", "(Ub, -np.asarray(Sb), Vb)", "(Ub, np.asarray(Sb), Vb)"),
    ("eigenvalue index shift", "k = np.arange(1, n + 1, dtype=np.float64)", "k = np.arange(0, n, dtype=np.float64)"),
    ("DST scale", "out = -Y[1:N].imag / math.sqrt(2.0 * N)", "out = -Y[1:N].imag / math.sqrt(N)"),
    ("pivot ties to the larger index", "np.argmin(np.where(tied, cols[j:], n + 1))",
     "np.argmax(np.where(tied, cols[j:], -1))"),
    ("QDEIM safeguard missing at the first pass", "if (not new or first) and", "if (not new) and"),
    ("guess weights ignored", "return warm_start(dst1(U0) * S0[None, :], dst1(V0))",
     "return warm_start(dst1(U0), dst1(V0))"),
    ("r_sig counted against the last singular value", "r_sig = int(np.count_nonzero(S_prev > tol * S_prev[0]))",
     "r_sig = int(np.count_nonzero(S_prev > tol * S_prev[-1]))"),
    ("no stop at a fixed point", "if stop_at_fixed_point and pre_prev is not None and pre == pre_prev:",
     "if False:"),
]


def mutated_oracle(old, new):
    with open(ORACLE_SRC) as f:
        src = f.read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    name = "crossdeim_mutant"
    mod = types.ModuleType(name)
    sys.modules[name] = mod  # dataclasses look their module up while the class is created
    try:
        exec(compile(src.replace(old, new), name, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def warm_start_pin_holds(mod) -> bool:
    """The warm start of module `mod` reproduces the dense F^ (the pin of the warm start)."""
    n = 63
    U, s, V = workloads.make("n4095_r10_fp64", 3, n=n)
    Uh, Vh = mod.spectral_factors(n, U, s, V)
    U1, S1, V1 = mod.warm_start(Uh, Vh)
    Fh = bf.sine_matrix(n) @ ((U * (s / (n + 1) ** 2)[None, :]) @ V.T) @ bf.sine_matrix(n)
    return np.linalg.norm((U1 * S1[None, :]) @ V1.T - Fh) <= 1e-14 * np.linalg.norm(Fh)


@pytest.mark.parametrize("mutation", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(mutation):
    name, old, new = mutation
    mod = mutated_oracle(old, new)
    try:
        if not warm_start_pin_holds(mod):
            return
    except Exception:
        return
    for case in CASES:
        n, U, s, V, r_max, tol, maxiter, kw = case_inputs(case)
        try:
            o = mod.solve(n, U, s, V, r_max, tol, maxiter, **kw)
        except Exception:
            return  # the mutant breaks outright
        b = bf.solve(n, U, s, V, r_max, tol, maxiter, **kw)
        if disagreements(o, b):
            return
    pytest.fail(f"planted mistake not caught: {name}")
