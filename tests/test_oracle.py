"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

None of these tests retypes an oracle formula to compare it with itself: each checks an
oracle function against an independent route (brute force, closed form, the 3-point
stencil, a library routine, an invariant or an exact-arithmetic identity).
"""
import math

import numpy as np
import pytest
import scipy.fft

import workloads
from oracle import crossdeim as cd
from oracle import dense

EPS = np.finfo(np.float64).eps


def brute_Z(n):
    """Dense orthonormal DST-I matrix; i*k is reduced mod 2(n+1) in integers before sin."""
    N = n + 1
    i = np.arange(1, n + 1, dtype=np.int64)
    ik = np.mod(np.outer(i, i), 2 * N)
    return math.sqrt(2.0 / N) * np.sin(np.pi * ik.astype(np.float64) / N)


def tridiag(n):
    return 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


# --------------------------------------------------------------------------------------
# Section 3: eigenpairs of T
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 7, 63, 255])
def test_eigenvalues_are_eigenvalues_of_T(n):
    lam = cd.eigenvalues(n)
    ref = np.linalg.eigvalsh(tridiag(n))  # LAPACK, independent of the closed form
    assert np.max(np.abs(np.sort(lam) - ref)) <= 4 * n * EPS  # LAPACK backward error bound, ||T|| < 4
    assert np.all(lam > 0) and np.all(lam < 4) and np.all(np.diff(lam) > 0)


@pytest.mark.parametrize("n", [7, 63, 255])
def test_eigenvectors_residual(n):
    lam = cd.eigenvalues(n)
    Z = brute_Z(n)
    res = tridiag(n) @ Z - Z * lam[None, :]
    assert np.max(np.abs(res)) <= 1e-14


def test_eigenvalue_small_mode_no_cancellation():
    # 2(1 - cos x) loses all digits for tiny x; the oracle's value must match the Taylor series
    n = 1048575
    x = math.pi / (n + 1)
    taylor = x * x - x ** 4 / 12.0 + x ** 6 / 360.0
    assert abs(cd.eigenvalues(n)[0] - taylor) <= 4 * EPS * taylor
    assert abs(2 * (1 - math.cos(x)) - taylor) > 1e-7 * taylor  # the literal form cancels


# --------------------------------------------------------------------------------------
# Orthonormal DST-I (Sections 3 and 3.2)
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 7, 15, 255, 1023])
def test_dst_matches_brute_force(n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 3))
    ref = brute_Z(n) @ X
    got = cd.dst1(X)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref))) * math.log2(n + 1)


@pytest.mark.parametrize("n", [15, 1023, 65535])
def test_dst_is_involution_and_isometry(n):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((n, 2))
    Y = cd.dst1(X)
    assert np.allclose(np.linalg.norm(Y, axis=0), np.linalg.norm(X, axis=0), rtol=1e-13, atol=0)
    assert np.max(np.abs(cd.dst1(Y) - X)) <= 1e-13


@pytest.mark.parametrize("n,k", [(255, 1), (255, 17), (4095, 50), (65535, 3)])
def test_dst_maps_sine_to_unit_vector(n, k):
    x = workloads.grid(n)
    y = cd.dst1(np.sin(k * np.pi * x))
    e = np.zeros(n)
    e[k - 1] = math.sqrt((n + 1) / 2.0)
    assert np.max(np.abs(y - e)) <= 1e-12 * math.sqrt(n)


@pytest.mark.parametrize("n", [7, 255, 4095])
def test_dst_matches_scipy(n):
    rng = np.random.default_rng(7)
    X = rng.standard_normal((n, 2))
    ref = scipy.fft.dst(X, type=1, norm="ortho", axis=0)
    assert np.max(np.abs(cd.dst1(X) - ref)) <= 1e-13


# --------------------------------------------------------------------------------------
# eq. g_for_p: the spectrally divided solution, from factors vs dense
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [31, 63])
def test_fibers_equal_dense_spectral_solution(n):
    U, s, V = workloads.make("n255_r5_fp64", seed=3, n=n)
    F = (U * s) @ V.T
    h = 1.0 / (n + 1)
    Z = brute_Z(n)
    lam = np.linalg.eigvalsh(tridiag(n))
    Wh = h * h * (Z.T @ F @ Z) / (lam[:, None] + lam[None, :])
    Uh, Vh = cd.spectral_factors(n, U, s, V)
    lam_o = cd.eigenvalues(n)
    J = [0, 5, n - 1, 17]
    I = [3, 0, n - 2]
    scale = np.max(np.abs(Wh))
    assert np.max(np.abs(cd.columns(Uh, Vh, lam_o, J) - Wh[:, J])) <= 1e-13 * scale
    assert np.max(np.abs(cd.rows(Uh, Vh, lam_o, I) - Wh[I, :])) <= 1e-13 * scale


# --------------------------------------------------------------------------------------
# Section 3.1: dense solve satisfies the 5-point equation; sine modes in closed form
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [63, 255])
def test_dense_solve_residual(n):
    U, s, V = workloads.make("n255_r5_fp64", seed=0, n=n)
    F = (U * s) @ V.T
    W = dense.dense_solve(F)
    h = 1.0 / (n + 1)
    T = tridiag(n)
    res = T @ W + W @ T.T - h * h * F  # explicit matrices, no DST involved
    assert np.linalg.norm(res) <= 1e-13 * 4 * np.linalg.norm(W)  # rounding relative to ||T|| ||W||
    assert np.allclose(dense.laplacian_apply(W), T @ W + W @ T.T, rtol=0, atol=1e-15)


def closed_form_sine(n, modes):
    """W for F = sum a sin(k pi x) sin(l pi y): a s_k s_l^T / ((4/h^2)(sin^2(k pi h/2) + sin^2(l pi h/2)))."""
    x = workloads.grid(n)
    h = 1.0 / (n + 1)
    W = np.zeros((n, n))
    for k, l, a in modes:
        den = (4.0 / h ** 2) * (math.sin(k * math.pi * h / 2) ** 2 + math.sin(l * math.pi * h / 2) ** 2)
        W += a * np.outer(np.sin(k * math.pi * x), np.sin(l * math.pi * x)) / den
    return W


def test_dense_solve_sine_closed_form():
    n = 255
    modes = [(3, 7, 1.5), (40, 2, -0.25)]
    U, s, V = workloads.sine_rhs(n, modes)
    W = dense.dense_solve((U * s) @ V.T)
    ref = closed_form_sine(n, modes)
    assert np.max(np.abs(W - ref)) <= 1e-14 * np.max(np.abs(ref)) * 10


# --------------------------------------------------------------------------------------
# Algorithm 1 (scross)
# --------------------------------------------------------------------------------------
def test_scross_reconstructs_exact_rank():
    # lambda = 1/2 makes W^ = U^ V^^T exactly; with |I| = |J| = rank the cross is exact
    rng = np.random.default_rng(11)
    n, p = 200, 6
    A = rng.standard_normal((n, p))
    B = rng.standard_normal((n, p))
    lam = np.full(n, 0.5)
    for I, J in [(list(rng.choice(n, p, replace=False)), list(rng.choice(n, p, replace=False))),
                 (list(range(p + 3)), list(range(10, 10 + p))),
                 (list(range(p)), list(range(20, 20 + p + 4)))]:
        cr = cd.scross(A, B, lam, I, J)
        G = A @ B.T
        X = (cr.U * cr.S) @ cr.V.T
        assert np.linalg.norm(X - G) <= 1e-12 * np.linalg.norm(G)
        assert cr.S.size == p
        assert np.allclose(cr.U.T @ cr.U, np.eye(p), atol=1e-13)
        assert np.allclose(cr.V.T @ cr.V, np.eye(p), atol=1e-13)


def test_scross_interpolates_and_matches_cross_formula():
    n = 127
    U, s, V = workloads.make("n255_r5_fp64", seed=2, n=n)
    Uh, Vh = cd.spectral_factors(n, U, s, V)
    lam = cd.eigenvalues(n)
    G = cd.columns(Uh, Vh, lam, range(n))
    I = [0, 2, 4, 7]
    J = [1, 0, 3, 6]
    cr = cd.scross(Uh, Vh, lam, I, J)
    X = (cr.U * cr.S) @ cr.V.T
    C = G[:, J]
    R = G[I, :]
    Gij = G[np.ix_(I, J)]
    assert np.linalg.cond(Gij) < 1e8
    ref = C @ np.linalg.solve(Gij, R)  # G(:,J) G(I,J)^+ G(I,:) in eq. (1)
    sc = np.linalg.norm(G)
    assert np.linalg.norm(X - ref) <= 1e-9 * sc
    assert np.linalg.norm(X[I, :] - R) <= 1e-9 * sc
    assert np.linalg.norm(X[:, J] - C) <= 1e-9 * sc
    # diag(R_C) of the unpivoted QR: |R_ll| = distance of column l from the span of the previous ones
    for l in range(len(J)):
        prev = C[:, :l]
        resid = C[:, l] - prev @ np.linalg.lstsq(prev, C[:, l], rcond=None)[0] if l else C[:, 0]
        assert abs(abs(cr.rC[l]) - np.linalg.norm(resid)) <= 1e-10 * np.linalg.norm(C)


def test_scross_else_branch_same_as_first_branch_when_square():
    # |J| > |I| takes the second branch; for an exact-rank W^ both branches give W^
    rng = np.random.default_rng(5)
    n, p = 90, 4
    A = rng.standard_normal((n, p))
    B = rng.standard_normal((n, p))
    lam = np.full(n, 0.5)
    c1 = cd.scross(A, B, lam, list(range(8)), list(range(30, 34)))  # |J| <= |I|
    c2 = cd.scross(A, B, lam, list(range(4)), list(range(30, 38)))  # |J| >  |I|
    for cr in (c1, c2):
        assert np.linalg.norm((cr.U * cr.S) @ cr.V.T - A @ B.T) <= 1e-12 * np.linalg.norm(A @ B.T)


def test_pinv_matches_numpy_with_same_cutoff():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((12, 5)) @ np.diag([1, 1e-3, 1e-8, 1e-15, 1e-17]) @ rng.standard_normal((5, 5))
    ref = np.linalg.pinv(A, rcond=12 * EPS)
    assert np.allclose(cd.pinv(A), ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


# --------------------------------------------------------------------------------------
# Algorithm 3 (leverage scores) and the index-set update
# --------------------------------------------------------------------------------------
def test_leverage_scores_sum_and_basis_invariance():
    rng = np.random.default_rng(0)
    n, r = 300, 7
    Q, _ = np.linalg.qr(rng.standard_normal((n, r)))
    pi = cd.leverage_scores(Q, r)
    assert abs(pi.sum() - r) <= 1e-12
    O, _ = np.linalg.qr(rng.standard_normal((r, r)))
    assert np.max(np.abs(cd.leverage_scores(Q @ O, r) - pi)) <= 1e-14
    # the SVD basis of the same space gives the same scores
    Us = np.linalg.svd(Q @ rng.standard_normal((r, r)), full_matrices=False)[0]
    assert np.max(np.abs(cd.leverage_scores(Us, r) - pi)) <= 1e-14


def test_select_brute_force():
    rng = np.random.default_rng(4)
    n = 40
    U = rng.standard_normal((n, 5))
    U[[3, 9, 12], :] = 0.0  # exact ties at zero go to the smaller index
    U[20] = U[21]  # an exact tie between two nonzero scores
    prev = [5, 1, 30]
    sel = cd.select(U, 3, prev, p_max=10)
    pi = np.sum(U[:, :3] ** 2, axis=1)
    cands = sorted((i for i in range(n) if i not in prev), key=lambda i: (-pi[i], i))
    assert sel.indices[:3] == prev
    assert sel.new == sorted(cands[:3])
    # cap: only p_max - |prev| new indices
    assert len(cd.select(U, 5, prev, p_max=4).new) == 1
    # all candidates tie at zero -> smallest indices outside prev
    Z = np.zeros((n, 2))
    assert cd.select(Z, 2, [0, 2], p_max=8).new == [1, 3]


def test_prune_relative_threshold():
    assert cd.prune([4, 7, 9], np.array([2.0, -1e-13, 5e-12]), 1e-12) == [4, 9]
    assert cd.prune([4, 7], np.array([1e-30, 1e-43]), 1e-12) == [4]


# --------------------------------------------------------------------------------------
# Norm of a factored difference (rho of Algorithm 4 and the error metric)
# --------------------------------------------------------------------------------------
def test_lr_norm_matches_dense_and_resolves_tiny_differences():
    rng = np.random.default_rng(9)
    n = 60
    Ua, _ = np.linalg.qr(rng.standard_normal((n, 5)))
    Va, _ = np.linalg.qr(rng.standard_normal((n, 5)))
    Sa = np.array([3.0, 2.0, 1.0, 0.5, 1e-3])
    dn = np.linalg.norm((Ua * Sa) @ Va.T)
    assert abs(cd.lr_norm([(Ua, Sa, Va)]) - dn) <= 1e-14 * dn
    Ub, Sb, Vb = rng.standard_normal((n, 3)), rng.standard_normal(3), rng.standard_normal((n, 3))
    d = (Ua * Sa) @ Va.T - (Ub * Sb) @ Vb.T
    assert abs(cd.lr_diff_norm(Ua, Sa, Va, Ub, Sb, Vb) - np.linalg.norm(d)) <= 1e-13 * np.linalg.norm(d)
    # a 1e-12 relative perturbation: the Gram identity ||A||^2 + ||B||^2 - 2<A,B> cannot see it
    E = rng.standard_normal((n, 1))
    Up = np.hstack([Ua, E])
    Sp = np.concatenate([Sa, [1e-12 * np.linalg.norm(Sa)]])
    Vp = np.hstack([Va, rng.standard_normal((n, 1))])
    exact = 1e-12 * np.linalg.norm(Sa) * np.linalg.norm(E) * np.linalg.norm(Vp[:, -1])
    got = cd.lr_diff_norm(Up, Sp, Vp, Ua, Sa, Va)
    assert abs(got - exact) <= 1e-3 * exact


# --------------------------------------------------------------------------------------
# Algorithm 4: the whole solve
# --------------------------------------------------------------------------------------
def best_rank_err(W, r):
    sv = np.linalg.svd(W, compute_uv=False)
    return math.sqrt(float(np.sum(sv[r:] ** 2))) / float(np.linalg.norm(sv))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_solve_n255_against_dense(seed):
    w = workloads.CONFIGS["n255_r5_fp64"]
    U, s, V = workloads.make(w, seed)
    res = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    W = dense.dense_solve((U * s) @ V.T)
    err = np.linalg.norm((res.U * res.S) @ res.V.T - W) / np.linalg.norm(W)
    assert err <= max(100 * best_rank_err(W, res.rank), 1e-12)
    assert res.rank <= w.r_max
    assert np.allclose(res.U.T @ res.U, np.eye(res.rank), atol=1e-12)


def test_solve_n4095_against_dense_and_sine_part():
    w = workloads.CONFIGS["n4095_r10_fp64"]
    U, s, V = workloads.make(w, 0)
    res = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    W = dense.dense_solve((U * s) @ V.T)
    err = np.linalg.norm((res.U * res.S) @ res.V.T - W) / np.linalg.norm(W)
    assert err <= max(100 * best_rank_err(W, res.rank), 1e-12)
    # the sine part of the RHS alone has a closed-form solution
    _, _, _, info = workloads.bump_rhs(w.n, 0, w.n_bumps, w.width_lo, w.width_hi, w.n_sines)
    modes = [(int(k), int(l), float(b)) for k, l, b in zip(info["kx"], info["ky"], info["b"])]
    Us, ss, Vs = workloads.sine_rhs(w.n, modes)
    rs = cd.solve(w.n, Us, ss, Vs, w.r_max, w.tol, w.maxiter)
    ref = closed_form_sine(w.n, modes)
    assert rs.rank == len({(k, l) for k, l, _ in modes})
    assert np.linalg.norm((rs.U * rs.S) @ rs.V.T - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("n", [255, 1048575])
def test_solve_manufactured_sine_rank_one(n):
    k, l, a = 5, 9, 2.0
    U, s, V = workloads.sine_rhs(n, [(k, l, a)])
    res = cd.solve(n, U, s, V, 8, 1e-10, 10)
    assert res.rank == 1
    h = 1.0 / (n + 1)
    den = (4.0 / h ** 2) * (math.sin(k * math.pi * h / 2) ** 2 + math.sin(l * math.pi * h / 2) ** 2)
    x = workloads.grid(n)
    ref_u = np.sin(k * math.pi * x)[:, None]
    ref_v = np.sin(l * math.pi * x)[:, None]
    e = cd.rel_err((res.U, res.S, res.V), (ref_u, np.array([a / den]), ref_v))
    assert e <= 1e-13
    # the sine row/column are selected; every extra row/column of W^ is zero and is pruned
    assert (k - 1) in res.trace[0].I_pre and (l - 1) in res.trace[0].J_pre
    assert res.I == [k - 1] and res.J == [l - 1]


def factored_residual(n, res, U, s, V):
    """||T W + W T - h^2 F||_F in factored form, T applied by the stencil (no DST)."""
    h = 1.0 / (n + 1)
    TU = dense.tridiag_apply(res.U)
    TV = dense.tridiag_apply(res.V)
    return cd.lr_norm([(TU, res.S, res.V), (res.U, res.S, TV), (U, -h * h * np.asarray(s), V)])


def test_solve_residual_large_n():
    w = workloads.CONFIGS["n65535_r20_fp64"]
    n = 16383
    U, s, V = workloads.make(w, 0, n=n)
    res = cd.solve(n, U, s, V, w.r_max, w.tol, w.maxiter)
    Wn = cd.lr_norm([(res.U, res.S, res.V)])
    # ||T E + E T|| <= 8 ||E||; the solve error is far below 1e-6 relative
    assert factored_residual(n, res, U, s, V) <= 8 * 1e-6 * Wn
    assert res.status in (cd.STATUS_OK, cd.STATUS_STAGNATED)


def test_fixed_point_exit_is_exact():
    w = workloads.CONFIGS["n255_r5_fp64"]
    U, s, V = workloads.make(w, 0)
    a = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    b = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, stop_at_fixed_point=False)
    assert a.status == cd.STATUS_STAGNATED and b.status == cd.STATUS_NOT_CONVERGED
    assert b.iters == w.maxiter
    assert np.array_equal(a.U, b.U) and np.array_equal(a.S, b.S) and np.array_equal(a.V, b.V)


def test_status_and_degenerate_inputs():
    n = 63
    z = np.zeros((n, 2))
    res = cd.solve(n, z, np.ones(2), z, 8, 1e-10, 5)
    assert res.rank == 1 and res.S[0] == 0.0 and res.status == cd.STATUS_OK
    U, s, V = workloads.make("n255_r5_fp64", 0, n=n)
    r1 = cd.solve(n, U, s, V, 16, 1e-10, 1)
    assert r1.status == cd.STATUS_NOT_CONVERGED and r1.iters == 1
    r2 = cd.solve(n, U, s, V, 3, 1e-14, 20)
    assert r2.status == cd.STATUS_STAGNATED and r2.rank <= 3
    r0 = cd.solve(n, U, s, V, 16, 1e-10, 0)
    assert r0.iters == 0 and r0.rank >= 1


# --------------------------------------------------------------------------------------
# Planted mistakes in the oracle must be caught by the pins above
# --------------------------------------------------------------------------------------
def test_planted_mistakes_are_caught(monkeypatch):
    n = 63
    U, s, V = workloads.make("n255_r5_fp64", 0, n=n)
    F = (U * s) @ V.T
    h = 1.0 / (n + 1)
    T = tridiag(n)

    def residual_ok():
        W = dense.dense_solve(F)
        return np.linalg.norm(T @ W + W @ T - h * h * F) <= 1e-13 * np.linalg.norm(h * h * F)

    assert residual_ok()
    good_eig = cd.eigenvalues
    monkeypatch.setattr(dense, "eigenvalues", lambda m: 4.0 * np.sin(np.arange(m) * np.pi / (2.0 * (m + 1))) ** 2 + 1e-3)
    assert not residual_ok()  # an index shift in lambda
    monkeypatch.setattr(dense, "eigenvalues", good_eig)
    good_dst = cd.dst1
    monkeypatch.setattr(dense, "dst1", lambda X: good_dst(X) * 1.0001)
    assert not residual_ok()  # a wrong DST scale
    monkeypatch.setattr(dense, "dst1", good_dst)
    # a transposed core in scross breaks exact reconstruction
    rng = np.random.default_rng(1)
    A, B = rng.standard_normal((50, 4)), rng.standard_normal((50, 4))
    lam = np.full(50, 0.5)
    good_svd = np.linalg.svd

    def bad_svd(M, *a, **k):
        return good_svd(M.T if M.shape[0] == M.shape[1] and M.shape[0] == 4 else M, *a, **k)

    monkeypatch.setattr(cd.np.linalg, "svd", bad_svd)
    cr = cd.scross(A, B, lam, list(range(4)), list(range(10, 14)))
    monkeypatch.setattr(cd.np.linalg, "svd", good_svd)
    assert np.linalg.norm((cr.U * cr.S) @ cr.V.T - A @ B.T) > 1e-3 * np.linalg.norm(A @ B.T)
