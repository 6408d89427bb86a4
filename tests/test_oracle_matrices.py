"""Pins of the oracle's Cross-DEIM on the paper's test matrices (Section 4.2), on the CPU:

  * the entries against the formulas written the paper's way (1-based indices and grid);
  * the whole iteration against the dense brute-force implementation (Algorithm 1 as printed on
    the explicit matrix), pass by pass: ordered sets, pruned sizes, ranks, status, rho, the
    indicator and the final product, with leverage scores and with QDEIM;
  * the result within 100 times the best rank-r error of the dense SVD (Eckart-Young).
"""
import math

import numpy as np
import pytest

import brute_crossdeim as bf
import workloads
from oracle import crossdeim as cd


def test_entries_match_the_papers_formulas():
    n = 37
    i1 = np.arange(1, n + 1)  # 1-based
    H = 1.0 / (i1[:, None] + i1[None, :] - 1.0)  # the Hilbert matrix
    assert np.array_equal(cd.hilbert(n, range(n), range(n)), H)
    x = -1.0 + 2.0 * (i1 - 1) / (n - 1)
    K = np.power(np.abs(x[:, None] + x[None, :]) / 2.0, 5)
    assert np.allclose(cd.kmatrix(n, range(n), range(n)), K, rtol=4e-16, atol=0.0)
    # non-smooth along x + y = 0: zero on the anti-diagonal
    assert np.all(np.abs(np.diag(np.fliplr(cd.kmatrix(n, range(n), range(n))))) <= 1e-75)


def _dense(kind, n):
    return cd.MATRICES[kind](n, np.arange(n), np.arange(n))


@pytest.mark.parametrize("kind,n,tol,selector,seed", [
    ("hilbert", 31, 1e-9, "ls", 0), ("hilbert", 63, 1e-9, "ls", 1), ("hilbert", 63, 1e-9, "qdeim", 2),
    ("k", 31, 1e-6, "ls", 3), ("k", 63, 1e-6, "ls", 4), ("k", 63, 1e-6, "qdeim", 5),
])
def test_oracle_equals_dense_brute_force(kind, n, tol, selector, seed):
    U0, V0 = workloads.matrix_guess(n, 4, seed)
    o = cd.solve_matrix(kind, n, U0, V0, 32, tol, 15, selector=selector)
    b = bf.solve_matrix(_dense(kind, n), U0, V0, 32, tol, 15, selector=selector)
    assert len(o.trace) == len(b["passes"])
    for to, tb in zip(o.trace, b["passes"]):
        assert to.I_pre == tb.I_pre and to.J_pre == tb.J_pre, f"pass {to.k}"
        assert to.I == tb.I and to.J == tb.J and to.rank == tb.rank and to.branch == tb.branch
        if math.isfinite(tb.rho):
            # the K matrix's early iterates interpolate at nearly dependent rows (eta ~ 1e9), so
            # the two routes' rounding moves rho by up to ~1e-9 relative
            assert abs(to.rho - tb.rho) <= 1e-7 * max(tb.rho, 1e-3)
    assert o.status == b["status"] and o.iters == b["iters"] and o.rank == b["rank"]
    Xo = (o.U * o.S[None, :]) @ o.V.T
    Xb = (b["U"] * b["S"][None, :]) @ b["V"].T
    assert np.linalg.norm(Xo - Xb) <= 1e-11 * np.linalg.norm(Xb)


@pytest.mark.parametrize("kind,tol", [("hilbert", 1e-9), ("k", 1e-6)])
def test_result_within_the_best_rank_r_error(kind, tol):
    n = 200
    G = _dense(kind, n)
    U0, V0 = workloads.matrix_guess(n, 8, 11)
    o = cd.solve_matrix(kind, n, U0, V0, 64, tol, 20)
    sv = np.linalg.svd(G, compute_uv=False)
    best = math.sqrt(float(np.sum(sv[o.rank:] ** 2)))
    err = np.linalg.norm((o.U * o.S[None, :]) @ o.V.T - G)
    assert err <= max(100.0 * best, 10 * tol * np.linalg.norm(G))
    assert o.status in (cd.STATUS_OK, cd.STATUS_STAGNATED)


def test_zero_guess_is_rejected():
    with pytest.raises(ValueError):
        cd.solve_matrix("hilbert", 31, np.zeros((31, 2)), np.zeros((31, 2)), 8, 1e-9, 5)
