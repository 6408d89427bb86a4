"""Dense brute-force Cross-DEIM Poisson solve for tiny grids (n <= 127).

TEST INFRASTRUCTURE ONLY. It pins the oracle: it shares no code with oracle/ (nor with
the GPU library) and takes a different route through every step, so that a mistake in
either implementation shows up as a disagreement.

  * the spectral solution W^ is formed in full, h^2 (Z F Z) ./ (lambda_i + lambda_j), with
    a dense sine matrix Z built entry by entry (the product i k reduced modulo 2(n+1) in
    integers before the sine is taken);
  * the warm start is the SVD of the dense n x n matrix F^ = Z U_F diag(h^2 sigma) V_F^T Z;
  * Algorithm 1 runs as printed: Q(I,:) W = R is solved for the full |J| x n matrix W (or
    Z(J,:) W = C^T for the |I| x n one) by a truncated-SVD pseudo-inverse, and the SVD of
    that wide matrix gives the iterate (the oracle takes the SVD of a |J| x |I| core instead);
  * leverage-score selection ranks the whole complement with one sort;
  * rho is the norm of the dense difference of two iterates, eta_1 and eta_2 the spectral
    norms of pseudo-inverses;
  * the final rank is found by scanning r upwards.

The readings of the paper's silent or garbled passages are the same as the oracle's (they
define the method being tested); each step below names the passage it follows.
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence

import numpy as np

EPS = float(np.finfo(np.float64).eps)


def sine_matrix(n: int) -> np.ndarray:
    """Z(i, k) = sqrt(2/(n+1)) sin(pi i k / (n+1)), i, k = 1..n (Section 3)."""
    i = np.arange(1, n + 1, dtype=np.int64)
    ik = np.outer(i, i) % (2 * (n + 1))
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.pi * ik.astype(np.float64) / (n + 1))


def lam(n: int) -> np.ndarray:
    """Eigenvalues of tridiag(-1, 2, -1): 2 - 2 cos(pi k/(n+1)) = 4 sin^2(pi k/(2(n+1)))."""
    return 4.0 * np.sin(np.pi * np.arange(1, n + 1) / (2.0 * (n + 1))) ** 2


def spectral_solution(n: int, U_F, sigma, V_F) -> np.ndarray:
    """W^ = h^2 (Z F Z) ./ (lambda_i + lambda_j) as a dense n x n matrix (Section 3.1)."""
    Z = sine_matrix(n)
    h = 1.0 / (n + 1)
    F = (np.asarray(U_F) * np.asarray(sigma)[None, :]) @ np.asarray(V_F).T
    L = lam(n)
    return h * h * (Z @ F @ Z) / (L[:, None] + L[None, :])


def pinv_trunc(A: np.ndarray) -> np.ndarray:
    """Pseudo-inverse with the singular values <= max(rows, cols) eps sigma_1 dropped."""
    m, k = A.shape
    if m == 0 or k == 0:
        return np.zeros((k, m))
    Ua, s, Vt = np.linalg.svd(A, full_matrices=False)
    out = np.zeros((k, m))
    if s[0] == 0.0:
        return out
    for l in range(s.size):
        if s[l] > max(m, k) * EPS * s[0]:
            out += np.outer(Vt[l], Ua[:, l]) / s[l]
    return out


def trunc_svd(W: np.ndarray, rows: int, cols: int):
    """SVD of W kept above max(|I|, |J|) eps sigma_1 (Algorithm 1's truncated SVD)."""
    Ua, s, Vt = np.linalg.svd(W, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return Ua[:, :0], s[:0], Vt[:0]
    r = 0
    while r < s.size and s[r] > max(rows, cols) * EPS * s[0]:
        r += 1
    return Ua[:, :r], s[:r], Vt[:r]


def scross_dense(G: np.ndarray, I: Sequence[int], J: Sequence[int]):
    """Algorithm 1 on an explicit matrix G, step by step."""
    I = list(I)
    J = list(J)
    C = G[:, J]
    R = G[I, :]
    Q, RC = np.linalg.qr(C)
    Z, RR = np.linalg.qr(R.T)
    k, l = len(J), len(I)
    if k <= l:
        W = pinv_trunc(Q[I, :]) @ R  # Q(I,:) W = R, |J| x n
        Uh, s, Vt = trunc_svd(W, l, k)
        U = Q @ Uh
        V = Vt.T
    else:
        W = pinv_trunc(Z[J, :]) @ C.T  # Z(J,:) W = C^T, |I| x m
        Ut, s, Vht = trunc_svd(W.T, l, k)  # W^T = U S V^^T
        U = Ut
        V = Z @ Vht.T
    return U, s, V, np.diag(RC).copy(), np.diag(RR).copy(), k <= l


def leverage_pick(U: np.ndarray, r_sig: int, taken: Sequence[int], count: int) -> List[int]:
    """Algorithm 3 ranking: the `count` largest squared row norms of U(:, :r_sig) outside
    `taken` (ties, and scores at the (64 eps)^2 rounding floor, to the smaller index),
    returned in ascending index order."""
    n = U.shape[0]
    score = np.array([float(np.dot(U[i, :r_sig], U[i, :r_sig])) for i in range(n)])
    top = score.max() if n else 0.0
    score[score <= (64.0 * EPS) ** 2 * top] = 0.0
    taken = set(int(i) for i in taken)
    ranked = sorted((i for i in range(n) if i not in taken), key=lambda i: (-score[i], i))
    return sorted(ranked[:count])


def gram_schmidt_pivots(A: np.ndarray, count: int) -> List[int]:
    """Column-pivoted QR order by classical Gram-Schmidt with reorthogonalization: at each
    step the column farthest from the span of the chosen ones. Squared distances within
    1e-12 (relative) of the largest tie, those at the (64 eps)^2 floor of the largest
    squared column norm count as 0, and ties go to the smaller index."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    basis = np.zeros((m, 0))
    chosen: List[int] = []
    floor = (64.0 * EPS) ** 2 * max(float(np.dot(A[:, c], A[:, c])) for c in range(n))
    for _ in range(min(count, m, n)):
        R = A - basis @ (basis.T @ A)
        R = R - basis @ (basis.T @ R)
        d = np.array([float(np.dot(R[:, c], R[:, c])) for c in range(n)])
        d[d <= floor] = 0.0
        d[chosen] = -1.0
        top = d.max()
        best = min(c for c in range(n) if d[c] >= top * (1.0 - 1e-12) and d[c] >= 0.0)
        chosen.append(best)
        nb = R[:, best] / math.sqrt(d[best]) if d[best] > 0 else np.zeros(m)
        basis = np.hstack([basis, nb[:, None]])
    return chosen


def qdeim_pick(U: np.ndarray, r_sig: int, prev: Sequence[int], p_max: int, first: bool) -> List[int]:
    """Algorithm 2 (QDEIM) with Algorithm 4's union and safeguard (deterministic extra index)."""
    out = list(int(i) for i in prev)
    added = False
    for i in gram_schmidt_pivots(U[:, :r_sig].T, r_sig):
        if len(out) < p_max and i not in out:
            out.append(i)
            added = True
    if (not added or first) and len(out) < min(p_max, U.shape[0]):
        out.append(leverage_pick(U, r_sig, out, 1)[0])
    return out


def smallest_sv(A: np.ndarray) -> float:
    """sigma_min as 1 / ||A^+||_2 (no truncation), 0 for a singular or empty A."""
    if A.size == 0:
        return 0.0
    P = np.linalg.pinv(A, rcond=0.0)
    nrm = float(np.linalg.norm(P, 2))
    return 0.0 if not math.isfinite(nrm) or nrm == 0.0 else 1.0 / nrm


class Pass:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def cross_deim_dense(G, it, r_max, tol, maxiter, prune_tau=1e-12, replay=None, selector="ls"):
    """Algorithm 4 on a dense G from the starting iterate it = (U, S, V)."""
    Up, Sp, Vp = it
    I: List[int] = []
    J: List[int] = []
    prev_pre = None
    passes = []
    status = 1
    iters = 0
    for k in range(maxiter):
        r_sig = int(np.sum(Sp > tol * Sp[0]))
        if replay is not None and k < len(replay):
            Ipre = [int(i) for i in replay[k][0]]
            Jpre = [int(j) for j in replay[k][1]]
        elif selector == "qdeim":
            Ipre = qdeim_pick(Up, r_sig, I, r_max, k == 0)
            Jpre = qdeim_pick(Vp, r_sig, J, r_max, k == 0)
        else:
            s_I = max(0, min(r_sig, r_max - len(I)))
            s_J = max(0, min(r_sig, r_max - len(J)))
            Ipre = I + leverage_pick(Up, r_sig, I, s_I)
            Jpre = J + leverage_pick(Vp, r_sig, J, s_J)
        if prev_pre is not None and (Ipre, Jpre) == prev_pre:
            status = 2
            break
        U, S, V, rC, rR, branch = scross_dense(G, Ipre, Jpre)
        iters += 1
        aR, aC = np.abs(rR), np.abs(rC)
        I = [i for i, d in zip(Ipre, aR) if d >= prune_tau * aR.max()]
        J = [j for j, d in zip(Jpre, aC) if d >= prune_tau * aC.max()]
        nrm = math.sqrt(float(np.sum(S * S)))
        s1 = smallest_sv(U[I, :])
        s2 = smallest_sv(V[J, :])
        eta1 = math.inf if s1 == 0.0 else 1.0 / s1
        eta2 = math.inf if s2 == 0.0 else 1.0 / s2
        ind = min(eta1 * (1.0 + eta2), eta2 * (1.0 + eta1)) * float(S.min()) / nrm
        if k == 0:
            rho = math.inf
        else:
            rho = float(np.linalg.norm((U * S) @ V.T - (Up * Sp) @ Vp.T)) / nrm
        passes.append(Pass(k=k, I_pre=Ipre, J_pre=Jpre, I=list(I), J=list(J), rank=S.size, S=S.copy(),
                           rho=rho, indicator=ind, eta1=eta1, eta2=eta2, branch=branch))
        Up, Sp, Vp = U, S, V
        prev_pre = (Ipre, Jpre)
        if max(rho, ind) < tol:
            status = 0
            break
    return Up, Sp, Vp, status, iters, passes, I, J


def final_rank_scan(Sp, tol, r_max):
    """Smallest r whose tail of squared singular values is below (tol ||S||)^2, scanning upwards."""
    total = float(np.sum(Sp * Sp))
    r = 0
    while r < Sp.size and float(np.sum(Sp[r:] ** 2)) >= (tol * math.sqrt(total)) ** 2:
        r += 1
    return max(min(r, r_max), 1)


def solve(n, U_F, sigma, V_F, r_max, tol, maxiter, prune_tau=1e-12, warm=None, replay=None,
          selector="ls"):
    """Algorithm 4 on the dense W^; returns a dict with the physical factors and the trace."""
    Z = sine_matrix(n)
    G = spectral_solution(n, U_F, sigma, V_F)
    h = 1.0 / (n + 1)
    Fh = Z @ ((np.asarray(U_F) * (h * h * np.asarray(sigma))[None, :]) @ np.asarray(V_F).T) @ Z
    rF = np.asarray(U_F).shape[1]

    def start(M, rank_cap):
        Ua, s, Vt = np.linalg.svd(M)
        if s[0] == 0.0:
            return None
        r = int(np.sum(s > rank_cap * EPS * s[0]))
        return Ua[:, :r], s[:r], Vt[:r].T

    it = start(Fh, rF)
    if it is None:
        z = np.zeros((n, 1))
        return {"U": z, "S": np.zeros(1), "V": z, "rank": 1, "status": 0, "iters": 0, "passes": []}
    if warm is not None:
        U0, S0, V0 = warm
        S0 = np.ones(np.asarray(U0).shape[1]) if S0 is None else np.asarray(S0)
        g = start(Z @ ((np.asarray(U0) * S0[None, :]) @ np.asarray(V0).T) @ Z, np.asarray(U0).shape[1])
        if g is not None:
            it = g
    Up, Sp, Vp, status, iters, passes, I, J = cross_deim_dense(G, it, r_max, tol, maxiter, prune_tau, replay,
                                                              selector)
    r = final_rank_scan(Sp, tol, r_max)
    return {"U": Z @ Up[:, :r], "S": Sp[:r].copy(), "V": Z @ Vp[:, :r], "rank": r, "status": status,
            "iters": iters, "passes": passes, "I": I, "J": J}


def solve_matrix(G, U0, V0, r_max, tol, maxiter, prune_tau=1e-12, selector="ls"):
    """Algorithm 4 on an explicit dense matrix G, started from the SVD of U0 V0^T (truncated at
    r0 eps sigma_1); returns a dict as solve (no sine transforms)."""
    M = np.asarray(U0) @ np.asarray(V0).T
    Ua, s, Vt = np.linalg.svd(M)
    r0 = np.asarray(U0).shape[1]
    r = int(np.sum(s > r0 * EPS * s[0]))
    it = (Ua[:, :r], s[:r], Vt[:r].T)
    Up, Sp, Vp, status, iters, passes, I, J = cross_deim_dense(G, it, r_max, tol, maxiter, prune_tau, None,
                                                              selector)
    r = final_rank_scan(Sp, tol, r_max)
    return {"U": Up[:, :r], "S": Sp[:r].copy(), "V": Vp[:, :r], "rank": r, "status": status,
            "iters": iters, "passes": passes, "I": I, "J": J}
