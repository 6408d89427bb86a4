"""Cross-DEIM low-rank Poisson solve, written out in plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke entry point and the
benchmark's CPU-baseline leg, never by the GPU library.

The solver (Section 3.2): the right-hand side F = U_F diag(sigma) V_F^T is moved to
the sine basis with the orthonormal DST-I, the spectrally divided solution
W^(i,j) = h^2 F^(i,j) / (lambda_i + lambda_j) (Section 3.1, eq. g_for_p) is
approximated by Cross-DEIM (Algorithm 4) without ever forming it, and the factors
are moved back with the same DST.

Readings of passages that are silent, ambiguous or garbled (each is also listed in
the design notes of the repository):
  * eigenvalues: 2(1 - cos(pi k/(n+1))) is evaluated as 4 sin^2(pi k/(2(n+1))),
    equal in exact arithmetic, without the cancellation at small k.
  * index selection: Algorithm 3 samples at random; here the leverage scores of the
    leading r_sig columns choose the top r_sig indices from the complement of the
    current set (ties and scores below a rounding floor go to the smaller index);
    the new indices are appended in ascending index order after the old ones (the
    paper notes that leverage-score sets are unordered); the set size is capped at
    r_max. This replaces the union and the random safeguard of
    Algorithm 4 (the paper allows dropping the safeguard for leverage scores).
  * r_sig = #{sigma_l > eps * sigma_1} of the previous iterate.
  * the warm start U_{-1}, V_{-1} is the truncated SVD of F^ itself (the paper only
    asks for an initial guess of the singular vector matrices).
  * Algorithm 1 roles: k = |J| and l = |I|; the first branch (|J| <= |I|) solves
    Q(I,:) W = G(I,:); the second solves with Z(J,:) (written Z(:,J) in the
    listing). Both solves use the pseudo-inverse with the default relative cutoff
    max(rows, cols) * eps of torch.linalg.pinv, the routine the paper names; the
    "truncated SVD" of the core uses the same cutoff with max(|I|, |J|).
  * the pruning thresholds of Algorithm 4 are relative to max |diag R|; all flags
    are computed before anything is removed; the second loop runs over J.
  * eta_1, eta_2 are the norms of the pseudo-inverses of U_k(I_k,:), V_k(J_k,:)
    (the DEIM error constants), on the pruned sets.
  * eps is relative to ||S_k||_F in rho, in the indicator and in the final
    truncation; the loop makes exactly maxiter passes; no stop at k = 0; when the
    pre-prune index sets repeat, the iteration has reached a fixed point and the
    previous iterate is returned.
  * QDEIM selection (Algorithm 2, QDEIM branch, as Algorithm 4's index selection): the
    first r_sig pivots of the column-pivoted QR of U_{k-1}(:, :r_sig)^T, pivoting on
    the largest remaining column norm (ties to the smaller index); the indices not
    already in I_{k-1} are appended in pivot order (Algorithm 4's union; QDEIM sets
    are ordered). Algorithm 4's safeguard appends one more index when nothing
    was added or at k = 0; the paper draws it at random, here it is the index outside
    the set with the largest leverage score (ties and noise to the smaller index),
    and it is added to the current set rather than to I*_k alone.
  * sampled leverage scores (Algorithm 3 as stated): row i is kept with probability
    p_i = min(1, c pi_i / r_sig) with c = rho r_sig, i.e. p_i = min(1, rho pi_i) for the floored
    score pi_i = sum_{eta < r_sig} U(i, eta)^2 (Algorithm 3's 1/k normalization with k = r_sig;
    the paper fixes only the order of c); the uniform u_i comes from the counter-based generator
    Philox4x32-10 with counter (i mod 2^32, i / 2^32, pass, side) and key (seed mod 2^32,
    seed / 2^32), u_i = 53 bits of its first two outputs / 2^53, and i is kept when u_i < p_i.
    The kept rows outside I_{k-1} are taken by (score descending, index ascending) up to the cap
    and appended in ascending index order; when none was kept (and the cap allows), the
    safeguard of Algorithm 4 appends a random index of the complement: the one with the
    largest -1 - u_i (computed in FP64; ties to the smaller index).
  * the test matrices of Section 4.2 are square (m = n) with 0-based indices: H(i, j) =
    1/(1 + i + j) is then the Hilbert matrix, and K uses the grid x_i = -1 + 2 i/(n - 1) on
    both sides. Cross-DEIM on them starts from the truncated SVD of a given guess U0 V0^T
    (Algorithm 4's inputs; the tests draw seeded Gaussian guesses) and returns the cross
    approximation itself, truncated as the Poisson solve.
  * the initial guess U0, V0 of Algorithm 4 is given in physical space (the space of
    the solver's output factors, e.g. a previous solution U_W, S, V_W) with optional
    weights S0: the warm start is then the truncated SVD of
    DST(U0) diag(S0) DST(V0)^T, computed exactly as the default warm start from the
    right-hand side.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

EPS = float(np.finfo(np.float64).eps)

STATUS_OK = 0
STATUS_NOT_CONVERGED = 1
STATUS_STAGNATED = 2

#: Leverage scores at or below FLOOR_REL * max(pi) are rounding noise; they count as 0.
FLOOR_REL = (64.0 * EPS) ** 2
#: Pivoted QR: squared column norms within this relative distance of the largest are ties.
PIVOT_TIE_REL = 1e-12


# ----------------------------------------------------------------------------------------
# Section 3: eigenpairs of T = tridiag(-1, 2, -1), and the orthonormal DST-I
# ----------------------------------------------------------------------------------------
def eigenvalues(n: int) -> np.ndarray:
    """lambda_k = 2(1 - cos(pi k/(n+1))) = 4 sin^2(pi k/(2(n+1))), k = 1..n (Section 3)."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return 4.0 * np.sin(k * np.pi / (2.0 * (n + 1))) ** 2


def dst1(X: np.ndarray) -> np.ndarray:
    """Orthonormal DST-I along axis 0: (Z x)_i = sqrt(2/(n+1)) sum_k x_k sin(i k pi/(n+1)).

    Z holds the eigenvectors z_k of T (Section 3); it is symmetric and orthogonal, so
    DST(DST(x)) = x as Section 3.2 requires. Computed through the DFT of the odd
    extension [0, x, 0, -reverse(x)] of length 2(n+1), whose imaginary part is
    -2 sum_k x_k sin(pi i k/(n+1)).
    """
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    n = X.shape[0]
    N = n + 1
    ext = np.zeros((2 * N, X.shape[1]))
    ext[1:N] = X
    ext[N + 1 :] = -X[::-1]
    Y = np.fft.fft(ext, axis=0)
    out = -Y[1:N].imag / math.sqrt(2.0 * N)
    return out[:, 0] if vec else out


def spectral_factors(n: int, U_F: np.ndarray, sigma: np.ndarray, V_F: np.ndarray):
    """U^ = DST(U_F) diag(h^2 sigma), V^ = DST(V_F) (Section 3.2).

    With these, W^(i,j) = sum_t U^(i,t) V^(j,t) / (lambda_i + lambda_j), i.e. eq. g_for_p
    with F^ = DST(U_F) S_F DST(V_F)^T; the h^2 and sigma factors are folded into U^.
    """
    h = 1.0 / (n + 1)
    Uh = dst1(U_F) * (h * h * np.asarray(sigma, dtype=np.float64))[None, :]
    Vh = dst1(V_F)
    return Uh, Vh


# ----------------------------------------------------------------------------------------
# Section 3.1, eq. g_for_p: entries, columns and rows of W^
# ----------------------------------------------------------------------------------------
def columns(Uh: np.ndarray, Vh: np.ndarray, lam: np.ndarray, J: Sequence[int]) -> np.ndarray:
    """C = W^(:, J), an n x |J| array."""
    J = np.asarray(J, dtype=np.int64)
    return (Uh @ Vh[J].T) / (lam[:, None] + lam[J][None, :])


def rows(Uh: np.ndarray, Vh: np.ndarray, lam: np.ndarray, I: Sequence[int]) -> np.ndarray:
    """R = W^(I, :), an |I| x n array."""
    I = np.asarray(I, dtype=np.int64)
    return (Uh[I] @ Vh.T) / (lam[I][:, None] + lam[None, :])


# ----------------------------------------------------------------------------------------
# Linear-algebra steps used by Algorithm 1
# ----------------------------------------------------------------------------------------
def thin_qr(X: np.ndarray):
    """Householder QR, X = Q R with Q n x k orthonormal and R k x k upper triangular."""
    Q, R = np.linalg.qr(X, mode="reduced")
    return Q, R


def pinv(A: np.ndarray) -> np.ndarray:
    """Pseudo-inverse by SVD; singular values <= max(m, n) * eps * sigma_1 are dropped."""
    m, k = A.shape
    if m == 0 or k == 0:
        return np.zeros((k, m))
    Ua, s, Vt = np.linalg.svd(A, full_matrices=False)
    if s[0] == 0.0:
        return np.zeros((k, m))
    keep = s > max(m, k) * EPS * s[0]
    return (Vt[keep].T / s[keep][None, :]) @ Ua[:, keep].T


def sigma_min(A: np.ndarray) -> float:
    """Smallest of the min(rows, cols) singular values of A."""
    if A.size == 0:
        return 0.0
    return float(np.linalg.svd(A, compute_uv=False)[-1])


@dataclasses.dataclass
class Cross:
    U: np.ndarray  # n x r, orthonormal columns
    S: np.ndarray  # r, descending
    V: np.ndarray  # n x r
    rC: np.ndarray  # diag(R_C), one per index of J
    rR: np.ndarray  # diag(R_R), one per index of I
    branch: bool = True  # True: |J| <= |I| (solve with Q(I,:)); False: solve with Z(J,:)


def scross(Uh, Vh, lam, I: Sequence[int], J: Sequence[int]) -> Cross:
    """Algorithm 1: stabilized cross approximation from the fibers W^(:,J), W^(I,:).

    C = W^(:,J) = Q R_C and R^T = W^(I,:)^T = Z R_R (thin QRs). With k = |J|, l = |I|:
      k <= l: W = Q(I,:)^+ R = [Q(I,:)^+ R_R^T] Z^T;
      k >  l: W^T = Z(J,:)^+ C^T, i.e. W = Q [R_C (Z(J,:)^+)^T] Z^T.
    Either way the approximation is Q M Z^T with a |J| x |I| core M, so the truncated
    SVD of M = U^ S V~^T gives U = Q U^, V = Z V~ (the SVD of the |J| x n matrix in the
    listing has the same singular values and left factor).
    """
    return scross_fibers(columns(Uh, Vh, lam, J), rows(Uh, Vh, lam, I).T, I, J)


def scross_fibers(C: np.ndarray, Rt: np.ndarray, I: Sequence[int], J: Sequence[int]) -> Cross:
    """Algorithm 1 from the fibers C = G(:, J) (n x |J|) and R^T = G(I, :)^T (n x |I|) of any G."""
    I = list(I)
    J = list(J)
    Q, RC = thin_qr(C)
    Zq, RR = thin_qr(Rt)
    if len(J) <= len(I):
        M = pinv(Q[I, :]) @ RR.T
    else:
        M = RC @ pinv(Zq[J, :]).T
    A, s, Bt = np.linalg.svd(M, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        r = 0
    else:
        r = int(np.count_nonzero(s > max(len(I), len(J)) * EPS * s[0]))
    return Cross(Q @ A[:, :r], s[:r].copy(), Zq @ Bt[:r].T, np.diag(RC).copy(), np.diag(RR).copy(),
                 len(J) <= len(I))


# ----------------------------------------------------------------------------------------
# Algorithm 3 (leverage scores) and the index-set update of Algorithm 4
# ----------------------------------------------------------------------------------------
def leverage_scores(U: np.ndarray, r_sig: int) -> np.ndarray:
    """pi_i = sum over the leading r_sig columns of U(i, eta)^2 (Algorithm 3; the 1/k factor
    does not change the ranking and is left out)."""
    return np.sum(U[:, :r_sig] ** 2, axis=1)


@dataclasses.dataclass
class Selection:
    indices: List[int]  # old indices, then the new ones in selection order
    new: List[int]
    gap: float  # (score of last taken - score of first left) / max score; inf if none left


def select(U: np.ndarray, r_sig: int, I_prev: Sequence[int], p_max: int) -> Selection:
    """Append the r_sig highest leverage scores outside I_prev to I_prev (capped at p_max)."""
    n = U.shape[0]
    pi = leverage_scores(U, r_sig)
    top = float(pi.max()) if n else 0.0
    score = np.where(pi <= FLOOR_REL * top, 0.0, pi)
    free = np.ones(n, dtype=bool)
    free[np.asarray(list(I_prev), dtype=np.int64)] = False
    cand = np.nonzero(free)[0]
    order = cand[np.lexsort((cand, -score[cand]))]
    s = max(0, min(r_sig, p_max - len(I_prev), order.size))
    # Leverage-score sets carry no order (Algorithm 4 notes this); the new indices are
    # appended in ascending index order so that rounding in equal scores cannot reorder them.
    new = sorted(int(i) for i in order[:s])
    if s < order.size and s > 0 and top > 0.0:
        gap = float(score[order[s - 1]] - score[order[s]]) / top
    else:
        gap = math.inf
    return Selection(list(I_prev) + new, new, gap)


def pivoted_qr_order(A: np.ndarray, count: int) -> tuple:
    """First `count` pivots of Householder QR with column pivoting of A (m x n, Algorithm 2).

    Step j picks, among the columns not yet pivoted, the one whose trailing part (rows j..m-1
    after the j reflectors so far) has the largest squared norm. Squared norms within
    PIVOT_TIE_REL of the largest count as equal, and those at or below FLOOR_REL times the
    largest initial one as 0: ties go to the smaller column index (rounding in the updates
    must not decide between columns that are equal in exact arithmetic). The norms are
    recomputed at every step. Returns (pivots, gaps): gaps[j] is the relative margin of step
    j's choice over the best column outside the tie (inf when there is none).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    m, n = A.shape
    count = min(count, m, n)
    cols = np.arange(n)
    piv: List[int] = []
    gaps: List[float] = []
    floor = FLOOR_REL * float(np.max(np.sum(A * A, axis=0))) if A.size else 0.0
    for j in range(count):
        nrm2 = np.sum(A[j:, j:] ** 2, axis=0)
        nrm2 = np.where(nrm2 <= floor, 0.0, nrm2)
        best = float(nrm2.max())
        tied = nrm2 >= best * (1.0 - PIVOT_TIE_REL)
        c = j + int(np.argmin(np.where(tied, cols[j:], n + 1)))
        rest = nrm2[~tied]
        gaps.append(math.inf if rest.size == 0 or best == 0.0 else (best - float(rest.max())) / best)
        A[:, [j, c]] = A[:, [c, j]]
        cols[[j, c]] = cols[[c, j]]
        piv.append(int(cols[j]))
        x = A[j:, j].copy()
        alpha = x[0]
        xn = float(np.linalg.norm(x))
        if xn == 0.0:
            continue
        beta = -math.copysign(xn, alpha)
        v = x.copy()
        v[0] = alpha - beta
        v /= v[0]
        tau = (beta - alpha) / beta
        A[j:, j:] -= tau * np.outer(v, v @ A[j:, j:])
    return piv, gaps


def qdeim_select(U: np.ndarray, r_sig: int, I_prev: Sequence[int], p_max: int, first: bool) -> Selection:
    """QDEIM index update (Algorithm 2 QDEIM branch; Algorithm 4's selection, union and safeguard).

    I* = the first r_sig pivots of the column-pivoted QR of U(:, :r_sig)^T; the pivots not in
    I_prev are appended in pivot order. If that adds nothing, or at the first pass, the index
    outside the set with the largest leverage score is appended as well (the safeguard; the
    paper picks it at random). The set is capped at p_max.
    """
    n = U.shape[0]
    piv, gaps = pivoted_qr_order(U[:, :r_sig].T, r_sig)
    have = set(int(i) for i in I_prev)
    out = list(int(i) for i in I_prev)
    new: List[int] = []
    for i in piv:
        if len(out) >= p_max:
            break
        if i not in have:
            out.append(i)
            new.append(i)
            have.add(i)
    if (not new or first) and len(out) < p_max and len(out) < n:
        pi = leverage_scores(U, r_sig)
        top = float(pi.max()) if n else 0.0
        score = np.where(pi <= FLOOR_REL * top, 0.0, pi)
        cand = np.array([i for i in range(n) if i not in have], dtype=np.int64)
        order = cand[np.lexsort((cand, -score[cand]))]
        extra = int(order[0])
        out.append(extra)
        new.append(extra)
    gap = min(gaps) if gaps else math.inf
    return Selection(out, new, gap)


# Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
# SC 2011): ten rounds of two 32 x 32 -> 64-bit multiplications on a 4 x 32-bit counter, the
# 2 x 32-bit key bumped by two Weyl constants between rounds.
PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """The four 32-bit outputs for counters (c0, c1, c2, c3) (arrays) and key (k0, k1)."""
    mask = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x, dtype=np.uint64) & mask for x in (c0, c1, c2, c3)]
    k0 = np.uint64(k0) & mask
    k1 = np.uint64(k1) & mask
    for _ in range(10):
        p0 = np.uint64(PHILOX_M[0]) * c[0]
        p1 = np.uint64(PHILOX_M[1]) * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & mask, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & mask]
        k0 = (k0 + np.uint64(PHILOX_W[0])) & mask
        k1 = (k1 + np.uint64(PHILOX_W[1])) & mask
    return c


def sample_uniforms(n: int, k: int, side: int, seed: int) -> np.ndarray:
    """u_i in [0, 1), i < n, for pass k and side (0: rows I, 1: columns J)."""
    i = np.arange(n, dtype=np.uint64)
    x = philox4x32_10(i & np.uint64(0xFFFFFFFF), i >> np.uint64(32), np.full(n, k, dtype=np.uint64),
                      np.full(n, side, dtype=np.uint64), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    r53 = ((x[1] << np.uint64(32)) | x[0]) >> np.uint64(11)
    return r53.astype(np.float64) * 2.0 ** -53


def sampled_select(U: np.ndarray, r_sig: int, I_prev: Sequence[int], p_max: int, rho: float, u: np.ndarray) -> Selection:
    """Algorithm 3 as stated, with Algorithm 4's union and its safeguard:
    rows outside I_prev are kept with probability min(1, rho pi_i) (u_i < p_i); the kept ones
    with the highest scores fill the set up to p_max (appended in ascending index order); if none
    was kept, the row of the complement with the largest -1 - u_i is appended."""
    n = U.shape[0]
    pi = leverage_scores(U, r_sig)
    top = float(pi.max()) if n else 0.0
    score = np.where(pi <= FLOOR_REL * top, 0.0, pi)
    prob = np.minimum(1.0, rho * score)
    free = np.ones(n, dtype=bool)
    free[np.asarray(list(I_prev), dtype=np.int64)] = False
    kept = np.nonzero(free & (u < prob))[0]
    order = kept[np.lexsort((kept, -score[kept]))]
    room = max(0, min(p_max, n) - len(I_prev))
    s = min(room, order.size)
    new = sorted(int(i) for i in order[:s])
    if s == 0 and room > 0:
        cand = np.nonzero(free)[0]
        key = -1.0 - u[cand]
        new = [int(cand[np.lexsort((cand, -key))][0])]
    return Selection(list(I_prev) + new, new, math.inf)


def prune(idx: Sequence[int], diag: np.ndarray, tau: float) -> List[int]:
    """Drop idx[l] where |diag[l]| < tau * max|diag| (Algorithm 4, redundant rows/columns)."""
    a = np.abs(np.asarray(diag))
    if a.size == 0:
        return []
    keep = a >= tau * a.max()
    return [int(i) for i, kp in zip(idx, keep) if kp]


# ----------------------------------------------------------------------------------------
# Frobenius norms of factored matrices (the rho of Algorithm 4, and error metrics)
# ----------------------------------------------------------------------------------------
def lr_norm(terms) -> float:
    """|| sum_i U_i diag(s_i) V_i^T ||_F for a list of (U_i, s_i, V_i), without forming it.

    [U_1 .. U_m] = Q_a R_a and [V_1 .. V_m] = Q_b R_b (Householder), so the sum equals
    Q_a R_a diag(s) R_b^T Q_b^T and its norm is || R_a diag(s) R_b^T ||_F.
    """
    A = np.hstack([np.asarray(t[0], dtype=np.float64) for t in terms])
    B = np.hstack([np.asarray(t[2], dtype=np.float64) for t in terms])
    d = np.concatenate([np.asarray(t[1], dtype=np.float64).ravel() for t in terms])
    if d.size == 0:
        return 0.0
    _, Ra = np.linalg.qr(A, mode="reduced")
    _, Rb = np.linalg.qr(B, mode="reduced")
    return float(np.linalg.norm((Ra * d[None, :]) @ Rb.T))


def lr_diff_norm(Ua, Sa, Va, Ub, Sb, Vb) -> float:
    """|| Ua diag(Sa) Va^T - Ub diag(Sb) Vb^T ||_F."""
    return lr_norm([(Ua, Sa, Va), (Ub, -np.asarray(Sb), Vb)])


def rel_err(a, b) -> float:
    """|| A - B ||_F / || B ||_F for factored A = (U, S, V), B = (U, S, V)."""
    den = lr_norm([b])
    return lr_diff_norm(*a, *b) / den if den > 0 else lr_norm([a])


# ----------------------------------------------------------------------------------------
# Algorithm 4: Cross-DEIM, warm started, applied to W^ (Section 3.2)
# ----------------------------------------------------------------------------------------
@dataclasses.dataclass
class IterRecord:
    k: int
    I_pre: List[int]
    J_pre: List[int]
    I: List[int]
    J: List[int]
    r_sig_in: int
    rank: int
    S: np.ndarray
    rho: float
    indicator: float
    eta1: float
    eta2: float
    gapI: float
    gapJ: float
    branch: bool = True  # |J_pre| <= |I_pre|: Algorithm 1 solves with Q(I,:)


@dataclasses.dataclass
class Result:
    U: np.ndarray  # n x r, physical-space factors
    S: np.ndarray  # r
    V: np.ndarray  # n x r
    rank: int
    status: int
    iters: int  # number of scross calls made
    I: List[int]  # pruned index sets of the returned iterate
    J: List[int]
    rho: float
    indicator: float
    trace: List[IterRecord]
    Uk: Optional[np.ndarray] = None  # spectral factors of the returned iterate (untruncated)
    Sk: Optional[np.ndarray] = None
    Vk: Optional[np.ndarray] = None


def warm_start(Uh: np.ndarray, Vh: np.ndarray):
    """U_{-1}, S_{-1}, V_{-1}: truncated SVD of F^ = U^ V^^T from the two thin QRs."""
    Qu, Ru = thin_qr(Uh)
    Qv, Rv = thin_qr(Vh)
    A, s, Bt = np.linalg.svd(Ru @ Rv.T)
    if s.size == 0 or s[0] == 0.0:
        return None
    r = int(np.count_nonzero(s > Uh.shape[1] * EPS * s[0]))
    return Qu @ A[:, :r], s[:r].copy(), Qv @ Bt[:r].T


def warm_start_from(n: int, U0: np.ndarray, S0: Optional[np.ndarray], V0: np.ndarray):
    """Warm start from a given guess (Algorithm 4 inputs U0, V0), in physical space.

    The guess is moved to the sine basis like the right-hand side (Section 3.2) and its
    truncated SVD, DST(U0) diag(S0) DST(V0)^T = U_{-1} S_{-1} V_{-1}^T, is the starting
    iterate; S0 = None means unit weights.
    """
    U0 = np.asarray(U0, dtype=np.float64)
    V0 = np.asarray(V0, dtype=np.float64)
    S0 = np.ones(U0.shape[1]) if S0 is None else np.asarray(S0, dtype=np.float64)
    return warm_start(dst1(U0) * S0[None, :], dst1(V0))


def indicator(U, S, V, I, J):
    """min(eta1 (1 + eta2), eta2 (1 + eta1)) * S_min / ||S||_F (Algorithm 4 stopping test)."""
    s1 = sigma_min(U[np.asarray(I, dtype=np.int64), :])
    s2 = sigma_min(V[np.asarray(J, dtype=np.int64), :])
    eta1 = math.inf if s1 == 0.0 else 1.0 / s1
    eta2 = math.inf if s2 == 0.0 else 1.0 / s2
    nrm = float(np.linalg.norm(S))
    val = min(eta1 * (1.0 + eta2), eta2 * (1.0 + eta1)) * float(S[-1]) / nrm
    return val, eta1, eta2


def final_rank(S: np.ndarray, tol: float, r_max: int) -> int:
    """Smallest r with sum_{l > r} S_l^2 < (tol ||S||_F)^2, clamped to [1, r_max]."""
    nrm2 = float(np.sum(S * S))
    thr = (tol * math.sqrt(nrm2)) ** 2
    tail = 0.0
    r_star = S.size
    # walk from the end: tail(r) = sum_{l >= r} S_l^2 (0-based), r* = smallest r with tail < thr
    for r in range(S.size, -1, -1):
        if r < S.size:
            tail += float(S[r]) ** 2
        if tail < thr:
            r_star = r
        else:
            break
    return max(min(r_star, r_max), 1)


def _cross_deim(n, fibers, ws, r_max, tol, maxiter, prune_tau, stop_at_fixed_point, replay, selector,
                ls_oversampling, seed):
    """Algorithm 4 from the starting iterate ws = (U_{-1}, S_{-1}, V_{-1}); fibers(I, J) returns
    (G(:, J), G(I, :)^T). Returns the last iterate, status, passes and the trace."""
    if selector not in ("ls", "qdeim", "ls_sampled"):
        raise ValueError(f"unknown selector {selector!r}")
    U_prev, S_prev, V_prev = ws
    I: List[int] = []
    J: List[int] = []
    pre_prev = None
    trace: List[IterRecord] = []
    status = STATUS_NOT_CONVERGED
    rho = math.inf
    ind = math.inf
    iters = 0
    for k in range(maxiter):
        r_sig = int(np.count_nonzero(S_prev > tol * S_prev[0]))
        if replay is not None and k < len(replay):
            rI = [int(i) for i in replay[k][0]]
            rJ = [int(j) for j in replay[k][1]]
            selI = Selection(rI, [i for i in rI if i not in I], math.inf)
            selJ = Selection(rJ, [j for j in rJ if j not in J], math.inf)
        elif selector == "qdeim":
            selI = qdeim_select(U_prev, r_sig, I, r_max, k == 0)
            selJ = qdeim_select(V_prev, r_sig, J, r_max, k == 0)
        elif selector == "ls_sampled":
            selI = sampled_select(U_prev, r_sig, I, r_max, ls_oversampling, sample_uniforms(n, k, 0, seed))
            selJ = sampled_select(V_prev, r_sig, J, r_max, ls_oversampling, sample_uniforms(n, k, 1, seed))
        else:
            selI = select(U_prev, r_sig, I, r_max)
            selJ = select(V_prev, r_sig, J, r_max)
        pre = (selI.indices, selJ.indices)
        if stop_at_fixed_point and pre_prev is not None and pre == pre_prev:
            status = STATUS_STAGNATED
            break
        C, Rt = fibers(selI.indices, selJ.indices)
        cr = scross_fibers(C, Rt, selI.indices, selJ.indices)
        iters += 1
        I = prune(selI.indices, cr.rR, prune_tau)
        J = prune(selJ.indices, cr.rC, prune_tau)
        ind, eta1, eta2 = indicator(cr.U, cr.S, cr.V, I, J)
        nrm = float(np.linalg.norm(cr.S))
        if k == 0:
            rho = math.inf
        else:
            rho = lr_diff_norm(cr.U, cr.S, cr.V, U_prev, S_prev, V_prev) / nrm
        trace.append(
            IterRecord(k, selI.indices, selJ.indices, I, J, r_sig, cr.S.size, cr.S, rho, ind,
                       eta1, eta2, selI.gap, selJ.gap, cr.branch)
        )
        U_prev, S_prev, V_prev = cr.U, cr.S, cr.V
        pre_prev = pre
        if max(rho, ind) < tol:
            status = STATUS_OK
            break
    return U_prev, S_prev, V_prev, status, iters, I, J, rho, ind, trace


def solve(
    n: int,
    U_F: np.ndarray,
    sigma: np.ndarray,
    V_F: np.ndarray,
    r_max: int,
    tol: float,
    maxiter: int,
    prune_tau: float = 1e-12,
    stop_at_fixed_point: bool = True,
    warm=None,
    replay=None,
    selector: str = "ls",
    ls_oversampling: float = 2.0,
    seed: int = 0,
) -> Result:
    """Low-rank Poisson solve: -Lap u = f, u = 0 on the boundary of the unit square.

    Returns W ~= U diag(S) V^T on the n x n interior grid (Sections 3.2 and Algorithm 4).
    warm: optional (U0, S0, V0), the initial guess of Algorithm 4 in physical space (S0 may be
    None); default (and for a zero guess): the right-hand side itself. replay: optional list of (I, J) index sets
    used for passes 0, 1, ... instead of selecting them (a diagnostic). selector: "ls"
    (leverage scores, Algorithm 3, the top r_sig), "ls_sampled" (Algorithm 3's random sampling,
    p_i = min(1, ls_oversampling pi_i) drawn with Philox4x32-10 keyed by seed) or "qdeim"
    (Algorithm 2).
    """
    if selector not in ("ls", "qdeim", "ls_sampled"):
        raise ValueError(f"unknown selector {selector!r}")
    U_F = np.asarray(U_F, dtype=np.float64)
    V_F = np.asarray(V_F, dtype=np.float64)
    lam = eigenvalues(n)
    Uh, Vh = spectral_factors(n, U_F, sigma, V_F)
    ws = warm_start(Uh, Vh)
    if ws is not None and warm is not None:
        guess = warm_start_from(n, *warm)
        if guess is not None:  # a zero guess leaves the start from the right-hand side
            ws = guess
    if ws is None:  # F = 0: the solution is 0
        z = np.zeros((n, 1))
        return Result(z, np.zeros(1), z.copy(), 1, STATUS_OK, 0, [], [], 0.0, 0.0, [])

    def fibers(I, J):
        return columns(Uh, Vh, lam, J), rows(Uh, Vh, lam, I).T

    U_prev, S_prev, V_prev, status, iters, I, J, rho, ind, trace = _cross_deim(
        n, fibers, ws, r_max, tol, maxiter, prune_tau, stop_at_fixed_point, replay, selector, ls_oversampling, seed)
    r = final_rank(S_prev, tol, r_max)
    U_out = dst1(U_prev[:, :r])
    V_out = dst1(V_prev[:, :r])
    return Result(U_out, S_prev[:r].copy(), V_out, r, status, iters, I, J, rho, ind, trace,
                  U_prev, S_prev, V_prev)


# ----------------------------------------------------------------------------------------
# Cross-DEIM on the paper's test matrices (Section 4.2): G given entrywise
# ----------------------------------------------------------------------------------------
def hilbert(n: int, I: Sequence[int], J: Sequence[int]) -> np.ndarray:
    """H(i, j) = 1/(1 + i + j) with 0-based i, j (the Hilbert matrix 1/(i + j - 1), 1-based)."""
    i = np.asarray(I, dtype=np.float64)[:, None]
    j = np.asarray(J, dtype=np.float64)[None, :]
    return 1.0 / (1.0 + i + j)


def kmatrix(n: int, I: Sequence[int], J: Sequence[int]) -> np.ndarray:
    """K(i, j) = (|x_i + y_j| / 2)^5 on the grid x_i = y_i = -1 + 2 i/(n - 1), i = 0..n-1
    (Section 4.2, 1-based there); the fifth power is formed as ((t t)(t t)) t."""
    x = -1.0 + 2.0 * np.asarray(I, dtype=np.float64) / (n - 1)
    y = -1.0 + 2.0 * np.asarray(J, dtype=np.float64) / (n - 1)
    t = np.abs(x[:, None] + y[None, :]) / 2.0
    t2 = t * t
    return (t2 * t2) * t


MATRICES = {"hilbert": hilbert, "k": kmatrix}


def solve_matrix(kind: str, n: int, U0: np.ndarray, V0: np.ndarray, r_max: int, tol: float, maxiter: int,
                 prune_tau: float = 1e-12, selector: str = "ls", ls_oversampling: float = 2.0, seed: int = 0,
                 replay=None) -> Result:
    """Cross-DEIM (Algorithm 4 with Algorithm 1) on the n x n test matrix `kind` ("hilbert" or
    "k"), started from the truncated SVD of the guess U0 V0^T (Algorithm 4's inputs U0, V0;
    truncated at r0 eps sigma_1 as the Poisson warm start). Returns G ~= U diag(S) V^T."""
    g = MATRICES[kind]
    ws = warm_start(np.asarray(U0, dtype=np.float64), np.asarray(V0, dtype=np.float64))
    if ws is None:
        raise ValueError("the initial guess is zero")

    def fibers(I, J):
        all_rows = np.arange(n)
        return g(n, all_rows, J), g(n, I, all_rows).T

    U_prev, S_prev, V_prev, status, iters, I, J, rho, ind, trace = _cross_deim(
        n, fibers, ws, r_max, tol, maxiter, prune_tau, True, replay, selector, ls_oversampling, seed)
    r = final_rank(S_prev, tol, r_max)
    return Result(U_prev[:, :r].copy(), S_prev[:r].copy(), V_prev[:, :r].copy(), r, status, iters, I, J, rho,
                  ind, trace, U_prev, S_prev, V_prev)
