"""Seeded synthetic right-hand sides for the low-rank Poisson solver.

This module is shared by the tests, the benchmark and the CPU oracle's callers. It
holds no arithmetic of the solver: it only draws random numbers and samples
Gaussian bumps and sine modes on the grid, so that the GPU path and the oracle
see identical inputs.

The paper's Poisson test (Section 4.2) uses an analytic, separable right-hand
side on an equidistant grid with n interior points per dimension and spacing
h = 1/(n+1) (Section 3, eq. matrix_poisson). The workloads below keep that
structure -- F = sum_k a_k g_k(x) h_k(y), stored as factors U (n x r), sigma (r),
V (n x r) -- with seeded centres, widths and amplitudes instead of the paper's
single bump.

Recipe (numpy.random.default_rng(seed), PCG64), draw order:
    cx[K], cy[K], wx[K], wy[K], a[K], then for the sine modes kx[M], ky[M], b[M].
Bump g(x; c, w) = exp(-(x - c)^2 / (2 w^2)), w is the standard deviation.
Sine mode s_k(x) = sin(k pi x); its discrete solution is known in closed form.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Workload",
    "CONFIGS",
    "grid",
    "bump_rhs",
    "sine_rhs",
    "make",
    "served_stream",
    "sketch_matrix",
    "matrix_guess",
    "MATRIX_CONFIGS",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One Poisson solve: grid size, RHS recipe and solver settings."""

    name: str
    n: int
    n_bumps: int
    width_lo: float
    width_hi: float
    n_sines: int
    r_max: int
    tol: float
    maxiter: int
    precision: str  # "fp64" or "mixed"
    centre_lo: float = 0.2
    centre_hi: float = 0.8
    sine_kmax: int = 50

    @property
    def rank(self) -> int:
        return self.n_bumps + self.n_sines


# The five workloads: FP64 n=255 (rank 5, cap 16, 10 iterations); FP64 n=4095 (rank 10
# incl. two sine modes, cap 32); mixed n=65535 (rank 20, cap 64); n=1048575 (rank 30,
# cap 64); and the served mix (see served_stream).
CONFIGS = {
    "n255_r5_fp64": Workload("n255_r5_fp64", 255, 5, 0.05, 0.2, 0, 16, 1e-10, 10, "fp64"),
    "n4095_r10_fp64": Workload("n4095_r10_fp64", 4095, 8, 0.05, 0.2, 2, 32, 1e-10, 20, "fp64"),
    "n65535_r20_mixed": Workload("n65535_r20_mixed", 65535, 20, 0.01, 0.1, 0, 64, 1e-10, 20, "mixed"),
    "n65535_r20_fp64": Workload("n65535_r20_fp64", 65535, 20, 0.01, 0.1, 0, 64, 1e-10, 20, "fp64"),
    "n1048575_r30_fp64": Workload("n1048575_r30_fp64", 1048575, 30, 0.002, 0.05, 0, 64, 1e-10, 20, "fp64"),
    "n1048575_r30_mixed": Workload("n1048575_r30_mixed", 1048575, 30, 0.002, 0.05, 0, 64, 1e-10, 20, "mixed"),
}


def grid(n: int) -> np.ndarray:
    """Interior grid points x_i = i h, i = 1..n, h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    return np.arange(1, n + 1, dtype=np.float64) * h


def _bump(x: np.ndarray, c: float, w: float) -> np.ndarray:
    return np.exp(-((x - c) ** 2) / (2.0 * w * w))


def bump_rhs(
    n: int,
    seed: int,
    n_bumps: int,
    width_lo: float,
    width_hi: float,
    n_sines: int = 0,
    centre_lo: float = 0.2,
    centre_hi: float = 0.8,
    sine_kmax: int = 50,
):
    """Return (U, sigma, V, info): column-major FP64 factors of the separable RHS.

    U[:, k] = g(x; cx_k, wx_k), V[:, k] = g(y; cy_k, wy_k), sigma_k = a_k for the bumps,
    then U[:, K+m] = sin(kx_m pi x), V[:, K+m] = sin(ky_m pi y), sigma = b_m for the sine
    modes. The factors are not orthonormal and sigma is signed.
    """
    rng = np.random.default_rng(seed)
    K = n_bumps
    cx = rng.uniform(centre_lo, centre_hi, K)
    cy = rng.uniform(centre_lo, centre_hi, K)
    wx = rng.uniform(width_lo, width_hi, K)
    wy = rng.uniform(width_lo, width_hi, K)
    a = rng.standard_normal(K)
    kx = rng.integers(1, sine_kmax + 1, n_sines)
    ky = rng.integers(1, sine_kmax + 1, n_sines)
    b = rng.standard_normal(n_sines)
    x = grid(n)
    r = K + n_sines
    U = np.empty((n, r), order="F")
    V = np.empty((n, r), order="F")
    for k in range(K):
        U[:, k] = _bump(x, cx[k], wx[k])
        V[:, k] = _bump(x, cy[k], wy[k])
    for m in range(n_sines):
        U[:, K + m] = np.sin(kx[m] * np.pi * x)
        V[:, K + m] = np.sin(ky[m] * np.pi * x)
    sigma = np.concatenate([a, b]).astype(np.float64)
    info = {"cx": cx, "cy": cy, "wx": wx, "wy": wy, "a": a, "kx": kx, "ky": ky, "b": b}
    return U, sigma, V, info


def bump_rhs_device(n: int, seed: int, n_bumps: int, width_lo: float, width_hi: float, device,
                    centre_lo: float = 0.2, centre_hi: float = 0.8):
    """bump_rhs drawn with the same seeded parameters, evaluated on a torch device in FP64.

    Returns (U, sigma, V) as column-major (n, r) CUDA tensors; used where thousands of
    right-hand sides are needed at once (the served stream).
    """
    import torch

    rng = np.random.default_rng(seed)
    K = n_bumps
    cx = rng.uniform(centre_lo, centre_hi, K)
    cy = rng.uniform(centre_lo, centre_hi, K)
    wx = rng.uniform(width_lo, width_hi, K)
    wy = rng.uniform(width_lo, width_hi, K)
    a = rng.standard_normal(K)
    x = torch.arange(1, n + 1, dtype=torch.float64, device=device) * (1.0 / (n + 1))

    def cols(c, w):
        c = torch.as_tensor(c, dtype=torch.float64, device=device)[:, None]
        w = torch.as_tensor(w, dtype=torch.float64, device=device)[:, None]
        return torch.exp(-((x[None, :] - c) ** 2) / (2.0 * w * w))  # (K, n): column-major (n, K)

    U = cols(cx, wx).t()
    V = cols(cy, wy).t()
    return U, torch.as_tensor(a, dtype=torch.float64, device=device), V


def sine_rhs(n: int, modes: Sequence[tuple]):
    """RHS made only of separable sine modes [(kx, ky, amplitude), ...]."""
    x = grid(n)
    r = len(modes)
    U = np.empty((n, r), order="F")
    V = np.empty((n, r), order="F")
    sigma = np.empty(r)
    for m, (kx, ky, amp) in enumerate(modes):
        U[:, m] = np.sin(kx * np.pi * x)
        V[:, m] = np.sin(ky * np.pi * x)
        sigma[m] = amp
    return U, sigma, V


def make(config: str | Workload, seed: int = 0, n: Optional[int] = None):
    """Factors for a named workload; `n` overrides the grid size (same recipe)."""
    w = CONFIGS[config] if isinstance(config, str) else config
    nn = w.n if n is None else n
    U, s, V, _ = bump_rhs(
        nn, seed, w.n_bumps, w.width_lo, w.width_hi, w.n_sines, w.centre_lo, w.centre_hi, w.sine_kmax
    )
    return U, s, V


@dataclasses.dataclass(frozen=True)
class Request:
    idx: int
    arrival_s: float
    n: int
    rank: int
    precision: str
    seed: int


def served_stream(
    count: int = 2000,
    rate_per_s: float = 1000.0,
    seed: int = 2026,
    sizes: Sequence[int] = (1023, 4095, 16383, 65535, 262143),
    weights: Sequence[float] = (0.3, 0.3, 0.2, 0.15, 0.05),
    rank_lo: int = 2,
    rank_hi: int = 20,
    p_mixed: float = 0.5,
) -> List[Request]:
    """Poisson arrivals of solve requests of mixed size, rank and precision.

    Request i draws its RHS with seed 1000 + i (bumps with widths in U(0.05, 0.2)).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, count)
    t = np.cumsum(gaps)
    ns = rng.choice(np.asarray(sizes), size=count, p=np.asarray(weights) / np.sum(weights))
    ranks = rng.integers(rank_lo, rank_hi + 1, count)
    mixed = rng.uniform(0.0, 1.0, count) < p_mixed
    return [
        Request(i, float(t[i]), int(ns[i]), int(ranks[i]), "mixed" if mixed[i] else "fp64", 1000 + i)
        for i in range(count)
    ]


def sketch_matrix(n: int, k: int = 64, seed: int = 777) -> np.ndarray:
    """Seeded n x k standard Gaussian test matrix (C order), for comparing two low-rank
    solutions at sizes where the n x n product cannot be formed: ||Om^T (A - B) Om'||_F
    estimates ||A - B||_F up to the factor k."""
    return np.random.default_rng(seed).standard_normal((n, k))


def matrix_guess(n: int, r0: int, seed: int = 0):
    """Seeded initial guess (U0, V0) for Cross-DEIM on a test matrix: two n x r0 standard
    Gaussian matrices (column-major), drawn U0 first."""
    rng = np.random.default_rng(seed)
    U0 = np.asfortranarray(rng.standard_normal((n, r0)))
    V0 = np.asfortranarray(rng.standard_normal((n, r0)))
    return U0, V0


# Cross-DEIM on the paper's test matrices (Section 4.2: the Hilbert matrix to 1e-9 and the K
# matrix to 1e-6); three sizes each, rank cap 64, a seeded rank-8 Gaussian initial guess.
MATRIX_CONFIGS = {
    "hilbert_n1000": ("hilbert", 1000, 1e-9),
    "hilbert_n16384": ("hilbert", 16384, 1e-9),
    "hilbert_n262144": ("hilbert", 262144, 1e-9),
    "k_n1000": ("k", 1000, 1e-6),
    "k_n16384": ("k", 16384, 1e-6),
    "k_n262144": ("k", 262144, 1e-6),
}
