"""Dense full-rank checks of the Poisson solve (small n only).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke entry point and the
benchmark's CPU-baseline leg, never by the GPU library.
"""
from __future__ import annotations

import numpy as np

from .crossdeim import dst1, eigenvalues


def dense_solve(F: np.ndarray) -> np.ndarray:
    """Section 3.1: F^ = Z^T F Z, W^(i,j) = h^2 F^(i,j)/(lambda_i + lambda_j), W = Z W^ Z^T."""
    F = np.asarray(F, dtype=np.float64)
    n = F.shape[0]
    h = 1.0 / (n + 1)
    lam = eigenvalues(n)
    Fh = dst1(dst1(F).T).T
    Wh = h * h * Fh / (lam[:, None] + lam[None, :])
    return dst1(dst1(Wh).T).T


def tridiag_apply(X: np.ndarray) -> np.ndarray:
    """T X with T = tridiag(-1, 2, -1), applied along axis 0 by the 3-point stencil."""
    X = np.asarray(X, dtype=np.float64)
    Y = 2.0 * X
    Y[1:] -= X[:-1]
    Y[:-1] -= X[1:]
    return Y


def laplacian_apply(W: np.ndarray) -> np.ndarray:
    """T W + W T^T, the left side of eq. matrix_poisson (5-point stencil, times h^2)."""
    return tridiag_apply(W) + tridiag_apply(W.T).T
