"""GPU parity of the stage kernels exposed through the C-ABI: DST-I and the TSQR.

Compared element by element with the CPU oracle (FP64 NumPy) on seeded inputs."""
import math

import numpy as np
import pytest

import workloads
from oracle import crossdeim as cd

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def to_dev(a):
    torch = _torch()
    from paper_2607_06021_amd import fortran

    return fortran(torch.from_numpy(np.ascontiguousarray(a)).cuda())


def to_np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,ncols", [(7, 1), (255, 5), (1023, 8), (4095, 7), (65535, 6), (262143, 3)])
def test_dst_fp64_matches_oracle(n, ncols):
    from paper_2607_06021_amd import Solver

    print(f"dst fp64 n={n} ncols={ncols}", flush=True)
    rng = np.random.default_rng(n + ncols)
    X = rng.standard_normal((n, ncols))
    scale = rng.standard_normal(ncols)
    torch = _torch()
    with Solver(n, min(8, n), 1e-10) as s:
        Y = to_np(s.dst1(to_dev(X), scale=torch.from_numpy(scale).cuda(), mul=0.5))
        torch.cuda.synchronize()
    ref = cd.dst1(X) * scale[None, :] * 0.5
    err = np.max(np.abs(Y - ref)) / np.max(np.abs(ref))
    print(f"  max rel err {err:.2e}")
    assert err <= 1e-14 * math.log2(n + 1)


# n + 1 not a power of two (Bluestein): tiny grids, the one-pass FFT (M <= 4096), the four-step
# FFT, the paper's grid sizes n = 2^k, column counts that leave half a pair and that take two
# rounds of column pairs
@pytest.mark.parametrize("n,ncols", [(2, 1), (3, 2), (5, 3), (100, 5), (1000, 9), (1024, 4), (4096, 20),
                                     (16384, 7), (65536, 3), (262144, 2)])
def test_dst_general_n_matches_oracle(n, ncols):
    from paper_2607_06021_amd import Solver

    print(f"dst general n={n} ncols={ncols}", flush=True)
    rng = np.random.default_rng(n + 7 * ncols)
    X = rng.standard_normal((n, ncols))
    scale = rng.standard_normal(ncols)
    torch = _torch()
    with Solver(n, min(32, n), 1e-10) as s:
        Xd = to_dev(X)
        Y = to_np(s.dst1(Xd, scale=torch.from_numpy(scale).cuda(), mul=0.5))
        Y32 = to_np(s.dst1(Xd, precision="mixed"))
        back = to_np(s.dst1(s.dst1(Xd)))
        torch.cuda.synchronize()
    ref = cd.dst1(X)
    err = np.max(np.abs(Y - ref * scale[None, :] * 0.5)) / np.max(np.abs(ref * scale[None, :] * 0.5))
    e32 = np.max(np.abs(Y32 - ref)) / np.max(np.abs(ref))
    einv = np.max(np.abs(back - X)) / np.max(np.abs(X))
    print(f"  max rel err fp64 {err:.2e} fp32 {e32:.2e} involution {einv:.2e}")
    lg = math.log2(4 * (n + 1))
    assert err <= 2e-15 * lg
    assert e32 <= 2e-6 * lg
    assert einv <= 4e-15 * lg


@pytest.mark.parametrize("n", [255, 65535])
def test_dst_fp32_and_involution(n):
    from paper_2607_06021_amd import Solver

    print(f"dst mixed/involution n={n}", flush=True)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((n, 4))
    _torch()
    with Solver(n, 8, 1e-10) as s:
        Xd = to_dev(X)
        Y32 = to_np(s.dst1(Xd, precision="mixed"))
        Y = s.dst1(Xd)
        back = to_np(s.dst1(Y))
    ref = cd.dst1(X)
    e32 = np.max(np.abs(Y32 - ref)) / np.max(np.abs(ref))
    print(f"  fp32 rel err {e32:.2e}")
    assert e32 <= 2e-6
    assert np.max(np.abs(back - X)) <= 1e-13 * math.log2(n + 1)


def _ill_conditioned(n, p, rng, kappa=1e12):
    Q, _ = np.linalg.qr(rng.standard_normal((n, p)))
    W, _ = np.linalg.qr(rng.standard_normal((p, p)))
    s = np.logspace(0, -np.log10(kappa), p)
    return (Q * s[None, :]) @ W


# widths that fill the four columns of a wave partly (2, 3, 33, 63), blocks shorter than one
# 64-row group of lanes (n = 63) or ragged (255 rows in the last block), and a tree of several
# levels over partly filled stacked factors (p < p_max)
@pytest.mark.parametrize("n,p,kind", [(255, 5, "rand"), (4095, 32, "rand"), (4095, 64, "ill"), (65535, 64, "ill"),
                                      (65535, 20, "deficient"), (131071, 1, "rand"),
                                      (1023, 64, "fibers"), (63, 3, "rand"), (63, 63, "rand"),
                                      (127, 2, "rand"), (511, 63, "ill"), (16383, 33, "rand")])
def test_tsqr_matches_householder(n, p, kind):
    from paper_2607_06021_amd import Solver

    print(f"tsqr n={n} p={p} kind={kind}", flush=True)
    rng = np.random.default_rng(p)
    if kind == "rand":
        A = rng.standard_normal((n, p))
    elif kind == "ill":
        A = _ill_conditioned(n, p, rng)
    elif kind == "deficient":
        A = rng.standard_normal((n, p))
        A[:, 5] = A[:, 2] * 3.0  # exactly dependent column
        A[:, 9] = 0.0            # zero column
    else:  # columns of W^ at random J: the matrices the solver factors
        U, s, V = workloads.make("n255_r5_fp64", 1, n=n)
        Uh, Vh = cd.spectral_factors(n, U, s, V)
        A = cd.columns(Uh, Vh, cd.eigenvalues(n), rng.choice(n, p, replace=False))
    _torch()
    with Solver(n, p, 1e-10) as s:
        Qd, Rd = s.tsqr(to_dev(A))
        Q, R = to_np(Qd), to_np(Rd)
    nrm = np.linalg.norm(A)
    assert np.array_equal(np.tril(R, -1), np.zeros_like(R))
    orth = np.linalg.norm(Q.T @ Q - np.eye(p))
    recon = np.linalg.norm(Q @ R - A) / nrm
    Rref = np.linalg.qr(A, mode="r")
    # after an exactly dependent column Q holds an arbitrary orthonormal direction, which
    # changes the later diagonal entries: compare the columns before it, and check that the
    # dependent ones are at rounding level
    lim = 5 if kind == "deficient" else p
    if kind == "fibers":  # numerically rank deficient: stop at the first |R_ll| at rounding level
        dref = np.abs(np.diag(Rref))
        small = np.nonzero(dref < 1e-13 * dref.max())[0]
        lim = int(small[0]) if small.size else p
    ddiff = np.max(np.abs(np.abs(np.diag(R)[:lim]) - np.abs(np.diag(Rref)[:lim]))) / nrm
    if kind == "deficient":
        assert abs(R[5, 5]) <= 1e-14 * nrm and abs(R[9, 9]) <= 1e-14 * nrm
    print(f"  |QtQ-I| {orth:.2e}  |QR-A|/|A| {recon:.2e}  diag diff {ddiff:.2e}")
    assert recon <= 1e-14 * math.sqrt(p) * 10
    assert ddiff <= 1e-14 * math.sqrt(p) * 10
    assert orth <= 1e-13 * math.sqrt(p)
    if kind not in ("deficient", "fibers"):
        # R agrees with LAPACK's up to the sign of each row
        sg = np.sign(np.diag(R)) * np.sign(np.diag(Rref))
        assert np.linalg.norm(R - sg[:, None] * Rref) <= 1e-12 * math.sqrt(p) * nrm * (1e4 if kind == "ill" else 1)


def test_tsqr_on_rank_deficient_fibers_of_a_solve():
    """The QR inputs of a rank-1 solve at the rank cap (6 of 16 columns exactly dependent):
    Q must stay orthonormal and the cross approximation built from it must match the one
    built from LAPACK's Q."""
    from paper_2607_06021_amd import Solver

    n = 255
    U, s, V = workloads.make("n255_r5_fp64", 0, n=n)
    U, s, V = U[:, :1], s[:1], V[:, :1]
    mats = []
    orig = cd.thin_qr

    def cap(X):
        mats.append(X.copy())
        return orig(X)

    cd.thin_qr = cap
    try:
        cd.solve(n, U, s, V, 16, 1e-10, 10)
    finally:
        cd.thin_qr = orig
    print(f"captured {len(mats)} QR inputs", flush=True)
    _torch()
    worst = 0.0
    with Solver(n, 16, 1e-10) as sol:
        for X in mats:
            Qd, Rd = sol.tsqr(to_dev(X))
            Q, R = to_np(Qd), to_np(Rd)
            p = X.shape[1]
            orth = np.linalg.norm(Q.T @ Q - np.eye(p))
            recon = np.linalg.norm(Q @ R - X) / np.linalg.norm(X)
            worst = max(worst, orth)
            assert orth <= 1e-13 * math.sqrt(p), (p, orth)
            assert recon <= 1e-14 * math.sqrt(p) * 10, (p, recon)
    print(f"  worst |QtQ-I| {worst:.2e}")
