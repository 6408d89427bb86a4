"""QDEIM index selection on the GPU (Algorithm 2 in Algorithm 4) against the oracle's, through
the C-ABI: identical ordered index sets at every pass (the pivots of the column-pivoted QR of
U(:, :r_sig)^T appended in pivot order, plus the safeguard index), the same pruned sizes,
ranks, status and pass count, and a relative error <= 1e-10 (FP64) or <= 1e-5 (mixed)."""
import numpy as np
import pytest

import workloads
from oracle import crossdeim as cd
from test_gpu_solve import compare_fp64, dev

pytestmark = pytest.mark.gpu


def gpu_qdeim(n, U, s, V, r_max, tol, maxiter, precision="fp64"):
    from paper_2607_06021_amd import Solver

    with Solver(n, r_max, tol, maxiter=maxiter, precision=precision, selector="qdeim") as sol:
        Uo, So, Vo, r, info = sol.solve(dev(U), dev(s), dev(V))
        return {
            "U": Uo[:, :r].cpu().numpy(), "S": So.cpu().numpy(), "V": Vo[:, :r].cpu().numpy(), "rank": r,
            "info": info.as_dict(), "sets": sol.index_sets(), "trace": sol.trace(),
            "Ufull": Uo.cpu().numpy(), "Vfull": Vo.cpu().numpy(),
        }


@pytest.mark.parametrize("name,seed", [("n255_r5_fp64", 0), ("n255_r5_fp64", 1), ("n255_r5_fp64", 2),
                                       ("n4095_r10_fp64", 0), ("n4095_r10_fp64", 1)])
def test_qdeim_fp64_parity(name, seed):
    w = workloads.CONFIGS[name]
    U, s, V = workloads.make(w, seed)
    print(f"qdeim {name} seed {seed}", flush=True)
    o = cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, selector="qdeim")
    g = gpu_qdeim(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    compare_fp64(g, o, f"qdeim {name} seed {seed}")


@pytest.fixture(scope="module")
def oracle_n65535():
    w = workloads.CONFIGS["n65535_r20_fp64"]
    U, s, V = workloads.make(w, 0)
    return w, (U, s, V), cd.solve(w.n, U, s, V, w.r_max, w.tol, w.maxiter, selector="qdeim")


def test_qdeim_n65535_fp64_parity(oracle_n65535):
    w, (U, s, V), o = oracle_n65535
    print("qdeim n=65535 fp64", flush=True)
    g = gpu_qdeim(w.n, U, s, V, w.r_max, w.tol, w.maxiter)
    compare_fp64(g, o, "qdeim n65535")


def test_qdeim_n65535_mixed_error(oracle_n65535):
    w, (U, s, V), o = oracle_n65535
    print("qdeim n=65535 mixed", flush=True)
    g = gpu_qdeim(w.n, U, s, V, w.r_max, w.tol, w.maxiter, precision="mixed")
    e = cd.rel_err((g["U"], g["S"][: g["rank"]], g["V"]), (o.U, o.S, o.V))
    print(f"  mixed qdeim: status {g['info']['status']} iters {g['info']['iters']} rank {g['rank']} "
          f"rel err vs FP64 oracle {e:.3e}", flush=True)
    assert e <= 1e-5


def test_qdeim_sine_modes_and_safeguard():
    """Two sine modes: the spectral solution has exactly two nonzero rows and columns, so after
    the first pass QDEIM's pivots are all old indices and only the safeguard adds one."""
    n = 255
    U, s, V = workloads.sine_rhs(n, [(5, 9, 2.0), (12, 3, -0.7)])
    print("qdeim sine modes", flush=True)
    o = cd.solve(n, U, s, V, 8, 1e-10, 10, selector="qdeim")
    g = gpu_qdeim(n, U, s, V, 8, 1e-10, 10)
    compare_fp64(g, o, "qdeim sines")
    assert sorted(g["sets"][0]) == [4, 11] and sorted(g["sets"][1]) == [2, 8]
