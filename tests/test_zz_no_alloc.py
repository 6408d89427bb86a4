"""The allocation-free thin QR (lrp_tsqr_noalloc, static per-GPU workspace) against the
context-based lrp_tsqr, through the C-ABI: two calls in a row (the second smaller), each
bitwise equal to the context entry point with the same tree (p_max = ncols), and a size beyond
the fixed workspace rejected on the host."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _fortran_dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def _noalloc(A):
    torch = _torch()
    from paper_2607_06021_amd import lrp as L
    from paper_2607_06021_amd.lrp import empty_fortran

    n, p = A.shape
    Q = empty_fortran(n, p, torch.float64, A.device)
    R = empty_fortran(p, p, torch.float64, A.device)
    s = torch.cuda.current_stream()
    rc = L.lib().lrp_tsqr_noalloc(n, p, A.data_ptr(), A.stride(1), Q.data_ptr(), Q.stride(1), R.data_ptr(),
                                  R.stride(1), ctypes.c_void_p(s.cuda_stream))
    assert rc == 0, L.strerror(rc)
    s.synchronize()
    return Q.cpu().numpy(), R.cpu().numpy()


def _with_context(A):
    from paper_2607_06021_amd import Solver

    n, p = A.shape
    with Solver(n, p, 1e-10) as sol:
        Q, R = sol.tsqr(A)
        return Q.cpu().numpy(), R.cpu().numpy()


def test_noalloc_tsqr_matches_context_entry_point_twice():
    _torch()
    rng = np.random.default_rng(7)
    for n, p in ((16383, 64), (4095, 20)):
        print(f"noalloc tsqr n={n} p={p}", flush=True)
        A = _fortran_dev(rng.standard_normal((n, p)))
        Qn, Rn = _noalloc(A)
        Qc, Rc = _with_context(A)
        An = A.cpu().numpy()
        print(f"  |QR-A|/|A| {np.linalg.norm(Qn @ Rn - An) / np.linalg.norm(An):.2e}, "
              f"bitwise equal Q {np.array_equal(Qn, Qc)} R {np.array_equal(Rn, Rc)}", flush=True)
        assert np.array_equal(Qn, Qc) and np.array_equal(Rn, Rc)
        assert np.array_equal(np.tril(Rn, -1), np.zeros_like(Rn))


def test_noalloc_tsqr_rejects_sizes_beyond_its_workspace():
    from paper_2607_06021_amd import lrp as L

    # checked on the host before anything is enqueued: no device pointer is touched
    A = ctypes.c_void_p(256)
    Q = ctypes.c_void_p(1 << 40)
    R = ctypes.c_void_p(1 << 41)
    assert L.lib().lrp_tsqr_noalloc(32767, 64, A, 32767, Q, 32767, R, 64, None) == L.LRP_ESIZE
    assert L.lib().lrp_tsqr_noalloc(32661, 65, A, 32661, Q, 32661, R, 65, None) == L.LRP_EINVAL
    assert L.lib().lrp_tsqr_noalloc(100, 8, A, 99, Q, 100, R, 8, None) == L.LRP_EINVAL
