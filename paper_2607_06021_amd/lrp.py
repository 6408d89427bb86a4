"""ctypes binding of liblrp.so (include/lrp.h), the HIP low-rank Poisson solver.

Argument marshalling only: every step of a solve runs in the library's HIP kernels.
PyTorch provides device memory and the stream. Matrices cross the boundary column-major:
an n x r factor is passed as a torch tensor of shape (n, r) whose transpose is contiguous
(``t.t().is_contiguous()``), i.e. the storage of an (r, n) row-major tensor.
"""
from __future__ import annotations

import ctypes
import math
import os
import re
from typing import Dict, List, Optional, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrp.so")
HEADER = os.path.join(HERE, "..", "include", "lrp.h")

LRP_OK, LRP_NOT_CONVERGED, LRP_STAGNATED = 0, 1, 2
LRP_EINVAL, LRP_ENOMEM, LRP_EDEVICE, LRP_ENUMERIC, LRP_ESIZE = -1, -2, -3, -4, -5
LRP_FP64, LRP_MIXED = 0, 1

_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_dbl = ctypes.c_double
_c_vp = ctypes.c_void_p


class Opts(ctypes.Structure):
    _fields_ = [("maxiter", _c_i32), ("precision", _c_i32), ("prune_tau", _c_dbl), ("stream", _c_vp),
                ("flags", _c_i32), ("selector", _c_i32), ("ls_oversampling", _c_dbl), ("seed", ctypes.c_uint64),
                ("matrix", _c_i32), ("reserved", _c_i32)]


LRP_FLAG_PROFILE = 1
LRP_SEL_LEVERAGE, LRP_SEL_QDEIM, LRP_SEL_LEVERAGE_SAMPLED = 0, 1, 2
_SELECTORS = {"ls": LRP_SEL_LEVERAGE, "qdeim": LRP_SEL_QDEIM, "ls_sampled": LRP_SEL_LEVERAGE_SAMPLED}
LRP_MAT_POISSON, LRP_MAT_HILBERT, LRP_MAT_K = 0, 1, 2
_MATRICES = {"poisson": LRP_MAT_POISSON, "hilbert": LRP_MAT_HILBERT, "k": LRP_MAT_K}


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", _c_i32), ("ms", _c_dbl)]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", _c_i32),
        ("iters", _c_i32),
        ("rank", _c_i32),
        ("nI", _c_i32),
        ("nJ", _c_i32),
        ("rho", _c_dbl),
        ("indicator", _c_dbl),
        ("ms", ctypes.c_float),
    ]

    def as_dict(self) -> Dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Request(ctypes.Structure):
    _fields_ = [
        ("n", _c_i64), ("r_F", _c_i32), ("r_max", _c_i32), ("tol", _c_dbl), ("maxiter", _c_i32),
        ("precision", _c_i32), ("U_F", _c_vp), ("ldu", _c_i64), ("sigma_F", _c_vp), ("V_F", _c_vp),
        ("ldv", _c_i64), ("U_out", _c_vp), ("ldou", _c_i64), ("S_out", _c_vp), ("V_out", _c_vp),
        ("ldov", _c_i64),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", _c_i64), ("completed", _c_i64), ("failed", _c_i64), ("queued", _c_i64),
                ("active", _c_i64), ("bytes_in_use", _c_i64), ("bytes_budget", _c_i64), ("contexts", _c_i32),
                ("grouping", _c_i32), ("passes", _c_i64), ("pass_launches", _c_i64)]

    def as_dict(self) -> Dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class LrpError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {strerror(code)} (code {code})")
        self.code = code


_LIB: Optional[ctypes.CDLL] = None


def header_functions() -> List[str]:
    """Names of the functions declared in include/lrp.h."""
    with open(HEADER) as f:
        text = f.read()
    return re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lrp_\w+)\s*\(", text, flags=re.M)


def lib() -> ctypes.CDLL:
    """Load liblrp.so; raises if the library has not been built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_06021_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    L.lrp_create.argtypes = [P(_c_vp), _c_i64, _c_i32, _c_dbl, P(Opts)]
    L.lrp_create.restype = ctypes.c_int
    L.lrp_solve.argtypes = [_c_vp, _c_i32, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp,
                            _c_vp, _c_i64, P(_c_i32), P(Info)]
    L.lrp_solve.restype = ctypes.c_int
    L.lrp_get_index_sets.argtypes = [_c_vp, P(_c_i64), P(_c_i32), P(_c_i64), P(_c_i32)]
    L.lrp_get_index_sets.restype = ctypes.c_int
    L.lrp_get_trace.argtypes = [_c_vp, P(_c_i32), P(_c_i32), P(_c_i32), P(_c_i32), P(_c_i32), P(_c_i32),
                                P(_c_i32), P(_c_i32), P(_c_dbl), P(_c_dbl), P(_c_i32), P(_c_i32), P(_c_i32)]
    L.lrp_get_trace.restype = ctypes.c_int
    L.lrp_set_guess.argtypes = [_c_vp, _c_i32, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64]
    L.lrp_set_guess.restype = ctypes.c_int
    L.lrp_set_index_sets.argtypes = [_c_vp, _c_i32, P(_c_i64), P(_c_i32), P(_c_i64), P(_c_i32)]
    L.lrp_set_index_sets.restype = ctypes.c_int
    L.lrp_destroy.argtypes = [_c_vp]
    L.lrp_destroy.restype = ctypes.c_int
    L.lrp_strerror.argtypes = [ctypes.c_int]
    L.lrp_strerror.restype = ctypes.c_char_p
    L.lrp_dst1.argtypes = [_c_vp, _c_i32, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_dbl, _c_i32]
    L.lrp_dst1.restype = ctypes.c_int
    L.lrp_tsqr.argtypes = [_c_vp, _c_i32, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64]
    L.lrp_tsqr.restype = ctypes.c_int
    L.lrp_server_create.argtypes = [P(_c_vp), _c_i64, _c_i32]
    L.lrp_server_create.restype = ctypes.c_int
    L.lrp_server_submit.argtypes = [_c_vp, P(Request), P(_c_i64)]
    L.lrp_server_submit.restype = ctypes.c_int
    L.lrp_server_poll.argtypes = [_c_vp, _c_i64, P(_c_i32), P(_c_i32), P(_c_i32), P(Info), P(_c_dbl)]
    L.lrp_server_poll.restype = ctypes.c_int
    L.lrp_server_wait.argtypes = [_c_vp, _c_i64, P(_c_i32), P(_c_i32), P(Info), P(_c_dbl)]
    L.lrp_server_wait.restype = ctypes.c_int
    L.lrp_server_times.argtypes = [_c_vp, _c_i64, P(_c_dbl), P(_c_dbl)]
    L.lrp_server_times.restype = ctypes.c_int
    L.lrp_server_release.argtypes = [_c_vp, _c_i64]
    L.lrp_server_release.restype = ctypes.c_int
    L.lrp_server_get_stats.argtypes = [_c_vp, P(ServerStats)]
    L.lrp_server_get_stats.restype = ctypes.c_int
    L.lrp_server_set_grouping.argtypes = [_c_vp, _c_i32]
    L.lrp_server_set_grouping.restype = ctypes.c_int
    L.lrp_server_destroy.argtypes = [_c_vp]
    L.lrp_server_destroy.restype = ctypes.c_int
    L.lrp_context_bytes.argtypes = [_c_i64, _c_i32, _c_i32, _c_i32]
    L.lrp_context_bytes.restype = ctypes.c_int64
    L.lrp_get_profile.argtypes = [_c_vp, P(_c_i32), P(KernelTime)]
    L.lrp_get_profile.restype = ctypes.c_int
    L.lrp_cross_solve.argtypes = [_c_vp, _c_i32, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64,
                                  P(_c_i32), P(Info)]
    L.lrp_cross_solve.restype = ctypes.c_int
    L.lrp_tsqr_noalloc.argtypes = [_c_i64, _c_i32, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp, _c_i64, _c_vp]
    L.lrp_tsqr_noalloc.restype = ctypes.c_int
    L.lrp_tsqr_noalloc_max_bytes.argtypes = []
    L.lrp_tsqr_noalloc_max_bytes.restype = ctypes.c_int64
    _LIB = L
    return L


def strerror(code: int) -> str:
    return lib().lrp_strerror(code).decode()


def _check(code: int, where: str, warn_ok: bool = False) -> int:
    if code < 0 or (code > 0 and not warn_ok):
        raise LrpError(code, where)
    return code


def _colmajor(t, n: int):
    """Pointer and leading dimension of a column-major (n, c) torch tensor."""
    if t.dim() != 2 or t.shape[0] != n:
        raise ValueError(f"expected an ({n}, c) matrix, got {tuple(t.shape)}")
    if t.stride(0) != 1:
        raise ValueError("matrix must be column-major (t.t().is_contiguous())")
    return t.data_ptr(), max(t.stride(1), n)


def fortran(t):
    """Column-major copy of a 2-D tensor (same shape)."""
    return t.t().contiguous().t()


def empty_fortran(n: int, c: int, dtype, device):
    import torch

    return torch.empty((c, n), dtype=dtype, device=device).t()


class Solver:
    """A library context: grid size n (n+1 a power of two), rank cap r_max, tolerance tol."""

    def __init__(self, n: int, r_max: int, tol: float, maxiter: int = 20, precision: str = "fp64",
                 prune_tau: float = 0.0, stream=None, profile: bool = False, selector: str = "ls",
                 ls_oversampling: float = 2.0, seed: int = 0, matrix: str = "poisson"):
        import torch

        self.n, self.r_max, self.tol = int(n), int(r_max), float(tol)
        self.maxiter = int(maxiter)
        self.precision = precision
        if stream is None:
            # a stream of its own (never the null stream), so that HIP events recorded on
            # self.stream bracket exactly the library's kernels
            stream = torch.cuda.Stream()
        self.stream = stream
        if selector not in _SELECTORS:
            raise ValueError(f"unknown selector {selector!r}")
        if matrix not in _MATRICES:
            raise ValueError(f"unknown matrix {matrix!r}")
        o = Opts(self.maxiter, LRP_MIXED if precision == "mixed" else LRP_FP64, float(prune_tau),
                 _c_vp(stream.cuda_stream), LRP_FLAG_PROFILE if profile else 0, _SELECTORS[selector],
                 float(ls_oversampling), int(seed), _MATRICES[matrix], 0)
        h = _c_vp()
        _check(lib().lrp_create(ctypes.byref(h), self.n, self.r_max, self.tol, ctypes.byref(o)), "lrp_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lrp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def profile(self) -> dict:
        """Per-kernel device time of the last solve (context created with profile=True):
        {name: (launches, ms)}, from HIP events recorded around every launch."""
        cap = 64
        arr = (KernelTime * cap)()
        cnt = _c_i32(cap)
        _check(lib().lrp_get_profile(self._h, ctypes.byref(cnt), arr), "lrp_get_profile")
        return {arr[q].name.decode(): (int(arr[q].launches), float(arr[q].ms)) for q in range(min(cnt.value, cap))}

    # ------------------------------------------------------------------------------------
    def solve(self, U_F, sigma, V_F, out=None, guess=None):
        """Solve with F = U_F diag(sigma) V_F^T (FP64 CUDA tensors, factors column-major).

        guess: optional (U0, S0, V0), the initial guess of Algorithm 4 in physical space
        (column-major (n, r0) FP64 CUDA tensors; S0 a vector of r0 weights or None).
        Returns (U, S, V, rank, info): U, V are (n, r_max) column-major with zero columns
        beyond `rank`, S has r_max entries.
        """
        import torch

        n, rm = self.n, self.r_max
        if guess is not None:
            U0, S0, V0 = guess
            p0, ld0 = _colmajor(U0, n)
            q0, lq0 = _colmajor(V0, n)
            if U0.shape[1] != V0.shape[1] or (S0 is not None and tuple(S0.shape) != (U0.shape[1],)):
                raise ValueError("guess factors must have matching column counts")
            for t in (U0, V0) + ((S0,) if S0 is not None else ()):
                if t.dtype != torch.float64 or not t.is_cuda:
                    raise ValueError("guess factors must be float64 CUDA tensors")
            if S0 is not None and not S0.is_contiguous():
                raise ValueError("S0 must be contiguous")
            _check(lib().lrp_set_guess(self._h, U0.shape[1], p0, ld0, S0.data_ptr() if S0 is not None else None,
                                       q0, lq0), "lrp_set_guess")
        rF = U_F.shape[1]
        pu, ldu = _colmajor(U_F, n)
        pv, ldv = _colmajor(V_F, n)
        if sigma.dim() != 1 or sigma.shape[0] != rF or not sigma.is_contiguous():
            raise ValueError("sigma must be a contiguous vector of length r_F")
        for t in (U_F, V_F, sigma):
            if t.dtype != torch.float64 or not t.is_cuda:
                raise ValueError("inputs must be float64 CUDA tensors")
        if out is None:
            Uo = empty_fortran(n, rm, torch.float64, U_F.device)
            Vo = empty_fortran(n, rm, torch.float64, U_F.device)
            So = torch.empty(rm, dtype=torch.float64, device=U_F.device)
        else:
            Uo, So, Vo = out
        puo, lduo = _colmajor(Uo, n)
        pvo, ldvo = _colmajor(Vo, n)
        r = _c_i32(0)
        info = Info()
        self._order()
        code = lib().lrp_solve(self._h, rF, pu, ldu, sigma.data_ptr(), pv, ldv, puo, lduo, So.data_ptr(),
                               pvo, ldvo, ctypes.byref(r), ctypes.byref(info))
        _check(code, "lrp_solve", warn_ok=True)
        return Uo, So, Vo, int(r.value), info

    def cross(self, U0, V0, out=None):
        """Cross-DEIM on the context's test matrix from the guess U0 V0^T (column-major (n, r0)
        FP64 CUDA tensors). Returns (U, S, V, rank, info) as solve."""
        import torch

        n, rm = self.n, self.r_max
        p0, ld0 = _colmajor(U0, n)
        q0, lq0 = _colmajor(V0, n)
        if U0.shape[1] != V0.shape[1]:
            raise ValueError("U0 and V0 must have the same number of columns")
        for t in (U0, V0):
            if t.dtype != torch.float64 or not t.is_cuda:
                raise ValueError("inputs must be float64 CUDA tensors")
        if out is None:
            Uo = empty_fortran(n, rm, torch.float64, U0.device)
            Vo = empty_fortran(n, rm, torch.float64, U0.device)
            So = torch.empty(rm, dtype=torch.float64, device=U0.device)
        else:
            Uo, So, Vo = out
        puo, lduo = _colmajor(Uo, n)
        pvo, ldvo = _colmajor(Vo, n)
        r = _c_i32(0)
        info = Info()
        self._order()
        code = lib().lrp_cross_solve(self._h, U0.shape[1], p0, ld0, q0, lq0, puo, lduo, So.data_ptr(), pvo, ldvo,
                                     ctypes.byref(r), ctypes.byref(info))
        _check(code, "lrp_cross_solve", warn_ok=True)
        return Uo, So, Vo, int(r.value), info

    def _order(self):
        """Make the context stream wait for work already queued on the caller's stream."""
        import torch

        cur = torch.cuda.current_stream()
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def index_sets(self) -> Tuple[List[int], List[int]]:
        I = (_c_i64 * self.r_max)()
        J = (_c_i64 * self.r_max)()
        nI, nJ = _c_i32(), _c_i32()
        _check(lib().lrp_get_index_sets(self._h, I, ctypes.byref(nI), J, ctypes.byref(nJ)), "lrp_get_index_sets")
        return list(I[: nI.value]), list(J[: nJ.value])

    def trace(self) -> List[Dict]:
        m = self.maxiter
        rm = self.r_max
        cnt = _c_i32(m)
        Ip = (_c_i32 * (m * rm))()
        Jp = (_c_i32 * (m * rm))()
        nIp, nJp, nI, nJ, rk, br, rt, sw = [(_c_i32 * m)() for _ in range(8)]
        ind, rho = (_c_dbl * m)(), (_c_dbl * m)()
        _check(lib().lrp_get_trace(self._h, ctypes.byref(cnt), Ip, nIp, Jp, nJp, nI, nJ, rk, ind, rho, br, rt, sw),
               "lrp_get_trace")
        out = []
        for k in range(cnt.value):
            out.append({
                "k": k,
                "I_pre": list(Ip[k * rm: k * rm + nIp[k]]),
                "J_pre": list(Jp[k * rm: k * rm + nJp[k]]),
                "nI": nI[k],
                "nJ": nJ[k],
                "rank": rk[k],
                "indicator": ind[k],
                "rho": rho[k],
                "branch": bool(br[k]),
                "route": "qr" if rt[k] == 0 else "jacobi",
                "sweeps": sw[k],
            })
        return out

    def set_index_sets(self, sets):
        """Replay: passes 0 .. len(sets)-1 of the following solves use sets[k] = (I, J) as their
        index sets; an empty list switches replay off."""
        m, rm = len(sets), self.r_max
        I = (_c_i64 * max(1, m * rm))()
        J = (_c_i64 * max(1, m * rm))()
        nI = (_c_i32 * max(1, m))()
        nJ = (_c_i32 * max(1, m))()
        for k, (Ik, Jk) in enumerate(sets):
            nI[k], nJ[k] = len(Ik), len(Jk)
            for q, v in enumerate(Ik[:rm]):
                I[k * rm + q] = int(v)
            for q, v in enumerate(Jk[:rm]):
                J[k * rm + q] = int(v)
        _check(lib().lrp_set_index_sets(self._h, m, I, nI, J, nJ), "lrp_set_index_sets")

    def dst1(self, X, scale=None, mul: float = 1.0, precision: str = "fp64"):
        """Orthonormal DST-I of the columns of X (n x c, column-major FP64 CUDA tensor)."""
        import torch

        px, ldx = _colmajor(X, self.n)
        Y = empty_fortran(self.n, X.shape[1], torch.float64, X.device)
        py, ldy = _colmajor(Y, self.n)
        ps = scale.data_ptr() if scale is not None else None
        self._order()
        _check(lib().lrp_dst1(self._h, X.shape[1], px, ldx, py, ldy, ps, float(mul),
                              LRP_MIXED if precision == "mixed" else LRP_FP64), "lrp_dst1")
        torch.cuda.current_stream().wait_stream(self.stream)
        return Y

    def tsqr(self, A):
        """Thin Householder QR of A (n x c, column-major FP64 CUDA tensor): returns Q, R."""
        import torch

        pa, lda = _colmajor(A, self.n)
        c = A.shape[1]
        Q = empty_fortran(self.n, c, torch.float64, A.device)
        R = empty_fortran(c, c, torch.float64, A.device)
        pq, ldq = _colmajor(Q, self.n)
        self._order()
        _check(lib().lrp_tsqr(self._h, c, pa, lda, pq, ldq, R.data_ptr(), c), "lrp_tsqr")
        return Q, R


class Server:
    """A solve queue with continuous admission (lrp_server_*): submit requests, poll them."""

    def __init__(self, budget_bytes: int, max_active: int = 8, grouping: bool = True):
        h = _c_vp()
        _check(lib().lrp_server_create(ctypes.byref(h), int(budget_bytes), int(max_active)), "lrp_server_create")
        self._h = h
        self._keep: Dict[int, tuple] = {}
        if not grouping:
            self.set_grouping(False)

    def set_grouping(self, enabled: bool):
        """Same-stage grouping of ready passes on or off (only while nothing is queued or active)."""
        _check(lib().lrp_server_set_grouping(self._h, 1 if enabled else 0), "lrp_server_set_grouping")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lrp_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, n: int, U_F, sigma, V_F, r_max: int, tol: float, maxiter: int = 20,
               precision: str = "fp64", out=None, sync: bool = True) -> int:
        """Queue one solve; returns its ticket. Outputs default to new (n, r_max) tensors.

        The inputs must be complete on the device when the server reads them: with sync=True
        the caller's current stream is synchronized first.
        """
        import torch

        pu, ldu = _colmajor(U_F, n)
        pv, ldv = _colmajor(V_F, n)
        if out is None:
            Uo = empty_fortran(n, r_max, torch.float64, U_F.device)
            Vo = empty_fortran(n, r_max, torch.float64, U_F.device)
            So = torch.empty(r_max, dtype=torch.float64, device=U_F.device)
        else:
            Uo, So, Vo = out
        puo, lduo = _colmajor(Uo, n)
        pvo, ldvo = _colmajor(Vo, n)
        if sync:
            torch.cuda.current_stream().synchronize()
        req = Request(n, U_F.shape[1], r_max, tol, maxiter, LRP_MIXED if precision == "mixed" else LRP_FP64,
                      pu, ldu, sigma.data_ptr(), pv, ldv, puo, lduo, So.data_ptr(), pvo, ldvo)
        t = _c_i64()
        _check(lib().lrp_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "lrp_server_submit")
        self._keep[t.value] = (U_F, sigma, V_F, Uo, So, Vo)
        return t.value

    def poll(self, ticket: int):
        """None while running; else (U, S, V, rank, status, info, latency_ms, queue_ms, run_ms):
        latency from submission, split into the wait for admission and the run after it."""
        done, st, rk, lat = _c_i32(), _c_i32(), _c_i32(), _c_dbl()
        info = Info()
        _check(lib().lrp_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(rk),
                                     ctypes.byref(info), ctypes.byref(lat)), "lrp_server_poll")
        if not done.value:
            return None
        return self._result(ticket, st.value, rk.value, info, lat.value)

    def wait(self, ticket: int):
        st, rk, lat = _c_i32(), _c_i32(), _c_dbl()
        info = Info()
        _check(lib().lrp_server_wait(self._h, ticket, ctypes.byref(st), ctypes.byref(rk), ctypes.byref(info),
                                     ctypes.byref(lat)), "lrp_server_wait")
        return self._result(ticket, st.value, rk.value, info, lat.value)

    def _result(self, ticket, status, rank, info, lat):
        qms, rms = _c_dbl(), _c_dbl()
        _check(lib().lrp_server_times(self._h, ticket, ctypes.byref(qms), ctypes.byref(rms)), "lrp_server_times")
        bufs = self._keep.pop(ticket)
        lib().lrp_server_release(self._h, ticket)
        return bufs[3], bufs[4], bufs[5], rank, status, info, lat, qms.value, rms.value

    def stats(self) -> Dict:
        st = ServerStats()
        _check(lib().lrp_server_get_stats(self._h, ctypes.byref(st)), "lrp_server_get_stats")
        return st.as_dict()


def context_bytes(n: int, r_max: int, maxiter: int = 20, precision: str = "fp64") -> int:
    return int(lib().lrp_context_bytes(n, r_max, maxiter, LRP_MIXED if precision == "mixed" else LRP_FP64))
