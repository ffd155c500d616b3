"""MI355X-native low-rank Fourier-Galerkin homogenisation (liblrfg).

Python binding of the C ABI in include/lrfg.h.  PyTorch provides device
memory (the workspace and device-resident inputs) and the HIP stream; every
step of the solve runs in the library's HIP kernels.

    from paper_1902_07455_amd import Solver
    s = Solver(d=3, N=(135, 135, 135), format="full", solver_tol=1e-8)
    res = s.solve(full=a)          # a: numpy array or torch tensor
    res.A_H                        # (d, d)
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import LrfgError, check, lib

__all__ = ["Solver", "SolveResult", "LrfgError", "lib", "fft_lines", "mode_op", "full_op",
           "gemm", "syevj", "gram_cut", "compress_tt", "compress_tucker", "tucker_round", "tt_round", "abi_version", "ga_double_grid", "device_check", "prof_enable", "prof_read", "prof_work", "Server",
           "Completion"]

_FORMATS = {"full": _lib.FORMAT_FULL, "cp": _lib.FORMAT_CP, "tucker": _lib.FORMAT_TUCKER,
            "tt": _lib.FORMAT_TT}
_SOLVERS = {"pcg": _lib.SOLVER_PCG, "mr": _lib.SOLVER_MR}
_PRECS = {"fp64": _lib.PREC_FP64, "fp32": _lib.PREC_MIXED_FP32, "bf16": _lib.PREC_MIXED_BF16}


def abi_version() -> int:
    return lib().lrfg_abi_version()


def ga_double_grid(N: int) -> int:
    """The double grid of the Ga discretisation for N points per axis: the
    smallest odd 3^a 5^b >= 2N - 1, or 2N - 1 when that exceeds 2048."""
    m = lib().lrfg_ga_double_grid(int(N))
    if m < 0:
        check(m)
    return m


def device_check() -> int:
    return lib().lrfg_device_check()


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class _Held:
    """Keeps host/device buffers alive while a call runs; yields pointers."""

    def __init__(self, device):
        self.keep = []
        self.device = device

    def ptr(self, x, dtype=np.float64):
        """Pointer and on-device flag for a numpy array or torch tensor."""
        if x is None:
            return None, 0
        torch = _torch() if not isinstance(x, np.ndarray) else None
        if torch is not None and isinstance(x, torch.Tensor):
            t = x.detach()
            if t.dtype != torch.float64:
                raise TypeError("FP64 tensors expected")
            t = t.contiguous()
            self.keep.append(t)
            return t.data_ptr(), int(t.is_cuda)
        arr = np.ascontiguousarray(np.asarray(x, dtype=dtype))
        self.keep.append(arr)
        return arr.ctypes.data, 0


@dataclasses.dataclass
class SolveResult:
    A_H: np.ndarray
    iters: np.ndarray
    res_hist: np.ndarray
    ranks: np.ndarray
    status: np.ndarray
    rc: int
    setup_ms: float
    solve_ms: float


_INCLUSIONS = {"square": 1, "cube": 1, "ball": 2}


def _fill_coeff(c, h, full=None, cp=None, tt=None, tucker=None, inclusion=None):
    """Fill an lrfg_coeff from numpy arrays or torch tensors (kept alive by h);
    inclusion: dict(shape="square"|"cube"|"ball", size=, inside=, outside=)
    (the Ga discretisation's coefficient)."""
    on_dev = 0
    if inclusion is not None:
        c.inclusion = _INCLUSIONS[inclusion["shape"]]
        c.incl_size = float(inclusion["size"])
        c.incl_inside = float(inclusion["inside"])
        c.incl_outside = float(inclusion["outside"])
    elif full is not None:
        ptr, on_dev = h.ptr(full)
        c.full = ptr
    elif cp is not None:
        w, fac = cp
        ptr, on_dev = h.ptr(w)
        c.weights = ptr
        c.rank = int(len(w))
        for i, f in enumerate(fac):
            c.factors[i] = h.ptr(f)[0]
    elif tt is not None:
        for i, G in enumerate(tt):
            c.tt_cores[i], on_dev = h.ptr(G)
            c.tt_ranks[i] = int(G.shape[0])
        c.tt_ranks[len(tt)] = int(tt[-1].shape[2])
    elif tucker is not None:
        core, frames = tucker
        c.tucker_core, on_dev = h.ptr(core)
        for i, F in enumerate(frames):
            c.tucker_frames[i] = h.ptr(F)[0]
            c.tucker_ranks[i] = int(F.shape[1])
    else:
        raise ValueError("give one of full / cp / tt / tucker")
    c.on_device = on_dev


def _result_buffers(r, nE, d, max_iter):
    """Host arrays behind one lrfg_result."""
    A = np.zeros((nE, nE))
    iters = np.zeros(nE, dtype=np.int32)
    hist = np.zeros((nE, max_iter))
    ranks = np.zeros((nE, d + 1), dtype=np.int32)
    status = np.zeros(nE, dtype=np.int32)
    r.A_H = A.ctypes.data
    r.iters = iters.ctypes.data
    r.res_hist = hist.ctypes.data
    r.ranks = ranks.ctypes.data
    r.status = status.ctypes.data
    return A, iters, hist, ranks, status


def _make_problem(d, N, format="full", rank_cap=0, trunc_tol=0.0, solver_tol=1e-10, max_iter=1000,
                  solver="pcg", precision="fp64", precond_terms=0, oversample=0, seed=0, coeff_rank=0,
                  aniso=None, rank_start=0, discretisation="gani"):
    p = _lib.Problem()
    p.d = int(d)
    Ns = list(N) + [1] * (3 - len(N))
    for i in range(3):
        p.N[i] = int(Ns[i])
    p.format = _FORMATS[format]
    p.rank_cap = int(rank_cap)
    p.trunc_tol = float(trunc_tol)
    p.solver_tol = float(solver_tol)
    p.max_iter = int(max_iter)
    p.solver = _SOLVERS[solver]
    p.precision = _PRECS[precision]
    p.precond_terms = int(precond_terms)
    p.oversample = int(oversample)
    p.seed = int(seed)
    p.coeff_rank = int(coeff_rank)
    p.flags = 0
    if aniso is not None:
        B = np.asarray(aniso, dtype=np.float64)
        if B.shape != (int(d), int(d)):
            raise ValueError("aniso must be a d x d matrix")
        for i, v in enumerate(B.reshape(-1)):
            p.aniso[i] = float(v)
    p.rank_start = int(rank_start)
    p.discretisation = {"gani": 0, "ga": 1}[discretisation]
    return p


class Solver:
    """A plan plus its device workspace, reusable across solves."""

    def __init__(self, d: int, N: Sequence[int], format: str = "full", rank_cap: int = 0,
                 trunc_tol: float = 0.0, solver_tol: float = 1e-10, max_iter: int = 1000,
                 solver: str = "pcg", precision: str = "fp64", precond_terms: int = 0,
                 oversample: int = 0, seed: int = 0, max_nE: Optional[int] = None,
                 coeff_rank: int = 0, device: str = "cuda:0", aniso=None, rank_start: int = 0,
                 discretisation: str = "gani"):
        L = lib()
        p = _make_problem(d, N, format, rank_cap, trunc_tol, solver_tol, max_iter, solver, precision,
                          precond_terms, oversample, seed, coeff_rank, aniso, rank_start, discretisation)
        self.problem = p
        self.d = int(d)
        self.max_iter = int(max_iter)
        self._plan = C.c_void_p()
        check(L.lrfg_plan_create(C.byref(p), C.byref(self._plan)))
        self.max_nE = int(max_nE or d)
        nb = C.c_size_t()
        check(L.lrfg_plan_workspace_bytes(self._plan, self.max_nE, C.byref(nb)))
        self.workspace_bytes = int(nb.value)
        self.device = device
        self._ws = None

    def workspace(self):
        if self._ws is None:
            torch = _torch()
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def solve(self, full=None, cp=None, tt=None, tucker=None, E=None, stream=None, inclusion=None) -> SolveResult:
        """full: nodal values; cp: (weights (R,), [factors (R, N_i)]);
        tt: list of cores [r_{i-1}][N_i][r_i]; tucker: (core (r_1, r_2, r_3),
        [frames (N_i, r_i)]); inclusion: dict(shape, size, inside, outside)
        for discretisation="ga".  E: (nE, d) or None."""
        return self.solve_batch([dict(full=full, cp=cp, tt=tt, tucker=tucker, inclusion=inclusion)], E=E,
                                stream=stream)[0]

    def solve_batch(self, coeffs, E=None, stream=None):
        """Several microstructures of this problem in one batched solve
        (lrfg_solve_batch): coeffs is a list of dicts with one of the keys
        full / cp / tt (as in solve).  Needs max_nE >= len(coeffs) * nE.
        Returns one SolveResult per microstructure."""
        L = lib()
        torch = _torch()
        h = _Held(self.device)
        cs = (_lib.Coeff * len(coeffs))()
        for k, kw in enumerate(coeffs):
            _fill_coeff(cs[k], h, kw.get("full"), kw.get("cp"), kw.get("tt"), kw.get("tucker"), kw.get("inclusion"))
        d = self.d
        if E is None:
            nE = d
            Eptr = None
        else:
            Earr = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(-1, d))
            nE = Earr.shape[0]
            h.keep.append(Earr)
            Eptr = Earr.ctypes.data
        rs = (_lib.Result * len(coeffs))()
        bufs = [_result_buffers(rs[k], nE, d, self.max_iter) for k in range(len(coeffs))]
        ws = self.workspace()
        with torch.cuda.device(torch.device(self.device)):
            sh = _stream_handle(stream)
            rc = L.lrfg_solve_batch(self._plan, cs, len(coeffs), Eptr, nE, C.c_void_p(ws.data_ptr()),
                                    self.workspace_bytes, C.c_void_p(sh), rs)
        check(rc, allow=(_lib.OK, _lib.NOT_CONVERGED, _lib.RANK_LIMITED))
        out = []
        for k, (A, iters, hist, ranks, status) in enumerate(bufs):
            rck = (_lib.NOT_CONVERGED if np.any(status == _lib.NOT_CONVERGED) else
                   _lib.RANK_LIMITED if np.any(status == _lib.RANK_LIMITED) else _lib.OK)
            out.append(SolveResult(A, iters, hist, ranks, status, rck, rs[k].setup_ms, rs[k].solve_ms))
        return out

    def close(self):
        """Destroy the plan and release its device workspace."""
        if self._plan:
            lib().lrfg_plan_destroy(self._plan)
            self._plan = C.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclasses.dataclass
class Completion:
    tag: int
    status: int
    batch_size: int
    queue_ms: float
    run_ms: float
    total_ms: float
    workspace_bytes: int
    result: SolveResult


class Server:
    """Continuous-batching request loop (lrfg_server_*): queued requests are
    admitted by workspace footprint in a device pool of pool_bytes, batched
    with queued requests of the same problem (up to max_batch per solve), and
    run as sessions on their own threads and HIP streams that share `slots`
    device permits in turns of iteration blocks."""

    def __init__(self, slots: int = 2, max_batch: int = 8, pool_bytes: int = 8 << 30, device: str = "cuda:0"):
        torch = _torch()
        dev = torch.device(device)
        self.device = device
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=dev)
        self._h = C.c_void_p()
        check(lib().lrfg_server_create(dev.index or 0, int(slots), int(max_batch), C.c_void_p(self.pool.data_ptr()),
                                       int(pool_bytes), C.byref(self._h)))
        self._pending = {}
        self._next = 0

    def submit(self, problem: dict, full=None, cp=None, tt=None, tucker=None, E=None,
               tag: Optional[int] = None) -> int:
        """Queue one request; problem holds Solver's keyword arguments
        (d, N, format, rank_cap, ...).  Returns its tag."""
        h = _Held(self.device)
        pr = _make_problem(**problem)
        c = _lib.Coeff()
        _fill_coeff(c, h, full, cp, tt, tucker)
        d = pr.d
        if E is None:
            nE, Eptr = d, None
        else:
            Earr = np.ascontiguousarray(np.asarray(E, dtype=np.float64).reshape(-1, d))
            nE = Earr.shape[0]
            h.keep.append(Earr)
            Eptr = Earr.ctypes.data
        r = _lib.Result()
        bufs = _result_buffers(r, nE, d, pr.max_iter)
        if tag is None:
            tag = self._next
        self._next = max(self._next, int(tag)) + 1
        torch = _torch()
        with torch.cuda.device(torch.device(self.device)):
            sh = _stream_handle(None)  # the caller's current stream: device inputs are ordered after it
        check(lib().lrfg_server_submit(self._h, C.byref(pr), C.byref(c), Eptr, nE, C.byref(r), int(tag),
                                       C.c_void_p(sh)))
        self._pending[int(tag)] = (h, pr, c, r, bufs)
        return int(tag)

    def poll(self, timeout_ms: int = 0, max_n: int = 256):
        """Completed requests (waits up to timeout_ms for the first; < 0: until one)."""
        done = (_lib.Completion * max_n)()
        n = C.c_int()
        check(lib().lrfg_server_poll(self._h, done, max_n, C.byref(n), int(timeout_ms)))
        out = []
        for k in range(n.value):
            c = done[k]
            h, pr, coeff, r, (A, iters, hist, ranks, status) = self._pending.pop(int(c.tag))
            res = SolveResult(A, iters, hist, ranks, status, int(c.status), r.setup_ms, r.solve_ms)
            out.append(Completion(int(c.tag), int(c.status), int(c.batch_size), float(c.queue_ms),
                                  float(c.run_ms), float(c.total_ms), int(c.workspace_bytes), res))
        return out

    def pending(self) -> int:
        return int(lib().lrfg_server_pending(self._h))

    def drain(self):
        """Wait for every submitted request; returns their completions."""
        out = []
        while self._pending:
            out += self.poll(timeout_ms=1000)
        return out

    def close(self):
        if self._h:
            lib().lrfg_server_destroy(self._h)
            self._h = C.c_void_p()
            self._pending.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prof_enable(kernel: Optional[str]):
    """Time every later launch of `kernel` with HIP events (None: off)."""
    check(lib().lrfg_prof_enable(kernel.encode() if kernel else None))


def prof_read():
    """(launch count, summed milliseconds) of the timed kernel."""
    n = C.c_int()
    ms = C.c_double()
    check(lib().lrfg_prof_read(C.byref(n), C.byref(ms)))
    return int(n.value), float(ms.value)


def prof_work() -> float:
    """Summed algorithmic work (FLOPs or bytes) of the timed launches."""
    w = C.c_double()
    check(lib().lrfg_prof_work(C.byref(w)))
    return float(w.value)


# ---------------------------------------------------------------- op level
def _ws_tensor(nbytes, device):
    torch = _torch()
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def fft_lines(x, outer: int, N: int, inner: int, direction: int, stream=None):
    """In-place batched 1-D DFT of a complex128 CUDA tensor viewed as
    [outer][N][inner]; direction -1 = F_N (with 1/N), +1 = inverse."""
    L = lib()
    ws = _ws_tensor(L.lrfg_fft_workspace_bytes(N), x.device)
    check(L.lrfg_fft_lines(C.c_void_p(x.data_ptr()), outer, N, inner, direction,
                           C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(_stream_handle(stream))))
    return x


def mode_op(x, outer: int, N: int, inner: int, op: int, t: float = 0.0, stream=None):
    """In-place real circulant along the middle index of a float64 CUDA
    tensor [outer][N][inner]: op 0 derivative, op 1 heat kernel exp(-t k^2),
    op 2 projection onto the frequencies |k| <= t."""
    L = lib()
    ws = _ws_tensor(L.lrfg_fft_workspace_bytes(N), x.device)
    check(L.lrfg_mode_op(C.c_void_p(x.data_ptr()), outer, N, inner, op, float(t),
                         C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(_stream_handle(stream))))
    return x


def full_op(which: int, N, a, u, out, stream=None):
    """Full-grid K (which 0) or P^-1 (which 1) on complex128 half spectra."""
    L = lib()
    Nc = (C.c_int * 3)(*[int(n) for n in N])
    ws = _ws_tensor(L.lrfg_full_op_workspace_bytes(Nc), u.device)
    aptr = C.c_void_p(a.data_ptr()) if a is not None else None
    check(L.lrfg_full_op(which, Nc, aptr, C.c_void_p(u.data_ptr()), C.c_void_p(out.data_ptr()),
                         C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(_stream_handle(stream))))
    return out


def gemm(A, B, C_, ta=False, tb=False, alpha=1.0, beta=0.0, stream=None, precision: str = "fp64"):
    """C_ = alpha op(A) op(B) + beta C_ on float64 CUDA tensors of shape
    (batch, rows, cols) (contiguous); returns C_.  precision "fp32" / "bf16":
    operands rounded to that type, FP32 accumulation (lrfg_gemm_mixed)."""
    L = lib()
    bt = C_.shape[0]
    m, n = C_.shape[1], C_.shape[2]
    k = A.shape[1] if ta else A.shape[2]
    ws = _ws_tensor(L.lrfg_gemm_workspace_bytes(m, n, k, bt), C_.device)
    sA = A.shape[1] * A.shape[2] if A.shape[0] > 1 else 0
    sB = B.shape[1] * B.shape[2] if B.shape[0] > 1 else 0
    check(L.lrfg_gemm_mixed(_PRECS[precision], int(ta), int(tb), m, n, k, float(alpha), C.c_void_p(A.data_ptr()),
                            A.shape[2], sA, C.c_void_p(B.data_ptr()), B.shape[2], sB, float(beta),
                            C.c_void_p(C_.data_ptr()), n, m * n, bt, C.c_void_p(ws.data_ptr()), ws.numel(),
                            C.c_void_p(_stream_handle(stream))))
    return C_


def syevj(A, stream=None):
    """Batched symmetric eigendecomposition of a (batch, n, n) float64 CUDA
    tensor: (W descending, V with eigenvectors as columns)."""
    torch = _torch()
    bt, n = A.shape[0], A.shape[1]
    W = torch.empty((bt, n), dtype=torch.float64, device=A.device)
    V = torch.empty((bt, n, n), dtype=torch.float64, device=A.device)
    check(lib().lrfg_syevj(n, C.c_void_p(A.data_ptr()), bt, C.c_void_p(W.data_ptr()),
                           C.c_void_p(V.data_ptr()), C.c_void_p(_stream_handle(stream))))
    return W, V


def gram_cut(G, c: int, tol: float = 0.0, stream=None):
    """Truncation basis of a (batch, n, n) float64 CUDA tensor of PSD Gram
    matrices: (S (batch, n, c) kept eigenvectors, kept (batch,), sweeps
    (batch,)) as tensors."""
    torch = _torch()
    bt, n = G.shape[0], G.shape[1]
    G = G.contiguous()
    S = torch.empty((bt, n, c), dtype=torch.float64, device=G.device)
    kept = torch.empty((bt,), dtype=torch.int32, device=G.device)
    sweeps = torch.empty((bt,), dtype=torch.int32, device=G.device)
    check(lib().lrfg_gram_cut(n, c, C.c_void_p(G.data_ptr()), bt, float(tol), C.c_void_p(S.data_ptr()),
                              C.c_void_p(kept.data_ptr()), C.c_void_p(sweeps.data_ptr()),
                              C.c_void_p(_stream_handle(stream))))
    return S, kept, sweeps


def tucker_round(frames, core, cap: int, tol: float = 0.0, oversample: int = 10, seed: int = 0, stream=None):
    """Truncate nE Tucker tensors: frames[j] (nE, N_j, r_j) and core
    (nE, r_1, r_2, r_3) float64 CUDA tensors.  Returns (frames, core, kept
    ranks (3, nE))."""
    torch = _torch()
    L = lib()
    nE = core.shape[0]
    Ns = [int(F.shape[1]) for F in frames]
    rin = [int(F.shape[2]) for F in frames]
    Nc = (C.c_int * 3)(*Ns)
    Rc = (C.c_int * 3)(*rin)
    nb = L.lrfg_tucker_round_workspace_bytes(Nc, Rc, int(cap), int(oversample), nE)
    if nb == 0:
        raise LrfgError(-1, "bad tucker_round sizes")
    ws = _ws_tensor(nb, core.device)
    c = [min(cap, n) for n in Ns]
    fo = [torch.empty((nE, Ns[j], c[j]), dtype=torch.float64, device=core.device) for j in range(3)]
    co = torch.empty((nE, c[0], c[1], c[2]), dtype=torch.float64, device=core.device)
    fi = [F.contiguous() for F in frames]
    ci = core.contiguous()
    ip = (C.c_void_p * 3)(*[F.data_ptr() for F in fi])
    op = (C.c_void_p * 3)(*[F.data_ptr() for F in fo])
    ranks = (C.c_int * 3)()
    kept = (C.c_int * (3 * nE))()
    check(L.lrfg_tucker_round(Nc, Rc, ip, C.c_void_p(ci.data_ptr()), int(cap), float(tol), int(oversample),
                              int(seed), op, C.c_void_p(co.data_ptr()), ranks, kept, nE,
                              C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(_stream_handle(stream))))
    return fo, co, np.array(list(kept), dtype=np.int32).reshape(3, nE)


def compress_tt(a, cap: int, tol: float = 0.0, oversample: int = 10, seed: int = 0, stream=None):
    """Full field a (float64 CUDA tensor, 2 or 3 dims) -> (TT cores
    [r_{j-1}][N_j][r_j] as CUDA tensors with the nominal ranks, kept ranks)."""
    torch = _torch()
    L = lib()
    d = a.dim()
    Ns = list(a.shape) + [1] * (3 - d)
    Nc = (C.c_int * 3)(*Ns)
    nb = L.lrfg_compress_workspace_bytes(d, Nc, int(cap), int(oversample))
    if nb == 0:
        raise LrfgError(-1, "bad compression sizes")
    ws = _ws_tensor(nb, a.device)
    c = [1] * 4
    if d == 3:
        c[1] = min(cap, Ns[0], Ns[1] * Ns[2])
        c[2] = min(cap, Ns[2], Ns[0] * Ns[1])
    else:
        c[1] = min(cap, Ns[0], Ns[1])
    outs = [torch.empty((c[j], Ns[j], c[j + 1]), dtype=torch.float64, device=a.device) for j in range(d)]
    optr = (C.c_void_p * 3)(*([o.data_ptr() for o in outs] + [0] * (3 - d)))
    ranks = (C.c_int * 4)()
    kept = (C.c_int * 2)()
    a = a.contiguous()
    check(L.lrfg_compress_tt(d, Nc, C.c_void_p(a.data_ptr()), int(cap), float(tol), int(oversample), int(seed),
                             optr, ranks, kept, C.c_void_p(ws.data_ptr()), ws.numel(),
                             C.c_void_p(_stream_handle(stream))))
    return outs, [int(kept[j]) for j in range(d - 1)]


def compress_tucker(a, cap: int, tol: float = 0.0, oversample: int = 10, seed: int = 0, stream=None):
    """Full field a (float64 CUDA tensor, 3 dims) -> ((core (c_1, c_2, c_3),
    [frames (N_j, c_j)]) as CUDA tensors with the nominal ranks, kept ranks)."""
    torch = _torch()
    L = lib()
    Ns = list(a.shape)
    Nc = (C.c_int * 3)(*Ns)
    nb = L.lrfg_compress_tucker_workspace_bytes(Nc, int(cap), int(oversample))
    if nb == 0:
        raise LrfgError(-1, "bad compression sizes")
    ws = _ws_tensor(nb, a.device)
    c = [min(cap, n) for n in Ns]
    frames = [torch.empty((Ns[j], c[j]), dtype=torch.float64, device=a.device) for j in range(3)]
    core = torch.empty(tuple(c), dtype=torch.float64, device=a.device)
    fptr = (C.c_void_p * 3)(*[F.data_ptr() for F in frames])
    ranks = (C.c_int * 3)()
    kept = (C.c_int * 3)()
    a = a.contiguous()
    check(L.lrfg_compress_tucker(Nc, C.c_void_p(a.data_ptr()), int(cap), float(tol), int(oversample), int(seed),
                                 fptr, C.c_void_p(core.data_ptr()), ranks, kept, C.c_void_p(ws.data_ptr()),
                                 ws.numel(), C.c_void_p(_stream_handle(stream))))
    return (core, frames), [int(kept[j]) for j in range(3)]


def tt_round(cores, cap: int, tol: float = 0.0, oversample: int = 10, seed: int = 0, stream=None):
    """Truncate nE trains given as float64 CUDA tensors cores[j] of shape
    (nE, r_{j-1}, N_j, r_j).  Returns (out cores, kept ranks (2, nE))."""
    torch = _torch()
    L = lib()
    d = len(cores)
    nE = cores[0].shape[0]
    Ns = [int(G.shape[2]) for G in cores] + [1] * (3 - d)
    rin = [1] + [int(G.shape[3]) for G in cores[:-1]] + [1] + [1] * (3 - d)
    Nc = (C.c_int * 3)(*Ns)
    Rc = (C.c_int * 4)(*rin[:4])
    nb = L.lrfg_tt_round_workspace_bytes(d, Nc, Rc, cap, oversample, nE)
    if nb == 0:
        raise LrfgError(-1, "bad tt_round sizes")
    ws = _ws_tensor(nb, cores[0].device)
    c = [1] * 4
    if d == 3:
        c[1] = min(cap, Ns[0], Ns[1] * Ns[2])
        c[2] = min(cap, Ns[2], Ns[0] * Ns[1])
    else:
        c[1] = min(cap, Ns[0], Ns[1])
    outs = [torch.empty((nE, c[j], Ns[j], c[j + 1]), dtype=torch.float64, device=cores[0].device)
            for j in range(d)]
    ins = [G.contiguous() for G in cores]
    ip = (C.c_void_p * 3)(*[G.data_ptr() for G in ins] + [0] * (3 - d))
    op = (C.c_void_p * 3)(*[G.data_ptr() for G in outs] + [0] * (3 - d))
    ranks = (C.c_int * 4)()
    kept = (C.c_int * (2 * nE))()
    check(L.lrfg_tt_round(d, Nc, Rc, ip, cap, float(tol), oversample, seed, op, ranks, kept, nE,
                          C.c_void_p(ws.data_ptr()), nb, C.c_void_p(_stream_handle(stream))))
    return outs, np.array(list(kept)).reshape(2, nE)
