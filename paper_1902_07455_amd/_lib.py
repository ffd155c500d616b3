"""ctypes binding of liblrfg.so (argument marshalling only).

The structures mirror include/lrfg.h field by field.  Loading fails loudly
when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrfg.so")

FORMAT_FULL, FORMAT_CP, FORMAT_TUCKER, FORMAT_TT = 0, 1, 2, 3
SOLVER_PCG, SOLVER_MR = 0, 1
PREC_FP64, PREC_MIXED_FP32, PREC_MIXED_BF16 = 0, 1, 2

OK, NOT_CONVERGED, EINVAL, ECOEFF, EWORKSPACE, EDEVICE, EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5
RANK_LIMITED = 2

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class Problem(C.Structure):
    _fields_ = [
        ("d", C.c_int),
        ("N", C.c_int * 3),
        ("format", C.c_int),
        ("rank_cap", C.c_int),
        ("trunc_tol", C.c_double),
        ("solver_tol", C.c_double),
        ("max_iter", C.c_int),
        ("solver", C.c_int),
        ("precision", C.c_int),
        ("precond_terms", C.c_int),
        ("oversample", C.c_int),
        ("seed", C.c_uint64),
        ("coeff_rank", C.c_int),
        ("flags", C.c_uint32),
        ("aniso", C.c_double * 9),
        ("rank_start", C.c_int),
        ("discretisation", C.c_int),
    ]


class Coeff(C.Structure):
    _fields_ = [
        ("on_device", C.c_int),
        ("full", C.c_void_p),
        ("rank", C.c_int),
        ("weights", C.c_void_p),
        ("factors", C.c_void_p * 3),
        ("tt_ranks", C.c_int * 4),
        ("tt_cores", C.c_void_p * 3),
        ("tucker_ranks", C.c_int * 3),
        ("tucker_core", C.c_void_p),
        ("tucker_frames", C.c_void_p * 3),
        ("inclusion", C.c_int),
        ("incl_size", C.c_double),
        ("incl_inside", C.c_double),
        ("incl_outside", C.c_double),
    ]


class Result(C.Structure):
    _fields_ = [
        ("A_H", C.c_void_p),
        ("iters", C.c_void_p),
        ("res_hist", C.c_void_p),
        ("ranks", C.c_void_p),
        ("status", C.c_void_p),
        ("setup_ms", C.c_double),
        ("solve_ms", C.c_double),
    ]


class Completion(C.Structure):
    _fields_ = [
        ("tag", C.c_uint64),
        ("status", C.c_int),
        ("batch_size", C.c_int),
        ("queue_ms", C.c_double),
        ("run_ms", C.c_double),
        ("total_ms", C.c_double),
        ("workspace_bytes", C.c_size_t),
    ]


class LrfgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lrfg status {status}: {msg}")
        self.status = status


_LIB = None

EXPORTS = [
    "lrfg_abi_version", "lrfg_status_string", "lrfg_last_error", "lrfg_device_check",
    "lrfg_plan_create", "lrfg_plan_workspace_bytes", "lrfg_solve", "lrfg_solve_batch", "lrfg_server_create", "lrfg_server_submit",
    "lrfg_server_poll", "lrfg_server_pending", "lrfg_server_destroy", "lrfg_plan_destroy",
    "lrfg_fft_workspace_bytes", "lrfg_fft_lines", "lrfg_mode_op",
    "lrfg_full_op_workspace_bytes", "lrfg_full_op", "lrfg_prof_enable", "lrfg_prof_read", "lrfg_prof_work",
    "lrfg_gemm_workspace_bytes", "lrfg_gemm", "lrfg_gemm_mixed", "lrfg_syevj", "lrfg_gram_cut", "lrfg_compress_workspace_bytes", "lrfg_tucker_round_workspace_bytes", "lrfg_tucker_round", "lrfg_compress_tt", "lrfg_compress_tucker_workspace_bytes", "lrfg_compress_tucker", "lrfg_tt_round_workspace_bytes",
    "lrfg_tt_round", "lrfg_solve_noalloc", "lrfg_ga_double_grid",
]


def lib():
    """The loaded library (raises if liblrfg.so is missing)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with "
                          "`python -m paper_1902_07455_amd.build`")
    # torch first: its HIP runtime is then the one liblrfg.so binds to, so
    # the process holds a single runtime (device memory and streams come
    # from torch)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    L.lrfg_abi_version.restype = C.c_int
    L.lrfg_ga_double_grid.argtypes = [C.c_int]
    L.lrfg_ga_double_grid.restype = C.c_int
    L.lrfg_status_string.restype = C.c_char_p
    L.lrfg_status_string.argtypes = [C.c_int]
    L.lrfg_last_error.restype = C.c_char_p
    L.lrfg_device_check.restype = C.c_int
    L.lrfg_plan_create.argtypes = [C.POINTER(Problem), C.POINTER(C.c_void_p)]
    L.lrfg_plan_create.restype = C.c_int
    L.lrfg_plan_workspace_bytes.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_size_t)]
    L.lrfg_plan_workspace_bytes.restype = C.c_int
    L.lrfg_solve.argtypes = [C.c_void_p, C.POINTER(Coeff), C.c_void_p, C.c_int, C.c_void_p,
                             C.c_size_t, C.c_void_p, C.POINTER(Result)]
    L.lrfg_solve.restype = C.c_int
    L.lrfg_solve_noalloc.argtypes = [C.c_void_p, C.POINTER(Coeff), C.c_void_p, C.c_int, C.c_void_p,
                                     C.POINTER(Result)]
    L.lrfg_solve_noalloc.restype = C.c_int
    L.lrfg_solve_batch.argtypes = [C.c_void_p, C.POINTER(Coeff), C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                   C.c_size_t, C.c_void_p, C.POINTER(Result)]
    L.lrfg_solve_batch.restype = C.c_int
    L.lrfg_server_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]
    L.lrfg_server_create.restype = C.c_int
    L.lrfg_server_submit.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(Coeff), C.c_void_p, C.c_int,
                                     C.POINTER(Result), C.c_uint64, C.c_void_p]
    L.lrfg_server_submit.restype = C.c_int
    L.lrfg_server_poll.argtypes = [C.c_void_p, C.POINTER(Completion), C.c_int, C.POINTER(C.c_int), C.c_int]
    L.lrfg_server_poll.restype = C.c_int
    L.lrfg_server_pending.argtypes = [C.c_void_p]
    L.lrfg_server_pending.restype = C.c_int
    L.lrfg_server_destroy.argtypes = [C.c_void_p]
    L.lrfg_server_destroy.restype = None
    L.lrfg_plan_destroy.argtypes = [C.c_void_p]
    L.lrfg_plan_destroy.restype = None
    L.lrfg_fft_workspace_bytes.argtypes = [C.c_int]
    L.lrfg_fft_workspace_bytes.restype = C.c_size_t
    L.lrfg_fft_lines.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                 C.c_size_t, C.c_void_p]
    L.lrfg_fft_lines.restype = C.c_int
    L.lrfg_mode_op.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                               C.c_void_p, C.c_size_t, C.c_void_p]
    L.lrfg_mode_op.restype = C.c_int
    L.lrfg_full_op_workspace_bytes.argtypes = [C.POINTER(C.c_int)]
    L.lrfg_full_op_workspace_bytes.restype = C.c_size_t
    L.lrfg_full_op.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_size_t, C.c_void_p]
    L.lrfg_full_op.restype = C.c_int
    L.lrfg_gemm_workspace_bytes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
    L.lrfg_gemm_workspace_bytes.restype = C.c_size_t
    L.lrfg_gemm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                            C.c_void_p, C.c_longlong, C.c_longlong, C.c_void_p, C.c_longlong,
                            C.c_longlong, C.c_double, C.c_void_p, C.c_longlong, C.c_longlong,
                            C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]
    L.lrfg_gemm.restype = C.c_int
    L.lrfg_gemm_mixed.argtypes = [C.c_int] + L.lrfg_gemm.argtypes
    L.lrfg_gemm_mixed.restype = C.c_int
    L.lrfg_syevj.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    L.lrfg_syevj.restype = C.c_int
    L.lrfg_gram_cut.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_void_p]
    L.lrfg_gram_cut.restype = C.c_int
    L.lrfg_tucker_round_workspace_bytes.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int, C.c_int,
                                                    C.c_int]
    L.lrfg_tucker_round_workspace_bytes.restype = C.c_size_t
    L.lrfg_tucker_round.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_void_p), C.c_void_p,
                                    C.c_int, C.c_double, C.c_int, C.c_uint64, C.POINTER(C.c_void_p), C.c_void_p,
                                    C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_int, C.c_void_p, C.c_size_t,
                                    C.c_void_p]
    L.lrfg_tucker_round.restype = C.c_int
    L.lrfg_compress_workspace_bytes.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_int, C.c_int]
    L.lrfg_compress_workspace_bytes.restype = C.c_size_t
    L.lrfg_compress_tt.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_void_p, C.c_int, C.c_double, C.c_int,
                                   C.c_uint64, C.POINTER(C.c_void_p), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.c_void_p, C.c_size_t, C.c_void_p]
    L.lrfg_compress_tt.restype = C.c_int
    L.lrfg_compress_tucker_workspace_bytes.argtypes = [C.POINTER(C.c_int), C.c_int, C.c_int]
    L.lrfg_compress_tucker_workspace_bytes.restype = C.c_size_t
    L.lrfg_compress_tucker.argtypes = [C.POINTER(C.c_int), C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_uint64,
                                       C.POINTER(C.c_void_p), C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.c_void_p, C.c_size_t, C.c_void_p]
    L.lrfg_compress_tucker.restype = C.c_int
    L.lrfg_tt_round_workspace_bytes.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                                C.c_int, C.c_int, C.c_int]
    L.lrfg_tt_round_workspace_bytes.restype = C.c_size_t
    L.lrfg_tt_round.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_void_p), C.c_int, C.c_double, C.c_int, C.c_uint64,
                                C.POINTER(C.c_void_p), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]
    L.lrfg_tt_round.restype = C.c_int
    L.lrfg_prof_enable.argtypes = [C.c_char_p]
    L.lrfg_prof_enable.restype = C.c_int
    L.lrfg_prof_read.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.lrfg_prof_read.restype = C.c_int
    L.lrfg_prof_work.argtypes = [C.POINTER(C.c_double)]
    L.lrfg_prof_work.restype = C.c_int
    _LIB = L
    return L


def check(status: int, allow=(OK,)) -> int:
    if status in allow:
        return status
    L = lib()
    msg = L.lrfg_last_error().decode() or L.lrfg_status_string(status).decode()
    raise LrfgError(status, msg)
