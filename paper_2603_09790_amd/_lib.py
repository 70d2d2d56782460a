"""ctypes loader and signatures of libsspcg.so (declared in include/sspcg.h)."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsspcg.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_HIP, ERR_BREAKDOWN, ERR_WORKSPACE, ERR_NONFINITE, ERR_UNSUPPORTED = -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
GRAM_FGS, GRAM_CHOLESKY = 0, 1
F64, F32 = 0, 1
BASIS = {"chebyshev": 0, "monomial": 1}
MATRIX_FP32 = 1
MATRIX_FULL_STORAGE = 2
MAX_S = 16
POLL_BYTES = 256      # SSPCG_POLL_BYTES
STATIC_SCRATCH_BYTES = 64 * 1024 * 1024   # SSPCG_STATIC_SCRATCH_BYTES
HIST_STRIDE = 4       # doubles per outer iteration in the s-step history

# Every symbol the header declares, in header order.
EXPORTS = [
    "sspcg_abi_version", "sspcg_status_string", "sspcg_last_error", "sspcg_default_params",
    "sspcg_matrix_scratch_bytes", "sspcg_matrix_aux_bytes",
    "sspcg_matrix_create", "sspcg_matrix_update_values", "sspcg_matrix_destroy",
    "sspcg_matrix_info", "sspcg_workspace_bytes", "sspcg_solve", "sspcg_solve_static",
    "sspcg_pcg_solve", "sspcg_interval_work_bytes", "sspcg_interval",
    "sspcg_kernel_work_bytes", "sspcg_spmv", "sspcg_mpk", "sspcg_block_update_gram",
    "sspcg_gram_rect", "sspcg_fgs", "sspcg_xr_update", "sspcg_csr_value_grad",
    "sspcg_diffusion7_assemble", "sspcg_diffusion7_theta_grad", "sspcg_stream_triad",
]


class Params(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("max_refine", ctypes.c_int32), ("gram", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("sweep_tol", ctypes.c_double), ("basis", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("inner_iters_total", ctypes.c_int32),
                ("relres", ctypes.c_double), ("relres_true", ctypes.c_double),
                ("device_ms", ctypes.c_double)]


PHASES = ["spmv", "gram_update", "gram_rect", "fgs", "norm", "xr"]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 6), ("ms", ctypes.c_double * 6),
                ("outer_iters", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {ph: dict(launches=self.launches[i], ms=self.ms[i]) for i, ph in enumerate(PHASES)} \
            | {"outer_iters": self.outer_iters}


class SSPCGError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: status {status} ({detail})")


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library.  Raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2603_09790_amd/build.py` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "sspcg_abi_version": (ctypes.c_int, []),
        "sspcg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "sspcg_last_error": (ctypes.c_char_p, []),
        "sspcg_default_params": (None, [ctypes.POINTER(Params)]),
        "sspcg_matrix_scratch_bytes": (SZ, [I32]),
        "sspcg_matrix_aux_bytes": (ctypes.c_int, [I32, I32, P, P, P, I32, P, SZ, P,
                                                  ctypes.POINTER(SZ)]),
        "sspcg_matrix_create": (ctypes.c_int, [I32, I32, P, P, P, I32, P, SZ, P,
                                               ctypes.POINTER(P)]),
        "sspcg_matrix_update_values": (ctypes.c_int, [P, P, P]),
        "sspcg_matrix_destroy": (ctypes.c_int, [P]),
        "sspcg_matrix_info": (ctypes.c_int, [P] + [ctypes.POINTER(I64)] * 7),
        "sspcg_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(Params), ctypes.POINTER(SZ)]),
        "sspcg_solve": (ctypes.c_int, [P, P, P, ctypes.POINTER(Params), P, SZ, P, P,
                                       ctypes.POINTER(Result), P, ctypes.POINTER(Profile)]),
        "sspcg_solve_static": (ctypes.c_int, [P, P, P, ctypes.POINTER(Params), P, P,
                                              ctypes.POINTER(Result)]),
        "sspcg_pcg_solve": (ctypes.c_int, [P, P, P, ctypes.POINTER(Params), P, SZ, P, P,
                                           ctypes.POINTER(Result), P]),
        "sspcg_interval_work_bytes": (ctypes.c_int, [P, I32, ctypes.POINTER(SZ)]),
        "sspcg_interval": (ctypes.c_int, [P, I32, I32, D, P, P, SZ, P, ctypes.POINTER(D),
                                          ctypes.POINTER(D), ctypes.POINTER(I32)]),
        "sspcg_kernel_work_bytes": (SZ, [I32]),
        "sspcg_spmv": (ctypes.c_int, [P, I32, P, P, P]),
        "sspcg_mpk": (ctypes.c_int, [P, I32, P, I32, D, D, I32, P, P, I64, P]),
        "sspcg_block_update_gram": (ctypes.c_int, [I64, I32, I32, P, P, P, P, P, P, I64, P, P,
                                                   P, SZ, P]),
        "sspcg_gram_rect": (ctypes.c_int, [I64, I32, I32, P, P, I64, P, P, SZ, P]),
        "sspcg_fgs": (ctypes.c_int, [I32, I32, P, P, I32, D, I32, P, P, P]),
        "sspcg_xr_update": (ctypes.c_int, [P, I32, I32, P, P, P, I64, P, P, P, P, P, SZ, P]),
        "sspcg_csr_value_grad": (ctypes.c_int, [P, P, P, P, P]),
        "sspcg_diffusion7_assemble": (ctypes.c_int, [P, P, P, P]),
        "sspcg_diffusion7_theta_grad": (ctypes.c_int, [P, P, P, P, P]),
        "sspcg_stream_triad": (ctypes.c_int, [I64, P, P, D, P, P]),
    }
    assert list(sig) == EXPORTS
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().sspcg_last_error().decode()


def status_string(st: int) -> str:
    return lib().sspcg_status_string(st).decode()


def check(st: int, where: str, allow=(OK,)) -> int:
    if st not in allow:
        raise SSPCGError(st, where, f"{status_string(st)}: {last_error()}")
    return st
