"""ctypes binding of libks.so (the C ABI declared in include/ks.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libks.so")

KS_OK, KS_MAXITER, KS_BREAKDOWN, KS_STAGNATED, KS_NONFINITE = 0, 1, 2, 3, 4
KS_EINVAL, KS_ENOMEM, KS_EHIP, KS_EDEVICE, KS_ETOOLARGE = -1, -2, -3, -4, -5
KS_CG, KS_GMRES, KS_BICGSTAB, KS_JACOBI, KS_GAUSS_SEIDEL = 0, 1, 2, 3, 4
KS_FP64, KS_IR_FP32, KS_IR_BF16, KS_IR_LU32, KS_IR_CHOL32 = 0, 1, 2, 3, 4
KS_DT_F64, KS_DT_F32, KS_DT_BF16 = 0, 1, 2
KS_FLAG_TIMING = 1
KS_FLAG_STOP_BACKWARD = 2
KS_FLAG_SYMMETRIC = 4
KS_FLAG_NO_PERSIST = 8
KS_MAX_RESTART = 128
KS_MAX_NRHS = 64

STATUS_NAMES = {0: "ok", 1: "maxiter", 2: "breakdown", 3: "stagnated", 4: "nonfinite",
                -1: "einval", -2: "enomem", -3: "ehip", -4: "edevice", -5: "etoolarge"}

# every symbol declared in include/ks.h
EXPORTS = ("ks_params_init", "ks_workspace_bytes", "ks_workspace_bytes_borrowed", "ks_create",
           "ks_solve", "ks_column_info", "ks_arnoldi", "ks_free", "ks_strerror", "ks_gemv",
           "ks_gemm_mr_workspace_bytes", "ks_gemm_mr",
           "ks_symv_workspace_bytes", "ks_symv", "ks_symv_f32", "ks_symv_noalloc", "ks_lu32_factor", "ks_chol32_factor", "ks_convert", "ks_read_ceiling", "ks_server_create", "ks_server_submit",
           "ks_server_step", "ks_server_poll", "ks_server_stats", "ks_server_free")


class KsParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("lda", ctypes.c_int64),
        ("precision", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("restart", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("inner_tol", ctypes.c_double),
        ("poll_every", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("nrhs", ctypes.c_int32),
        ("timing_every", ctypes.c_int32),
    ]


class KsInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iters", ctypes.c_int32),
        ("outer_iters", ctypes.c_int32),
        ("restarts", ctypes.c_int32),
        ("rel_res", ctypes.c_double),
        ("backward_err", ctypes.c_double),
        ("elapsed_ms", ctypes.c_double),
        ("gemv_ms", ctypes.c_double),
        ("gemv_calls", ctypes.c_int32),
        ("precision_used", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, "?")
        return d


_lock = threading.Lock()
_lib = None


class KsError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({code})")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libks.so (once).  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1511_07207_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        PP = ctypes.POINTER(KsParams)
        L.ks_params_init.argtypes = [PP, i32, i32]
        L.ks_params_init.restype = ctypes.c_int
        L.ks_workspace_bytes.argtypes = [PP, ctypes.POINTER(sz)]
        L.ks_workspace_bytes.restype = ctypes.c_int
        L.ks_workspace_bytes_borrowed.argtypes = [PP, ctypes.POINTER(sz)]
        L.ks_workspace_bytes_borrowed.restype = ctypes.c_int
        L.ks_create.argtypes = [ctypes.POINTER(vp), PP, vp, vp, sz, vp]
        L.ks_create.restype = ctypes.c_int
        L.ks_solve.argtypes = [vp, vp, vp, ctypes.POINTER(KsInfo)]
        L.ks_solve.restype = ctypes.c_int
        L.ks_column_info.argtypes = [vp, i32, ctypes.POINTER(KsInfo)]
        L.ks_column_info.restype = ctypes.c_int
        L.ks_arnoldi.argtypes = [vp, vp, i32, vp, vp, ctypes.POINTER(i32)]
        L.ks_arnoldi.restype = ctypes.c_int
        L.ks_free.argtypes = [vp]
        L.ks_free.restype = None
        L.ks_strerror.argtypes = [ctypes.c_int]
        L.ks_strerror.restype = ctypes.c_char_p
        L.ks_gemv.argtypes = [i32, i64, i32, vp, vp, vp, vp]
        L.ks_gemv.restype = ctypes.c_int
        L.ks_gemm_mr_workspace_bytes.argtypes = [i32, i32, i32, ctypes.POINTER(sz)]
        L.ks_gemm_mr_workspace_bytes.restype = ctypes.c_int
        L.ks_gemm_mr.argtypes = [i32, i64, i32, vp, i32, vp, i64, vp, vp, sz, vp]
        L.ks_gemm_mr.restype = ctypes.c_int
        L.ks_symv_workspace_bytes.argtypes = [i32, ctypes.POINTER(sz)]
        L.ks_symv_workspace_bytes.restype = ctypes.c_int
        L.ks_symv.argtypes = [i32, i64, vp, vp, vp, vp, sz, vp]
        L.ks_symv.restype = ctypes.c_int
        L.ks_symv_f32.argtypes = [i32, i64, vp, vp, vp, vp, sz, vp]
        L.ks_symv_f32.restype = ctypes.c_int
        L.ks_symv_noalloc.argtypes = [i32, i64, vp, vp, vp, vp]
        L.ks_symv_noalloc.restype = ctypes.c_int
        L.ks_lu32_factor.argtypes = [i32, i64, vp, i64, vp, vp, ctypes.POINTER(i32), vp]
        L.ks_lu32_factor.restype = ctypes.c_int
        L.ks_chol32_factor.argtypes = [i32, i64, vp, i64, vp, ctypes.POINTER(i32), vp]
        L.ks_chol32_factor.restype = ctypes.c_int
        L.ks_convert.argtypes = [i32, i64, vp, i32, i64, vp, vp]
        L.ks_convert.restype = ctypes.c_int
        L.ks_read_ceiling.argtypes = [vp, sz, vp, vp]
        L.ks_read_ceiling.restype = ctypes.c_int
        L.ks_server_create.argtypes = [ctypes.POINTER(vp), sz, i32, i32, vp]
        L.ks_server_create.restype = ctypes.c_int
        L.ks_server_submit.argtypes = [vp, PP, vp, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
        L.ks_server_submit.restype = ctypes.c_int
        L.ks_server_step.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.ks_server_step.restype = ctypes.c_int
        L.ks_server_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(KsInfo),
                                     i32, ctypes.POINTER(i32)]
        L.ks_server_poll.restype = ctypes.c_int
        L.ks_server_stats.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.ks_server_stats.restype = ctypes.c_int
        L.ks_server_free.argtypes = [vp]
        L.ks_server_free.restype = None
        _lib = L
        return L


def check(rc: int, where: str) -> int:
    if rc < 0:
        raise KsError(rc, where)
    return rc
