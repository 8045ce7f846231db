"""Plain binary64 CPU oracle for the dense Krylov solvers (ctypes over ks_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg may use this package; the product library and
its Python binding never import it.

Functions and the passages of the paper they follow:

* ``cg``      conjugate gradient, Krylov section (prose description; the
              Hestenes-Stiefel form of Golub and Van Loan)
* ``gmres``   restarted GMRES(m): Arnoldi step as printed in the GMRES
              pseudo-code, least squares by Givens rotations (Saad), restart
              from the current iterate
* ``bicgstab`` BiCGSTAB as listed in the paper (omega as a quotient; the
              residual and rho updates the listing omits restored)
* ``arnoldi`` the Arnoldi basis and unrotated Hessenberg matrix alone
* ``lu_factor`` / ``lu_solve``  right-looking LU with partial pivoting and the
              two triangular solves (direct methods section)
* ``metrics`` relative residual and normwise backward error

Parity status of each function is recorded in the test suite's pins.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ks_oracle.c")
_LIB = os.path.join(_HERE, "libks_oracle.so")
_lock = threading.Lock()
_lib = None

STATUS = {0: "ok", 1: "maxiter", 2: "breakdown", 3: "stagnated", 4: "nonfinite", -1: "einval"}


def build(force: bool = False) -> str:
    """Compile ks_oracle.c with gcc into libks_oracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_LIB)
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        P = ctypes.POINTER
        pd, pi = P(d), P(i)
        lib.ko_cg.argtypes = [i, pd, l, pd, pd, d, i, pi, pi, pd, pd, i]
        lib.ko_cg.restype = i
        lib.ko_gmres.argtypes = [i, pd, l, pd, pd, d, i, i, pi, pi, pd, pd, i, pd, i]
        lib.ko_gmres.restype = i
        lib.ko_bicgstab.argtypes = [i, pd, l, pd, pd, d, i, pi, pi, pd]
        lib.ko_bicgstab.restype = i
        pf = ctypes.POINTER(ctypes.c_float)
        lib.ko_lu32_block.argtypes = [i, pd, l, pf, l, pi, i]
        lib.ko_lu32_block.restype = i
        lib.ko_lu32_apply.argtypes = [i, pf, l, pi, pd, pd]
        lib.ko_lu32_apply.restype = None
        lib.ko_gmres_ir_lu.argtypes = [i, pd, l, pd, pd, d, i, d, i, i, i, pi, pi, pd]
        lib.ko_gmres_ir_lu.restype = i
        lib.ko_chol32_block.argtypes = [i, pd, l, pf, l, i]
        lib.ko_chol32_block.restype = i
        lib.ko_chol32_apply.argtypes = [i, pf, l, pd, pd]
        lib.ko_chol32_apply.restype = None
        lib.ko_cg_ir_chol.argtypes = [i, pd, l, pd, pd, d, d, i, i, i, pi, pi, pd]
        lib.ko_cg_ir_chol.restype = i
        for name in ("ko_jacobi", "ko_gauss_seidel"):
            getattr(lib, name).argtypes = [i, pd, l, pd, pd, d, i, pi, pd]
            getattr(lib, name).restype = i
        lib.ko_arnoldi.argtypes = [i, pd, l, pd, i, pd, pd]
        lib.ko_arnoldi.restype = i
        lib.ko_lu_factor.argtypes = [i, pd, l, pi]
        lib.ko_lu_factor.restype = i
        lib.ko_lu_solve.argtypes = [i, pd, l, pi, pd, pd]
        lib.ko_lu_solve.restype = i
        lib.ko_metrics.argtypes = [i, pd, l, pd, pd, pd]
        lib.ko_metrics.restype = i
        lib.ko_matvec.argtypes = [i, pd, l, pd, pd]
        lib.ko_matvec.restype = None
        lib.ko_matvec_rows.argtypes = [i, pd, l, pi, i, pd, pd]
        lib.ko_matvec_rows.restype = None
        lib.ko_residual.argtypes = [i, pd, l, pd, pd, pd]
        lib.ko_residual.restype = None
        lib.ko_norm_inf_mat.argtypes = [i, pd, l]
        lib.ko_norm_inf_mat.restype = d
        lib.ko_dot.argtypes = [i, pd, pd]
        lib.ko_dot.restype = d
        lib.ko_set_threads.argtypes = [i]
        lib.ko_set_threads.restype = None
        lib.ko_get_threads.argtypes = []
        lib.ko_get_threads.restype = i
        _lib = lib
        return lib


def _pd(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _mat(A) -> tuple[np.ndarray, int]:
    A = np.asarray(A, dtype=np.float64)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    if not A.flags.c_contiguous:
        A = np.ascontiguousarray(A)
    return A, A.shape[1]


def _vec(v, n) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
    if v.size != n:
        raise ValueError("vector length mismatch")
    return v


def set_threads(t: int) -> None:
    _load().ko_set_threads(int(t))


def get_threads() -> int:
    return int(_load().ko_get_threads())


def matvec(A, x) -> np.ndarray:
    A, lda = _mat(A)
    n = A.shape[0]
    x = _vec(x, n)
    y = np.empty(n)
    _load().ko_matvec(n, _pd(A), lda, _pd(x), _pd(y))
    return y


def matvec_rows(A, rows, x) -> np.ndarray:
    """Rows `rows` of A x (plain left-to-right sums), for sampled checks."""
    A, lda = _mat(A)
    n = A.shape[0]
    x = _vec(x, n)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.intc))
    if rows.size and (rows.min() < 0 or rows.max() >= n):
        raise ValueError("row index out of range")
    y = np.empty(rows.size)
    _load().ko_matvec_rows(n, _pd(A), lda, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           int(rows.size), _pd(x), _pd(y))
    return y


def residual(A, b, x) -> np.ndarray:
    A, lda = _mat(A)
    n = A.shape[0]
    b, x = _vec(b, n), _vec(x, n)
    r = np.empty(n)
    _load().ko_residual(n, _pd(A), lda, _pd(b), _pd(x), _pd(r))
    return r


def norm_inf(A) -> float:
    A, lda = _mat(A)
    return float(_load().ko_norm_inf_mat(A.shape[0], _pd(A), lda))


def metrics(A, b, x) -> dict:
    """rel_res = ||b-Ax||_2/||b||_2, eta_inf = ||b-Ax||_inf/(||A||_inf||x||_inf+||b||_inf)."""
    A, lda = _mat(A)
    n = A.shape[0]
    b, x = _vec(b, n), _vec(x, n)
    out = np.zeros(3)
    rc = _load().ko_metrics(n, _pd(A), lda, _pd(b), _pd(x), _pd(out))
    if rc != 0:
        raise ValueError("ko_metrics: bad arguments")
    return dict(rel_res=float(out[0]), eta_inf=float(out[1]), res_norm=float(out[2]))


def cg(A, b, x0=None, tol=1e-10, max_iter=None, hist=False):
    """Conjugate gradient; returns (x, info). info: status, iters, restarts, rel_res[, hist]."""
    A, lda = _mat(A)
    n = A.shape[0]
    b = _vec(b, n)
    x = np.zeros(n) if x0 is None else _vec(x0, n).copy()
    max_iter = 2 * n if max_iter is None else int(max_iter)
    it, rs, rr = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    h = np.zeros(max(max_iter, 1)) if hist else None
    st = _load().ko_cg(n, _pd(A), lda, _pd(b), _pd(x), float(tol), max_iter, ctypes.byref(it),
                       ctypes.byref(rs), ctypes.byref(rr), _pd(h) if hist else None,
                       max_iter if hist else 0)
    info = dict(status=int(st), status_name=STATUS.get(int(st), "?"), iters=it.value,
                restarts=rs.value, rel_res=rr.value)
    if hist:
        info["hist"] = h[: it.value].copy()
    return x, info


def gmres(A, b, x0=None, tol=1e-10, max_iter=None, restart=30, hist=False):
    """Restarted GMRES(m); returns (x, info). info: status, iters, cycles, rel_res[, est, cres]."""
    A, lda = _mat(A)
    n = A.shape[0]
    b = _vec(b, n)
    x = np.zeros(n) if x0 is None else _vec(x0, n).copy()
    max_iter = 10 * n if max_iter is None else int(max_iter)
    it, cy, rr = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    est = np.zeros(max(max_iter, 1)) if hist else None
    ccap = max_iter + 2
    cres = np.zeros(ccap) if hist else None
    st = _load().ko_gmres(n, _pd(A), lda, _pd(b), _pd(x), float(tol), max_iter, int(restart),
                          ctypes.byref(it), ctypes.byref(cy), ctypes.byref(rr),
                          _pd(est) if hist else None, max_iter if hist else 0,
                          _pd(cres) if hist else None, ccap if hist else 0)
    info = dict(status=int(st), status_name=STATUS.get(int(st), "?"), iters=it.value,
                cycles=cy.value, rel_res=rr.value)
    if hist:
        info["est"] = est[: it.value].copy()
        info["cres"] = cres[: cy.value + 1].copy()
    return x, info


def bicgstab(A, b, x0=None, tol=1e-10, max_iter=None):
    """BiCGSTAB; returns (x, info). iters counts products with A (two per iteration)."""
    A, lda = _mat(A)
    n = A.shape[0]
    b = _vec(b, n)
    x = np.zeros(n) if x0 is None else _vec(x0, n).copy()
    max_iter = 20 * n if max_iter is None else int(max_iter)
    it, rs, rr = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    st = _load().ko_bicgstab(n, _pd(A), lda, _pd(b), _pd(x), float(tol), max_iter,
                             ctypes.byref(it), ctypes.byref(rs), ctypes.byref(rr))
    return x, dict(status=int(st), status_name=STATUS.get(int(st), "?"), iters=it.value,
                   restarts=rs.value, rel_res=rr.value)


def _stationary(fn, A, b, x0, tol, max_iter):
    A, lda = _mat(A)
    n = A.shape[0]
    b = _vec(b, n)
    x = np.zeros(n) if x0 is None else _vec(x0, n).copy()
    max_iter = 20 * n if max_iter is None else int(max_iter)
    it, rr = ctypes.c_int(0), ctypes.c_double(0.0)
    st = fn(n, _pd(A), lda, _pd(b), _pd(x), float(tol), max_iter, ctypes.byref(it),
            ctypes.byref(rr))
    return x, dict(status=int(st), status_name=STATUS.get(int(st), "?"), iters=it.value,
                   rel_res=rr.value)


def jacobi(A, b, x0=None, tol=1e-10, max_iter=None):
    """Jacobi iteration D x(k+1) = b - (L + U) x(k); returns (x, info)."""
    return _stationary(_load().ko_jacobi, A, b, x0, tol, max_iter)


def gauss_seidel(A, b, x0=None, tol=1e-10, max_iter=None):
    """Gauss-Seidel forward sweeps (D + L) x(k+1) = b - U x(k); returns (x, info)."""
    return _stationary(_load().ko_gauss_seidel, A, b, x0, tol, max_iter)


def _pf(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _pi(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def lu32_block(A, b=16):
    """The block LU in binary32 on fl32(A). Returns (LU float32 n x n, piv, singular)."""
    A, lda = _mat(A)
    n = A.shape[0]
    LU = np.zeros((n, n), dtype=np.float32)
    piv = np.zeros(n, dtype=np.int32)
    sing = _load().ko_lu32_block(n, _pd(A), lda, _pf(LU), n, _pi(piv), int(b))
    if sing < 0:
        raise ValueError("ko_lu32_block: bad arguments")
    return LU, piv, int(sing)


def lu32_apply(LU, piv, v):
    """U^-1 L^-1 P v in binary64 with the binary32 factors."""
    LU = np.ascontiguousarray(LU, dtype=np.float32)
    n = LU.shape[0]
    piv = np.ascontiguousarray(piv, dtype=np.int32)
    v = _vec(v, n)
    z = np.zeros(n)
    _load().ko_lu32_apply(n, _pf(LU), n, _pi(piv), _pd(v), _pd(z))
    return z


def gmres_ir_lu(A, b, x0=None, tol=1e-12, restart=30, inner_tol=1e-4, max_inner=None,
                max_outer=30, nb=16):
    """GMRES-IR: binary64 refinement, GMRES(restart) on the system left-
    preconditioned by the binary32 block LU of A. Returns (x, info)."""
    A, lda = _mat(A)
    n = A.shape[0]
    b = _vec(b, n)
    x = np.zeros(n) if x0 is None else _vec(x0, n).copy()
    max_inner = 10 * n if max_inner is None else int(max_inner)
    o, it, eta = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    st = _load().ko_gmres_ir_lu(n, _pd(A), lda, _pd(b), _pd(x), float(tol), int(restart),
                                float(inner_tol), max_inner, int(max_outer), int(nb),
                                ctypes.byref(o), ctypes.byref(it), ctypes.byref(eta))
    return x, dict(status=int(st), status_name=STATUS.get(int(st), "?"), outer_iters=o.value,
                   inner_iters=it.value, eta_inf=eta.value)


def chol32_block(A, nb=64):
    """Binary32 block Cholesky of the binary32 rounding of symmetric A (lower
    triangle read; block width nb).  Returns (L float32 lower, not_pd) where
    not_pd = 0, or 1 + the first column whose pivot is not positive."""
    A, lda = _mat(A)
    n = A.shape[0]
    L = np.zeros((n, n), dtype=np.float32)
    s = _load().ko_chol32_block(n, _pd(A), lda, _pf(L), n, int(nb))
    if s < 0:
        raise ValueError("ko_chol32_block: bad arguments")
    return L, int(s)


def chol32_apply(L, v):
    """z = L^-T L^-1 v in binary64 with the binary32 factor widened."""
    L = np.ascontiguousarray(L, dtype=np.float32)
    n = L.shape[0]
    v = _vec(v, n)
    z = np.zeros(n)
    _load().ko_chol32_apply(n, _pf(L), n, _pd(v), _pd(z))
    return z


def cg_ir_chol(A, b, x0=None, tol=1e-12, inner_tol=1e-4, max_inner=None, max_outer=30, nb=64):
    """CG-IR: binary64 refinement, CG in binary64 preconditioned with the
    binary32 block Cholesky of A. Returns (x, info)."""
    A, lda = _mat(A)
    n = A.shape[0]
    b = _vec(b, n)
    x = np.zeros(n) if x0 is None else _vec(x0, n).copy()
    max_inner = 10 * n if max_inner is None else int(max_inner)
    o, it, eta = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    st = _load().ko_cg_ir_chol(n, _pd(A), lda, _pd(b), _pd(x), float(tol), float(inner_tol),
                               max_inner, int(max_outer), int(nb), ctypes.byref(o), ctypes.byref(it),
                               ctypes.byref(eta))
    return x, dict(status=int(st), status_name=STATUS.get(int(st), "?"), outer_iters=o.value,
                   inner_iters=it.value, eta_inf=eta.value)


def arnoldi(A, v0, k):
    """k Arnoldi steps (MGS twice). Returns (V n x (k'+1), H (k'+1) x k', k')."""
    A, lda = _mat(A)
    n = A.shape[0]
    v0 = _vec(v0, n)
    V = np.zeros((k + 1, n))
    H = np.zeros((k + 1, k))
    done = _load().ko_arnoldi(n, _pd(A), lda, _pd(v0), int(k), _pd(V), _pd(H))
    if done < 0:
        raise ValueError("ko_arnoldi: bad arguments")
    return V[: done + 1].T.copy(), H[: done + 1, :done].copy(), done


def lu_factor(A):
    """GEPP as listed in the paper. Returns (LU, piv, singular_index)."""
    A, lda = _mat(A)
    LU = A.copy()
    n = A.shape[0]
    piv = np.zeros(n, dtype=np.intc)
    s = _load().ko_lu_factor(n, _pd(LU), lda, piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return LU, piv, int(s)


def lu_solve(LU, piv, b):
    LU, lda = _mat(LU)
    n = LU.shape[0]
    b = _vec(b, n)
    x = np.zeros(n)
    piv = np.ascontiguousarray(piv, dtype=np.intc)
    _load().ko_lu_solve(n, _pd(LU), lda, piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                        _pd(b), _pd(x))
    return x


def gepp_solve(A, b):
    LU, piv, s = lu_factor(A)
    if s:
        raise np.linalg.LinAlgError(f"singular pivot at step {s}")
    return lu_solve(LU, piv, b)
