"""Python front end of the dense Krylov library.

Tensors are torch tensors on the GPU (torch supplies device memory and the
current stream); all arithmetic happens in libks.so's HIP kernels.

    x, info = solve(A, b)                       # CG, binary64, tol 1e-10
    x, info = solve(A, b, method="gmres", restart=30)
    x, info = solve(A, b, precision="fp32", tol=1e-12)   # FP32 inner + FP64 IR
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as N

_METHODS = {"cg": N.KS_CG, "gmres": N.KS_GMRES, "bicgstab": N.KS_BICGSTAB,
            "jacobi": N.KS_JACOBI, "gauss_seidel": N.KS_GAUSS_SEIDEL}
_PRECISIONS = {"fp64": N.KS_FP64, "fp32": N.KS_IR_FP32, "bf16": N.KS_IR_BF16,
               "lu32": N.KS_IR_LU32, "chol32": N.KS_IR_CHOL32}
_PREC_NAMES = {v: k for k, v in _PRECISIONS.items()}


def _stream_handle() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _check_matrix(A: torch.Tensor) -> int:
    if not (isinstance(A, torch.Tensor) and A.is_cuda and A.dtype == torch.float64):
        raise TypeError("A must be a float64 CUDA tensor")
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    if A.stride(1) != 1 or A.stride(0) < A.shape[1]:
        raise ValueError("A must be row-major with unit column stride")
    return int(A.stride(0))


def make_params(n: int, method: str = "cg", lda: int | None = None, tol: float = 1e-10,
                max_iter: int | None = None, restart: int = 30, precision: str = "fp64",
                inner_tol: float = 1e-4, max_outer: int = 30, poll_every: int = 0,
                timing: bool = False, nrhs: int = 1, stop_backward: bool = False,
                symmetric: bool = False, timing_every: int = 0, persist: bool = True) -> N.KsParams:
    p = N.KsParams()
    N.check(N.lib().ks_params_init(ctypes.byref(p), int(n), _METHODS[method]), "ks_params_init")
    p.lda = int(lda if lda is not None else n)
    p.tol = float(tol)
    if max_iter is not None:
        p.max_iter = int(max_iter)
    p.restart = int(restart)
    p.precision = _PRECISIONS[precision]
    p.inner_tol = float(inner_tol)
    p.max_outer = int(max_outer)
    p.poll_every = int(poll_every)
    p.flags = ((N.KS_FLAG_TIMING if timing else 0) | (N.KS_FLAG_STOP_BACKWARD if stop_backward else 0)
               | (N.KS_FLAG_SYMMETRIC if symmetric else 0) | (0 if persist else N.KS_FLAG_NO_PERSIST))
    p.nrhs = int(nrhs)
    p.timing_every = int(timing_every)
    return p


class Solver:
    """A solver bound to one matrix A (create once, solve many right-hand sides).

    The workspace is a torch uint8 tensor owned by this object; A must stay
    alive and unmodified while the solver exists (it is read in place when
    aligned).
    """

    def __init__(self, A: torch.Tensor, method: str = "cg", **kw):
        lda = _check_matrix(A)
        n = A.shape[0]
        self.A = A
        self.n = n
        self.params = make_params(n, method=method, lda=lda, **kw)
        L = N.lib()
        need = ctypes.c_size_t(0)
        aligned = A.data_ptr() % 16 == 0 and (lda * 8) % 16 == 0
        fn = L.ks_workspace_bytes_borrowed if aligned else L.ks_workspace_bytes
        N.check(fn(ctypes.byref(self.params), ctypes.byref(need)), "ks_workspace_bytes")
        nbytes = int(need.value) + 256
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = ctypes.c_void_p(base + off)
        self._ws_bytes = nbytes - off
        h = ctypes.c_void_p()
        N.check(L.ks_create(ctypes.byref(h), ctypes.byref(self.params), _ptr(A), self._ws_ptr,
                            self._ws_bytes, _stream_handle()), "ks_create")
        self._h = h

    def solve(self, b: torch.Tensor, x0: torch.Tensor | None = None, out: torch.Tensor | None = None):
        """Solve A x = b; returns (x, info dict).  x is a new tensor unless `out` is given.

        With nrhs = s > 1, b is n x s (one right-hand side per column); the
        result is n x s and info["columns"] lists each column's outcome.
        """
        if self.params.nrhs > 1:
            return self._solve_multi(b, x0)
        if not (b.is_cuda and b.dtype == torch.float64 and b.numel() == self.n and b.is_contiguous()):
            raise ValueError("b must be a contiguous float64 CUDA vector of length n")
        if out is None:
            out = torch.zeros(self.n, dtype=torch.float64, device=b.device)
            if x0 is not None:
                out.copy_(x0.reshape(-1))
        elif x0 is not None:
            out.copy_(x0.reshape(-1))
        info = N.KsInfo()
        rc = N.lib().ks_solve(self._h, _ptr(b), _ptr(out), ctypes.byref(info))
        N.check(rc, "ks_solve")
        d = info.as_dict()
        d["precision_used"] = _PREC_NAMES.get(d["precision_used"], d["precision_used"])
        return out, d

    def _solve_multi(self, B: torch.Tensor, X0: torch.Tensor | None = None):
        s = self.params.nrhs
        if not (B.is_cuda and B.dtype == torch.float64 and tuple(B.shape) == (self.n, s)):
            raise ValueError(f"B must be a float64 CUDA tensor of shape ({self.n}, {s})")
        Bc = B.t().contiguous()          # column-major n x s: right-hand side j contiguous
        Xc = torch.zeros((s, self.n), dtype=torch.float64, device=B.device)
        if X0 is not None:
            Xc.copy_(X0.t())
        info = N.KsInfo()
        N.check(N.lib().ks_solve(self._h, _ptr(Bc), _ptr(Xc), ctypes.byref(info)), "ks_solve")
        d = info.as_dict()
        d["precision_used"] = _PREC_NAMES.get(d["precision_used"], d["precision_used"])
        cols = []
        for j in range(s):
            ci = N.KsInfo()
            N.check(N.lib().ks_column_info(self._h, j, ctypes.byref(ci)), "ks_column_info")
            cols.append(ci.as_dict())
        d["columns"] = cols
        return Xc.t(), d

    def arnoldi(self, v0: torch.Tensor, k: int):
        """k Arnoldi steps from v0: returns (V n x (k'+1), H (k'+1) x k', k')."""
        V = torch.zeros((k + 1, self.n), dtype=torch.float64, device=v0.device)
        H = torch.zeros((k + 1, k), dtype=torch.float64, device=v0.device)
        kd = ctypes.c_int32(0)
        N.check(N.lib().ks_arnoldi(self._h, _ptr(v0.contiguous()), int(k), _ptr(V), _ptr(H),
                                   ctypes.byref(kd)), "ks_arnoldi")
        kd = kd.value
        return V[: kd + 1].T, H[: kd + 1, :kd], kd

    def close(self):
        if getattr(self, "_h", None):
            N.lib().ks_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server (binary64 CG / GMRES(m)).

    submit() queues a solve and returns a ticket; step() runs one scheduling
    tick; poll() returns the finished (ticket, x, info) triples.  The tensors
    of a request are kept referenced here until it is returned.
    """

    def __init__(self, mem_budget_bytes: int = 64 << 30, max_inflight: int = 1024,
                 chunk: int = 16):
        h = ctypes.c_void_p()
        N.check(N.lib().ks_server_create(ctypes.byref(h), int(mem_budget_bytes), int(max_inflight),
                                         int(chunk), _stream_handle()), "ks_server_create")
        self._h = h
        self._live = {}

    def submit(self, A: torch.Tensor, b: torch.Tensor, x0: torch.Tensor | None = None,
               method: str = "cg", **kw) -> int:
        lda = _check_matrix(A)
        n = A.shape[0]
        p = make_params(n, method=method, lda=lda, **kw)
        x = torch.zeros(n, dtype=torch.float64, device=A.device)
        if x0 is not None:
            x.copy_(x0.reshape(-1))
        t = ctypes.c_uint64(0)
        N.check(N.lib().ks_server_submit(self._h, ctypes.byref(p), _ptr(A), _ptr(b), _ptr(x),
                                         ctypes.byref(t)), "ks_server_submit")
        self._live[t.value] = (A, b, x)
        return t.value

    def step(self):
        a, q = ctypes.c_int32(0), ctypes.c_int32(0)
        N.check(N.lib().ks_server_step(self._h, ctypes.byref(a), ctypes.byref(q)), "ks_server_step")
        return a.value, q.value

    def poll(self, cap: int = 4096):
        tickets = (ctypes.c_uint64 * cap)()
        infos = (N.KsInfo * cap)()
        k = ctypes.c_int32(0)
        N.check(N.lib().ks_server_poll(self._h, tickets, infos, cap, ctypes.byref(k)), "ks_server_poll")
        out = []
        for i in range(k.value):
            t = tickets[i]
            _, _, x = self._live.pop(t)
            d = infos[i].as_dict()
            d["precision_used"] = _PREC_NAMES.get(d["precision_used"], d["precision_used"])
            out.append((t, x, d))
        return out

    def stats(self):
        b, a, q = ctypes.c_size_t(0), ctypes.c_int32(0), ctypes.c_int32(0)
        N.check(N.lib().ks_server_stats(self._h, ctypes.byref(b), ctypes.byref(a), ctypes.byref(q)),
                "ks_server_stats")
        return dict(bytes_in_use=b.value, inflight=a.value, queued=q.value)

    def close(self):
        if getattr(self, "_h", None):
            N.lib().ks_server_free(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(A: torch.Tensor, b: torch.Tensor, x0: torch.Tensor | None = None, method: str = "cg",
          **kw):
    """One-shot solve of A x = b (see Solver for the keyword arguments)."""
    s = Solver(A, method=method, **kw)
    try:
        return s.solve(b, x0=x0)
    finally:
        s.close()


def gemv(A: torch.Tensor, v: torch.Tensor, y: torch.Tensor | None = None,
         lda: int | None = None, n: int | None = None) -> torch.Tensor:
    """y = A v with the solvers' GEMV kernel.  A: float64 / float32 / bfloat16 row-major."""
    dt = {torch.float64: N.KS_DT_F64, torch.float32: N.KS_DT_F32,
          torch.bfloat16: N.KS_DT_BF16}[A.dtype]
    n = A.shape[0] if n is None else n
    lda = A.stride(0) if lda is None else lda
    vdt = torch.float64 if A.dtype == torch.float64 else torch.float32
    if y is None:
        y = torch.empty(n, dtype=vdt, device=A.device)
    N.check(N.lib().ks_gemv(int(n), int(lda), dt, _ptr(A), _ptr(v), _ptr(y), _stream_handle()),
            "ks_gemv")
    return y


def gemm_mr(A: torch.Tensor, P: torch.Tensor, Q: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Q = A P on the matrix cores (the lockstep CG's product).  A: float64 or
    float32 n x n row-major; P: n x s of A's dtype, s <= 64, stored column by
    column (P.t() contiguous, as Q is returned)."""
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("gemm_mr: A must be float64 or float32")
    if P.dtype != A.dtype or P.dim() != 2:
        raise TypeError("gemm_mr: P must be an n x s matrix of A's dtype")
    n, s = P.shape
    Pc = P.t().contiguous()  # s x n: column j of P contiguous
    dt = N.KS_DT_F64 if A.dtype == torch.float64 else N.KS_DT_F32
    sz = ctypes.c_size_t(0)
    N.check(N.lib().ks_gemm_mr_workspace_bytes(int(n), int(s), dt, ctypes.byref(sz)),
            "ks_gemm_mr_workspace_bytes")
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(sz.value, dtype=torch.uint8, device=A.device)
    Qc = torch.empty((s, n), dtype=A.dtype, device=A.device)
    N.check(N.lib().ks_gemm_mr(int(n), int(A.stride(0)), dt, _ptr(A), int(s), _ptr(Pc), int(n),
                               _ptr(Qc), _ptr(workspace), sz.value, _stream_handle()), "ks_gemm_mr")
    if Q is None:
        return Qc.t()
    Q.copy_(Qc.t())
    return Q


def symv(A: torch.Tensor, x: torch.Tensor, y: torch.Tensor | None = None,
         n: int | None = None, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """y = A x for symmetric A (float64, or float32 with float32 x, y and
    accumulation), reading only its lower triangle."""
    if A.dtype not in (torch.float64, torch.float32):
        raise TypeError("symv: A must be float64 or float32")
    n = A.shape[0] if n is None else n
    sz = ctypes.c_size_t(0)
    N.check(N.lib().ks_symv_workspace_bytes(int(n), ctypes.byref(sz)), "ks_symv_workspace_bytes")
    if workspace is None or workspace.numel() < sz.value:
        workspace = torch.empty(sz.value, dtype=torch.uint8, device=A.device)
    if y is None:
        y = torch.empty(n, dtype=A.dtype, device=A.device)
    fn = N.lib().ks_symv if A.dtype == torch.float64 else N.lib().ks_symv_f32
    N.check(fn(int(n), int(A.stride(0)), _ptr(A), _ptr(x), _ptr(y), _ptr(workspace), sz.value,
               _stream_handle()), "ks_symv")
    return y


def symv_noalloc(A: torch.Tensor, x: torch.Tensor, y: torch.Tensor | None = None,
                 n: int | None = None) -> torch.Tensor:
    """y = A x for symmetric float64 A from its lower triangle, with the tile
    partials in the library's fixed device array instead of a workspace
    (n <= KS_SYMV_NOALLOC_MAX_N; calls on one GPU must not overlap)."""
    if A.dtype != torch.float64:
        raise TypeError("symv_noalloc: A must be float64")
    n = A.shape[0] if n is None else n
    if y is None:
        y = torch.empty(n, dtype=A.dtype, device=A.device)
    N.check(N.lib().ks_symv_noalloc(int(n), int(A.stride(0)), _ptr(A), _ptr(x), _ptr(y),
                                    _stream_handle()), "ks_symv_noalloc")
    return y


def lu32_factor(A: torch.Tensor) -> tuple[torch.Tensor, torch.Tensor, int]:
    """Binary32 block LU with partial pivoting of a float64 matrix.
    Returns (LU float32 n x n, piv int32, info)."""
    if A.dtype != torch.float64:
        raise TypeError("lu32_factor: A must be float64")
    n = A.shape[0]
    LU = torch.empty((n, n), dtype=torch.float32, device=A.device)
    piv = torch.empty(n, dtype=torch.int32, device=A.device)
    info = ctypes.c_int32(0)
    N.check(N.lib().ks_lu32_factor(int(n), int(A.stride(0)), _ptr(A), int(n), _ptr(LU), _ptr(piv),
                                   ctypes.byref(info), _stream_handle()), "ks_lu32_factor")
    return LU, piv, int(info.value)


def chol32_factor(A: torch.Tensor) -> tuple[torch.Tensor, int]:
    """Binary32 block Cholesky of a symmetric float64 matrix.
    Returns (F float32 n x ldl with L on and below the diagonal and L^T above
    it, info); ldl = n rounded up to a multiple of 4."""
    if A.dtype != torch.float64:
        raise TypeError("chol32_factor: A must be float64")
    n = A.shape[0]
    ldl = (n + 3) // 4 * 4
    F = torch.empty((n, ldl), dtype=torch.float32, device=A.device)
    info = ctypes.c_int32(0)
    N.check(N.lib().ks_chol32_factor(int(n), int(A.stride(0)), _ptr(A), int(ldl), _ptr(F),
                                     ctypes.byref(info), _stream_handle()), "ks_chol32_factor")
    return F, int(info.value)


def convert(A: torch.Tensor, dtype: torch.dtype, lda_dst: int | None = None) -> torch.Tensor:
    """Low-precision copy of a float64 matrix with the library's rounding rule."""
    n = A.shape[0]
    lda_dst = n if lda_dst is None else lda_dst
    dt = {torch.float32: N.KS_DT_F32, torch.bfloat16: N.KS_DT_BF16, torch.float64: N.KS_DT_F64}[dtype]
    out = torch.empty((n, lda_dst), dtype=dtype, device=A.device)
    N.check(N.lib().ks_convert(int(n), int(A.stride(0)), _ptr(A), dt, int(lda_dst), _ptr(out),
                               _stream_handle()), "ks_convert")
    return out


def read_ceiling(buf: torch.Tensor, sink: torch.Tensor) -> None:
    """Stream-read every byte of buf (the memory read ceiling kernel)."""
    N.check(N.lib().ks_read_ceiling(_ptr(buf), buf.numel() * buf.element_size(), _ptr(sink),
                                    _stream_handle()), "ks_read_ceiling")
