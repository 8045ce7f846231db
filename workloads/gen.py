"""Seeded generators for the dense test systems.

The paper gives only the sizes of its systems (2000-20000 unknowns for the
iterative methods, Results section) and never describes the matrices, so the
systems here are synthetic:

* SPD:  A = Q diag(lam) Q^T with Q the orthogonal factor of the QR
  factorisation of an n x n N(0,1) matrix, lam_i = kappa**u_i with
  u_i ~ U[0,1) and the two end points pinned (u = 0 and u = 1) so that
  cond_2(A) = kappa up to rounding; A is then symmetrised once,
  A <- (A + A^T)/2, so that it is exactly symmetric in binary64.
* nonsymmetric: A = diag(D) + G/sqrt(n), D ~ U[2,4], G ~ N(0,1).
* nonsymmetric with a swept condition number:
  A = diag(lam) + 0.25 G/sqrt(n), lam log-uniform on [1, kappa] with pinned
  end points.
* x_true ~ N(0,1), b = A x_true, x0 = 0.

Two back ends draw the same recipe:

* ``backend="numpy"``: PCG64 streams keyed by
  ``SeedSequence([seed, config_id, *key, role])`` (role 0 = G, 1 = lam/D,
  2 = x_true), QR and products by numpy/LAPACK on the host.  Used for every
  system the CPU oracle solves.
* ``backend="torch"``: the same keys hashed to a 64-bit seed for torch's
  device generator, QR and products by torch on the GPU.  The O(n^3) QR is
  minutes-to-hours on the host at n = 16384/32768, so the full-size systems
  are built on the device; their bit streams differ from the numpy ones but
  the distribution is the same.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Any, Sequence

import numpy as np

ROLE_G, ROLE_LAM, ROLE_X = 0, 1, 2


@dataclasses.dataclass
class Problem:
    """A dense system A x = b with its known solution.

    ``A`` is row-major n x n binary64, ``b`` and ``x_true`` have n rows (and
    nrhs columns for the multi-right-hand-side case).  For ``backend="numpy"``
    they are numpy arrays, for ``backend="torch"`` torch tensors on the device.
    """

    A: Any
    b: Any
    x_true: Any
    kind: str
    n: int
    kappa: float | None
    meta: dict


def seed_words(seed: int, config_id: int, key: Sequence[int], role: int) -> list[int]:
    return [int(seed), int(config_id), *[int(k) for k in key], int(role)]


def _np_rng(seed, config_id, key, role) -> np.random.Generator:
    ss = np.random.SeedSequence(seed_words(seed, config_id, key, role))
    return np.random.Generator(np.random.PCG64(ss))


def _torch_seed(seed, config_id, key, role) -> int:
    ss = np.random.SeedSequence(seed_words(seed, config_id, key, role))
    return int(ss.generate_state(1, np.uint64)[0] & np.uint64(0x7FFFFFFFFFFFFFFF))


def _pinned_exponents(u: np.ndarray) -> np.ndarray:
    u = np.array(u, dtype=np.float64)
    if u.size >= 1:
        u[0] = 0.0
    if u.size >= 2:
        u[-1] = 1.0
    return u


def _log_uniform(rng: np.random.Generator, n: int, kappa: float) -> np.ndarray:
    u = _pinned_exponents(rng.random(n))
    return np.power(float(kappa), u)


def _rhs_numpy(A, n, nrhs, seed, config_id, key):
    rng = _np_rng(seed, config_id, key, ROLE_X)
    if nrhs == 1:
        x = rng.standard_normal(n)
    else:
        x = rng.standard_normal((n, nrhs))
    b = A @ x
    return x, b


def _torch():
    import torch

    return torch


def _device_rng(device, seed, config_id, key, role):
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(_torch_seed(seed, config_id, key, role))
    return g


def _rhs_torch(A, n, nrhs, seed, config_id, key, device):
    torch = _torch()
    g = _device_rng(device, seed, config_id, key, ROLE_X)
    shape = (n,) if nrhs == 1 else (n, nrhs)
    x = torch.randn(shape, dtype=torch.float64, device=device, generator=g)
    b = A @ x
    return x, b


def _lam_torch(n, kappa, seed, config_id, key, device):
    torch = _torch()
    g = _device_rng(device, seed, config_id, key, ROLE_LAM)
    u = torch.rand(n, dtype=torch.float64, device=device, generator=g)
    if n >= 1:
        u[0] = 0.0
    if n >= 2:
        u[-1] = 1.0
    return torch.pow(torch.tensor(float(kappa), dtype=torch.float64, device=device), u)


def spd_problem(n: int, kappa: float, seed: int = 0, config_id: int = 0,
                key: Sequence[int] = (), nrhs: int = 1, backend: str = "numpy",
                device: str = "cuda", q_form: str = "qr") -> Problem:
    """SPD system with cond_2(A) = kappa (recipe in the module docstring).

    q_form="identity" takes Q = I, i.e. A = diag(lambda) stored densely: the
    same spectrum and the same bytes per matrix-vector product, for hardware
    counter runs in which the QR library call cannot run under the profiler.
    """
    if q_form == "identity":
        if backend == "numpy":
            lam = _log_uniform(_np_rng(seed, config_id, key, ROLE_LAM), n, kappa)
            A = np.diag(lam)
            x, b = _rhs_numpy(A, n, nrhs, seed, config_id, key)
        else:
            torch = _torch()
            lam = _lam_torch(n, kappa, seed, config_id, key, device)
            A = torch.diag(lam).contiguous()
            x, b = _rhs_torch(A, n, nrhs, seed, config_id, key, device)
        return Problem(A, b, x, "spd", n, float(kappa),
                       dict(seed=seed, config_id=config_id, key=list(key), backend=backend,
                            q_form=q_form))
    if backend == "numpy":
        lam = _log_uniform(_np_rng(seed, config_id, key, ROLE_LAM), n, kappa)
        G = _np_rng(seed, config_id, key, ROLE_G).standard_normal((n, n))
        Q, _ = np.linalg.qr(G)
        del G
        A = (Q * lam) @ Q.T
        del Q
        A = 0.5 * (A + A.T)
        A = np.ascontiguousarray(A)
        x, b = _rhs_numpy(A, n, nrhs, seed, config_id, key)
    elif backend == "torch":
        torch = _torch()
        lam = _lam_torch(n, kappa, seed, config_id, key, device)
        g = _device_rng(device, seed, config_id, key, ROLE_G)
        G = torch.randn((n, n), dtype=torch.float64, device=device, generator=g)
        Q, _ = torch.linalg.qr(G)
        del G
        A = (Q * lam) @ Q.T
        del Q
        A = 0.5 * (A + A.T)
        A = A.contiguous()
        x, b = _rhs_torch(A, n, nrhs, seed, config_id, key, device)
    else:
        raise ValueError(f"unknown backend {backend!r}")
    return Problem(A, b, x, "spd", n, float(kappa),
                   dict(seed=seed, config_id=config_id, key=list(key), backend=backend))


def nonsym_problem(n: int, seed: int = 0, config_id: int = 0, key: Sequence[int] = (),
                   nrhs: int = 1, backend: str = "numpy", device: str = "cuda") -> Problem:
    """A = diag(D) + G/sqrt(n) with D ~ U[2,4] and G ~ N(0,1)."""
    if backend == "numpy":
        D = 2.0 + 2.0 * _np_rng(seed, config_id, key, ROLE_LAM).random(n)
        A = _np_rng(seed, config_id, key, ROLE_G).standard_normal((n, n))
        A *= 1.0 / math.sqrt(n)
        A[np.arange(n), np.arange(n)] += D
        x, b = _rhs_numpy(A, n, nrhs, seed, config_id, key)
    elif backend == "torch":
        torch = _torch()
        gD = _device_rng(device, seed, config_id, key, ROLE_LAM)
        D = 2.0 + 2.0 * torch.rand(n, dtype=torch.float64, device=device, generator=gD)
        g = _device_rng(device, seed, config_id, key, ROLE_G)
        A = torch.randn((n, n), dtype=torch.float64, device=device, generator=g)
        A *= 1.0 / math.sqrt(n)
        A.diagonal().add_(D)
        x, b = _rhs_torch(A, n, nrhs, seed, config_id, key, device)
    else:
        raise ValueError(f"unknown backend {backend!r}")
    return Problem(A, b, x, "nonsym", n, None,
                   dict(seed=seed, config_id=config_id, key=list(key), backend=backend))


def nonsym_swept_problem(n: int, kappa: float, seed: int = 0, config_id: int = 0,
                         key: Sequence[int] = (), backend: str = "numpy",
                         device: str = "cuda") -> Problem:
    """A = diag(lam) + 0.25 G/sqrt(n), lam log-uniform on [1, kappa]."""
    if backend == "numpy":
        lam = _log_uniform(_np_rng(seed, config_id, key, ROLE_LAM), n, kappa)
        A = _np_rng(seed, config_id, key, ROLE_G).standard_normal((n, n))
        A *= 0.25 / math.sqrt(n)
        A[np.arange(n), np.arange(n)] += lam
        x, b = _rhs_numpy(A, n, 1, seed, config_id, key)
    elif backend == "torch":
        torch = _torch()
        lam = _lam_torch(n, kappa, seed, config_id, key, device)
        g = _device_rng(device, seed, config_id, key, ROLE_G)
        A = torch.randn((n, n), dtype=torch.float64, device=device, generator=g)
        A *= 0.25 / math.sqrt(n)
        A.diagonal().add_(lam)
        x, b = _rhs_torch(A, n, 1, seed, config_id, key, device)
    else:
        raise ValueError(f"unknown backend {backend!r}")
    return Problem(A, b, x, "nonsym_swept", n, float(kappa),
                   dict(seed=seed, config_id=config_id, key=list(key), backend=backend))


def multi_rhs_problem(n: int, kappa: float, nrhs: int, seed: int = 0, config_id: int = 3,
                      backend: str = "numpy", device: str = "cuda") -> Problem:
    """One SPD matrix with nrhs right-hand sides B = A X_true (X_true ~ N(0,1))."""
    return spd_problem(n, kappa, seed=seed, config_id=config_id, nrhs=nrhs,
                       backend=backend, device=device)


@dataclasses.dataclass
class Request:
    index: int
    arrival_s: float
    kind: str          # "cg" (SPD) or "gmres" (D + G/sqrt(n))
    n: int
    kappa: float | None
    key: tuple


def stream_requests(count: int, rate_per_s: float, seed: int = 0, n_lo: int = 256,
                    n_hi: int = 8192, kappa_lo: float = 1e2, kappa_hi: float = 1e5,
                    config_id: int = 4) -> list[Request]:
    """Request stream: Poisson arrivals, log-uniform n, 50/50 CG/GMRES mix.

    Request i's matrix is drawn from keys ``[seed, config_id, i, role]``.
    """
    rng = _np_rng(seed, config_id, (), 7)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(int)
    kinds = rng.random(count) < 0.5
    kap = np.exp(rng.uniform(math.log(kappa_lo), math.log(kappa_hi), size=count))
    out = []
    for i in range(count):
        if kinds[i]:
            out.append(Request(i, float(arrivals[i]), "cg", int(ns[i]), float(kap[i]), (i,)))
        else:
            out.append(Request(i, float(arrivals[i]), "gmres", int(ns[i]), None, (i,)))
    return out


def request_problem(req: Request, seed: int = 0, config_id: int = 4, backend="numpy",
                    device="cuda") -> Problem:
    if req.kind == "cg":
        return spd_problem(req.n, req.kappa, seed=seed, config_id=config_id, key=req.key,
                           backend=backend, device=device)
    return nonsym_problem(req.n, seed=seed, config_id=config_id, key=req.key,
                          backend=backend, device=device)
