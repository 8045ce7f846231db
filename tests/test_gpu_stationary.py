"""Jacobi and Gauss-Seidel on the GPU against the CPU oracle, through the C ABI.

Both are contractions on the test matrices (diagonal plus a scaled Gaussian,
Jacobi spectral radius about 0.36), so rounding differences do not grow from
step to step: after a fixed number of updates the GPU iterate must equal the
oracle's element by element within 1e-11 * max|x| (each update adds about
n u |A||x| of rounding, n <= 2049, damped by 1 / (1 - rho)).  Solves to a
tolerance must stop after the same number of updates as the oracle, give or
take one (the residual can sit on the threshold within rounding), with a true
relative residual (oracle metrics) within the tolerance and the solution
within 1e-8 of the oracle's.

The sizes span the Gauss-Seidel substitution blocks (64 rows, two per
launch) and the product chunks (512 columns) with ragged tails: n = 1, 7, 64,
65, 128, 130, 191, 513, 1000, 2049.
"""
import numpy as np
import pytest

import oracle
from workloads import nonsym_problem, spd_problem

pytestmark = pytest.mark.gpu

METHODS = {"jacobi": oracle.jacobi, "gauss_seidel": oracle.gauss_seidel}


def _t(x, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(device)


def _solve(device, A, b, method, x0=None, **kw):
    from paper_1511_07207_amd import krylov

    x, info = krylov.solve(_t(A, device), _t(b, device),
                           None if x0 is None else _t(x0, device), method=method, **kw)
    return x.cpu().numpy(), info


@pytest.mark.parametrize("method", list(METHODS))
@pytest.mark.parametrize("n,steps,seed", [(1, 1, 0), (7, 3, 1), (64, 4, 2), (65, 4, 3),
                                          (128, 3, 8), (130, 5, 4), (191, 3, 9), (513, 6, 5),
                                          (1000, 3, 6), (2049, 5, 7)])
def test_iterates_match_oracle_step_by_step(device, method, n, steps, seed):
    print(f"{method} n={n} steps={steps} seed={seed}", flush=True)
    p = nonsym_problem(n, seed=seed, config_id=6)
    xo, io = METHODS[method](p.A, p.b, tol=1e-300, max_iter=steps)
    # the limit, except where a step solves the system exactly (n = 1)
    assert io["status_name"] == ("ok" if n == 1 else "maxiter") and io["iters"] == steps
    x, info = _solve(device, p.A, p.b, method, tol=1e-300, max_iter=steps)
    assert info["status_name"] == io["status_name"] and info["iters"] == steps, info
    err = np.abs(x - xo).max()
    assert err <= 1e-11 * np.abs(xo).max(), err / np.abs(xo).max()


@pytest.mark.parametrize("method", list(METHODS))
@pytest.mark.parametrize("n,seed", [(100, 10), (512, 11), (1000, 12), (2049, 13)])
def test_converged_solve_matches_oracle(device, method, n, seed):
    print(f"{method} n={n} seed={seed} tol 1e-10", flush=True)
    p = nonsym_problem(n, seed=seed, config_id=6)
    xo, io = METHODS[method](p.A, p.b, tol=1e-10, max_iter=500)
    assert io["status_name"] == "ok", io
    x, info = _solve(device, p.A, p.b, method, tol=1e-10, max_iter=500)
    assert info["status_name"] == "ok", info
    assert abs(info["iters"] - io["iters"]) <= 1, (info["iters"], io["iters"])
    m = oracle.metrics(p.A, p.b, x)
    assert m["rel_res"] <= 1e-10
    slack = np.sqrt(n) * 2.0 ** -53
    assert abs(info["rel_res"] - m["rel_res"]) <= 1e-3 * m["rel_res"] + slack
    assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)


@pytest.mark.parametrize("method", list(METHODS))
def test_warm_start_and_backward_error_stop(device, method):
    n = 300
    p = nonsym_problem(n, seed=20, config_id=6)
    x0 = np.random.default_rng(21).standard_normal(n)
    xo, io = METHODS[method](p.A, p.b, x0=x0, tol=1e-300, max_iter=4)
    x, info = _solve(device, p.A, p.b, method, x0=x0, tol=1e-300, max_iter=4)
    assert info["iters"] == 4
    assert np.abs(x - xo).max() <= 1e-11 * np.abs(xo).max()
    # stop on the normwise backward error instead of the relative residual
    x, info = _solve(device, p.A, p.b, method, tol=1e-13, max_iter=500, stop_backward=True)
    assert info["status_name"] == "ok", info
    assert oracle.metrics(p.A, p.b, x)["eta_inf"] <= 1e-13 * (1 + 1e-6)


@pytest.mark.parametrize("method", list(METHODS))
def test_special_cases(device, method):
    n = 70
    p = nonsym_problem(n, seed=30, config_id=6)
    # b = 0: x = 0 without an update
    x, info = _solve(device, p.A, np.zeros(n), method, x0=np.ones(n), tol=1e-10)
    assert info["status_name"] == "ok" and info["iters"] == 0 and not x.any()
    # exact start: integer system, x0 = x*
    rng = np.random.default_rng(31)
    A = rng.integers(-3, 4, size=(n, n)).astype(float)
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1) + 1
    xs = rng.integers(-5, 6, size=n).astype(float)
    x, info = _solve(device, A, A @ xs, method, x0=xs, tol=1e-12)
    assert info["status_name"] == "ok" and info["iters"] == 0
    # a zero on the diagonal: breakdown before any update, as the oracle
    Z = p.A.copy()
    Z[40, 40] = 0.0
    _, io = METHODS[method](Z, p.b, tol=1e-10)
    _, info = _solve(device, Z, p.b, method, tol=1e-10)
    assert io["status_name"] == info["status_name"] == "breakdown" and info["iters"] == 0
    # a non-finite right-hand side
    bn = p.b.copy()
    bn[3] = np.nan
    _, info = _solve(device, p.A, bn, method, tol=1e-10)
    assert info["status_name"] == "nonfinite"
    # diagonal A: exact after one update
    d = rng.uniform(1, 3, n)
    x, info = _solve(device, np.diag(d), p.b, method, tol=1e-14)
    assert info["status_name"] == "ok" and info["iters"] == 1
    np.testing.assert_array_equal(x, p.b / d) if method == "jacobi" else \
        np.testing.assert_allclose(x, p.b / d, rtol=2 ** -51)


def test_jacobi_divergence_and_gauss_seidel_on_spd(device):
    """Unit diagonal, off-diagonal 0.9 (SPD): Jacobi diverges (iteration
    matrix eigenvalue -0.9 (n - 1)), Gauss-Seidel converges, on both sides."""
    n = 20
    A = np.full((n, n), 0.9) + 0.1 * np.eye(n)
    b = np.random.default_rng(40).standard_normal(n)
    _, io = oracle.jacobi(A, b, tol=1e-10, max_iter=30)
    _, info = _solve(device, A, b, "jacobi", tol=1e-10, max_iter=30)
    assert io["status_name"] == info["status_name"] == "maxiter"
    assert info["iters"] == 30
    xo, io = oracle.gauss_seidel(A, b, tol=1e-10, max_iter=20000)
    x, info = _solve(device, A, b, "gauss_seidel", tol=1e-10, max_iter=20000)
    assert io["status_name"] == info["status_name"] == "ok"
    assert abs(info["iters"] - io["iters"]) <= max(1, io["iters"] // 100), (info["iters"], io["iters"])
    assert oracle.metrics(A, b, x)["rel_res"] <= 1e-10


def test_gauss_seidel_on_spd_workload(device):
    """An SPD matrix of the CG workload (kappa 1e2): Gauss-Seidel converges."""
    n = 300
    p = spd_problem(n, 1e2, seed=50, config_id=6)
    xo, io = oracle.gauss_seidel(p.A, p.b, tol=1e-8, max_iter=5000)
    x, info = _solve(device, p.A, p.b, "gauss_seidel", tol=1e-8, max_iter=5000)
    assert io["status_name"] == info["status_name"] == "ok", (io, info)
    assert abs(info["iters"] - io["iters"]) <= max(1, io["iters"] // 100), (info["iters"], io["iters"])
    assert oracle.metrics(p.A, p.b, x)["rel_res"] <= 1e-8
