"""BiCGSTAB on the GPU against the CPU oracle, through the C ABI.

Bars as for the other methods: true relative residual <= tol and the
solution within 1e-8 (relative) of the oracle's at condition numbers up to
1e4.  The number of products with A must lie within 1% (at least 2) of the
oracle's plus the oracle's own rounding spread: the largest change of the
oracle's count when every entry of A moves by one unit in the last place
(three seeded perturbations).  BiCGSTAB's residual is not monotone, so once
the iteration runs long enough for rounding to matter the step at which it
first meets the tolerance moves by several percent under such a change (the
SPD case below moves by about 7%); on the well-conditioned cases the spread
is 0 and the bar is the plain 1%.
"""
import numpy as np
import pytest

import oracle
from workloads import nonsym_problem, nonsym_swept_problem, spd_problem

pytestmark = pytest.mark.gpu


def _t(x, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(device)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _rounding_spread(A, b, count, tol, max_iter):
    spread = 0
    for k in range(3):
        sgn = np.random.default_rng(1000 + k).choice([-1.0, 1.0], size=A.shape)
        Ap = A + sgn * np.spacing(A)
        _, io = oracle.bicgstab(Ap, b, tol=tol, max_iter=max_iter)
        spread = max(spread, abs(io["iters"] - count))
    return spread


def _iters_close(a, b, spread):
    return abs(a - b) <= max(2, int(0.01 * b)) + spread


CASES = [("nonsym", 512, 0), ("nonsym", 1000, 1), ("nonsym", 2049, 2), ("nonsym", 100, 3),
         ("spd", 777, 4), ("swept", 600, 5)]


def _problem(kind, n, seed):
    if kind == "nonsym":
        return nonsym_problem(n, seed=seed, config_id=5)
    if kind == "spd":
        return spd_problem(n, 1e3, seed=seed, config_id=5)
    return nonsym_swept_problem(n, 1e2, seed=seed, config_id=5)


@pytest.mark.parametrize("kind,n,seed", CASES)
def test_bicgstab_matches_oracle(device, kind, n, seed):
    from paper_1511_07207_amd import krylov

    print(f"bicgstab {kind} n={n} seed={seed}", flush=True)
    p = _problem(kind, n, seed)
    xo, io = oracle.bicgstab(p.A, p.b, tol=1e-10, max_iter=20 * n)
    assert io["status"] == 0, io
    x, info = krylov.solve(_t(p.A, device), _t(p.b, device), method="bicgstab", tol=1e-10,
                           max_iter=20 * n)
    x = x.cpu().numpy()
    assert info["status"] == 0, info
    m = oracle.metrics(p.A, p.b, x)
    assert m["rel_res"] <= 1e-10
    slack = np.sqrt(n) * 2.0 ** -53
    assert abs(info["rel_res"] - m["rel_res"]) <= 1e-3 * m["rel_res"] + slack
    assert abs(info["backward_err"] - m["eta_inf"]) <= 1e-3 * m["eta_inf"] + slack
    assert _rel(x, xo) <= 1e-8
    spread = _rounding_spread(p.A, p.b, io["iters"], 1e-10, 20 * n)
    assert _iters_close(info["iters"], io["iters"], spread), (info["iters"], io["iters"], spread)


def test_bicgstab_first_iterate_equals_oracle(device):
    # two products = one full iteration: the iterate is fixed by the recurrence
    # alone, so the two sides agree to rounding
    from paper_1511_07207_amd import krylov

    p = nonsym_problem(300, seed=7, config_id=5)
    xo, io = oracle.bicgstab(p.A, p.b, tol=1e-15, max_iter=2)
    x, info = krylov.solve(_t(p.A, device), _t(p.b, device), method="bicgstab", tol=1e-15,
                           max_iter=2)
    assert io["status"] == 1 and info["status"] == 1 and info["iters"] == 2
    assert _rel(x.cpu().numpy(), xo) <= 1e-13


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_bicgstab_mixed_precision(device, precision):
    from paper_1511_07207_amd import krylov

    n = 1024
    p = nonsym_problem(n, seed=8, config_id=5)
    print(f"bicgstab IR {precision} n={n}", flush=True)
    x, info = krylov.solve(_t(p.A, device), _t(p.b, device), method="bicgstab",
                           precision=precision, tol=1e-12, max_iter=20 * n)
    assert info["status"] == 0, info
    m = oracle.metrics(p.A, p.b, x.cpu().numpy())
    assert m["eta_inf"] <= 1e-12 * (1 + 1e-6)
    assert info["outer_iters"] >= 1


def test_bicgstab_special_cases(device):
    import torch

    from paper_1511_07207_amd import krylov

    n = 300
    p = nonsym_problem(n, seed=9, config_id=5)
    A = _t(p.A, device)
    # b = 0 gives x = 0 at once
    x, info = krylov.solve(A, torch.zeros(n, dtype=torch.float64, device=device),
                           x0=torch.ones(n, dtype=torch.float64, device=device), method="bicgstab")
    assert info["status"] == 0 and info["iters"] == 0 and float(x.abs().max()) == 0.0
    # exact initial guess: no product in the loop
    x, info = krylov.solve(A, _t(p.b, device), x0=_t(p.x_true, device), method="bicgstab", tol=1e-10)
    assert info["status"] == 0 and info["iters"] == 0
    # identity: the half step after one product is exact
    b = np.random.default_rng(1).standard_normal(n)
    x, info = krylov.solve(_t(np.eye(n), device), _t(b, device), method="bicgstab", tol=1e-12)
    assert info["status"] == 0 and info["iters"] == 1
    assert np.array_equal(x.cpu().numpy(), b)
    # product budget
    x, info = krylov.solve(A, _t(p.b, device), method="bicgstab", tol=1e-14, max_iter=7)
    assert info["status"] == 1 and info["iters"] == 7
    _, io = oracle.bicgstab(p.A, p.b, tol=1e-14, max_iter=7)
    assert io["iters"] == 7
    # non-finite right-hand side
    bb = p.b.copy()
    bb[3] = np.nan
    _, info = krylov.solve(A, _t(bb, device), method="bicgstab")
    assert info["status"] == 4


def test_bicgstab_timing_counts_every_product(device):
    from paper_1511_07207_amd import krylov

    n = 2048
    p = nonsym_problem(n, seed=10, config_id=5)
    _, info = krylov.solve(_t(p.A, device), _t(p.b, device), method="bicgstab", tol=1e-10,
                           timing=True)
    assert info["status"] == 0
    assert info["gemv_calls"] == info["iters"]
    assert 0.0 < info["gemv_ms"] < info["elapsed_ms"]


def test_bicgstab_stop_on_backward_error(device):
    from paper_1511_07207_amd import krylov

    n = 1500
    p = nonsym_problem(n, seed=11, config_id=5)
    x, info = krylov.solve(_t(p.A, device), _t(p.b, device), method="bicgstab", tol=1e-13,
                           stop_backward=True)
    assert info["status"] == 0
    m = oracle.metrics(p.A, p.b, x.cpu().numpy())
    assert m["eta_inf"] <= 1e-13 * (1 + 1e-6)
    assert abs(info["backward_err"] - m["eta_inf"]) <= 1e-3 * m["eta_inf"] + np.sqrt(n) * 2.0 ** -53
