"""Mixed-precision refinement over the condition-number sweep of the
refinement workload (binary64 outer residual and update, inner solve on a
binary32 or bfloat16 copy of A, stop at the normwise backward error
eta_inf = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf) <= 1e-12):

  * SPD A = Q diag(lambda) Q^T, CG inner solve;
  * nonsymmetric A = diag(lambda) + 0.25 G / sqrt(n), GMRES(50) inner solve;

with lambda log-uniform on [1, kappa], kappa in {1e2, 1e4, 1e6}.

At n = 1024 every cell is checked against the oracle: eta_inf of the returned
x computed by the oracle's own residual, and the forward error against the
binary64 oracle run to its attainable accuracy.  Two cells cannot converge
and are asserted as such: bfloat16 copies of the SPD matrices are indefinite
from kappa = 1e4 on (the solve must promote to binary32 or binary64 and still
converge), and restarted GMRES(50) stalls on the nonsymmetric kappa = 1e6
matrix (the oracle's binary64 GMRES(50) stops near eta_inf = 5e-8 after
20000 products), so the refinement must end with MAXITER or STAGNATED and a
backward error it reports truthfully; GMRES-IR with the binary32 LU
preconditioner is the method that solves that cell.

At n = 32768 the cells the benchmark does not already cover are checked by
their properties on a host copy of A (the oracle's residual and backward error
of the returned x; the forward error against x_true within cond(A) times the
backward-error bound).
"""
import numpy as np
import pytest

import oracle
from workloads import nonsym_swept_problem, spd_problem

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
ETA = 1e-12


def _t(a, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check_reported_eta(info, m, n):
    assert abs(info["backward_err"] - m["eta_inf"]) <= 1e-3 * m["eta_inf"] + np.sqrt(n) * U


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_spd_cg_refinement_cells(device, kappa, prec):
    from paper_1511_07207_amd import krylov

    n = 1024
    print(f"C3 cell SPD CG-IR kappa={kappa:g} {prec} n={n}", flush=True)
    p = spd_problem(n, kappa, seed=5, config_id=2)
    A, b = _t(p.A, device), _t(p.b, device)
    # the general inner product, and (binary32) the lower-triangle one the
    # benchmark times
    variants = [False, True] if prec == "fp32" else [False]
    xo, io = oracle.cg(p.A, p.b, tol=1e-14, max_iter=40 * n)
    for sym in variants:
        x, info = krylov.solve(A, b, method="cg", precision=prec, tol=ETA, max_iter=20 * n,
                               symmetric=sym)
        print(f"  symmetric={sym}: status {info['status_name']} outer {info['outer_iters']} "
              f"inner {info['iters']} precision_used {info['precision_used']} "
              f"eta {info['backward_err']:.2e}", flush=True)
        assert info["status"] == 0, info
        xh = x.cpu().numpy()
        m = oracle.metrics(p.A, p.b, xh)
        assert m["eta_inf"] <= ETA
        _check_reported_eta(info, m, n)
        assert _rel(xh, xo) <= max(1e-8, 100 * kappa * 1e-14)
        if prec == "bf16" and kappa >= 1e4:
            # the bfloat16 copy is indefinite: the solve promoted
            assert info["precision_used"] in ("fp32", "fp64"), info
        if prec == "bf16" and kappa == 1e2:
            assert info["precision_used"] == "bf16", info


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("kappa", [1e2, 1e4])
def test_nonsym_gmres50_refinement_cells(device, kappa, prec):
    from paper_1511_07207_amd import krylov

    n = 1024
    print(f"C3 cell nonsym GMRES(50)-IR kappa={kappa:g} {prec} n={n}", flush=True)
    p = nonsym_swept_problem(n, kappa, seed=5, config_id=2)
    x, info = krylov.solve(_t(p.A, device), _t(p.b, device), method="gmres", restart=50,
                           precision=prec, tol=ETA, max_iter=20 * n)
    print(f"  status {info['status_name']} outer {info['outer_iters']} inner {info['iters']} "
          f"precision_used {info['precision_used']} eta {info['backward_err']:.2e}", flush=True)
    assert info["status"] == 0, info
    # the diagonal dominates: the bfloat16 copy stays a good preconditioner
    assert info["precision_used"] == prec, info
    xh = x.cpu().numpy()
    m = oracle.metrics(p.A, p.b, xh)
    assert m["eta_inf"] <= ETA
    _check_reported_eta(info, m, n)
    xo, io = oracle.gmres(p.A, p.b, tol=1e-14, restart=50, max_iter=40 * n)
    assert io["status"] == 0
    assert _rel(xh, xo) <= max(1e-8, 100 * kappa * 1e-14)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_nonsym_gmres50_refinement_stalls_at_kappa_1e6(device, prec):
    from paper_1511_07207_amd import krylov

    n, kappa = 1024, 1e6
    print(f"C3 cell nonsym GMRES(50)-IR kappa=1e6 {prec} n={n} (stalls)", flush=True)
    p = nonsym_swept_problem(n, kappa, seed=5, config_id=2)
    A, b = _t(p.A, device), _t(p.b, device)
    x, info = krylov.solve(A, b, method="gmres", restart=50, precision=prec, tol=ETA,
                           max_iter=1000, max_outer=12)
    print(f"  status {info['status_name']} outer {info['outer_iters']} inner {info['iters']} "
          f"precision_used {info['precision_used']} eta {info['backward_err']:.2e}", flush=True)
    assert info["status_name"] in ("maxiter", "stagnated"), info
    xh = x.cpu().numpy()
    assert np.all(np.isfinite(xh))
    m = oracle.metrics(p.A, p.b, xh)
    assert m["eta_inf"] > ETA
    _check_reported_eta(info, m, n)
    # progress was made, as binary64 GMRES(50) makes it (it never diverges)
    assert m["eta_inf"] < oracle.metrics(p.A, p.b, np.zeros(n))["eta_inf"]
    # the method that solves this cell: GMRES-IR with the binary32 LU
    x2, i2 = krylov.solve(A, b, method="gmres", restart=30, precision="lu32", tol=ETA)
    assert i2["status"] == 0, i2
    assert oracle.metrics(p.A, p.b, x2.cpu().numpy())["eta_inf"] <= ETA


# ----------------------------------------------------------- n = 32768

def _full_size_check(A_host, bh, xt, xh, info, n, kappa):
    m = oracle.metrics(A_host, bh, xh)
    print(f"  eta (oracle) {m['eta_inf']:.3e} rel_res {m['rel_res']:.3e}", flush=True)
    assert m["eta_inf"] <= ETA * (1 + 1e-6)
    _check_reported_eta(info, m, n)
    # forward error: ||x - x_true|| / ||x_true|| <= cond(A) * (backward-error
    # bound in the 2-norm: eta_inf times the n-dependent norm factors)
    assert np.linalg.norm(xh - xt) <= 4 * kappa * np.sqrt(n) * ETA * np.linalg.norm(xt) + 1e-12


@pytest.mark.parametrize("kappa", [1e2, 1e6])
def test_spd_full_size_kappa_cells(device, kappa):
    import torch

    from paper_1511_07207_amd import krylov

    n = 32768
    print(f"C3 SPD n={n} kappa={kappa:g}: generating", flush=True)
    p = spd_problem(n, kappa, seed=0, config_id=2, backend="torch", device="cuda")
    runs = [("fp32", True)] + ([("bf16", False)] if kappa <= 1e2 else [])
    results = []
    for prec, sym in runs:
        x, info = krylov.solve(p.A, p.b, method="cg", precision=prec, tol=ETA, max_iter=4 * n,
                               symmetric=sym)
        print(f"  {prec} symmetric={sym}: status {info['status_name']} outer "
              f"{info['outer_iters']} inner {info['iters']} used {info['precision_used']}",
              flush=True)
        assert info["status"] == 0, info
        results.append((x.cpu().numpy(), info))
        del x
    A_host = p.A.cpu().numpy()
    bh, xt = p.b.cpu().numpy(), p.x_true.cpu().numpy()
    del p
    torch.cuda.empty_cache()
    for xh, info in results:
        _full_size_check(A_host, bh, xt, xh, info, n, kappa)
    if kappa <= 1e2:
        assert results[1][1]["precision_used"] == "bf16"


def test_nonsym_full_size_kappa_1e4(device):
    import torch

    from paper_1511_07207_amd import krylov

    n, kappa = 32768, 1e4
    print(f"C3 nonsymmetric n={n} kappa=1e4: generating", flush=True)
    p = nonsym_swept_problem(n, kappa, seed=0, config_id=2, backend="torch", device="cuda")
    results = []
    for prec in ("fp32", "bf16"):
        x, info = krylov.solve(p.A, p.b, method="gmres", restart=50, precision=prec, tol=ETA,
                               max_iter=4 * n)
        print(f"  {prec}: status {info['status_name']} outer {info['outer_iters']} inner "
              f"{info['iters']} used {info['precision_used']}", flush=True)
        assert info["status"] == 0, info
        assert info["precision_used"] == prec, info
        results.append((x.cpu().numpy(), info))
        del x
    A_host = p.A.cpu().numpy()
    bh, xt = p.b.cpu().numpy(), p.x_true.cpu().numpy()
    del p
    torch.cuda.empty_cache()
    for xh, info in results:
        _full_size_check(A_host, bh, xt, xh, info, n, kappa)
