"""Binary32 block Cholesky on the GPU (trailing updates on the matrix cores)
and CG-IR preconditioned by it, against the oracle, through the C ABI.

Factor: the componentwise backward-error bound of the Cholesky factorization
in binary32, |A32 - L L^T| <= gamma_{n+1} |L| |L^T| (the matrix cores sum in
their own order, so the factor is not the oracle's bit for bit), within
rounding of the oracle's factor, L^T mirrored exactly into the upper
triangle, bit for bit on an exactly representable factor (every partial sum
exact, so any summation order gives L0), and the first non-positive pivot of
an indefinite matrix.  Sizes cross the 64-column blocks and the 64 x 64
update tiles with ragged tails, and (past 256) the 256-column outer blocks
whose rank-256 updates run in 128 x 128 tiles.

CG-IR: eta_inf <= 1e-12 checked by the oracle's residual, the forward error
against the binary64 oracle run to its attainable accuracy, outer steps
within one of the oracle's CG-IR, and statuses for b = 0 and an indefinite A.
"""
import numpy as np
import pytest

import oracle
from workloads import spd_problem

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
ETA = 1e-12


def _t(a, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    return G @ G.T / n + 0.5 * np.eye(n)


def _factor(A, device):
    from paper_1511_07207_amd import krylov

    F, info = krylov.chol32_factor(_t(A, device))
    n = A.shape[0]
    F = F.cpu().numpy()[:, :n]
    return F, info


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 127, 129, 200, 300, 513, 1500])
def test_chol32_factor_backward_error_and_oracle(device, n):
    print(f"chol32 factor n={n}", flush=True)
    A = _spd(n, 200 + n)
    F, info = _factor(A, device)
    assert info == 0
    L = np.tril(F).astype(np.float64)
    # the upper triangle holds L^T exactly
    np.testing.assert_array_equal(np.triu(F, 1), np.tril(F, -1).T)
    A32 = A.astype(np.float32).astype(np.float64)
    A32 = np.tril(A32) + np.tril(A32, -1).T
    gamma = (n + 1) * U32 / (1 - (n + 1) * U32)
    err = np.abs(A32 - L @ L.T)
    assert np.all(err <= gamma * (np.abs(L) @ np.abs(L).T) + 1e-300)
    assert np.all(np.diag(L) > 0)
    Lo, s = oracle.chol32_block(A, nb=64)
    assert s == 0
    Lo = Lo.astype(np.float64)
    # two binary32 factorizations of the same matrix: within the perturbation
    # bound of the factor (cond(A) n u32, as the oracle's pin against LAPACK)
    rel = np.linalg.norm(L - Lo) / np.linalg.norm(Lo)
    assert rel <= np.linalg.cond(A32) * n * U32


@pytest.mark.parametrize("n,seed", [(24, 120), (130, 121), (257, 122), (1100, 123)])
def test_chol32_factor_exact_system_bitwise(device, n, seed):
    print(f"chol32 exact factor n={n}", flush=True)
    rng = np.random.default_rng(seed)
    d = rng.choice([1.0, 2.0, 4.0], n)
    L0 = np.tril(rng.choice([-1.0, -0.5, 0.0, 0.5, 1.0], size=(n, n)), -1) * d[None, :] + np.diag(d)
    A = L0 @ L0.T
    F, info = _factor(A, device)
    assert info == 0
    np.testing.assert_array_equal(np.tril(F).astype(np.float64), L0)
    Lo, _ = oracle.chol32_block(A, nb=64)
    np.testing.assert_array_equal(np.tril(F), Lo)


def test_chol32_factor_reports_first_nonpositive_pivot(device):
    print("chol32 indefinite", flush=True)
    n = 150
    A = np.eye(n) * 2.0
    A[97, 97] = -1.0
    _, info = _factor(A, device)
    _, s = oracle.chol32_block(A, nb=64)
    assert info == s == 98
    B = _spd(n, 300)
    B[5, 5] = -50.0
    _, info = _factor(B, device)
    assert 1 <= info <= 6


@pytest.mark.parametrize("n,kappa,seed", [(300, 1e2, 0), (1000, 1e4, 1), (1000, 1e6, 2),
                                          (2048, 1e6, 3), (777, 1e5, 4)])
def test_cg_ir_chol_matches_oracle(device, n, kappa, seed):
    from paper_1511_07207_amd import krylov

    print(f"cg-ir chol32 n={n} kappa={kappa:g} seed={seed}", flush=True)
    p = spd_problem(n, kappa, seed=seed, config_id=2)
    x, info = krylov.solve(_t(p.A, device), _t(p.b, device), method="cg", precision="chol32",
                           tol=ETA, max_iter=n)
    print(f"  status {info['status_name']} outer {info['outer_iters']} inner {info['iters']} "
          f"eta {info['backward_err']:.2e}", flush=True)
    assert info["status"] == 0, info
    xh = x.cpu().numpy()
    m = oracle.metrics(p.A, p.b, xh)
    assert m["eta_inf"] <= ETA
    assert abs(info["backward_err"] - m["eta_inf"]) <= 1e-3 * m["eta_inf"] + np.sqrt(n) * 2.0 ** -53
    xo, io = oracle.cg_ir_chol(p.A, p.b, tol=ETA, max_inner=n)
    assert io["status"] == 0
    assert abs(info["outer_iters"] - io["outer_iters"]) <= 1, (info, io)
    # forward error against the oracle's CG-IR run to 1e-15
    xr, _ = oracle.cg_ir_chol(p.A, p.b, tol=1e-15, max_inner=n)
    assert np.linalg.norm(xh - xr) <= max(1e-8, 100 * kappa * 1e-14) * np.linalg.norm(xr)


def test_cg_ir_chol_special_cases(device):
    from paper_1511_07207_amd import krylov

    print("cg-ir chol32 b = 0, indefinite A", flush=True)
    p = spd_problem(200, 1e3, seed=7, config_id=2)
    x, info = krylov.solve(_t(p.A, device), _t(np.zeros(200), device), method="cg",
                           precision="chol32", tol=ETA)
    assert info["status"] == 0 and info["iters"] == 0 and not x.cpu().numpy().any()
    S = p.A.copy()
    S[3, 3] = -5.0
    _, info = krylov.solve(_t(S, device), _t(p.b, device), method="cg", precision="chol32", tol=ETA)
    assert info["status_name"] == "breakdown"


def test_cg_ir_chol_full_size_kappa_1e6(device):
    """The refinement workload's hardest SPD cell, n = 32768, cond 1e6."""
    import torch

    from paper_1511_07207_amd import krylov

    n, kappa = 32768, 1e6
    print(f"cg-ir chol32 n={n} kappa=1e6: generating", flush=True)
    p = spd_problem(n, kappa, seed=0, config_id=2, backend="torch", device="cuda")
    x, info = krylov.solve(p.A, p.b, method="cg", precision="chol32", tol=ETA, max_iter=500)
    print(f"  status {info['status_name']} outer {info['outer_iters']} inner {info['iters']} "
          f"eta {info['backward_err']:.2e}", flush=True)
    assert info["status"] == 0, info
    xh = x.cpu().numpy()
    del x
    A_host = p.A.cpu().numpy()
    bh, xt = p.b.cpu().numpy(), p.x_true.cpu().numpy()
    del p
    torch.cuda.empty_cache()
    m = oracle.metrics(A_host, bh, xh)
    print(f"  eta (oracle) {m['eta_inf']:.3e}", flush=True)
    assert m["eta_inf"] <= ETA * (1 + 1e-6)
    assert np.linalg.norm(xh - xt) <= 4 * kappa * np.sqrt(n) * ETA * np.linalg.norm(xt) + 1e-12


@pytest.mark.parametrize("n", [70, 777, 2048, 16383])
def test_cg_ir_chol_persistent_substitutions_bitwise(device, n):
    """The substitutions with L and L^T in one cooperative launch per sweep
    give the same solve, bit for bit, as one launch per 64-row step."""
    from paper_1511_07207_amd import krylov

    print(f"cg-ir chol32 persistent vs per-launch substitutions n={n}", flush=True)
    p = spd_problem(n, 1e5, seed=12, config_id=2, backend="torch", device="cuda")
    out = []
    for persist in (True, False):
        x, info = krylov.solve(p.A, p.b, method="cg", precision="chol32", tol=ETA, max_iter=n,
                               persist=persist)
        assert info["status"] == 0, info
        out.append((x.cpu().numpy(), info["iters"], info["outer_iters"]))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    assert out[0][1:] == out[1][1:]
