"""Binary32 block LU and GMRES-IR on the GPU against the CPU oracle, through
the C ABI.

Factorization.  Pivots are argmax decisions taken in binary32 on both sides,
but the GPU's elimination uses fused multiply-adds where the oracle rounds the
product and the difference separately, so a near-tie between two candidate
rows may resolve differently once n is large.  The bars: at n <= 300 the
pivots equal the oracle's and the factors agree within the binary32 rounding
bound; at every size the GPU factors satisfy the componentwise backward-error
bound of Gaussian elimination, |P A32 - L U| <= gamma_n |L||U| in binary32
(gamma_n = n u / (1 - n u), u = 2^-24), whatever valid pivots were chosen,
with |l_ij| <= 1; on an exactly representable L0 U0 the factors are bitwise
the oracle's.

GMRES-IR.  On nonsymmetric systems with condition numbers up to 1e6 (where
plain GMRES(50) stalls) both sides reach a normwise backward error <= 1e-12
(checked by the oracle's own residual) in the same number of refinement
steps give or take one, and the solutions agree within cond(A) times that
bound.
"""
import numpy as np
import pytest

import oracle
from workloads import nonsym_swept_problem

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _t(x, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(device)


def _parts(LU, piv):
    n = LU.shape[0]
    L = np.tril(LU.astype(np.float64), -1) + np.eye(n)
    Uf = np.triu(LU.astype(np.float64))
    perm = np.arange(n)
    for k, p in enumerate(piv):
        perm[[k, p]] = perm[[p, k]]
    return L, Uf, perm


def _gpu_lu(A, device):
    from paper_1511_07207_amd import krylov

    LU, piv, info = krylov.lu32_factor(_t(A, device))
    return LU.cpu().numpy(), piv.cpu().numpy(), info


@pytest.mark.parametrize("n", [1, 5, 16, 17, 100, 257, 300, 520])
def test_lu32_factor_matches_oracle(device, n):
    print(f"lu32 n={n}", flush=True)
    A = np.random.default_rng(100 + n).standard_normal((n, n))
    LU, piv, info = _gpu_lu(A, device)
    LUo, pivo, sing = oracle.lu32_block(A, b=16)
    assert info == sing == 0
    np.testing.assert_array_equal(piv, pivo)
    L, Uf, perm = _parts(LU, piv)
    Lo, Uo, _ = _parts(LUo, pivo)
    gamma = n * U32 / (1 - n * U32)
    bound = 2 * gamma * (np.abs(Lo) @ np.abs(Uo))
    # the difference of the two factorizations, measured as the product's
    assert np.all(np.abs(L @ Uf - Lo @ Uo) <= bound + 1e-300)


@pytest.mark.parametrize("n", [64, 1000, 1500, 2049, 2600, 5000])
def test_lu32_backward_error_bound(device, n):
    print(f"lu32 bound n={n}", flush=True)
    A = np.random.default_rng(200 + n).standard_normal((n, n))
    LU, piv, info = _gpu_lu(A, device)
    assert info == 0
    L, Uf, perm = _parts(LU, piv)
    A32 = A.astype(np.float32).astype(np.float64)
    gamma = n * U32 / (1 - n * U32)
    assert np.all(np.abs(A32[perm] - L @ Uf) <= gamma * (np.abs(L) @ np.abs(Uf)) + 1e-300)
    assert np.abs(np.tril(LU, -1)).max(initial=0.0) <= 1.0


@pytest.mark.parametrize("n", [4096, 32768])
def test_lu32_large_sampled_rows(device, n):
    """64 sampled rows of P A32 - L U against the bound, the pivots valid
    (row k or below at step k) and every multiplier at most 1 in magnitude;
    n = 32768 is the largest size (32 panel blocks at the first panel)."""
    print(f"lu32 n={n} (sampled rows): generating", flush=True)
    A = np.random.default_rng(300).standard_normal((n, n))
    LU, piv, info = _gpu_lu(A, device)
    print("  factored", flush=True)
    assert info == 0
    assert np.all(piv >= np.arange(n)) and np.all(piv < n)
    assert np.abs(np.tril(LU, -1)).max() <= 1.0
    perm = np.arange(n)
    for k, p in enumerate(piv):
        perm[[k, p]] = perm[[p, k]]
    rows = np.sort(np.random.default_rng(301).choice(n, 64, replace=False))
    # rows `rows` of the unit lower L (columns left of each row's own index)
    Lr = np.where(np.arange(n)[None, :] < rows[:, None], LU[rows].astype(np.float64), 0.0)
    Lr[np.arange(64), rows] = 1.0
    Uf = np.triu(LU).astype(np.float64)
    del LU
    A32 = A[perm[rows]].astype(np.float32).astype(np.float64)
    del A
    gamma = n * U32 / (1 - n * U32)
    lhs = np.abs(A32 - Lr @ Uf)
    np.abs(Uf, out=Uf)
    assert np.all(lhs <= gamma * (np.abs(Lr) @ Uf) + 1e-300)


@pytest.mark.parametrize("n,zero_col", [(40, 7), (1100, 20), (4501, 1500)])
def test_lu32_exact_factorization_bitwise(device, n, zero_col):
    """An exactly representable L0 U0 (every partial sum exact, so any order
    of summation gives L0 and U0, and partial pivoting keeps the diagonal:
    |u_kk| = 8 > |l_ik u_kk|); n = 1100 crosses the rank-256 trailing updates
    on the matrix cores and a two-block panel, n = 4501 five-block panels and
    ragged trailing tiles with rows not 16-byte aligned.  Against the oracle
    where it finishes in seconds, else against L0 and U0 themselves."""
    print(f"lu32 exact n={n}", flush=True)
    rng = np.random.default_rng(310)
    L0 = np.tril(rng.choice([-0.5, -0.25, 0.0, 0.25, 0.5], size=(n, n)), -1) + np.eye(n)
    U0 = np.triu(rng.integers(-3, 4, size=(n, n)).astype(float), 1) + np.diag(rng.choice([-8.0, 8.0], n))
    A = L0 @ U0
    LU, piv, info = _gpu_lu(A, device)
    assert info == 0
    np.testing.assert_array_equal(piv, np.arange(n))
    np.testing.assert_array_equal(np.tril(LU, -1), np.tril(L0, -1))
    np.testing.assert_array_equal(np.triu(LU), U0)
    with_oracle = n <= 2000
    if with_oracle:
        LUo, pivo, _ = oracle.lu32_block(A, b=16)
        np.testing.assert_array_equal(LU, LUo)
    # a zero column: reported as the first zero pivot (the columns before it
    # factor exactly as above, and it stays zero)
    S = A.copy()
    S[:, zero_col] = 0.0
    _, _, info = _gpu_lu(S, device)
    assert info == zero_col + 1
    if with_oracle:
        _, _, sing = oracle.lu32_block(S, b=16)
        assert sing == info


@pytest.mark.parametrize("n,kappa,seed", [(100, 1e6, 0), (300, 1e6, 1), (1000, 1e4, 2),
                                          (2049, 1e6, 3), (777, 1e2, 4)])
def test_gmres_ir_lu_matches_oracle(device, n, kappa, seed):
    from paper_1511_07207_amd import krylov

    print(f"gmres-ir lu32 n={n} kappa={kappa:g}", flush=True)
    p = nonsym_swept_problem(n, kappa, seed=seed, config_id=7)
    xo, io = oracle.gmres_ir_lu(p.A, p.b, tol=1e-12, restart=30, inner_tol=1e-4)
    assert io["status_name"] == "ok", io
    x, info = krylov.solve(_t(p.A, device), _t(p.b, device), method="gmres", restart=30,
                           precision="lu32", tol=1e-12, inner_tol=1e-4)
    x = x.cpu().numpy()
    assert info["status_name"] == "ok", info
    assert info["precision_used"] == "lu32"
    assert abs(info["outer_iters"] - io["outer_iters"]) <= 1, (info, io)
    m = oracle.metrics(p.A, p.b, x)
    assert m["eta_inf"] <= 1e-12 * (1 + 1e-6)
    assert abs(info["backward_err"] - m["eta_inf"]) <= 1e-3 * m["eta_inf"] + 1e-15
    assert np.linalg.norm(x - xo) <= 10 * kappa * 1e-12 * np.linalg.norm(xo)


def test_gmres_ir_lu_where_gmres_stalls(device):
    from paper_1511_07207_amd import krylov

    n = 1000
    p = nonsym_swept_problem(n, 1e6, seed=5, config_id=7)
    A, b = _t(p.A, device), _t(p.b, device)
    _, ig = krylov.solve(A, b, method="gmres", restart=50, tol=1e-10, max_iter=1500)
    assert ig["status_name"] == "maxiter"
    x, info = krylov.solve(A, b, method="gmres", restart=30, precision="lu32", tol=1e-12)
    assert info["status_name"] == "ok" and info["outer_iters"] <= 4, info
    assert oracle.metrics(p.A, p.b, x.cpu().numpy())["eta_inf"] <= 1e-12 * (1 + 1e-6)


def test_gmres_ir_lu_special_cases(device):
    from paper_1511_07207_amd import krylov

    n = 70
    p = nonsym_swept_problem(n, 1e3, seed=6, config_id=7)
    A = _t(p.A, device)
    x, info = krylov.solve(A, _t(np.zeros(n), device), _t(np.ones(n), device), method="gmres",
                           precision="lu32", tol=1e-12)
    assert info["status_name"] == "ok" and info["outer_iters"] == 0 and not x.cpu().numpy().any()
    # singular in binary32: a zero column
    S = p.A.copy()
    S[:, 9] = 0.0
    _, info = krylov.solve(_t(S, device), _t(p.b, device), method="gmres", precision="lu32",
                           tol=1e-12)
    _, io = oracle.gmres_ir_lu(S, p.b, tol=1e-12)
    assert info["status_name"] == io["status_name"] == "breakdown"
    # n = 1
    x, info = krylov.solve(_t(np.array([[4.0]]), device), _t(np.array([2.0]), device),
                           method="gmres", precision="lu32", tol=1e-14)
    assert info["status_name"] == "ok" and x.cpu().numpy()[0] == 0.5

def test_gmres_ir_lu_full_size_kappa_1e6(device):
    """The refinement workload's hardest nonsymmetric cell, n = 32768, cond
    1e6, where GMRES(50) in binary64 and the binary32 and bfloat16 inner
    solves stagnate: the LU-preconditioned GMRES-IR reaches eta_inf <= 1e-12
    (checked by the oracle's residual) in a few refinement steps."""
    import torch

    from paper_1511_07207_amd import krylov

    n, kappa = 32768, 1e6
    print(f"gmres-ir lu32 n={n} kappa=1e6: generating", flush=True)
    p = nonsym_swept_problem(n, kappa, seed=0, config_id=2, backend="torch", device="cuda")
    x, info = krylov.solve(p.A, p.b, method="gmres", restart=50, precision="lu32", tol=1e-12,
                           inner_tol=1e-4)
    print(f"  status {info['status_name']} outer {info['outer_iters']} inner {info['iters']} "
          f"eta {info['backward_err']:.2e}", flush=True)
    assert info["status_name"] == "ok", info
    assert info["outer_iters"] <= 6, info
    xh = x.cpu().numpy()
    del x
    A_host = p.A.cpu().numpy()
    bh, xt = p.b.cpu().numpy(), p.x_true.cpu().numpy()
    del p
    torch.cuda.empty_cache()
    m = oracle.metrics(A_host, bh, xh)
    print(f"  eta (oracle) {m['eta_inf']:.3e}", flush=True)
    assert m["eta_inf"] <= 1e-12 * (1 + 1e-6)
    assert np.linalg.norm(xh - xt) <= 4 * kappa * np.sqrt(n) * 1e-12 * np.linalg.norm(xt) + 1e-12


@pytest.mark.parametrize("n", [70, 777, 2049, 16384])
def test_gmres_ir_lu_persistent_substitutions_bitwise(device, n):
    """The preconditioner's substitutions in one cooperative launch per sweep
    (a block per row block, up to the 256 row blocks of n = 16384) give the
    same solve, bit for bit, as one launch per 64-row step."""
    from paper_1511_07207_amd import krylov

    print(f"gmres-ir lu32 persistent vs per-launch substitutions n={n}", flush=True)
    p = nonsym_swept_problem(n, 1e6, seed=11, config_id=7, backend="torch", device="cuda")
    out = []
    for persist in (True, False):
        x, info = krylov.solve(p.A, p.b, method="gmres", restart=30, precision="lu32", tol=1e-12,
                               persist=persist)
        assert info["status_name"] == "ok", info
        out.append((x.cpu().numpy(), info["iters"], info["outer_iters"]))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    assert out[0][1:] == out[1][1:]
