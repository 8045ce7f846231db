"""Lockstep multi-right-hand-side CG (A*P on the matrix cores) against the
oracle's one-column CG, column by column, through the C ABI."""
import numpy as np
import pytest

import oracle
from workloads import multi_rhs_problem, spd_problem

pytestmark = pytest.mark.gpu


def _t(x, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(device)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _iters_close(a, b, n):
    """1% (at least 2) while CG is in its exact-arithmetic regime (fewer than
    n/2 steps); 5% (at least 3) once it runs towards or past n steps, where loss of
    orthogonality makes the count depend on the summation order."""
    if b < n // 2:
        return abs(a - b) <= max(2, int(0.01 * b))
    return abs(a - b) <= max(3, int(0.05 * b))


@pytest.mark.parametrize("n,s,kappa", [(1000, 16, 1e3), (777, 5, 1e4), (2048, 64, 1e4),
                                       (130, 33, 1e2)])
def test_lockstep_cg_matches_oracle_per_column(device, n, s, kappa):
    from paper_1511_07207_amd import krylov

    print(f"mrhs n={n} s={s} kappa={kappa}", flush=True)
    p = multi_rhs_problem(n, kappa, s, seed=1)
    X, info = krylov.Solver(_t(p.A, device), method="cg", nrhs=s, tol=1e-10,
                            max_iter=10 * n).solve(_t(p.b, device))
    X = X.cpu().numpy()
    assert info["status"] == 0, info
    for j in range(s):
        xo, io = oracle.cg(p.A, p.b[:, j], tol=1e-10, max_iter=10 * n)
        cj = info["columns"][j]
        assert cj["status"] == 0
        m = oracle.metrics(p.A, p.b[:, j], X[:, j])
        assert m["rel_res"] <= 1e-10
        assert _rel(X[:, j], xo) <= 1e-8, j
        assert _iters_close(cj["iters"], io["iters"], n), (j, cj, io)


def test_lockstep_first_iterate_exact(device):
    # after one iteration every column is x1 = (b'b / b'Ab) b: checks the
    # contraction itself at rounding level
    from paper_1511_07207_amd import krylov

    n, s = 300, 20
    p = multi_rhs_problem(n, 50.0, s, seed=2)
    X, info = krylov.Solver(_t(p.A, device), method="cg", nrhs=s, tol=1e-300,
                            max_iter=1).solve(_t(p.b, device))
    X = X.cpu().numpy()
    for j in range(s):
        xo, io = oracle.cg(p.A, p.b[:, j], tol=1e-300, max_iter=1)
        assert info["columns"][j]["iters"] == 1
        assert _rel(X[:, j], xo) <= 1e-13


def test_lockstep_special_columns(device):
    from paper_1511_07207_amd import krylov

    n, s = 200, 6
    p = multi_rhs_problem(n, 100.0, s, seed=3)
    B = p.b.copy()
    B[:, 1] = 0.0                      # zero column: x = 0, 0 iterations
    X0 = np.zeros((n, s))
    X0[:, 2] = p.x_true[:, 2]          # exact initial guess: 0 iterations
    X, info = krylov.Solver(_t(p.A, device), method="cg", nrhs=s, tol=1e-10).solve(
        _t(B, device), x0=_t(X0, device))
    X = X.cpu().numpy()
    cols = info["columns"]
    assert cols[1]["status"] == 0 and cols[1]["iters"] == 0 and np.all(X[:, 1] == 0)
    assert cols[2]["status"] == 0 and cols[2]["iters"] == 0
    for j in (0, 3, 4, 5):
        xo, io = oracle.cg(p.A, B[:, j], tol=1e-10)
        assert _rel(X[:, j], xo) <= 1e-8


def test_lockstep_ir_fp32_backward_error(device):
    from paper_1511_07207_amd import krylov

    n, s = 1024, 16
    p = multi_rhs_problem(n, 1e3, s, seed=4)
    X, info = krylov.Solver(_t(p.A, device), method="cg", nrhs=s, precision="fp32", tol=1e-12,
                            max_iter=4 * n).solve(_t(p.b, device))
    X = X.cpu().numpy()
    assert info["status"] == 0, info
    for j in range(s):
        m = oracle.metrics(p.A, p.b[:, j], X[:, j])
        assert m["eta_inf"] <= 1e-12, (j, m)
        xo, _ = oracle.cg(p.A, p.b[:, j], tol=1e-14, max_iter=20 * n)
        assert _rel(X[:, j], xo) <= 1e-8


def test_lockstep_repeatable(device):
    import torch

    from paper_1511_07207_amd import krylov

    p = multi_rhs_problem(600, 1e3, 24, seed=5)
    solver = krylov.Solver(_t(p.A, device), method="cg", nrhs=24, tol=1e-10)
    X1, _ = solver.solve(_t(p.b, device))
    X2, _ = solver.solve(_t(p.b, device))
    torch.cuda.synchronize()
    assert torch.equal(X1, X2)


# ---- the contraction Q = A P on its own (ks_gemm_mr) -------------------------
# Integer entries small enough that every product and every partial sum is an
# integer below 2^24: binary32 and binary64 arithmetic are then exact in any
# summation order, so the product must equal the oracle's column by column
# bit for bit (a dropped, repeated or misplaced term changes it).  The sizes
# cover one split of K with a ragged end (777, 1000), several splits with
# and without the XCD grouping (2100, 4100, 4096) and 1 .. 4 tiles of 16
# columns.

def _padded(A, device, tdt):
    """A on the device with its rows 64-element aligned (the entry point wants
    16-byte row strides); a view of the n x n part."""
    import torch

    n = A.shape[0]
    lda = (n + 63) // 64 * 64
    buf = torch.zeros((n, lda), dtype=tdt, device=device)
    buf[:, :n] = _t(A, device).to(tdt)
    return buf[:, :n]


def _int_problem(n, s, amax, pmax, seed):
    rng = np.random.default_rng([seed, n, s])
    A = rng.integers(-amax, amax + 1, size=(n, n)).astype(np.float64)
    P = rng.integers(-pmax, pmax + 1, size=(n, s)).astype(np.float64)
    return A, P


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n,s", [(777, 5), (1000, 33), (2100, 64), (4100, 17), (4096, 64)])
def test_gemm_mr_exact_on_integers(device, dtype, n, s):
    import torch

    from paper_1511_07207_amd import krylov

    print(f"gemm_mr exact n={n} s={s} {dtype}", flush=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    A, P = _int_problem(n, s, 2, 3, seed=11)
    Q = krylov.gemm_mr(_padded(A, device, tdt), _t(P, device).to(tdt)).double().cpu().numpy()
    for j in range(s):
        np.testing.assert_array_equal(Q[:, j], oracle.matvec(A, P[:, j]), err_msg=f"column {j}")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gemm_mr_rounding_within_bound_and_repeatable(device, dtype):
    # random values: |q - q_exact| <= gamma_n sum_k |a_ik| |p_kj| for any
    # summation order (gamma_n = n u / (1 - n u), u the unit roundoff), the
    # exact value approximated by the oracle's binary64 sums of the same inputs
    import torch

    from paper_1511_07207_amd import krylov

    n, s = 2100, 40
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    rng = np.random.default_rng(12)
    A = rng.standard_normal((n, n))
    P = rng.standard_normal((n, s))
    Ad, Pd = _padded(A, device, tdt), _t(P, device).to(tdt)
    A_in, P_in = Ad.double().cpu().numpy(), Pd.double().cpu().numpy()  # the values multiplied
    Q1 = krylov.gemm_mr(Ad, Pd)
    Q2 = krylov.gemm_mr(Ad, Pd)
    torch.cuda.synchronize()
    assert torch.equal(Q1, Q2)
    Q = Q1.double().cpu().numpy()
    gamma = n * u / (1 - n * u)
    gamma64 = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)   # the oracle's own sums
    absA = np.abs(A_in)
    for j in range(s):
        ref = oracle.matvec(A_in, P_in[:, j])
        bound = (gamma + gamma64) * oracle.matvec(absA, np.abs(P_in[:, j])) * (1 + 1e-9)
        assert np.all(np.abs(Q[:, j] - ref) <= bound), j


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_gemm_mr_full_size_sampled_rows(device, dtype):
    # the lockstep benchmark's shape (n = 16384, 64 columns) in the launch
    # configuration the solver uses, entries in {-1, 0, 1}: exact, sampled rows
    import torch

    from paper_1511_07207_amd import krylov

    n, s = 16384, 64
    print(f"gemm_mr full size {dtype}", flush=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    A, P = _int_problem(n, s, 1, 1, seed=13)
    Q = krylov.gemm_mr(_t(A, device).to(tdt), _t(P, device).to(tdt)).double().cpu().numpy()
    rows = np.sort(np.random.default_rng(14).choice(n, 96, replace=False))
    rows[-1] = n - 1
    for j in range(s):
        np.testing.assert_array_equal(Q[rows, j], oracle.matvec_rows(A, rows, P[:, j]),
                                      err_msg=f"column {j}")
