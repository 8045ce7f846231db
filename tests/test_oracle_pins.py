"""Pins for the CPU oracle: each check ties it to something other than itself.

* exact-rational brute force of the Krylov iterates (CG: the A-norm minimiser
  over x0 + K_k; GMRES: the residual minimiser over x0 + K_k), solved with
  Python fractions, never with the oracle's own arithmetic;
* finite termination (CG in at most n steps, and in d steps for d distinct
  eigenvalues; full GMRES likewise) from the Krylov section's claims;
* the Arnoldi relation A V_k = V_{k+1} Hbar_k with orthonormal V;
* GMRES's non-increasing residual, and full GMRES <= CG on SPD systems;
* LAPACK (numpy.linalg.solve) and hand-worked fixtures for GEPP;
* special cases and the hand-worked backward-error example.
"""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import nonsym_problem, spd_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ exact helpers

def _fr_solve(M, v):
    """Solve M y = v exactly (Gauss-Jordan over Fractions, nonzero pivot)."""
    k = len(v)
    aug = [list(M[i]) + [v[i]] for i in range(k)]
    for c in range(k):
        p = next(r for r in range(c, k) if aug[r][c] != 0)
        aug[c], aug[p] = aug[p], aug[c]
        piv = aug[c][c]
        aug[c] = [e / piv for e in aug[c]]
        for r in range(k):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[c])]
    return [aug[i][k] for i in range(k)]


def _fr_matvec(A, x):
    return [sum((a * b for a, b in zip(row, x)), Fraction(0)) for row in A]


def _fr_krylov(A, r0, k):
    K = [r0]
    for _ in range(k - 1):
        K.append(_fr_matvec(A, K[-1]))
    return K  # list of k vectors


def _fr_dot(x, y):
    return sum((a * b for a, b in zip(x, y)), Fraction(0))


def exact_cg_iterate(A, b, k):
    """argmin over x in K_k(A, b) of ||x - x*||_A  (x0 = 0): (K'AK) y = K'b."""
    Af = [[Fraction(int(a)) for a in row] for row in A]
    bf = [Fraction(int(v)) for v in b]
    K = _fr_krylov(Af, bf, k)
    AK = [_fr_matvec(Af, kv) for kv in K]
    M = [[_fr_dot(K[i], AK[j]) for j in range(k)] for i in range(k)]
    rhs = [_fr_dot(K[i], bf) for i in range(k)]
    y = _fr_solve(M, rhs)
    n = len(bf)
    return np.array([float(sum((y[j] * K[j][i] for j in range(k)), Fraction(0))) for i in range(n)])


def exact_gmres_iterate(Af, bf, x0f, k):
    """argmin over x in x0 + K_k(A, r0) of ||b - A x||_2: (AK)'(AK) y = (AK)' r0."""
    r0 = [bi - ai for bi, ai in zip(bf, _fr_matvec(Af, x0f))]
    K = _fr_krylov(Af, r0, k)
    AK = [_fr_matvec(Af, kv) for kv in K]
    M = [[_fr_dot(AK[i], AK[j]) for j in range(k)] for i in range(k)]
    rhs = [_fr_dot(AK[i], r0) for i in range(k)]
    y = _fr_solve(M, rhs)
    n = len(bf)
    return [x0f[i] + sum((y[j] * K[j][i] for j in range(k)), Fraction(0)) for i in range(n)]


def _int_spd(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.integers(-3, 4, size=(n, n))
    return M.T @ M + 2 * np.eye(n, dtype=np.int64)


def _int_nonsym(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.integers(-2, 3, size=(n, n))
    return M + 6 * np.eye(n, dtype=np.int64)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


TINY = 1e-300  # a tolerance the iteration never meets: runs exactly max_iter steps


# ---------------------------------------------------------------- CG pins

@pytest.mark.parametrize("n,seed", [(4, 1), (5, 2), (6, 3)])
def test_cg_iterates_match_exact_rational_minimiser(n, seed):
    A = _int_spd(n, seed)
    b = np.random.default_rng(seed + 10).integers(-5, 6, size=n)
    for k in range(1, n + 1):
        x, info = oracle.cg(A.astype(float), b.astype(float), tol=TINY, max_iter=k)
        assert info["iters"] == k
        xe = exact_cg_iterate(A, b, k)
        assert _rel(x, xe) <= 1e-12, (k, _rel(x, xe))


def test_cg_finite_termination_at_most_n_steps():
    # exact arithmetic ends in <= n steps; with a spread spectrum rounding can
    # delay it by a few steps, so the pin uses a mild condition number
    for seed in range(3):
        p = spd_problem(16, 4.0, seed=seed, config_id=90)
        x, info = oracle.cg(p.A, p.b, tol=1e-10, max_iter=100)
        assert info["status"] == 0
        assert info["iters"] <= 16
        assert info["rel_res"] <= 1e-10


def test_cg_two_distinct_eigenvalues_two_steps():
    rng = np.random.default_rng(5)
    n = 40
    u = rng.standard_normal(n)
    A = np.eye(n) + np.outer(u, u)          # eigenvalues 1 and 1 + u'u
    b = rng.standard_normal(n)
    x, info = oracle.cg(A, b, tol=1e-10)
    assert info["status"] == 0 and info["iters"] == 2
    assert _rel(x, np.linalg.solve(A, b)) <= 1e-12


def test_cg_diagonal_d_distinct_values_d_steps():
    vals = np.array([1.0, 2.0, 5.0, 9.0])
    n = 32
    d = np.tile(vals, n // 4)
    A = np.diag(d)
    b = np.ones(n)
    x, info = oracle.cg(A, b, tol=1e-10)
    assert info["status"] == 0 and info["iters"] == 4
    assert _rel(x, b / d) <= 1e-13


def test_cg_energy_norm_strictly_decreasing():
    p = spd_problem(40, 1e3, seed=4, config_id=91)
    xs = np.linalg.solve(p.A, p.b)
    prev = np.inf
    for k in range(1, 30):
        x, _ = oracle.cg(p.A, p.b, tol=TINY, max_iter=k)
        e = x - xs
        en = float(e @ p.A @ e)
        assert en < prev
        prev = en


def test_cg_residuals_mutually_orthogonal():
    # r_i' r_j = 0 for i != j (exact arithmetic); checked on the first steps
    p = spd_problem(60, 50.0, seed=6, config_id=92)
    rs = []
    for k in range(0, 6):
        if k == 0:
            x = np.zeros(60)
        else:
            x, _ = oracle.cg(p.A, p.b, tol=TINY, max_iter=k)
        r = p.b - p.A @ x
        rs.append(r / np.linalg.norm(r))
    G = np.array([[a @ b for b in rs] for a in rs])
    assert np.max(np.abs(G - np.eye(len(rs)))) <= 1e-10


def test_cg_breakdown_on_indefinite():
    A = np.diag([1.0, -1.0, 2.0])
    b = np.array([1.0, 1.0, 0.0])   # p'Ap = 0 at step 1
    x, info = oracle.cg(A, b, tol=1e-10)
    assert info["status"] == 2


# ------------------------------------------------------------- GMRES pins

@pytest.mark.parametrize("n,seed", [(4, 1), (5, 2), (6, 3)])
def test_gmres_iterates_match_exact_least_squares(n, seed):
    A = _int_nonsym(n, seed)
    b = np.random.default_rng(seed + 20).integers(-5, 6, size=n)
    Af = [[Fraction(int(a)) for a in row] for row in A]
    bf = [Fraction(int(v)) for v in b]
    zero = [Fraction(0)] * n
    for k in range(1, n + 1):
        x, info = oracle.gmres(A.astype(float), b.astype(float), tol=TINY, max_iter=k, restart=n)
        assert info["iters"] == k
        xe = np.array([float(v) for v in exact_gmres_iterate(Af, bf, zero, k)])
        assert _rel(x, xe) <= 1e-12, (k, _rel(x, xe))


def test_gmres_restarted_iterates_match_composed_exact_minimisers():
    n, m = 6, 2
    A = _int_nonsym(n, 7)
    b = np.random.default_rng(8).integers(-5, 6, size=n)
    Af = [[Fraction(int(a)) for a in row] for row in A]
    bf = [Fraction(int(v)) for v in b]
    xe = [Fraction(0)] * n
    for cyc in range(1, 4):
        xe = exact_gmres_iterate(Af, bf, xe, m)
        x, info = oracle.gmres(A.astype(float), b.astype(float), tol=TINY, max_iter=m * cyc,
                               restart=m)
        assert info["cycles"] == cyc
        assert _rel(x, np.array([float(v) for v in xe])) <= 1e-12


def test_full_gmres_terminates_in_n_steps():
    p = nonsym_problem(24, seed=2, config_id=93)
    x, info = oracle.gmres(p.A, p.b, tol=1e-12, restart=24, max_iter=24)
    assert info["status"] == 0 and info["iters"] <= 24


def test_gmres_rank_one_perturbation_two_steps():
    rng = np.random.default_rng(9)
    n = 50
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    A = np.eye(n) + np.outer(u, v)
    assert abs(1 + v @ u) > 1e-3
    b = rng.standard_normal(n)
    x, info = oracle.gmres(A, b, tol=1e-10, restart=30)
    assert info["status"] == 0 and info["iters"] <= 2
    assert _rel(x, np.linalg.solve(A, b)) <= 1e-11


def test_arnoldi_relation_and_orthonormality():
    p = nonsym_problem(200, seed=3, config_id=94)
    v0 = np.random.default_rng(1).standard_normal(200)
    V, H, k = oracle.arnoldi(p.A, v0, 30)
    assert k == 30 and V.shape == (200, 31) and H.shape == (31, 30)
    AF = np.linalg.norm(p.A)
    assert np.linalg.norm(p.A @ V[:, :30] - V @ H) <= 1e-13 * AF
    assert np.linalg.norm(V.T @ V - np.eye(31)) <= 1e-13
    assert np.allclose(np.tril(H, -2), 0.0)               # upper Hessenberg
    assert np.all(np.diag(H, -1) > 0)
    # the first vector is v0 normalised
    assert _rel(V[:, 0], v0 / np.linalg.norm(v0)) <= 1e-15


def test_gmres_residual_non_increasing():
    p = nonsym_problem(300, seed=4, config_id=95)
    x, info = oracle.gmres(p.A, p.b, tol=1e-12, restart=5, max_iter=400, hist=True)
    assert info["status"] == 0
    cres = info["cres"]
    assert len(cres) >= 3
    assert np.all(cres[1:] <= cres[:-1] * (1 + 1e-12))
    est = info["est"]
    m = 5
    for c in range(info["cycles"]):
        seg = est[c * m:(c + 1) * m]
        assert np.all(seg[1:] <= seg[:-1] * (1 + 1e-12))


def test_full_gmres_residual_below_cg_on_spd():
    p = spd_problem(50, 200.0, seed=5, config_id=96)
    for k in range(1, 20):
        xc, _ = oracle.cg(p.A, p.b, tol=TINY, max_iter=k)
        xg, _ = oracle.gmres(p.A, p.b, tol=TINY, max_iter=k, restart=50)
        rc = np.linalg.norm(p.b - p.A @ xc)
        rg = np.linalg.norm(p.b - p.A @ xg)
        assert rg <= rc * (1 + 1e-10), k


# ---------------------------------------------------------- GEPP and solves

def _read_fixture(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows.setdefault(key, []).append([float(v) for v in vals])
    return rows


def test_gepp_hand_worked_3x3():
    fx = _read_fixture("gepp_3x3.txt")
    A, b = np.array(fx["A"]), np.array(fx["b"][0])
    LU, piv, s = oracle.lu_factor(A)
    assert s == 0
    assert list(piv) == [int(v) for v in fx["piv"][0]]
    assert np.array_equal(LU, np.array(fx["LU"]))
    assert np.array_equal(oracle.lu_solve(LU, piv, b), np.array(fx["x"][0]))


@pytest.mark.parametrize("n", [1, 2, 7, 33, 100])
def test_gepp_matches_lapack(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x = oracle.gepp_solve(A, b)
    xl = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    assert _rel(x, xl) <= 10 * kappa * n * np.finfo(float).eps


def test_gepp_detects_singular():
    A = np.array([[1.0, 2.0], [2.0, 4.0]])
    _, _, s = oracle.lu_factor(A)
    assert s == 2


def test_krylov_agrees_with_gepp_on_small_systems():
    p = spd_problem(64, 1e2, seed=7, config_id=97)
    xg = oracle.gepp_solve(p.A, p.b)
    x, info = oracle.cg(p.A, p.b, tol=1e-12)
    assert info["status"] == 0
    assert _rel(x, xg) <= 1e2 * 1e-12 * 10
    q = nonsym_problem(64, seed=7, config_id=97)
    xg = oracle.gepp_solve(q.A, q.b)
    x, info = oracle.gmres(q.A, q.b, tol=1e-12, restart=30)
    assert info["status"] == 0
    assert _rel(x, xg) <= 10 * np.linalg.cond(q.A) * 1e-12


def test_known_solution_error_bound():
    kappa = 1e3
    p = spd_problem(256, kappa, seed=8, config_id=98)
    x, info = oracle.cg(p.A, p.b, tol=1e-10)
    assert info["status"] == 0 and info["rel_res"] <= 1e-10
    u = np.finfo(float).eps / 2
    assert _rel(x, p.x_true) <= kappa * info["rel_res"] + kappa * 256 * u


# --------------------------------------------------------- special cases

def test_n_equals_one():
    A = np.array([[4.0]])
    b = np.array([3.0])
    x, info = oracle.cg(A, b, tol=1e-12)
    assert info["iters"] == 1 and abs(x[0] - 0.75) <= 1e-16
    x, info = oracle.gmres(A, b, tol=1e-12)
    assert info["iters"] == 1 and abs(x[0] - 0.75) <= 1e-16


def test_identity_one_step():
    b = np.random.default_rng(0).standard_normal(17)
    for solve in (oracle.cg, oracle.gmres):
        x, info = solve(np.eye(17), b, tol=1e-12)
        assert info["iters"] == 1 and np.array_equal(x, b)


def test_zero_rhs_returns_zero():
    A = np.eye(5) * 3
    for solve in (oracle.cg, oracle.gmres):
        x, info = solve(A, np.zeros(5), x0=np.ones(5))
        assert info["status"] == 0 and info["iters"] == 0 and np.all(x == 0)


def test_exact_initial_guess_zero_iterations():
    p = spd_problem(30, 10.0, seed=1, config_id=99)
    for solve in (oracle.cg, oracle.gmres):
        x, info = solve(p.A, p.b, x0=p.x_true, tol=1e-10)
        assert info["iters"] == 0 and info["status"] == 0


def test_nonfinite_rhs():
    b = np.array([1.0, np.nan, 0.0])
    for solve in (oracle.cg, oracle.gmres):
        _, info = solve(np.eye(3), b)
        assert info["status"] == 4


def test_maxiter_status():
    p = spd_problem(100, 1e4, seed=2, config_id=99)
    _, info = oracle.cg(p.A, p.b, tol=1e-12, max_iter=5)
    assert info["status"] == 1 and info["iters"] == 5
    q = nonsym_problem(100, seed=2, config_id=99)
    _, info = oracle.gmres(q.A, q.b, tol=1e-14, max_iter=7, restart=3)
    assert info["status"] == 1 and info["iters"] == 7 and info["cycles"] == 3


def test_backward_error_hand_worked_2x2():
    fx = _read_fixture("eta_inf_2x2.txt")
    A, b, x = np.array(fx["A"]), np.array(fx["b"][0]), np.array(fx["x"][0])
    m = oracle.metrics(A, b, x)
    assert m["eta_inf"] == fx["eta_inf"][0][0]
    assert abs(m["rel_res"] ** 2 - fx["rel_res_sq"][0][0]) <= 1e-16


# ------------------------------------------------------------ BiCGSTAB pins

def _fr_vec(v):
    return [Fraction(int(a)) for a in v]


def test_bicgstab_first_iterate_from_its_two_defining_conditions():
    # One BiCGSTAB step from x0 = 0 (r0 = b, p = r0) is fixed by two 1-D
    # conditions, computed here exactly and independently of the recurrence:
    #   alpha: the Galerkin condition r0'(r0 - alpha A r0) = 0
    #   omega: s - omega A s has least 2-norm, s = r0 - alpha A r0
    # and x1 = alpha r0 + omega s.
    for seed, n in [(1, 4), (2, 5), (3, 6)]:
        A = _int_nonsym(n, seed)
        b = np.random.default_rng(seed + 40).integers(-5, 6, size=n)
        Af = [[Fraction(int(a)) for a in row] for row in A]
        r0 = _fr_vec(b)
        Ar0 = _fr_matvec(Af, r0)
        alpha = _fr_dot(r0, r0) / _fr_dot(r0, Ar0)
        s = [a - alpha * c for a, c in zip(r0, Ar0)]
        As = _fr_matvec(Af, s)
        omega = _fr_dot(As, s) / _fr_dot(As, As)
        x1 = np.array([float(alpha * a + omega * c) for a, c in zip(r0, s)])
        x, info = oracle.bicgstab(A.astype(float), b.astype(float), tol=TINY, max_iter=2)
        assert info["iters"] == 2
        assert _rel(x, x1) <= 1e-13


def _fr_poly_apply(A, coeffs, v):
    """sum_i coeffs[i] A^i v, exactly."""
    out = [Fraction(0)] * len(v)
    w = list(v)
    for c in coeffs:
        out = [o + c * wi for o, wi in zip(out, w)]
        w = _fr_matvec(A, w)
    return out


def _fr_poly_mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def exact_bicgstab_iterate(A, b, k):
    """The k-th BiCGSTAB iterate from x0 = 0 (shadow residual r0 = b), built from
    the two objects that define it rather than from its recurrence:
      phi_k, the BiCG residual polynomial: degree k, phi_k(0) = 1 and
        phi_k(A) r0 orthogonal to r0, A' r0, ..., (A')^(k-1) r0
        (the Petrov-Galerkin conditions r0' A^j phi_k(A) r0 = 0, j < k);
      psi_k(t) = prod_j (1 - omega_j t), where omega_j minimises the 2-norm of
        (1 - omega A) s_j, s_j = psi_(j-1)(A) phi_j(A) r0.
    The residual is r_k = psi_k(A) phi_k(A) r0.  Since 1 - psi_k phi_k vanishes
    at 0, it equals t q(t) and x_k = q(A) r0 without any solve with A."""
    Af = [[Fraction(int(a)) for a in row] for row in A]
    r0 = _fr_vec(b)
    K = _fr_krylov(Af, r0, 2 * k + 1)          # r0, A r0, ..., A^(2k) r0
    mom = [_fr_dot(r0, K[i]) for i in range(2 * k + 1)]  # r0' A^i r0
    psi = [Fraction(1)]
    for j in range(1, k + 1):
        # phi_j = 1 + c_1 t + ... + c_j t^j from its j orthogonality conditions
        M = [[mom[i + m] for m in range(1, j + 1)] for i in range(j)]
        c = _fr_solve(M, [-mom[i] for i in range(j)])
        phi = [Fraction(1)] + c
        s = _fr_poly_apply(Af, _fr_poly_mul(psi, phi), r0)
        As = _fr_matvec(Af, s)
        omega = _fr_dot(As, s) / _fr_dot(As, As)
        psi = _fr_poly_mul(psi, [Fraction(1), -omega])
    P = _fr_poly_mul(psi, phi)                  # residual polynomial, P(0) = 1
    q = [-c for c in P[1:]]                      # 1 - P(t) = t q(t)
    x = _fr_poly_apply(Af, q, r0)
    return np.array([float(v) for v in x])


@pytest.mark.parametrize("k", [2, 3])
def test_bicgstab_later_iterates_from_polynomial_conditions(k):
    # Iterates past the first fix the recurrence's beta and rho: a beta
    # without its alpha / omega factor, or rho taken as r'r instead of r0'r,
    # changes phi_k and so x_k.
    for seed, n in [(1, 5), (2, 6), (5, 7)]:
        A = _int_nonsym(n, seed)
        b = np.random.default_rng(seed + 40).integers(-5, 6, size=n)
        xk = exact_bicgstab_iterate(A, b, k)
        x, info = oracle.bicgstab(A.astype(float), b.astype(float), tol=TINY, max_iter=2 * k)
        assert info["iters"] == 2 * k
        assert _rel(x, xk) <= 1e-12


def test_bicgstab_exact_iterate_construction_matches_first_step():
    # the polynomial construction at k = 1 is the first iterate's two conditions
    A = _int_nonsym(5, 9)
    b = np.random.default_rng(49).integers(-5, 6, size=5)
    x, _ = oracle.bicgstab(A.astype(float), b.astype(float), tol=TINY, max_iter=2)
    assert _rel(x, exact_bicgstab_iterate(A, b, 1)) <= 1e-13


def test_bicgstab_terminates_within_n_iterations():
    # In exact arithmetic phi_n(A) r0 = 0 (n conditions on a degree-n
    # polynomial with phi(0) = 1), so without breakdown the residual vanishes
    # after at most n iterations, 2n products.
    for seed in range(20):
        n = 6
        rng = np.random.default_rng(seed + 300)
        A = np.diag(rng.uniform(2.0, 4.0, n)) + rng.standard_normal((n, n)) / np.sqrt(n)
        b = rng.standard_normal(n)
        _, info = oracle.bicgstab(A, b, tol=1e-10, max_iter=2 * n)
        assert info["status"] == 0 and info["rel_res"] <= 1e-10 and info["iters"] <= 2 * n


def test_bicgstab_identity_half_step():
    b = np.random.default_rng(1).standard_normal(20)
    x, info = oracle.bicgstab(np.eye(20), b, tol=1e-12)
    assert info["status"] == 0 and info["iters"] == 1 and np.array_equal(x, b)


@pytest.mark.parametrize("kind", ["spd", "nonsym"])
def test_bicgstab_agrees_with_gepp(kind):
    if kind == "spd":
        p = spd_problem(80, 1e2, seed=11, config_id=97)
    else:
        p = nonsym_problem(80, seed=11, config_id=97)
    x, info = oracle.bicgstab(p.A, p.b, tol=1e-12)
    assert info["status"] == 0 and info["rel_res"] <= 1e-12
    xg = oracle.gepp_solve(p.A, p.b)
    assert _rel(x, xg) <= 10 * np.linalg.cond(p.A) * 1e-12


def test_bicgstab_special_cases():
    A = np.eye(5) * 2.0
    x, info = oracle.bicgstab(A, np.zeros(5), x0=np.ones(5))
    assert info["status"] == 0 and info["iters"] == 0 and np.all(x == 0)
    p = nonsym_problem(40, seed=3, config_id=97)
    x, info = oracle.bicgstab(p.A, p.b, x0=p.x_true, tol=1e-10)
    assert info["iters"] == 0 and info["status"] == 0
    _, info = oracle.bicgstab(np.eye(3), np.array([1.0, np.nan, 0.0]))
    assert info["status"] == 4
    _, info = oracle.bicgstab(p.A, p.b, tol=1e-14, max_iter=6)
    assert info["status"] == 1 and info["iters"] == 6


def test_matvec_rows_is_the_product_restricted():
    # the sampled-row product is the full product restricted to those rows,
    # pinned by exact integer arithmetic
    rng = np.random.default_rng(3)
    A = rng.integers(-9, 10, size=(37, 37)).astype(float)
    x = rng.integers(-9, 10, size=37).astype(float)
    rows = [0, 5, 36, 17, 17]
    y = oracle.matvec_rows(A, rows, x)
    exact = [sum(int(A[r, j]) * int(x[j]) for j in range(37)) for r in rows]
    assert y.tolist() == [float(v) for v in exact]


# ---------------------------------------------------- Jacobi / Gauss-Seidel
# The stationary iterations, pinned by exactness on diagonal and triangular
# matrices, by SciPy's forward substitution for the sweeps, by exact rational
# arithmetic for the iterates, and by the two convergence theorems that tell
# the methods apart (Stein-Rosenberg; Gauss-Seidel on SPD matrices).

def _fr_jacobi_step(A, b, x):
    n = len(b)
    return [(b[i] - sum(A[i][j] * x[j] for j in range(n) if j != i)) / A[i][i] for i in range(n)]


def _fr_gs_sweep(A, b, x):
    x = list(x)
    n = len(b)
    for i in range(n):
        x[i] = (b[i] - sum(A[i][j] * x[j] for j in range(n) if j != i)) / A[i][i]
    return x


def _small_int_system(seed, n=5):
    """Integer, strictly diagonally dominant A and integer b."""
    rng = np.random.default_rng(seed)
    A = rng.integers(-3, 4, size=(n, n)).astype(float)
    A[np.arange(n), np.arange(n)] = np.abs(A).sum(axis=1) + rng.integers(1, 4, size=n)
    b = rng.integers(-9, 10, size=n).astype(float)
    return A, b


@pytest.mark.parametrize("steps", [1, 2, 3])
def test_jacobi_iterates_match_exact_rational_steps(steps):
    A, b = _small_int_system(11)
    x, info = oracle.jacobi(A, b, tol=1e-300, max_iter=steps)
    assert info["status_name"] == "maxiter" and info["iters"] == steps
    Af = [[Fraction(int(v)) for v in row] for row in A]
    bf = [Fraction(int(v)) for v in b]
    xf = [Fraction(0)] * len(b)
    for _ in range(steps):
        xf = _fr_jacobi_step(Af, bf, xf)
    np.testing.assert_allclose(x, [float(v) for v in xf], rtol=1e-14, atol=0)


@pytest.mark.parametrize("steps", [1, 2, 3])
def test_gauss_seidel_iterates_match_exact_rational_sweeps(steps):
    A, b = _small_int_system(12)
    x, info = oracle.gauss_seidel(A, b, tol=1e-300, max_iter=steps)
    assert info["status_name"] == "maxiter" and info["iters"] == steps
    Af = [[Fraction(int(v)) for v in row] for row in A]
    bf = [Fraction(int(v)) for v in b]
    xf = [Fraction(0)] * len(b)
    for _ in range(steps):
        xf = _fr_gs_sweep(Af, bf, xf)
    np.testing.assert_allclose(x, [float(v) for v in xf], rtol=1e-14, atol=0)


def test_gauss_seidel_sweeps_are_forward_substitutions():
    """x1 = tril(A)^{-1} b and x2 = tril(A)^{-1} (b - triu(A, 1) x1) (SciPy)."""
    from scipy.linalg import solve_triangular

    p = nonsym_problem(300, seed=3, config_id=0)
    A, b = p.A, p.b
    x1, _ = oracle.gauss_seidel(A, b, tol=1e-300, max_iter=1)
    r1 = solve_triangular(np.tril(A), b, lower=True)
    np.testing.assert_allclose(x1, r1, rtol=1e-12, atol=1e-14 * np.abs(r1).max())
    x2, _ = oracle.gauss_seidel(A, b, tol=1e-300, max_iter=2)
    r2 = solve_triangular(np.tril(A), b - np.triu(A, 1) @ r1, lower=True)
    np.testing.assert_allclose(x2, r2, rtol=1e-12, atol=1e-14 * np.abs(r2).max())
    # Jacobi's first two steps from zero: b / d, then (b - (A - D) x1) / d
    d = np.diag(A)
    j1, _ = oracle.jacobi(A, b, tol=1e-300, max_iter=1)
    np.testing.assert_array_equal(j1, b / d)  # b_i - 0 = b_i exactly, one division
    j2, _ = oracle.jacobi(A, b, tol=1e-300, max_iter=2)
    np.testing.assert_allclose(j2, (b - (A - np.diag(d)) @ (b / d)) / d, rtol=1e-12)


def test_stationary_exact_cases():
    rng = np.random.default_rng(5)
    n = 40
    d = rng.uniform(1, 3, n) * rng.choice([-1, 1], n)
    b = rng.standard_normal(n)
    # diagonal A: Jacobi and Gauss-Seidel are exact after one update
    for fn in (oracle.jacobi, oracle.gauss_seidel):
        x, info = fn(np.diag(d), b, tol=1e-14)
        assert info["status_name"] == "ok" and info["iters"] == 1
        np.testing.assert_array_equal(x, b / d)
    # lower-triangular A: one Gauss-Seidel sweep is the exact forward solve
    L = np.tril(rng.standard_normal((n, n)) * 0.1, -1) + np.diag(d)
    x, info = oracle.gauss_seidel(L, b, tol=1e-12)
    assert info["status_name"] == "ok" and info["iters"] == 1
    # exact start and b = 0
    A, bi = _small_int_system(13)
    xs = np.linalg.solve(A, bi)
    for fn in (oracle.jacobi, oracle.gauss_seidel):
        x, info = fn(A, A @ xs, x0=xs, tol=1e-12)
        assert info["iters"] == 0 and info["status_name"] == "ok"
        x, info = fn(A, np.zeros(5), x0=np.ones(5), tol=1e-12)
        assert info["iters"] == 0 and info["status_name"] == "ok" and not x.any()


def test_stationary_breakdown_and_divergence():
    A, b = _small_int_system(14)
    Z = A.copy()
    Z[2, 2] = 0.0
    for fn in (oracle.jacobi, oracle.gauss_seidel):
        _, info = fn(Z, b, tol=1e-10)
        assert info["status_name"] == "breakdown" and info["iters"] == 0
    # [[1, 2], [2, 1]]: Jacobi's iteration matrix has spectral radius 2
    x, info = oracle.jacobi(np.array([[1.0, 2.0], [2.0, 1.0]]), np.array([1.0, 0.0]),
                            tol=1e-10, max_iter=40)
    assert info["status_name"] == "maxiter" and info["rel_res"] > 1e6


def test_gauss_seidel_converges_on_spd_where_jacobi_diverges():
    """SPD with unit diagonal and off-diagonal 0.9: Jacobi's iteration matrix
    has eigenvalue -1.8, while Gauss-Seidel converges for every SPD matrix."""
    n = 3
    A = np.full((n, n), 0.9) + 0.1 * np.eye(n)
    assert np.linalg.eigvalsh(A).min() > 0
    b = np.array([1.0, -2.0, 0.5])
    _, ij = oracle.jacobi(A, b, tol=1e-10, max_iter=200)
    assert ij["status_name"] == "maxiter"
    x, ig = oracle.gauss_seidel(A, b, tol=1e-10, max_iter=2000)
    assert ig["status_name"] == "ok"
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-8)


def test_stein_rosenberg_gauss_seidel_faster_on_m_matrix():
    """For an M-matrix (nonpositive off-diagonals, Jacobi convergent) the
    Gauss-Seidel spectral radius is the smaller: fewer sweeps to a tolerance."""
    rng = np.random.default_rng(6)
    n = 120
    A = -rng.uniform(0, 1, (n, n)) / n
    A[np.arange(n), np.arange(n)] = 0.0
    A[np.arange(n), np.arange(n)] = -A.sum(axis=1) * 1.25
    b = rng.standard_normal(n)
    xj, ij = oracle.jacobi(A, b, tol=1e-12)
    xg, ig = oracle.gauss_seidel(A, b, tol=1e-12)
    assert ij["status_name"] == "ok" and ig["status_name"] == "ok"
    assert ig["iters"] < ij["iters"]
    xs = np.linalg.solve(A, b)
    for x in (xj, xg):
        np.testing.assert_allclose(x, xs, rtol=1e-9, atol=1e-9 * np.abs(xs).max())


def test_stationary_on_the_nonsymmetric_workload():
    p = nonsym_problem(256, seed=0, config_id=0)
    for fn in (oracle.jacobi, oracle.gauss_seidel):
        x, info = fn(p.A, p.b, tol=1e-10)
        assert info["status_name"] == "ok" and info["rel_res"] <= 1e-10
        m = oracle.metrics(p.A, p.b, x)
        assert m["rel_res"] <= 1e-10
        np.testing.assert_allclose(x, p.x_true, rtol=1e-7, atol=1e-8)


# ----------------------------------------- binary32 block LU and GMRES-IR
# The block LU of the direct-methods section in binary32, pinned by the
# componentwise backward-error bound of Gaussian elimination, by the pivots
# of the binary64 GEPP (itself pinned to LAPACK above), by an exactly
# representable factorization it must reproduce bit for bit, blocked or not;
# its application M^-1 by SciPy's triangular solves; GMRES-IR by exactness
# when M = A and by convergence where unpreconditioned GMRES stalls.

def _lu_parts(LU, piv):
    n = LU.shape[0]
    L = np.tril(LU.astype(np.float64), -1) + np.eye(n)
    U = np.triu(LU.astype(np.float64))
    perm = np.arange(n)
    for k, p in enumerate(piv):
        perm[[k, p]] = perm[[p, k]]
    return L, U, perm


@pytest.mark.parametrize("n,b", [(1, 16), (50, 16), (200, 16), (200, 7), (200, 200)])
def test_lu32_backward_error_bound(n, b):
    rng = np.random.default_rng(60 + n + b)
    A = rng.standard_normal((n, n))
    LU, piv, sing = oracle.lu32_block(A, b=b)
    assert sing == 0
    L, U, perm = _lu_parts(LU, piv)
    A32 = A.astype(np.float32).astype(np.float64)
    u = 2.0 ** -24
    gamma = n * u / (1 - n * u)
    err = np.abs(A32[perm] - L @ U)
    assert np.all(err <= gamma * (np.abs(L) @ np.abs(U)) + 1e-300)
    assert np.abs(np.tril(LU, -1)).max(initial=0.0) <= 1.0  # partial pivoting: |l_ij| <= 1


def test_lu32_pivots_match_binary64_gepp():
    for seed in range(3):
        A = np.random.default_rng(70 + seed).standard_normal((120, 120))
        _, piv32, _ = oracle.lu32_block(A, b=16)
        _, piv64, _ = oracle.lu_factor(A)
        np.testing.assert_array_equal(piv32, piv64)


def _exact_lu_system(n, seed):
    """A = L0 U0 with dyadic |l| <= 1/2 (no row interchange) and integer U0:
    every intermediate of elimination is exact in binary32."""
    rng = np.random.default_rng(seed)
    L0 = np.tril(rng.choice([-0.5, -0.25, 0.0, 0.25, 0.5], size=(n, n)), -1) + np.eye(n)
    U0 = np.triu(rng.integers(-3, 4, size=(n, n)).astype(float), 1) + np.diag(rng.choice([-8.0, 8.0], n))
    return L0, U0, L0 @ U0


@pytest.mark.parametrize("b", [1, 4, 16, 24])
def test_lu32_reproduces_an_exact_factorization(b):
    n = 24
    L0, U0, A = _exact_lu_system(n, 80)
    LU, piv, sing = oracle.lu32_block(A, b=b)
    assert sing == 0
    np.testing.assert_array_equal(piv, np.arange(n))
    L, U, _ = _lu_parts(LU, piv)
    np.testing.assert_array_equal(L, L0)
    np.testing.assert_array_equal(U, U0)


def test_lu32_apply_is_the_two_triangular_solves():
    from scipy.linalg import solve_triangular

    n = 150
    A = np.random.default_rng(90).standard_normal((n, n))
    LU, piv, _ = oracle.lu32_block(A, b=16)
    L, U, perm = _lu_parts(LU, piv)
    v = np.random.default_rng(91).standard_normal(n)
    z = oracle.lu32_apply(LU, piv, v)
    ref = solve_triangular(U, solve_triangular(L, v[perm], lower=True, unit_diagonal=True))
    np.testing.assert_allclose(z, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_gmres_ir_lu_exact_preconditioner_and_special_cases():
    n = 24
    _, _, A = _exact_lu_system(n, 81)
    xs = np.random.default_rng(82).standard_normal(n)
    b = A @ xs
    # M = A exactly: one preconditioned GMRES step per refinement step, and
    # the first correction already meets binary64 accuracy
    x, info = oracle.gmres_ir_lu(A, b, tol=1e-14)
    assert info["status_name"] == "ok" and info["outer_iters"] == 1 and info["inner_iters"] == 1
    np.testing.assert_allclose(x, xs, rtol=1e-12)
    x, info = oracle.gmres_ir_lu(A, np.zeros(n), x0=np.ones(n), tol=1e-12)
    assert info["status_name"] == "ok" and info["outer_iters"] == 0 and not x.any()
    S = A.copy()
    S[:, 5] = 0.0
    _, info = oracle.gmres_ir_lu(S, b, tol=1e-12)
    assert info["status_name"] == "breakdown"


def test_gmres_ir_lu_converges_where_gmres_stalls():
    from workloads import nonsym_swept_problem

    p = nonsym_swept_problem(300, 1e6, seed=1, config_id=2)
    _, ig = oracle.gmres(p.A, p.b, tol=1e-10, restart=50, max_iter=1500)
    assert ig["status_name"] == "maxiter"
    x, info = oracle.gmres_ir_lu(p.A, p.b, tol=1e-12)
    assert info["status_name"] == "ok" and info["outer_iters"] <= 4, info
    assert oracle.metrics(p.A, p.b, x)["eta_inf"] <= 1e-12
    xs = np.linalg.solve(p.A, p.b)
    assert np.linalg.norm(x - xs) <= 1e6 * 1e-12 * 10 * np.linalg.norm(xs)


# --------------------------------------- binary32 block Cholesky and CG-IR
# The block Cholesky of the direct-methods section in binary32, pinned by the
# componentwise backward-error bound of the Cholesky factorization, by its
# independence of the block width (every sum subtracts its terms in the same
# order), by an exactly representable factor it must reproduce bit for bit,
# by LAPACK's Cholesky of the same binary32 matrix, and by refusing a matrix
# that is not positive definite; its application by SciPy's triangular
# solves; CG-IR by exactness when M = A and by convergence where plain CG
# needs thousands of iterations.

def _spd32(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    return G @ G.T / n + 0.5 * np.eye(n)


@pytest.mark.parametrize("n,b", [(1, 64), (70, 16), (200, 64), (200, 7), (200, 200)])
def test_chol32_backward_error_bound(n, b):
    A = _spd32(n, 100 + n + b)
    L, notpd = oracle.chol32_block(A, nb=b)
    assert notpd == 0
    L64 = L.astype(np.float64)
    assert not np.triu(L64, 1).any()
    A32 = A.astype(np.float32).astype(np.float64)
    A32 = np.tril(A32) + np.tril(A32, -1).T  # the lower triangle is what is read
    u = 2.0 ** -24
    gamma = (n + 1) * u / (1 - (n + 1) * u)
    err = np.abs(A32 - L64 @ L64.T)
    assert np.all(err <= gamma * (np.abs(L64) @ np.abs(L64).T) + 1e-300)
    assert np.all(np.diag(L64) > 0)


def test_chol32_independent_of_block_width_and_close_to_lapack():
    n = 150
    A = _spd32(n, 110)
    L1, _ = oracle.chol32_block(A, nb=1)
    for b in (2, 16, 64, 149, 150, 1000):
        Lb, s = oracle.chol32_block(A, nb=b)
        assert s == 0
        np.testing.assert_array_equal(Lb, L1)
    # LAPACK's Cholesky of the same binary32 matrix in binary64: the binary32
    # factor is within the perturbation bound of the factor (forward error of
    # order cond(A) n u32)
    A32 = A.astype(np.float32).astype(np.float64)
    A32 = np.tril(A32) + np.tril(A32, -1).T
    Lr = np.linalg.cholesky(A32)
    rel = np.linalg.norm(L1 - Lr) / np.linalg.norm(Lr)
    assert rel <= np.linalg.cond(A32) * n * 2.0 ** -24


def _exact_chol_system(n, seed):
    """A = L0 L0^T with L0 lower, diagonal in {1, 2, 4} and dyadic
    off-diagonal entries small enough that every partial sum is exact in
    binary32: the factorization must return L0 exactly."""
    rng = np.random.default_rng(seed)
    d = rng.choice([1.0, 2.0, 4.0], n)
    L0 = np.tril(rng.choice([-1.0, -0.5, 0.0, 0.5, 1.0], size=(n, n)), -1) * d[None, :] + np.diag(d)
    return L0, L0 @ L0.T


@pytest.mark.parametrize("b", [1, 4, 16, 24])
def test_chol32_reproduces_an_exact_factor(b):
    n = 24
    L0, A = _exact_chol_system(n, 120)
    L, s = oracle.chol32_block(A, nb=b)
    assert s == 0
    np.testing.assert_array_equal(L.astype(np.float64), L0)


def test_chol32_refuses_indefinite_and_reads_the_lower_triangle():
    n = 40
    A = _spd32(n, 130)
    A[17, 17] = -1.0
    _, s = oracle.chol32_block(A, nb=16)
    assert s >= 1 and s <= 18
    # the upper triangle is never read
    B = _spd32(n, 131)
    Bn = B.copy()
    Bn[np.triu_indices(n, 1)] = np.nan
    L1, _ = oracle.chol32_block(B, nb=8)
    L2, _ = oracle.chol32_block(Bn, nb=8)
    np.testing.assert_array_equal(L1, L2)


def test_chol32_apply_is_the_two_triangular_solves():
    from scipy.linalg import solve_triangular

    n = 150
    A = _spd32(n, 140)
    L, _ = oracle.chol32_block(A, nb=32)
    L64 = L.astype(np.float64)
    v = np.random.default_rng(141).standard_normal(n)
    z = oracle.chol32_apply(L, v)
    ref = solve_triangular(L64.T, solve_triangular(L64, v, lower=True), lower=False)
    np.testing.assert_allclose(z, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_cg_ir_chol_exact_preconditioner_and_special_cases():
    n = 24
    _, A = _exact_chol_system(n, 150)
    xs = np.random.default_rng(151).standard_normal(n)
    b = A @ xs
    # M = A exactly: the preconditioned residual z = A^-1 r makes the first
    # PCG step exact, and the first correction meets binary64 accuracy
    x, info = oracle.cg_ir_chol(A, b, tol=1e-14)
    assert info["status_name"] == "ok" and info["outer_iters"] == 1 and info["inner_iters"] == 1
    assert _rel(x, xs) <= np.linalg.cond(A) * 2.0 ** -52
    x, info = oracle.cg_ir_chol(A, np.zeros(n), x0=np.ones(n), tol=1e-12)
    assert info["status_name"] == "ok" and info["outer_iters"] == 0 and not x.any()
    S = A.copy()
    S[3, 3] = -5.0
    _, info = oracle.cg_ir_chol(S, b, tol=1e-12)
    assert info["status_name"] == "breakdown"


def test_cg_ir_chol_converges_in_few_steps_at_high_condition():
    p = spd_problem(300, 1e6, seed=2, config_id=2)
    _, ic = oracle.cg(p.A, p.b, tol=1e-10, max_iter=300)
    assert ic["status_name"] == "maxiter"
    x, info = oracle.cg_ir_chol(p.A, p.b, tol=1e-12)
    assert info["status_name"] == "ok" and info["outer_iters"] <= 5, info
    assert info["inner_iters"] <= 60, info
    assert oracle.metrics(p.A, p.b, x)["eta_inf"] <= 1e-12
    xs = np.linalg.solve(p.A, p.b)
    assert np.linalg.norm(x - xs) <= 1e6 * 1e-12 * 10 * np.linalg.norm(xs)
