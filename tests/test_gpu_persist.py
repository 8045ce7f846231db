"""Persistent small-n CG (one cooperative launch with a grid barrier between
iterations, n <= 1024) against the per-launch fused path it replaces
(KS_FLAG_NO_PERSIST): the same iterates bit for bit -- x, the iteration
count, the status and the reported residuals -- and, through the existing
parity tests, the oracle's solution.  Sizes cover one block of eight rows,
ragged last blocks, the 256- and 512-column chunks and the largest order the
persistent form takes; statuses cover convergence, the iteration limit, a
breakdown on an indefinite matrix, b = 0 and a non-finite b."""
import numpy as np
import pytest

import oracle
from workloads import spd_problem

pytestmark = pytest.mark.gpu


def _t(x, device):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).to(device)


def _both(A, b, device, **kw):
    from paper_1511_07207_amd import krylov

    out = []
    for persist in (True, False):
        x, info = krylov.solve(_t(A, device), _t(b, device), method="cg", persist=persist, **kw)
        out.append((x.cpu().numpy(), info))
    return out


def _same(a, b):
    (xa, ia), (xb, ib) = a, b
    assert np.array_equal(xa.view(np.int64), xb.view(np.int64))
    for k in ("status", "iters", "restarts"):
        assert ia[k] == ib[k], (k, ia, ib)
    for k in ("rel_res", "backward_err"):
        assert ia[k] == ib[k] or (np.isnan(ia[k]) and np.isnan(ib[k])), (k, ia, ib)


@pytest.mark.parametrize("n,kappa,seed", [(1, 1.0, 0), (7, 10.0, 1), (8, 10.0, 2), (64, 1e2, 3),
                                          (257, 1e2, 4), (300, 1e3, 5), (512, 1e3, 0),
                                          (777, 1e4, 6), (1023, 1e3, 7), (1024, 1e3, 8)])
def test_persistent_cg_bitwise_equal_to_per_launch(device, n, kappa, seed):
    print(f"persistent cg n={n} kappa={kappa:g} seed={seed}", flush=True)
    p = spd_problem(n, kappa, seed=seed, config_id=0)
    r = _both(p.A, p.b, device, tol=1e-10, max_iter=10 * n + 10)
    _same(*r)
    x, info = r[0]
    assert info["status"] == 0, info
    assert oracle.metrics(p.A, p.b, x)["rel_res"] <= 1e-10


def test_persistent_cg_c1_workload(device):
    """The latency workload: n = 512, cond 1e3, tol 1e-10, at most 512 iterations."""
    print("persistent cg C1 n=512", flush=True)
    p = spd_problem(512, 1e3, seed=0, config_id=0)
    r = _both(p.A, p.b, device, tol=1e-10, max_iter=512)
    _same(*r)
    xo, io = oracle.cg(p.A, p.b, tol=1e-10, max_iter=512)
    x, info = r[0]
    assert info["status"] == 0 and abs(info["iters"] - io["iters"]) <= max(2, io["iters"] // 100)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-8


def test_persistent_cg_iteration_limit(device):
    print("persistent cg max_iter", flush=True)
    p = spd_problem(600, 1e4, seed=9, config_id=0)
    r = _both(p.A, p.b, device, tol=1e-12, max_iter=37)
    _same(*r)
    assert r[0][1]["status_name"] == "maxiter" and r[0][1]["iters"] == 37


def test_persistent_cg_breakdown_and_special_inputs(device):
    print("persistent cg breakdown / b = 0 / NaN", flush=True)
    rng = np.random.default_rng(10)
    n = 200
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(-1.0, 2.0, n)
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    b = rng.standard_normal(n)
    r = _both(A, b, device, tol=1e-10, max_iter=4 * n)
    _same(*r)
    assert r[0][1]["status_name"] in ("breakdown", "maxiter", "ok")
    p = spd_problem(100, 10.0, seed=11, config_id=0)
    r = _both(p.A, np.zeros(100), device, tol=1e-10)
    _same(*r)
    assert r[0][1]["iters"] == 0 and not np.any(r[0][0])
    bn = p.b.copy()
    bn[3] = np.nan
    r = _both(p.A, bn, device, tol=1e-10)
    assert r[0][1]["status_name"] == r[1][1]["status_name"] == "nonfinite"


def test_persistent_cg_repeated_solves_bitwise(device):
    """A solver reused for several right-hand sides: the barrier flags start
    from zero in every launch."""
    import torch

    from paper_1511_07207_amd import krylov

    print("persistent cg repeated solves", flush=True)
    p = spd_problem(512, 1e3, seed=12, config_id=0)
    A = _t(p.A, device)
    s = krylov.Solver(A, method="cg", tol=1e-10)
    outs = []
    for _ in range(3):
        x = torch.zeros(512, dtype=torch.float64, device=device)
        _, info = s.solve(_t(p.b, device), out=x)
        outs.append((x.cpu().numpy(), info))
    s.close()
    for o in outs[1:]:
        _same(outs[0], o)
