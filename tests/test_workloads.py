"""The seeded generators produce the stated systems (CPU)."""
import math

import numpy as np

from workloads import nonsym_problem, nonsym_swept_problem, spd_problem, stream_requests
from workloads.gen import _np_rng


def test_spd_exact_symmetry_and_spectrum():
    kappa = 1e3
    p = spd_problem(256, kappa, seed=0, config_id=0)
    assert np.array_equal(p.A, p.A.T)
    ev = np.linalg.eigvalsh(p.A)
    assert abs(ev[0] - 1.0) <= 1e-11 and abs(ev[-1] / kappa - 1.0) <= 1e-12
    lam = np.sort(np.power(kappa, _pinned(256)))
    # eigenvalues equal the prescribed lambda set (so Q is orthogonal)
    assert np.max(np.abs(np.sort(ev) - lam) / lam) <= 1e-11
    assert np.linalg.norm(p.A @ p.x_true - p.b) <= 1e-12 * np.linalg.norm(p.b)


def _pinned(n):
    u = _np_rng(0, 0, (), 1).random(n)
    u[0], u[-1] = 0.0, 1.0
    return u


def test_seed_reproducibility_and_independence():
    a = spd_problem(64, 10.0, seed=3, config_id=1)
    b = spd_problem(64, 10.0, seed=3, config_id=1)
    c = spd_problem(64, 10.0, seed=4, config_id=1)
    assert np.array_equal(a.A, b.A) and np.array_equal(a.b, b.b)
    assert not np.array_equal(a.A, c.A)


def test_nonsym_structure():
    n = 1024
    p = nonsym_problem(n, seed=0, config_id=1)
    off = p.A - np.diag(np.diag(p.A))
    assert abs(off.std() * math.sqrt(n) - 1.0) < 0.01
    d = np.diag(p.A)
    assert d.min() > 2.0 - 5.0 / math.sqrt(n) and d.max() < 4.0 + 5.0 / math.sqrt(n)
    assert not np.array_equal(p.A, p.A.T)


def test_nonsym_swept_diagonal_span():
    p = nonsym_swept_problem(512, 1e4, seed=0, config_id=2)
    d = np.diag(p.A)
    assert d.min() < 1.2 and d.max() > 1e4 * 0.99


def test_stream_statistics():
    reqs = stream_requests(4096, rate_per_s=100.0, seed=0)
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 256 and ns.max() <= 8192
    mean_log = np.mean(np.log(ns))
    assert abs(mean_log - 0.5 * (math.log(256) + math.log(8192))) < 0.06
    frac_cg = np.mean([r.kind == "cg" for r in reqs])
    assert abs(frac_cg - 0.5) < 0.03
    gaps = np.diff([r.arrival_s for r in reqs])
    assert abs(gaps.mean() - 0.01) < 0.001
    kap = np.array([r.kappa for r in reqs if r.kind == "cg"])
    assert kap.min() >= 1e2 and kap.max() <= 1e5
