#!/usr/bin/env python3
"""Throughput benchmark of the dense Krylov solvers on one MI355X.

One step = one pass of the binary64 hot path over one batch of synthetic
input: a CG solve of the SPD system (n = 16384, cond_2 = 1e4) and a GMRES(30)
solve of the nonsymmetric system A = D + G/sqrt(n) (n = 16384), both from
x0 = 0 to relative residual 1e-10.  The matrices and right-hand sides are
generated on the device before timing (seeded; see workloads/gen.py) and the
solvers are created (A borrowed in place, ||A||_inf computed) before timing.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 16384]

Prints one JSON line (metric, value = solves/s, ...) with
  roofline:      the FP64 GEMV of the CG loop (the dominant kernel):
                 algorithmic bytes per launch / mean launch time measured with
                 HIP events on the library's stream during the timed steps;
  cpu_baseline:  the CPU oracle timed on a bounded sample of the same
                 systems (a few hundred iterations), scaled to the
                 iteration counts of a full step.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E datasheet
PROFILES = os.path.join(ROOT, "profiles")


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


# The solvers time their A*v launches with HIP event pairs on their own
# stream; each pair costs the stream a few microseconds, so only one launch
# in TIMING_EVERY is timed (the first of a solve always is): the launch
# averages come from a sample, the solve times carry almost none of the
# events' cost.
TIMING_EVERY = 16

# sources of the two CG products (general GEMV / symmetric lower-triangle product)
_PRODUCT_SOURCES = {
    "general": ("ks_gemv_body.h", "ks_gemv.hip", "ks_device.h", "ks_internal.h"),
    "symmetric": ("ks_symv.hip", "ks_device.h", "ks_internal.h"),
}
_PRODUCT_PROFILE = {"general": "cg_matvec_f64_n{n}_pmc.txt", "symmetric": "symv_f64_n{n}_pmc.txt"}


def kernel_source_hash(product: str = "general") -> str:
    import hashlib

    h = hashlib.sha256()
    for f in _PRODUCT_SOURCES[product]:
        with open(os.path.join(ROOT, "paper_1511_07207_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def product_bytes(n: int, product: str) -> float:
    """Algorithmic bytes of one timed CG product.  General: A once, p once, q
    once.  Symmetric: the lower triangle once and p once; its finishing launch
    also applies the iteration's update (x and r read and written, q never
    stored), which the same timed pair covers."""
    if product == "general":
        return 8.0 * n * n + 2 * 8.0 * n
    return 8.0 * n * (n + 1) / 2 + 5 * 8.0 * n


def load_traffic(n: int, product: str = "general"):
    """HBM bytes per CG product from the committed rocprofv3 PMC summary, or
    None if there is none for this size or the kernel source changed since."""
    path = os.path.join(PROFILES, _PRODUCT_PROFILE[product].format(n=n))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"^TRAFFIC_JSON (\{.*\})$", txt, re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("kernel_hash") != kernel_source_hash(product):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(spd, ns, cg_iters, gm_iters, steps_done):
    """Time the oracle on a bounded sample and scale to one step's iterations."""
    import numpy as np

    import oracle

    A1 = spd.A.cpu().numpy()
    b1 = spd.b.cpu().numpy()
    A2 = ns.A.cpu().numpy()
    b2 = ns.b.cpu().numpy()
    threads = oracle.get_threads()
    # about 10 s of oracle work on a 16-core host: a whole GMRES solve and up
    # to 1000 CG iterations
    s_cg = max(1, min(cg_iters, 1000))
    s_gm = max(1, gm_iters)
    t = time.perf_counter()
    _, i1 = oracle.cg(A1, b1, tol=1e-300, max_iter=s_cg)
    t_cg = time.perf_counter() - t
    t = time.perf_counter()
    _, i2 = oracle.gmres(A2, b2, tol=1e-300, max_iter=s_gm, restart=30)
    t_gm = time.perf_counter() - t
    est_step = t_cg * cg_iters / i1["iters"] + t_gm * gm_iters / i2["iters"]
    return {
        "value": 2.0 / est_step,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{i1['iters']} CG iterations ({t_cg:.1f} s) and {i2['iters']} GMRES(30) "
                   f"steps ({t_gm:.1f} s) of the same n={spd.n} systems, scaled to one step "
                   f"({cg_iters} CG + {gm_iters} GMRES iterations)"),
        "est_step_s": est_step,
    }


# ------------------------------------------------------------------ extra legs
def _timed(fn):
    import torch

    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t


def leg_c1(dev):
    """Plain CG, n = 512, kappa = 1e3, tol 1e-10, max 512 iterations."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import spd_problem

    p = spd_problem(512, 1e3, seed=0, config_id=0)
    A = torch.from_numpy(p.A).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    s = krylov.Solver(A, method="cg", tol=1e-10, max_iter=512)
    x = torch.zeros(512, dtype=torch.float64, device=dev)
    s.solve(b, out=x.zero_())
    lat, its = [], []
    for _ in range(30):
        (_, info), dt = _timed(lambda: s.solve(b, out=x.zero_()))
        lat.append(dt * 1e3)
        its.append(info["iters"])
    s.close()
    return {"n": 512, "kappa": 1e3, "iters": its[-1], "status": info["status_name"],
            "rel_res": info["rel_res"], "solves_per_s": round(1e3 / statistics.mean(lat), 2),
            "p50_ms": round(_pct(lat, 0.5), 3), "p99_ms": round(_pct(lat, 0.99), 3),
            "us_per_iteration": round(1e3 * statistics.median(lat) / its[-1], 2)}


def leg_c3(dev, n, kappa, spd_form="qr"):
    """Mixed precision vs binary64 at equal accuracy (backward error 1e-12)."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_swept_problem, spd_problem

    out = {"n": n, "eta_target": 1e-12}
    cases = [("spd_cg", kappa, "cg"), ("nonsym_gmres50", 1e2, "gmres")]
    for name, kap, method in cases:
        if method == "cg":
            prob = spd_problem(n, kap, seed=0, config_id=2, backend="torch", device="cuda",
                               q_form=spd_form)
        else:
            prob = nonsym_swept_problem(n, kap, seed=0, config_id=2, backend="torch", device="cuda")
        res = {"kappa": kap}
        # SPD: also binary64 and binary32-refined solves on the lower triangle
        # (the symmetric products: half the bytes per product)
        precs = ("fp64", "fp32", "bf16") + (("fp64_sym", "fp32_sym") if method == "cg" else ())
        for key in precs:
            prec, sym = key.split("_")[0], key.endswith("_sym")
            kw = dict(method=method, tol=1e-12, restart=50, timing=True, timing_every=TIMING_EVERY,
                      max_iter=4 * n, symmetric=sym)
            if prec == "fp64":
                kw["stop_backward"] = True
            else:
                kw["precision"] = prec
            (solver), tc = _timed(lambda: krylov.Solver(prob.A, **kw))
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            (_, info), dt = _timed(lambda: solver.solve(prob.b, out=x))
            # bytes per element of the timed matrix-vector products (mixed if a
            # bfloat16 solve fell back to binary32)
            e = {"fp64": 8, "fp32": 4, "bf16": 2}[prec] if info["precision_used"] == prec else None
            r = {"solves_per_s": round(1.0 / dt, 4), "solve_ms": round(dt * 1e3, 2),
                 "create_ms": round(tc * 1e3, 2), "status": info["status_name"],
                 "iters": info["iters"], "outer": info["outer_iters"],
                 "precision_used": info["precision_used"], "eta_inf": info["backward_err"],
                 "rel_res": info["rel_res"]}
            if e and info["gemv_calls"]:
                # algorithmic bytes of A per product: all of it, or the lower triangle
                ab = e * n * (n + 1) / 2 if sym else e * n * n
                r["gemv_gbs"] = round(ab / (info["gemv_ms"] / info["gemv_calls"] * 1e-3) / 1e9, 1)
            r["fwd_err_vs_x_true"] = float((x - prob.x_true).norm() / prob.x_true.norm())
            res[key] = r
            solver.close()
            del x
        f64 = res["fp64"]["solves_per_s"]
        for key in precs[1:]:
            res[key]["speedup_vs_fp64"] = round(res[key]["solves_per_s"] / f64, 3)
        out[name] = res
        del prob
        torch.cuda.empty_cache()
    return out


def leg_f1(dev, n):
    """BiCGSTAB on the nonsymmetric n = 16384 system of the main step, beside
    GMRES(30) on the same system: binary64 at relative residual 1e-10, then
    binary64 vs binary32 / bfloat16 inner solves at backward error 1e-12."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_problem

    prob = nonsym_problem(n, seed=0, config_id=1, backend="torch", device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    out = {"n": n, "system": "D + G/sqrt(n), D uniform in [2,4]"}
    runs = [("bicgstab_fp64", dict(method="bicgstab", tol=1e-10)),
            ("gmres30_fp64", dict(method="gmres", restart=30, tol=1e-10)),
            ("bicgstab_fp64_eta", dict(method="bicgstab", tol=1e-12, stop_backward=True)),
            ("bicgstab_fp32_eta", dict(method="bicgstab", tol=1e-12, precision="fp32")),
            ("bicgstab_bf16_eta", dict(method="bicgstab", tol=1e-12, precision="bf16"))]
    for name, kw in runs:
        s = krylov.Solver(prob.A, timing=True, timing_every=TIMING_EVERY, **kw)
        s.solve(prob.b, out=x.zero_())
        lat = []
        for _ in range(5):
            (_, info), dt = _timed(lambda: s.solve(prob.b, out=x.zero_()))
            lat.append(dt * 1e3)
        e = {"fp64": 8, "fp32": 4, "bf16": 2}[info["precision_used"]]
        r = {"status": info["status_name"], "iters": info["iters"], "outer": info["outer_iters"],
             "precision_used": info["precision_used"], "rel_res": info["rel_res"],
             "eta_inf": info["backward_err"], "solves_per_s": round(1e3 / statistics.mean(lat), 3),
             "p50_ms": round(_pct(lat, 0.5), 3)}
        if info["gemv_calls"] and info["outer_iters"] == 0:
            r["gemv_gbs"] = round((e * n * n + 16.0 * n) / (info["gemv_ms"] / info["gemv_calls"] * 1e-3) / 1e9, 1)
        out[name] = r
        s.close()
    out["bicgstab_over_gmres30"] = round(out["bicgstab_fp64"]["solves_per_s"]
                                         / out["gmres30_fp64"]["solves_per_s"], 3)
    for prec in ("fp32", "bf16"):
        out[f"bicgstab_{prec}_speedup_vs_fp64"] = round(
            out[f"bicgstab_{prec}_eta"]["solves_per_s"] / out["bicgstab_fp64_eta"]["solves_per_s"], 3)
    del prob, x
    return out


def leg_f3(dev, n):
    """Jacobi and Gauss-Seidel on the nonsymmetric n = 16384 system of the main
    step (D + G/sqrt(n), Jacobi spectral radius about 0.36), binary64 to
    relative residual 1e-10, beside GMRES(30) on the same system; then the
    four methods the paper times (Jacobi, Gauss-Seidel, GMRES(35), BiCGSTAB)
    at its tolerance 1e-4 over its size range."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_problem

    def run(prob, m, kw, reps):
        x = torch.zeros(m, dtype=torch.float64, device=dev)
        s = krylov.Solver(prob.A, timing=True, timing_every=TIMING_EVERY, **kw)
        s.solve(prob.b, out=x.zero_())
        lat = []
        for _ in range(reps):
            (_, info), dt = _timed(lambda: s.solve(prob.b, out=x.zero_()))
            lat.append(dt * 1e3)
        s.close()
        t = statistics.median(lat)
        r = {"status": info["status_name"], "iters": info["iters"], "rel_res": info["rel_res"],
             "p50_ms": round(t, 3), "solves_per_s": round(1e3 / statistics.mean(lat), 3)}
        if kw["method"] in ("jacobi", "gauss_seidel") and info["iters"]:
            # each update reads A once (Jacobi: the product; Gauss-Seidel: the
            # strict upper product and the substitution's lower triangle)
            r["ms_per_update"] = round(t / info["iters"], 4)
            r["update_gbs"] = round(8.0 * m * m * info["iters"] / (t * 1e-3) / 1e9, 1)
        return r

    prob = nonsym_problem(n, seed=0, config_id=1, backend="torch", device="cuda")
    out = {"n": n, "system": "D + G/sqrt(n), D uniform in [2,4]", "tol": 1e-10}
    for name, kw in (("jacobi", dict(method="jacobi", tol=1e-10)),
                     ("gauss_seidel", dict(method="gauss_seidel", tol=1e-10)),
                     ("gmres30", dict(method="gmres", restart=30, tol=1e-10))):
        out[name] = run(prob, n, kw, 5)
    del prob
    sweep = {}
    for m in (2000, 8000, 16000):
        prob = nonsym_problem(m, seed=0, config_id=1, backend="torch", device="cuda")
        row = {}
        for name, kw in (("jacobi", dict(method="jacobi")), ("gauss_seidel", dict(method="gauss_seidel")),
                         ("gmres35", dict(method="gmres", restart=35)), ("bicgstab", dict(method="bicgstab"))):
            r = run(prob, m, dict(kw, tol=1e-4), 5)
            row[name] = {"iters": r["iters"], "p50_ms": r["p50_ms"], "status": r["status"]}
        sweep[str(m)] = row
        del prob
    out["paper_tolerance_1e-4"] = sweep
    torch.cuda.empty_cache()
    return out


def leg_f4(dev):
    """GMRES-IR with the binary32 block LU: the factorization (in create) at
    the paper's direct-method sizes, and solves of the nonsymmetric kappa = 1e6
    family to backward error 1e-12, beside binary64 GMRES(50) on the same
    systems (which stalls there)."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_swept_problem

    out = {"system": "diag(lambda) + 0.25 G/sqrt(n), lambda log-uniform [1, kappa]",
           "kappa": 1e6, "eta_target": 1e-12}
    for m in (1000, 2000, 3000, 4096):
        prob = nonsym_swept_problem(m, 1e6, seed=0, config_id=8, backend="torch", device="cuda")
        x = torch.zeros(m, dtype=torch.float64, device=dev)
        creates = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s = krylov.Solver(prob.A, method="gmres", restart=30, precision="lu32", tol=1e-12)
            torch.cuda.synchronize()
            creates.append((time.perf_counter() - t0) * 1e3)
            if len(creates) < 3:
                s.close()
        s.solve(prob.b, out=x.zero_())
        lat = []
        for _ in range(3):
            (_, info), dt = _timed(lambda: s.solve(prob.b, out=x.zero_()))
            lat.append(dt * 1e3)
        s.close()
        tc = statistics.median(creates)
        r = {"create_ms": round(tc, 3),
             "factor_gflops": round(2.0 * m ** 3 / 3.0 / (tc * 1e-3) / 1e9, 1),
             "status": info["status_name"], "outer": info["outer_iters"], "inner": info["iters"],
             "eta_inf": info["backward_err"], "solve_ms": round(statistics.median(lat), 3)}
        s64 = krylov.Solver(prob.A, method="gmres", restart=50, tol=1e-12, stop_backward=True,
                            max_iter=1500)
        (_, i64), dt = _timed(lambda: s64.solve(prob.b, out=x.zero_()))
        s64.close()
        r["gmres50_fp64"] = {"status": i64["status_name"], "iters": i64["iters"],
                             "eta_inf": i64["backward_err"], "ms": round(dt * 1e3, 3)}
        out[str(m)] = r
        del prob, x
    torch.cuda.empty_cache()
    return out


def leg_c2p(dev, n):
    """The CG solve of the main step with either product: general GEMV (all of
    A per iteration) and the symmetric lower-triangle product."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import spd_problem

    prob = spd_problem(n, 1e4, seed=0, config_id=1, backend="torch", device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    out = {"n": n, "kappa": 1e4}
    for prod in ("general", "symmetric"):
        s = krylov.Solver(prob.A, method="cg", tol=1e-10, timing=True, timing_every=TIMING_EVERY, symmetric=(prod == "symmetric"))
        s.solve(prob.b, out=x.zero_())
        lat = []
        for _ in range(3):
            (_, info), dt = _timed(lambda: s.solve(prob.b, out=x.zero_()))
            lat.append(dt * 1e3)
        out[prod] = {"status": info["status_name"], "iters": info["iters"], "rel_res": info["rel_res"],
                     "solve_ms": round(statistics.median(lat), 2),
                     "product_ms": round(info["gemv_ms"] / max(info["gemv_calls"], 1), 4),
                     "product_gbs_algorithmic": round(product_bytes(n, prod) / (info["gemv_ms"] / max(info["gemv_calls"], 1) * 1e-3) / 1e9, 1)}
        s.close()
    out["symmetric_speedup"] = round(out["general"]["solve_ms"] / out["symmetric"]["solve_ms"], 3)
    del prob, x
    return out


def leg_c4(dev, n):
    """Lockstep CG on 64 right-hand sides (A*P on MFMA)."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import multi_rhs_problem

    s = 64
    prob = multi_rhs_problem(n, 1e4, s, seed=0, backend="torch", device="cuda")
    out = {"n": n, "nrhs": s, "kappa": 1e4}
    for prec, tol, peak in (("fp64", 1e-10, 78.6), ("fp32", 1e-12, 157.3)):
        solver = krylov.Solver(prob.A, method="cg", nrhs=s, tol=tol, precision=prec, timing=True, timing_every=TIMING_EVERY,
                               max_iter=4 * n)
        solver.solve(prob.b)
        (X, info), dt = _timed(lambda: solver.solve(prob.b))
        ms = info["gemv_ms"] / max(info["gemv_calls"], 1)
        tf = 2.0 * n * n * s / (ms * 1e-3) / 1e12
        out[prec] = {"solves_per_s": round(s / dt, 2), "status": info["status_name"],
                     "lockstep_iters": info["iters"], "outer": info["outer_iters"],
                     "max_rel_res": info["rel_res"], "max_eta_inf": info["backward_err"],
                     "gemm_ms": round(ms, 4), "gemm_tflops": round(tf, 2),
                     "mfma_peak_tflops": peak, "mfma_frac": round(tf / peak, 4)}
        solver.close()
    return out


def leg_c5(dev, count, pool_size, seed=0):
    """Serving: binary64 against mixed-precision requests at equal accuracy
    (normwise backward error <= 1e-12), over a pool of resident systems.
    Saturation throughput of each, then both under the same Poisson arrivals
    at 0.5x and 0.9x of the binary64 saturation rate (p50 / p99 latency)."""
    import math

    import numpy as np
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_problem, spd_problem

    rng = np.random.default_rng([seed, 4, 99])
    pool = []
    for i in range(pool_size):
        n = int(round(math.exp(rng.uniform(math.log(256), math.log(8192)))))
        if i % 2 == 0:
            kap = float(math.exp(rng.uniform(math.log(1e2), math.log(1e5))))
            prob = spd_problem(n, kap, seed=seed, config_id=4, key=(i,), backend="torch", device="cuda")
            pool.append(("cg", prob, kap))
        else:
            prob = nonsym_problem(n, seed=seed, config_id=4, key=(i,), backend="torch", device="cuda")
            pool.append(("gmres", prob, None))

    def kw_for(kind, kap, mode):
        kw = dict(method=kind, tol=1e-12)
        if kind == "gmres":
            kw["restart"] = 30
        if mode == "fp64":
            kw["stop_backward"] = True
        else:
            # inner precision: bfloat16 where its copy stays usable (GMRES on
            # D + G/sqrt(n); SPD up to kappa ~ 3e2), binary32 otherwise
            kw["precision"] = "bf16" if (kind == "gmres" or kap <= 3e2) else "fp32"
        return kw

    # request i: pool entry, fresh right-hand side b = A x_true
    reqs = []
    g = torch.Generator(device="cuda")
    g.manual_seed(seed * 1000003 + 17)
    order = rng.permutation(np.arange(count) % pool_size)
    for i in range(count):
        kind, prob, kap = pool[int(order[i])]
        xt = torch.randn(prob.n, dtype=torch.float64, device=dev, generator=g)
        reqs.append((kind, prob, kap, prob.A @ xt))
    torch.cuda.synchronize()

    def run(arrivals, mode):
        srv = krylov.Server(mem_budget_bytes=64 << 30, max_inflight=1024, chunk=16)
        t0 = time.perf_counter()
        pending = list(range(count))
        lat, statuses, etas, precs, peak_inflight = [], [], [], {}, 0
        tick_of = {}
        while True:
            now = time.perf_counter() - t0
            while pending and arrivals[pending[0]] <= now:
                i = pending.pop(0)
                kind, prob, kap, b = reqs[i]
                tick_of[srv.submit(prob.A, b, **kw_for(kind, kap, mode))] = i
            a, q = srv.step()
            peak_inflight = max(peak_inflight, a)
            done_t = time.perf_counter() - t0
            for t, x, info in srv.poll():
                lat.append(done_t - arrivals[tick_of[t]])
                statuses.append(info["status"])
                etas.append(info["backward_err"])
                precs[info["precision_used"]] = precs.get(info["precision_used"], 0) + 1
            if not pending and a == 0 and q == 0:
                break
            if a == 0 and q == 0 and pending:
                wait = arrivals[pending[0]] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
        total = time.perf_counter() - t0
        srv.close()
        lat_ms = [v * 1e3 for v in lat]
        return {"requests": count, "wall_s": round(total, 3),
                "throughput_req_per_s": round(count / total, 2),
                "p50_ms": round(_pct(lat_ms, 0.5), 2), "p99_ms": round(_pct(lat_ms, 0.99), 2),
                "all_ok": all(s == 0 for s in statuses) and len(statuses) == count,
                "max_backward_err": max(etas) if etas else None,
                "precision_used": precs, "peak_inflight": peak_inflight}

    out = {"pool": pool_size, "n_range": [256, 8192], "eta_target": 1e-12}
    sat64 = run([0.0] * count, "fp64")
    satmx = run([0.0] * count, "mixed")
    out["saturation"] = {"fp64": sat64, "mixed": satmx,
                         "mixed_over_fp64": round(satmx["throughput_req_per_s"]
                                                  / sat64["throughput_req_per_s"], 3)}
    lam = sat64["throughput_req_per_s"]
    for frac in (0.5, 0.9):
        gaps = rng.exponential(1.0 / (frac * lam), size=count)
        arr = list(np.cumsum(gaps) - gaps[0])
        out[f"rate_{frac}_of_fp64_saturation"] = {
            "offered_req_per_s": round(frac * lam, 2),
            "fp64": run(arr, "fp64"), "mixed": run(arr, "mixed")}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--spd-form", choices=("qr", "identity"), default="qr",
                    help="Q of the SPD matrix: QR of a Gaussian (default) or the identity "
                         "(same spectrum and bytes; for hardware-counter runs)")
    ap.add_argument("--legs", default="c1,c2p,c3,c4,c5,f1,f3,f4",
                    help="extra measurements after the timed steps (comma list of "
                         "c1,c2p,c3,c4,c5,f1,f3,f4; 'none' for the main step only)")
    ap.add_argument("--n3", type=int, default=32768, help="size of the mixed-precision leg")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-pool", type=int, default=32)
    ap.add_argument("--cg-product", choices=("symmetric", "general"), default="symmetric",
                    help="CG product: the symmetric kernel reading the lower triangle of A "
                         "(KS_FLAG_SYMMETRIC) or the general GEMV")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="before timing, copy A once with the library's binary64 copy kernel "
                         "(known bytes: 8 n^2 read + 8 n^2 written) to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library solves on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_problem, spd_problem

    dev = torch.device("cuda:0")
    n = args.n
    t0 = time.perf_counter()
    spd = spd_problem(n, 1e4, seed=0, config_id=1, backend="torch", device="cuda",
                      q_form=args.spd_form)
    ns = nonsym_problem(n, seed=0, config_id=1, backend="torch", device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated n={n} systems in {gen_s:.1f}s", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    sym = args.cg_product == "symmetric"
    cg = krylov.Solver(spd.A, method="cg", tol=1e-10, timing=True, timing_every=TIMING_EVERY, symmetric=sym)
    gm = krylov.Solver(ns.A, method="gmres", restart=30, tol=1e-10, timing=True, timing_every=TIMING_EVERY)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    xcg = torch.zeros(n, dtype=torch.float64, device=dev)
    xgm = torch.zeros(n, dtype=torch.float64, device=dev)
    # measured HBM read ceiling: the library's streaming-read kernel over A
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    krylov.read_ceiling(spd.A, sink)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        krylov.read_ceiling(spd.A, sink)
    ev1.record()
    torch.cuda.synchronize()
    read_ceiling_gbs = 8.0 * n * n / (ev0.elapsed_time(ev1) / 10 * 1e-3) / 1e9
    if args.calibration_copy:
        copy = krylov.convert(spd.A, torch.float64)
        torch.cuda.synchronize()
        del copy

    def step():
        xcg.zero_()
        t = time.perf_counter()
        _, icg = cg.solve(spd.b, out=xcg)
        t1 = time.perf_counter()
        xgm.zero_()
        _, igm = gm.solve(ns.b, out=xgm)
        t2 = time.perf_counter()
        return icg, igm, (t1 - t) * 1e3, (t2 - t1) * 1e3

    for w in range(args.warmup):
        step()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for k in range(args.steps):
        recs.append(step())
        print(f"[bench] step {k + 1}/{args.steps}: cg {recs[-1][2]:.1f} ms "
              f"({recs[-1][0]['iters']} it), gmres {recs[-1][3]:.1f} ms "
              f"({recs[-1][1]['iters']} it)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ok = all(r[0]["status"] == 0 and r[1]["status"] == 0 and r[0]["rel_res"] <= 1e-10
             and r[1]["rel_res"] <= 1e-10 for r in recs)
    solves = 2 * args.steps
    value = solves / elapsed
    ms_step = elapsed * 1e3 / args.steps
    # dominant kernel: the FP64 product of the CG loop, q = A p (the symmetric
    # product is two launches: the tiles of the lower triangle, then the
    # finishing sum that also applies the iteration's x and r update)
    gemv_ms = sum(r[0]["gemv_ms"] for r in recs)
    gemv_calls = sum(r[0]["gemv_calls"] for r in recs)
    gm_gemv_ms = sum(r[1]["gemv_ms"] for r in recs)
    gm_gemv_calls = sum(r[1]["gemv_calls"] for r in recs)
    bytes_per_launch = product_bytes(n, args.cg_product)
    gm_bytes = product_bytes(n, "general")
    avg_ms = gemv_ms / max(gemv_calls, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic(n, args.cg_product)
    cg_iters = recs[-1][0]["iters"]
    gm_iters = recs[-1][1]["iters"]
    out = {
        "metric": "solves/s (FP64 CG + GMRES(30), n=16384, rel. residual 1e-10)",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"CG on SPD n={n} (Q diag(lambda) Q^T, lambda log-uniform [1,1e4]) + "
                         f"GMRES(30) on D + G/sqrt(n), n={n}; x0=0, tol 1e-10; one of each per step"),
            "n": n, "kappa_spd": 1e4, "restart": 30, "tol": 1e-10, "spd_q": args.spd_form,
            "cg_product": ("symmetric: lower triangle of A read once per iteration"
                           if sym else "general: all of A read once per iteration"),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("symv_tile_kernel + symv_cg_finish_kernel "
                       "(q = A p from the lower triangle, fused with x += alpha p, r -= alpha q)"
                       if sym else
                       "cg_matvec_kernel<double> (q = A p, p'q partials)"),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "read_ceiling_gbs": round(read_ceiling_gbs, 1),
            "frac_of_read_ceiling": round(achieved / read_ceiling_gbs, 4),
            "traffic": traffic,
            "bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": round(avg_ms, 5),
            "launches": gemv_calls,
        },
        "valid": ok,
        "solves": {
            "cg": {"iters": cg_iters, "rel_res": recs[-1][0]["rel_res"],
                   "backward_err": recs[-1][0]["backward_err"],
                   "p50_ms": round(_pct([r[2] for r in recs], 0.5), 3),
                   "p99_ms": round(_pct([r[2] for r in recs], 0.99), 3)},
            "gmres": {"iters": gm_iters, "rel_res": recs[-1][1]["rel_res"],
                      "backward_err": recs[-1][1]["backward_err"],
                      "p50_ms": round(_pct([r[3] for r in recs], 0.5), 3),
                      "p99_ms": round(_pct([r[3] for r in recs], 0.99), 3),
                      "gemv_gbs": round(gm_bytes / (gm_gemv_ms / max(gm_gemv_calls, 1) * 1e-3) / 1e9, 1)},
        },
        "iterations_per_s": round((cg_iters + gm_iters) * args.steps / elapsed, 1),
        "create_ms": round(create_ms, 2),
        "generate_s": round(gen_s, 2),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(spd, ns, cg_iters, gm_iters, args.steps)
    else:
        out["cpu_baseline"] = None
    cg.close()
    gm.close()
    del spd, ns
    torch.cuda.empty_cache()
    legs = {}
    wanted = [] if args.legs == "none" else [x.strip() for x in args.legs.split(",") if x.strip()]
    for name in wanted:
        print(f"[bench] leg {name} ...", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        try:
            if name == "c1":
                legs[name] = leg_c1(dev)
            elif name == "c3":
                legs[name] = leg_c3(dev, args.n3, 1e4, args.spd_form)
            elif name == "c4":
                legs[name] = leg_c4(dev, n)
            elif name == "c5":
                legs[name] = leg_c5(dev, args.serve_requests, args.serve_pool)
            elif name == "f1":
                legs[name] = leg_f1(dev, n)
            elif name == "f3":
                legs[name] = leg_f3(dev, n)
            elif name == "f4":
                legs[name] = leg_f4(dev)
            elif name == "c2p":
                legs[name] = leg_c2p(dev, n)
            else:
                legs[name] = {"error": "unknown leg"}
        except Exception as e:  # a failing leg is reported, not fatal
            legs[name] = {"error": f"{type(e).__name__}: {e}"}
        legs.setdefault(name, {})["leg_wall_s"] = round(time.perf_counter() - t0, 1)
        print(f"[bench] leg {name} done in {legs[name]['leg_wall_s']}s", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    out["legs"] = legs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
