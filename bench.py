#!/usr/bin/env python3
"""Throughput benchmark of the dense Krylov solvers on one MI355X.

One step = one pass of the mixed-precision refinement path over the
refinement workload at n = 32768, cond = 1e4 (seeded, synthetic; see
workloads/gen.py):
  * SPD A = Q diag(lambda) Q^T, lambda log-uniform on [1, 1e4]: CG inner
    solves on the binary32 copy of A, reading its lower triangle;
  * nonsymmetric A = diag(lambda) + 0.25 G / sqrt(n), lambda log-uniform on
    [1, 1e4]: GMRES(50) inner solves on the bfloat16 copy of A;
with the residual, the update and GMRES's Givens rotations in binary64, from
x0 = 0 to normwise backward error eta_inf <= 1e-12.  The matrices and
right-hand sides are generated on the device and the solvers created (copies
made, ||A||_inf computed) before timing; `value` = solves/s over the timed
steps.  Beside it, the same two systems solved in binary64 (CG on the lower
triangle, GMRES(50)) stopping on the same backward error.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 32768]

Prints one JSON line (metric, value = mixed solves/s, ...) with
  roofline:      the product that takes most of a step's time: algorithmic
                 bytes per launch / mean launch time from HIP events on the
                 library's stream during the timed steps;
  cpu_baseline:  the binary64 CPU oracle on a bounded sample of the same two
                 systems (products of CG and GMRES(50)), scaled to the
                 iterations a binary64 solve to the same backward error takes.
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
# Relative tolerance of an inner solve on the bfloat16 copy: 8 units of
# bfloat16 roundoff (2^-8).  The copy perturbs A by about that much relative,
# so each refinement step can gain only a couple of digits whatever the inner
# solve does; running it further (the library's 1e-4 default, kept for
# binary32 copies, whose error is far below it) only costs products.
BF16_INNER_TOL = 2.0 ** -5

# sources of the timed products, and the committed counter summaries of each
_PRODUCT_SOURCES = {
    "general": ("ks_gemv_body.h", "ks_gemv.hip", "ks_device.h", "ks_internal.h"),
    "symmetric": ("ks_symv.hip", "ks_device.h", "ks_internal.h"),
    "symmetric32": ("ks_symv32.hip", "ks_device.h", "ks_internal.h"),
    "gmres_bf16": ("ks_gemv_body.h", "ks_gemv.hip", "ks_device.h", "ks_internal.h"),
}
_PRODUCT_PROFILE = {"general": "cg_matvec_f64_n{n}_pmc.txt", "symmetric": "symv_f64_n{n}_pmc.txt",
                    "symmetric32": "symv32_f32_n{n}_pmc.txt",
                    "gmres_bf16": "gm_matvec_bf16_n{n}_pmc.txt"}
_PRODUCT_KERNEL = {
    "general": "cg_matvec_kernel<double> (q = A p, p'q partials)",
    "symmetric": ("symv_tile_kernel + symv_cg_finish_kernel (q = A p from the lower triangle, "
                  "fused with x += alpha p, r -= alpha q)"),
    "symmetric32": ("symv32_tile_kernel + symv32_cg_finish_kernel (binary32 q = A p from the lower "
                    "triangle of the binary32 copy, fused with the inner CG's x, r update)"),
    "gmres_bf16": ("gm_matvec_kernel<bf16> (w = A v_k on the bfloat16 copy, binary32 "
                   "accumulation, ||w||^2 partials)"),
}


def kernel_source_hash(product: str = "general") -> str:
    import hashlib

    h = hashlib.sha256()
    for f in _PRODUCT_SOURCES[product]:
        with open(os.path.join(ROOT, "paper_1511_07207_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def product_bytes(n: int, product: str) -> float:
    """Algorithmic bytes of one timed product launch.
    general (binary64): A once, p in, q out.
    symmetric (binary64): the lower triangle once and p once; its finishing
      launch also applies the iteration's update (x and r read and written,
      q never stored), which the same timed pair covers.
    symmetric32: the same in binary32.
    gmres_bf16: the bfloat16 A once, v_k in and w out in binary32."""
    if product == "general":
        return 8.0 * n * n + 2 * 8.0 * n
    if product == "symmetric":
        return 8.0 * n * (n + 1) / 2 + 5 * 8.0 * n
    if product == "symmetric32":
        return 4.0 * n * (n + 1) / 2 + 5 * 4.0 * n
    if product == "gmres_bf16":
        return 2.0 * n * n + 2 * 4.0 * n
    raise ValueError(product)


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


def cpu_baseline(spd, ns, cg_iters, gm_iters):
    """Time the oracle on a bounded sample of the step's two systems (CG and
    GMRES(50) products in binary64), at all host threads and at one, and
    scale to the products of a binary64 solve to the same backward error."""
    import oracle

    A1 = spd.A.cpu().numpy()
    b1 = spd.b.cpu().numpy()
    A2 = ns.A.cpu().numpy()
    b2 = ns.b.cpu().numpy()
    threads = oracle.get_threads()
    res = {}
    for label, th, k in (("all_threads", threads, 12), ("one_thread", 1, 2)):
        oracle.set_threads(th)
        t = time.perf_counter()
        _, i1 = oracle.cg(A1, b1, tol=1e-300, max_iter=k)
        t_cg = time.perf_counter() - t
        t = time.perf_counter()
        _, i2 = oracle.gmres(A2, b2, tol=1e-300, max_iter=k, restart=50)
        t_gm = time.perf_counter() - t
        est = t_cg * cg_iters / i1["iters"] + t_gm * gm_iters / i2["iters"]
        res[label] = {"threads": th, "cg_products": i1["iters"], "cg_s": round(t_cg, 2),
                      "gmres_products": i2["iters"], "gmres_s": round(t_gm, 2),
                      "est_step_s": round(est, 2), "solves_per_s": 2.0 / est}
    oracle.set_threads(threads)
    allt = res["all_threads"]
    return {
        "value": allt["solves_per_s"],
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{allt['cg_products']} CG and {allt['gmres_products']} GMRES(50) products of the "
                   f"step's two n={spd.n} systems in binary64 ({allt['cg_s'] + allt['gmres_s']:.1f} s "
                   f"on {threads} threads), scaled to the {cg_iters} + {gm_iters} products a binary64 "
                   f"solve of each to eta_inf <= 1e-12 takes"),
        "est_step_s": allt["est_step_s"],
        "one_thread": {"value": res["one_thread"]["solves_per_s"], "cores": 1,
                       "sample": (f"{res['one_thread']['cg_products']} CG and "
                                  f"{res['one_thread']['gmres_products']} GMRES(50) products, "
                                  f"same scaling"),
                       "est_step_s": res["one_thread"]["est_step_s"]},
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
    """Plain CG, n = 512, kappa = 1e3, tol 1e-10, max 512 iterations: the
    persistent form (one cooperative launch per solve) and, beside it, one
    launch per iteration (same iterates)."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import spd_problem

    p = spd_problem(512, 1e3, seed=0, config_id=0)
    A = torch.from_numpy(p.A).to(dev)
    b = torch.from_numpy(p.b).to(dev)
    out = {"n": 512, "kappa": 1e3}
    for persist in (True, False):
        s = krylov.Solver(A, method="cg", tol=1e-10, max_iter=512, persist=persist)
        x = torch.zeros(512, dtype=torch.float64, device=dev)
        s.solve(b, out=x.zero_())
        lat, its = [], []
        for _ in range(50):
            (_, info), dt = _timed(lambda: s.solve(b, out=x.zero_()))
            lat.append(dt * 1e3)
            its.append(info["iters"])
        s.close()
        rec = {"iters": its[-1], "status": info["status_name"], "rel_res": info["rel_res"],
               "solves_per_s": round(1e3 / statistics.mean(lat), 2),
               "p50_ms": round(_pct(lat, 0.5), 3), "p99_ms": round(_pct(lat, 0.99), 3),
               "us_per_iteration": round(1e3 * statistics.median(lat) / its[-1], 2)}
        if persist:
            out.update(rec)
        else:
            out["one_launch_per_iteration"] = rec
    return out


def _solve_timed(solver, b, x, reps_fast=3, fast_s=1.0):
    """Solve once (warm-up); if that took under fast_s seconds, time reps_fast
    more solves and report their median, else report the first."""
    (_, info), dt = _timed(lambda: solver.solve(b, out=x.zero_()))
    if dt >= fast_s:
        return info, dt, 1
    lat = []
    for _ in range(reps_fast):
        (_, info), d = _timed(lambda: solver.solve(b, out=x.zero_()))
        lat.append(d)
    return info, statistics.median(lat), reps_fast


def leg_c3sweep(dev, n, spd_form="qr"):
    """The refinement workload over its condition-number sweep (n = 32768,
    kappa in 1e2, 1e4, 1e6; SPD with CG inner solves, nonsymmetric with
    GMRES(50) inner solves): binary64 stopping on the backward error against
    binary32 and bfloat16 inner solves, all to eta_inf <= 1e-12, and the
    factored preconditioners: CG-IR with the binary32 Cholesky factor (SPD)
    and GMRES(50)-IR with the binary32 LU (nonsymmetric), factorization in
    create timed apart.  In the nonsymmetric kappa = 1e6 cell the
    unpreconditioned solves stall (restarted GMRES(50) stops making progress
    near eta_inf = 1e-8): they run with a capped budget and are reported with
    the status and backward error they reached."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_swept_problem, spd_problem

    out = {"n": n, "eta_target": 1e-12}
    for kind in ("spd_cg", "nonsym_gmres50"):
        for kap in (1e2, 1e4, 1e6):
            if kind == "spd_cg":
                prob = spd_problem(n, kap, seed=0, config_id=2, backend="torch", device="cuda",
                                   q_form=spd_form)
                keys = ("fp64_sym", "fp32_sym", "bf16", "chol32")
            else:
                prob = nonsym_swept_problem(n, kap, seed=0, config_id=2, backend="torch",
                                            device="cuda")
                keys = ("fp64", "fp32", "bf16", "lu32")
            stall = kind == "nonsym_gmres50" and kap >= 1e6
            x = torch.zeros(n, dtype=torch.float64, device=dev)
            res = {}
            for key in keys:
                prec, sym = key.split("_")[0], key.endswith("_sym")
                kw = dict(method="cg" if kind == "spd_cg" else "gmres", tol=1e-12, restart=50,
                          timing=True, timing_every=TIMING_EVERY, max_iter=4 * n, symmetric=sym)
                if stall and prec != "lu32":
                    kw.update(max_iter=2000 if prec == "fp64" else 800, max_outer=4)
                if prec == "fp64":
                    kw["stop_backward"] = True
                else:
                    kw["precision"] = prec
                if prec == "bf16":
                    kw["inner_tol"] = BF16_INNER_TOL
                if prec in ("chol32", "lu32"):
                    kw["symmetric"] = False
                    kw["max_iter"] = 2000
                torch.cuda.synchronize()
                tc0 = time.perf_counter()
                solver = krylov.Solver(prob.A, **kw)
                torch.cuda.synchronize()
                create_ms = (time.perf_counter() - tc0) * 1e3
                info, dt, reps = _solve_timed(solver, prob.b, x)
                r = {"status": info["status_name"], "solve_ms": round(dt * 1e3, 2),
                     "solves_per_s": round(1.0 / dt, 4), "timed_solves": reps,
                     "iters": info["iters"], "outer": info["outer_iters"],
                     "precision_used": info["precision_used"], "eta_inf": info["backward_err"],
                     "fwd_err_vs_x_true": float((x - prob.x_true).norm() / prob.x_true.norm())}
                if prec in ("chol32", "lu32"):
                    # the binary32 factorization in ks_create: n^3 / 3 flops
                    # (Cholesky), 2 n^3 / 3 (LU)
                    fl = n ** 3 / 3.0 if prec == "chol32" else 2.0 * n ** 3 / 3.0
                    r["factor_ms"] = round(create_ms, 2)
                    r["factor_tflops"] = round(fl / (create_ms * 1e-3) / 1e12, 2)
                    r["factor_plus_solve_ms"] = round(create_ms + dt * 1e3, 2)
                if info["gemv_calls"] and info["precision_used"] == prec and prec not in ("chol32", "lu32"):
                    e = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
                    ab = e * n * (n + 1) / 2 if sym else e * n * n
                    r["gemv_gbs"] = round(ab / (info["gemv_ms"] / info["gemv_calls"] * 1e-3) / 1e9, 1)
                res[key] = r
                solver.close()
            f64 = res[keys[0]]
            for key in keys[1:]:
                if f64["status"] == "ok" and res[key]["status"] == "ok":
                    res[key]["speedup_vs_fp64"] = round(res[key]["solves_per_s"] / f64["solves_per_s"], 3)
            out[f"{kind}_kappa_{kap:g}"] = res
            print(f"[bench]   c3 sweep {kind} kappa={kap:g} done", file=sys.stderr, flush=True)
            del prob, x
            torch.cuda.empty_cache()
    return out


def leg_c2(dev, n, steps, spd_form="qr"):
    """Plain binary64 solves on one GPU: CG on the SPD system (n = 16384,
    cond 1e4, lower-triangle product) and GMRES(30) on D + G/sqrt(n), x0 = 0,
    relative residual 1e-10; `steps` timed pairs after one warm-up, with the
    roofline of the CG product (the symmetric tiles and the finishing sum that
    also applies the x, r update)."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_problem, spd_problem

    spd = spd_problem(n, 1e4, seed=0, config_id=1, backend="torch", device="cuda", q_form=spd_form)
    ns = nonsym_problem(n, seed=0, config_id=1, backend="torch", device="cuda")
    cg = krylov.Solver(spd.A, method="cg", tol=1e-10, timing=True, timing_every=TIMING_EVERY,
                       symmetric=True)
    gm = krylov.Solver(ns.A, method="gmres", restart=30, tol=1e-10, timing=True,
                       timing_every=TIMING_EVERY)
    xcg = torch.zeros(n, dtype=torch.float64, device=dev)
    xgm = torch.zeros(n, dtype=torch.float64, device=dev)
    cg.solve(spd.b, out=xcg.zero_())
    gm.solve(ns.b, out=xgm.zero_())
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        (_, icg), tc = _timed(lambda: cg.solve(spd.b, out=xcg.zero_()))
        (_, igm), tg = _timed(lambda: gm.solve(ns.b, out=xgm.zero_()))
        recs.append((icg, igm, tc * 1e3, tg * 1e3))
    el = time.perf_counter() - t0
    gemv_ms = sum(r[0]["gemv_ms"] for r in recs)
    calls = sum(r[0]["gemv_calls"] for r in recs)
    avg = gemv_ms / max(calls, 1)
    pb = product_bytes(n, "symmetric")
    out = {"n": n, "solves_per_s": round(2 * steps / el, 4), "steps": steps,
           "ok": all(r[0]["status"] == 0 and r[1]["status"] == 0 for r in recs),
           "cg": {"iters": recs[-1][0]["iters"], "rel_res": recs[-1][0]["rel_res"],
                  "p50_ms": round(_pct([r[2] for r in recs], 0.5), 3)},
           "gmres30": {"iters": recs[-1][1]["iters"], "rel_res": recs[-1][1]["rel_res"],
                       "p50_ms": round(_pct([r[3] for r in recs], 0.5), 3)},
           "symmetric_product": {"avg_launch_ms": round(avg, 5), "bytes_per_launch": pb,
                                 "achieved_gbs": round(pb / (avg * 1e-3) / 1e9, 1),
                                 "frac": round(pb / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "traffic": load_traffic(n, "symmetric")}}
    cg.close()
    gm.close()
    del spd, ns
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
            ("bicgstab_bf16_eta", dict(method="bicgstab", tol=1e-12, precision="bf16",
                                       inner_tol=BF16_INNER_TOL))]
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
    """Jacobi and Gauss-Seidel on the nonsymmetric n = 16384 system of the
    binary64 leg (D + G/sqrt(n), Jacobi spectral radius about 0.36), binary64
    to relative residual 1e-10, beside GMRES(30) on the same system."""
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
    torch.cuda.empty_cache()
    return out


def leg_f4(dev):
    """GMRES-IR with the binary32 block LU: the factorization (in create) at
    the paper's direct-method sizes and up to n = 16384, and solves of the nonsymmetric kappa = 1e6
    family to backward error 1e-12, beside binary64 GMRES(50) on the same
    systems (which stalls there)."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_swept_problem

    out = {"system": "diag(lambda) + 0.25 G/sqrt(n), lambda log-uniform [1, kappa]",
           "kappa": 1e6, "eta_target": 1e-12}
    for m in (1000, 2000, 4096, 8192, 16384):
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


def leg_chol(dev, n, spd_form="qr"):
    """CG-IR with the binary32 block Cholesky preconditioner on the refinement
    workload's hardest SPD cell (n = 32768, cond 1e6), beside binary32-refined
    CG on the lower triangle (the headline's SPD solver) at the same backward
    error: factorization time and TFLOP/s (n^3 / 3 flops, in ks_create) and
    solve time after the factorization."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import spd_problem

    prob = spd_problem(n, 1e6, seed=0, config_id=2, backend="torch", device="cuda", q_form=spd_form)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    out = {"n": n, "kappa": 1e6, "eta_target": 1e-12}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = krylov.Solver(prob.A, method="cg", precision="chol32", tol=1e-12, max_iter=2000)
    torch.cuda.synchronize()
    fact_ms = (time.perf_counter() - t0) * 1e3
    info, dt, reps = _solve_timed(s, prob.b, x)
    s.close()
    out["chol32"] = {"factor_ms": round(fact_ms, 2),
                     "factor_tflops": round(n ** 3 / 3.0 / (fact_ms * 1e-3) / 1e12, 2),
                     "status": info["status_name"], "outer": info["outer_iters"],
                     "inner": info["iters"], "eta_inf": info["backward_err"],
                     "solve_ms": round(dt * 1e3, 2), "timed_solves": reps,
                     "factor_plus_solve_ms": round(fact_ms + dt * 1e3, 2),
                     "fwd_err_vs_x_true": float((x - prob.x_true).norm() / prob.x_true.norm())}
    s = krylov.Solver(prob.A, method="cg", precision="fp32", symmetric=True, tol=1e-12,
                      max_iter=4 * n)
    info, dt, reps = _solve_timed(s, prob.b, x)
    s.close()
    out["fp32_sym"] = {"status": info["status_name"], "outer": info["outer_iters"],
                       "inner": info["iters"], "eta_inf": info["backward_err"],
                       "solve_ms": round(dt * 1e3, 2), "timed_solves": reps}
    del prob, x
    torch.cuda.empty_cache()
    return out


def leg_lu(dev, n):
    """GMRES(50)-IR with the binary32 block LU preconditioner on the
    refinement workload's hardest nonsymmetric cell (n = 32768, cond 1e6),
    where the unpreconditioned solves stall: factorization time and TFLOP/s
    (2 n^3 / 3 flops, in ks_create) and solve time after the factorization."""
    import torch

    from paper_1511_07207_amd import krylov
    from workloads import nonsym_swept_problem

    prob = nonsym_swept_problem(n, 1e6, seed=0, config_id=2, backend="torch", device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    out = {"n": n, "kappa": 1e6, "eta_target": 1e-12}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = krylov.Solver(prob.A, method="gmres", restart=50, precision="lu32", tol=1e-12, max_iter=2000)
    torch.cuda.synchronize()
    fact_ms = (time.perf_counter() - t0) * 1e3
    info, dt, reps = _solve_timed(s, prob.b, x)
    s.close()
    out["lu32"] = {"factor_ms": round(fact_ms, 2),
                   "factor_tflops": round(2.0 * n ** 3 / 3.0 / (fact_ms * 1e-3) / 1e12, 2),
                   "status": info["status_name"], "outer": info["outer_iters"],
                   "inner": info["iters"], "eta_inf": info["backward_err"],
                   "solve_ms": round(dt * 1e3, 2), "timed_solves": reps,
                   "factor_plus_solve_ms": round(fact_ms + dt * 1e3, 2),
                   "fwd_err_vs_x_true": float((x - prob.x_true).norm() / prob.x_true.norm())}
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


def leg_c5(dev, count, pool_size, seed=0, rates=(0.5, 0.9)):
    """Serving: binary64 against mixed-precision requests at equal accuracy
    (normwise backward error <= 1e-12; SPD requests with the lower-triangle
    product), over a pool of resident systems
    (n log-uniform on [256, 8192], half SPD CG with cond log-uniform on
    [1e2, 1e5], half GMRES(30) on D + G/sqrt(n)), each request with its own
    right-hand side.  Saturation throughput of each, then both under the same
    Poisson arrivals at the given fractions of the binary64 saturation rate
    (p50 / p99 latency)."""
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
        else:
            # SPD requests on the lower triangle (the binary64 products and the
            # binary32 inner products; bfloat16 inner solves keep the general one)
            kw["symmetric"] = True
        if mode == "fp64":
            kw["stop_backward"] = True
        else:
            # inner precision: bfloat16 where its copy stays usable (GMRES on
            # D + G/sqrt(n); SPD up to kappa ~ 3e2), binary32 otherwise
            kw["precision"] = "bf16" if (kind == "gmres" or kap <= 3e2) else "fp32"
            if kw["precision"] == "bf16":
                kw["inner_tol"] = BF16_INNER_TOL
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
                if len(lat) % 512 == 0:
                    print(f"[bench]     c5 {mode}: {len(lat)}/{count} requests done at {done_t:.1f} s",
                          file=sys.stderr, flush=True)
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
    for frac in rates:
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
    ap.add_argument("--n", type=int, default=32768, help="order of the step's two systems")
    ap.add_argument("--kappa", type=float, default=1e4, help="condition number of both systems")
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="timed binary64 steps at the same backward error (after one warm-up)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--spd-form", choices=("qr", "identity"), default="qr",
                    help="Q of the SPD matrix: QR of a Gaussian (default) or the identity "
                         "(same spectrum and bytes; for hardware-counter runs)")
    ap.add_argument("--legs", default="c1,c2,c3sweep,c4,c5,f1,f3,f4",
                    help="extra measurements after the timed steps (comma list of "
                         "c1,c2,c2p,c3sweep,c4,c5,f1,f3,f4,chol,lu; 'none' for the main step only)")
    ap.add_argument("--n2", type=int, default=16384, help="size of the binary64 legs (c2, c2p, c4, f1, f3)")
    ap.add_argument("--c2-steps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=1024)
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--serve-rates", default="0.5,0.9",
                    help="arrival rates of the serving leg as fractions of the binary64 saturation rate")
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
    from workloads import nonsym_swept_problem, spd_problem

    dev = torch.device("cuda:0")
    n, kap = args.n, args.kappa
    ETA = 1e-12
    t0 = time.perf_counter()
    spd = spd_problem(n, kap, seed=0, config_id=2, backend="torch", device="cuda",
                      q_form=args.spd_form)
    ns = nonsym_swept_problem(n, kap, seed=0, config_id=2, backend="torch", device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated the two n={n} systems in {gen_s:.1f}s", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    common = dict(tol=ETA, max_iter=4 * n, timing=True, timing_every=TIMING_EVERY)
    # mixed precision: binary32 CG on the lower triangle (a bfloat16 copy of
    # this SPD matrix is indefinite), bfloat16 GMRES(50) on the nonsymmetric one
    cg = krylov.Solver(spd.A, method="cg", precision="fp32", symmetric=True, **common)
    gm = krylov.Solver(ns.A, method="gmres", restart=50, precision="bf16", inner_tol=BF16_INNER_TOL,
                       **common)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    xcg = torch.zeros(n, dtype=torch.float64, device=dev)
    xgm = torch.zeros(n, dtype=torch.float64, device=dev)
    # measured HBM read ceiling: the library's streaming-read kernel over A
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    krylov.read_ceiling(spd.A, sink)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        krylov.read_ceiling(spd.A, sink)
    ev1.record()
    torch.cuda.synchronize()
    read_ceiling_gbs = 8.0 * n * n / (ev0.elapsed_time(ev1) / 5 * 1e-3) / 1e9
    if args.calibration_copy:
        copy = krylov.convert(spd.A, torch.float64)
        torch.cuda.synchronize()
        del copy

    def step(s1, s2):
        t = time.perf_counter()
        _, i1 = s1.solve(spd.b, out=xcg.zero_())
        t1 = time.perf_counter()
        _, i2 = s2.solve(ns.b, out=xgm.zero_())
        t2 = time.perf_counter()
        return i1, i2, (t1 - t) * 1e3, (t2 - t1) * 1e3

    def ok_rec(r):
        return (r[0]["status"] == 0 and r[1]["status"] == 0 and r[0]["backward_err"] <= ETA
                and r[1]["backward_err"] <= ETA)

    for w in range(args.warmup):
        step(cg, gm)
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for k in range(args.steps):
        recs.append(step(cg, gm))
        print(f"[bench] step {k + 1}/{args.steps}: spd cg-ir {recs[-1][2]:.1f} ms "
              f"({recs[-1][0]['iters']} inner, {recs[-1][0]['outer_iters']} outer), nonsym gmres50-ir "
              f"{recs[-1][3]:.1f} ms ({recs[-1][1]['iters']} inner, {recs[-1][1]['outer_iters']} outer)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ok = all(ok_rec(r) for r in recs)
    value = 2 * args.steps / elapsed
    ms_step = elapsed * 1e3 / args.steps
    xm_cg, xm_gm = xcg.clone(), xgm.clone()

    # binary64 at the same backward error: CG on the lower triangle, GMRES(50)
    cg64 = krylov.Solver(spd.A, method="cg", symmetric=True, stop_backward=True, **common)
    gm64 = krylov.Solver(ns.A, method="gmres", restart=50, stop_backward=True, **common)
    step(cg64, gm64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs64 = []
    for k in range(args.fp64_steps):
        recs64.append(step(cg64, gm64))
        print(f"[bench] binary64 step {k + 1}/{args.fp64_steps}: cg {recs64[-1][2]:.1f} ms "
              f"({recs64[-1][0]['iters']} it), gmres50 {recs64[-1][3]:.1f} ms "
              f"({recs64[-1][1]['iters']} it)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t0
    value64 = 2 * len(recs64) / el64 if recs64 else None
    ok64 = all(ok_rec(r) for r in recs64)
    cg64.close()
    gm64.close()

    # per-kernel accounting of the timed products: the one with most of the
    # step's time is the roofline kernel
    def prod_stats(idx, product):
        ms = sum(r[idx]["gemv_ms"] for r in recs)
        calls = sum(r[idx]["gemv_calls"] for r in recs)
        avg = ms / max(calls, 1)
        launches = recs[-1][idx]["iters"]
        pb = product_bytes(n, product)
        return {"product": product, "kernel": _PRODUCT_KERNEL[product], "avg_launch_ms": avg,
                "launches_per_solve": launches, "ms_per_solve": avg * launches,
                "bytes_per_launch": pb, "achieved_gbs": pb / (avg * 1e-3) / 1e9, "timed_launches": calls}

    ks = [prod_stats(0, "symmetric32"), prod_stats(1, "gmres_bf16")]
    dom = max(ks, key=lambda k: k["ms_per_solve"])
    other = ks[1] if dom is ks[0] else ks[0]
    traffic = load_traffic(n, dom["product"])

    def solve_summary(idx, rs):
        return {"inner_products": rs[-1][idx]["iters"], "outer_steps": rs[-1][idx]["outer_iters"],
                "precision_used": rs[-1][idx]["precision_used"],
                "backward_err": rs[-1][idx]["backward_err"], "rel_res": rs[-1][idx]["rel_res"],
                "p50_ms": round(_pct([r[2 + idx] for r in rs], 0.5), 3),
                "p99_ms": round(_pct([r[2 + idx] for r in rs], 0.99), 3)}

    def prec_name(v):
        return {0: "fp64", 1: "fp32", 2: "bf16", 3: "lu32"}.get(v, v) if isinstance(v, int) else v

    for rs in (recs, recs64):
        for r in rs:
            for i in (0, 1):
                r[i]["precision_used"] = prec_name(r[i]["precision_used"])
    fwd = {"spd_cg": float((xm_cg - spd.x_true).norm() / spd.x_true.norm()),
           "nonsym_gmres50": float((xm_gm - ns.x_true).norm() / ns.x_true.norm())}
    out = {
        "metric": "solves/s + GEMV HBM GB/s at 1e-12 backward err, mixed vs FP64; p50/p99 latency",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "mixed: f32 / bf16 inner products (f32 accumulation), f64 residual, update and Givens",
        "data": "synthetic",
        "config": {
            "workload": (f"mixed-precision refinement, n={n}, cond {kap:g}: CG-IR on SPD Q diag(lambda) Q^T "
                         f"(binary32 inner CG on the lower triangle) + GMRES(50)-IR on "
                         f"diag(lambda) + 0.25 G/sqrt(n) (bfloat16 inner GMRES), lambda log-uniform "
                         f"[1, {kap:g}]; x0 = 0; stop at eta_inf <= 1e-12; one of each per step"),
            "n": n, "kappa": kap, "eta_target": ETA, "restart": 50,
            "inner_tol": {"fp32": 1e-4, "bf16": BF16_INNER_TOL},
            "spd_q": args.spd_form, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom["kernel"],
            "achieved": round(dom["achieved_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dom["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "bytes_per_launch": dom["bytes_per_launch"],
            "avg_launch_ms": round(dom["avg_launch_ms"], 5),
            "timed_launches": dom["timed_launches"],
            "read_ceiling_gbs": round(read_ceiling_gbs, 1),
            "frac_of_read_ceiling": round(dom["achieved_gbs"] / read_ceiling_gbs, 4),
        },
        "other_product": {"kernel": other["kernel"], "achieved_gbs": round(other["achieved_gbs"], 1),
                          "frac": round(other["achieved_gbs"] / HBM_PEAK_GBS, 4),
                          "avg_launch_ms": round(other["avg_launch_ms"], 5),
                          "bytes_per_launch": other["bytes_per_launch"],
                          "traffic": load_traffic(n, other["product"])},
        "valid": ok,
        "solves": {"spd_cg_ir_fp32_lower": solve_summary(0, recs),
                   "nonsym_gmres50_ir_bf16": solve_summary(1, recs)},
        "fwd_err_vs_x_true": fwd,
        "fp64_equal_accuracy": {
            "solves_per_s": round(value64, 4) if value64 else None, "steps": len(recs64),
            "valid": ok64,
            "spd_cg_lower": solve_summary(0, recs64) if recs64 else None,
            "nonsym_gmres50": solve_summary(1, recs64) if recs64 else None,
        },
        "mixed_over_fp64": round(value / value64, 3) if value64 else None,
        "iterations_per_s": round(sum(r[0]["iters"] + r[1]["iters"] for r in recs) / elapsed, 1),
        "create_ms": round(create_ms, 2),
        "generate_s": round(gen_s, 2),
    }
    cg.close()
    gm.close()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(spd, ns, recs64[-1][0]["iters"] if recs64 else 1000,
                                           recs64[-1][1]["iters"] if recs64 else 1000)
        print("[bench] CPU oracle sample done", file=sys.stderr, flush=True)
    else:
        out["cpu_baseline"] = None
    del spd, ns, xcg, xgm, xm_cg, xm_gm
    torch.cuda.empty_cache()
    legs = {}
    wanted = [] if args.legs == "none" else [x.strip() for x in args.legs.split(",") if x.strip()]
    n2 = args.n2
    for name in wanted:
        print(f"[bench] leg {name} ...", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        try:
            if name == "c1":
                legs[name] = leg_c1(dev)
            elif name == "c2":
                legs[name] = leg_c2(dev, n2, args.c2_steps, args.spd_form)
            elif name == "c3sweep":
                legs[name] = leg_c3sweep(dev, n, args.spd_form)
            elif name == "c4":
                legs[name] = leg_c4(dev, n2)
            elif name == "c5":
                rates = [float(v) for v in args.serve_rates.split(",") if v.strip()]
                legs[name] = leg_c5(dev, args.serve_requests, args.serve_pool, rates=rates)
            elif name == "f1":
                legs[name] = leg_f1(dev, n2)
            elif name == "f3":
                legs[name] = leg_f3(dev, n2)
            elif name == "f4":
                legs[name] = leg_f4(dev)
            elif name == "c2p":
                legs[name] = leg_c2p(dev, n2)
            elif name == "chol":
                legs[name] = leg_chol(dev, n, args.spd_form)
            elif name == "lu":
                legs[name] = leg_lu(dev, n)
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
