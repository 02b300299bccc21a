#!/usr/bin/env python
"""Throughput of the IMEX-DG step on one MI355X.

Metric: DoF-updates/s per IMEX-RK2 step (F fields x N nodes per step), FP64 and FP32-inner, with
p50/p99 step latency.  Workload: 3D box 40 x 40 x 20 km, degree 4, 64 x 64 x 32 base hexahedra
with one 2:1 level below 3 km over a Gaussian hill (274,432 cells, 171.5 M DoFs), stratified
atmosphere, u = 10 m/s, dt = 0.6 s.  Inputs are synthetic and resident in HBM before timing.

Prints one JSON line.  The roofline object reports the dominant operator kernel class measured
live with HIP events around its launches on the solver's stream; cpu_baseline times the FP64
oracle (as it stands) on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f = math.floor(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def run_gpu(w, precision, steps, warmup, timing=True):
    import torch

    import paper_2408_08129_amd as P
    from paper_2408_08129_amd import cases

    opt = P.options(precision=precision, gmres_rtol=w.get("rtol", 1e-8), quad_extra=w.get("quad_extra", 0))
    s = P.Solver(cases.product_case(w), w["degree"], opt)
    U = s.init_state(w["ubar"])
    for i in range(warmup):
        s.step(U, w["dt"])
        print("[bench] warmup step %d done" % i, file=sys.stderr, flush=True)
    s.set_timing(timing)
    torch.cuda.synchronize()
    lat = []
    stats = []
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        st = s.step(U, w["dt"])
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        stats.append(st.as_dict(opt.fp_iters))
        print("[bench] step %d %.1f ms its %s" % (i, lat[-1], stats[-1]["gmres_iters"]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    out = dict(solver=s, U=U, lat=lat, stats=stats, total=total, dofs=s.nf * s.N, N=s.N,
               ncell=s.ncell, nf=s.nf)
    return out


KERNEL_NAMES = {
    "explicit_residual": "k_col_exp + 2:1 faces pass of k_cell<OpExplicit> (explicit residual)",
    "weak_gradient": "k_col<grad> + 2:1 faces pass of k_cell<OpGrad> (Helmholtz pass 1: h M^-1 B p)",
    "weak_divergence": "k_col<div> + 2:1 faces pass of k_cell<OpDiv> (Helmholtz pass 2: C w, penalty, mass)",
    "gs_dots": "k_gs_dots (Gram-Schmidt reduction pass)",
    "gs_update": "k_gs_update (Gram-Schmidt update pass)",
}
SOURCES = ("dg_ops.hip", "dg_helm.hip", "dg_solver.hip", "dg_internal.hpp", "dg_device.hpp")  # the kernels profiled


def source_sha256():
    import hashlib
    src = b"".join(open(os.path.join(ROOT, "paper_2408_08129_amd", "csrc", f), "rb").read() for f in SOURCES)
    return hashlib.sha256(src).hexdigest()


def measured_traffic(cls, workload):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (calibrated against a plain copy), or None if absent or if the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if source_sha256() != rec.get("source_sha256"):
        return None
    k = rec.get("classes", {}).get(cls)
    return k["hbm_bytes_per_launch"] if k else None


def roofline(res, workload="box3d_r4_hill"):
    """Dominant kernel over the timed region: its algorithmic bytes (reported by the library per
    launch, as designed) over its HIP-event-measured device time."""
    st = res["stats"]
    tk = {k: sum(s["t_kernel_ms"][k] for s in st) for k in st[0]["t_kernel_ms"]}
    nk = {k: sum(s["n_kernel"][k] for s in st) for k in st[0]["n_kernel"]}
    bk = {k: sum(s["bytes_kernel"][k] for s in st) for k in st[0]["bytes_kernel"]}
    cand = {k: tk[k] for k in KERNEL_NAMES if nk.get(k, 0) > 0}
    dom = max(cand, key=cand.get)
    avg_ms = tk[dom] / nk[dom]
    bytes_per_launch = bk[dom] / nk[dom]
    achieved = bk[dom] / (tk[dom] * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom, workload),
           "kernel": KERNEL_NAMES[dom], "avg_launch_ms": round(avg_ms, 4), "launches": nk[dom],
           "algorithmic_bytes_per_launch": round(bytes_per_launch)}
    out["by_class"] = {k: {"ms": round(tk[k], 2), "launches": nk[k],
                           "gbs": (round(bk[k] / (tk[k] * 1e-3) / 1e9, 1) if tk[k] > 0 and bk[k] > 0 else None)}
                       for k in tk if nk[k] > 0}
    return out


def cpu_baseline(w, budget_s=30.0):
    """FP64 oracle on a column sample of the workload (same cell sizes, refinement and height)."""
    import numpy as np

    from oracle import oracle as O
    from paper_2408_08129_amd import cases
    from tests import _common as C

    nx = int(os.environ.get("BENCH_CPU_COLUMNS", "2"))
    ws = cases.column_sample(w, nx, nx)
    o = O.Oracle(C.oracle_case(ws))
    U = o.initial_state(w["ubar"])
    t0 = time.perf_counter()
    st = {}
    o.step(U, w["dt"], rtol=w.get("rtol", 1e-8), stats=st)
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(o.nf * o.N / t, 1), "unit": "DoF-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "one FP64 IMEX-RK2 step of a %dx%d-column sample of the workload (%d cells, "
                      "%d DoFs, full height, same refinement), %.1f s, GMRES its %s"
                      % (nx, nx, o.ncell, o.nf * o.N, t, st.get("gmres_iters"))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="box3d_r4_hill")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--quad-extra", type=int, default=0,
                    help="over-integrate the explicit flux with degree + 1 + Q points per direction")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2408_08129_amd as P
    from paper_2408_08129_amd import cases

    P.lib()  # fails loudly if the HIP library is not built
    assert torch.cuda.is_available(), "needs a ROCm GPU"
    w = dict(cases.WORKLOADS[args.workload])
    w["rtol"] = 1e-8
    w["quad_extra"] = args.quad_extra

    r64 = run_gpu(w, P.DG_FP64, args.steps, args.warmup)
    value = r64["dofs"] * args.steps / r64["total"]
    line = {
        "metric": "DoF-updates/s per IMEX-RK2 step (FP64 vs FP32-inner) + p50/p99 step latency",
        "value": round(value, 1), "unit": "DoF-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r64["total"] / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": r64["ncell"], "dofs": r64["dofs"],
                   "degree": w["degree"], "dim": w["dim"], "dt": w["dt"], "gmres_rtol": w["rtol"],
                   "precision": "fp64", "quad_extra": args.quad_extra},
        "p50_step_ms": round(percentile(r64["lat"], 50), 3),
        "p99_step_ms": round(percentile(r64["lat"], 99), 3),
        "gmres_iters": [s["gmres_iters"] for s in r64["stats"]],
    }
    line["roofline"] = roofline(r64, args.workload)
    if not args.no_mixed:
        U64 = r64["U"]
        ref = U64.clone()
        del r64
        torch.cuda.empty_cache()
        r32 = run_gpu(w, P.DG_FP32_INNER, args.steps, args.warmup)
        v32 = r32["dofs"] * args.steps / r32["total"]
        # same number of steps from the same initial state: per-field difference to FP64
        # momentum components are measured against the largest momentum component: a component
        # that is zero up to rounding (flow along a ridge) has no scale of its own
        nf = r32["nf"]
        mscale = max(float(ref[f].abs().max()) for f in range(1, nf - 1))
        diff, adiff = [], []
        for f in range(nf):
            a, b = r32["U"][f], ref[f]
            scale = mscale if 1 <= f < nf - 1 else float(b.abs().max())
            adiff.append(float((a - b).abs().max()))
            diff.append(adiff[-1] / scale)
        line["fp32_inner"] = {
            "value": round(v32, 1), "unit": "DoF-updates/s",
            "ms_per_step": round(r32["total"] / args.steps * 1e3, 3),
            "p50_step_ms": round(percentile(r32["lat"], 50), 3),
            "p99_step_ms": round(percentile(r32["lat"], 99), 3),
            "gain_vs_fp64": round(v32 / value, 3),
            "max_rel_diff_vs_fp64_per_field": diff,
            "max_abs_diff_vs_fp64_per_field": adiff,
            "inner_iters": [s["gmres_iters"] for s in r32["stats"]],
            "outer_iters": [s["outer_iters"] for s in r32["stats"]],
        }
        del r32
    if args.calibrate_copy:
        a = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
