#!/usr/bin/env python
"""Throughput of the IMEX-DG step on one MI355X.

Metric: DoF-updates/s per IMEX-RK2 step (F fields x N nodes per step), FP64 and FP32-inner, with
p50/p99 step latency.  Default workload: the large 3D case, 128 x 128 x 128 base hexahedra on
128 x 128 x 32 km, degree 4, two 2:1 levels near a Gaussian ridge (h = 1 km, half-width 5 km):
2,183,168 cells, 1.364e9 DoFs, stratified atmosphere, u = 10 m/s, dt = 0.4 s.  Inputs are
synthetic and resident in HBM before timing.

Prints one JSON line.  The roofline object reports the Helmholtz apply (the two operator passes of
the pressure system) measured live with HIP events around its launches on the solver's stream,
against its algorithmic minimum of 3 words per node (p and h in, A p out); cpu_baseline times the
FP64 oracle (as it stands) on a bounded column sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
DEFAULT_WORKLOAD = "box3d_r4_ridge_large"


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

    extra = {}
    if w.get("enthalpy_split"):
        extra = dict(enthalpy_split=1, penalty_beta=float(w.get("penalty_beta", 0.0)))
    if w.get("gmres_restart"):
        extra["gmres_restart"] = int(w["gmres_restart"])
    if w.get("inner_restart"):
        extra["inner_restart"] = int(w["inner_restart"])
    opt = P.options(precision=precision, gmres_rtol=w.get("rtol", 1e-8), quad_extra=w.get("quad_extra", 0), **extra)
    t0 = time.perf_counter()
    s = P.Solver(cases.product_case(w), w["degree"], opt)
    U = s.init_state(w["ubar"])
    torch.cuda.synchronize()
    print("[bench] precision %d: setup %.1f s" % (precision, time.perf_counter() - t0), file=sys.stderr, flush=True)
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
    return dict(solver=s, U=U, lat=lat, stats=stats, total=total, dofs=s.nf * s.N, N=s.N,
                ncell=s.ncell, nf=s.nf)


KERNELS = {
    "helmholtz_apply": "k_col<grad> + k_col<div>, each followed by the 2:1-faces pass of k_cell "
                       "(Helmholtz apply A(h) p: pass 1 h M^-1 B p, pass 2 divergence, penalty, mass)",
    "explicit_residual": "k_col_exp + 2:1-faces pass of k_cell<OpExplicit> (explicit residual)",
}
SOURCES = ("dg_ops.hip", "dg_helm.hip", "dg_internal.hpp", "dg_device.hpp", "dg_solver.hip")  # the operator kernels and their launch tables


def source_sha256():
    src = b"".join(open(os.path.join(ROOT, "paper_2408_08129_amd", "csrc", f), "rb").read() for f in SOURCES)
    return hashlib.sha256(src).hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of a kernel from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (calibrated against a plain copy), or None if absent or if the kernel sources changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if source_sha256() != rec.get("source_sha256"):
        return None
    k = rec.get("kernels", {}).get(kernel)
    return k["hbm_bytes_per_launch"] if k else None


def roofline(res, workload):
    """The Helmholtz apply over the timed region: its algorithmic minimum bytes (3 words per node:
    p and h in, A p out) per apply over its HIP-event-measured device time (both passes)."""
    st = res["stats"]
    tk = {k: sum(s["t_kernel_ms"][k] for s in st) for k in st[0]["t_kernel_ms"]}
    nk = {k: sum(s["n_kernel"][k] for s in st) for k in st[0]["n_kernel"]}
    bk = {k: sum(s["bytes_kernel"][k] for s in st) for k in st[0]["bytes_kernel"]}
    N, nf = res["N"], res["nf"]
    napply = nk["helmholtz_pass1"]
    t_apply = tk["helmholtz_pass1"] + tk["helmholtz_pass2"]
    alg_apply = 3 * 8.0 * N                      # FP64: p, h in; A p out
    achieved = alg_apply * napply / (t_apply * 1e-3) / 1e9
    two_pass = (bk["helmholtz_pass1"] + bk["helmholtz_pass2"]) / (t_apply * 1e-3) / 1e9
    alg_exp = 2 * nf * 8.0 * N                   # U in, R out
    t_exp = tk["explicit_residual"]
    exp_gbs = alg_exp * nk["explicit_residual"] / (t_exp * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": measured_traffic("helmholtz_apply", workload),
           "kernel": KERNELS["helmholtz_apply"], "avg_launch_ms": round(t_apply / napply, 4),
           "launches": napply, "algorithmic_bytes_per_launch": round(alg_apply),
           "algorithmic_basis": "3 words per node (p, h in; A p out), FP64, N = %d nodes" % N,
           "two_pass_design": {"bytes_per_launch": round((bk["helmholtz_pass1"] + bk["helmholtz_pass2"]) / napply),
                               "achieved": round(two_pass, 1), "frac": round(two_pass / HBM_PEAK_GBS, 4),
                               "basis": "the passes' own reads and writes, incl. the d-word q round trip"},
           "explicit_residual": {"avg_launch_ms": round(t_exp / max(1, nk["explicit_residual"]), 4),
                                 "achieved": round(exp_gbs, 1), "frac": round(exp_gbs / HBM_PEAK_GBS, 4),
                                 "algorithmic_bytes_per_launch": round(alg_exp),
                                 "traffic": measured_traffic("explicit_residual", workload),
                                 "basis": "2 F words per node (U in, R out)"}}
    out["by_class"] = {k: {"ms": round(tk[k], 2), "launches": nk[k],
                           "gbs": (round(bk[k] / (tk[k] * 1e-3) / 1e9, 1) if tk[k] > 0 and bk[k] > 0 else None)}
                       for k in tk if nk[k] > 0}
    tp = {k: sum(s["t_phase_ms"][k] for s in st) / len(st) for k in st[0]["t_phase_ms"]}
    out["phase_ms_per_step"] = {k: round(v, 2) for k, v in tp.items()}
    return out


def accuracy_vs_oracle(workload):
    """GPU FP64 and FP32-inner against the stored FP64 oracle trajectory of a column sample of the
    workload (same cells, refinement and height; tests/golden, written by the oracle only):
    per-field max and L2 relative error at the stored sample of nodes."""
    import numpy as np
    import torch

    import paper_2408_08129_amd as P
    from paper_2408_08129_amd import cases
    gold = {"box3d_r4_ridge_large": "box3d_r4_ridge_large_column1x1_3steps",
            "box3d_r4_hill": "box3d_r4_hill_columns2x2_3steps"}.get(workload)
    path = os.path.join(ROOT, "tests", "golden", "%s.json" % gold) if gold else None
    if not path or not os.path.exists(path):
        return None
    g = json.load(open(path))
    base, cols = g["workload"].split("@")
    nx, ny = (int(v) for v in cols.split("x"))
    w = cases.column_sample(cases.WORKLOADS[base], nx, ny)
    out = {"sample": "%s, %d cells, %d steps, %d sampled nodes; oracle GMRES rtol 1e-12"
                     % (g["workload"], g["ncell"], g["steps"], len(g["node"]))}
    for name, prec in (("fp64", P.DG_FP64), ("fp32_inner", P.DG_FP32_INNER)):
        s = P.Solver(cases.product_case(w), w["degree"], P.options(precision=prec))
        U = s.init_state(g["ubar"])
        for _ in range(g["steps"]):
            s.step(U, g["dt"])
        torch.cuda.synchronize()
        cells = s.cell_table()
        index = {tuple(r): i for i, r in enumerate(cells.tolist())}
        idx = np.array([index[tuple(c)] * s.nloc + q for c, q in zip(g["cells"], g["node"])])
        Ug = U.cpu().numpy()[:, idx]
        ref = np.array(g["values"])
        wJ = np.array(g["wJ"])
        nf = g["nf"]
        mmax = max(g["field_max"][1:nf - 1])
        ml2 = max(math.sqrt(np.sum(wJ * ref[f] ** 2)) for f in range(1, nf - 1))
        mx, l2 = [], []
        for f in range(nf):
            mom = 1 <= f < nf - 1
            mx.append(float(np.max(np.abs(Ug[f] - ref[f]))) / (mmax if mom else g["field_max"][f]))
            l2.append(math.sqrt(np.sum(wJ * (Ug[f] - ref[f]) ** 2)) / (ml2 if mom else math.sqrt(np.sum(wJ * ref[f] ** 2))))
        out[name] = {"max_rel_per_field": mx, "l2_rel_per_field": l2}
        s.close()
    return out


def serving_leg(n=16, steps=5, max_cells=50000):
    """A bounded run of the ensemble server: n requests (Poisson arrivals, mean 0.25 s), 2D/3D
    members of 2k-max_cells cells at degree 3-4, steps each; FP32-inner and, on the same requests,
    FP64."""
    import paper_2408_08129_amd as P
    from paper_2408_08129_amd import cases, serve

    def info(w):
        return P.dg_mesh_info(cases.product_case(w), w["degree"], with_cells=False)[0]

    reqs = serve.draw_requests(n, 2408, 0.25, steps, max_cells=max_cells, mesh_info=info)
    out = {"workload": "%d requests, Poisson arrivals at 4/s, 2D/3D orography members of 2k-%dk cells at "
                       "degree 3-4, %d steps each, GMRES rtol 1e-8" % (n, max_cells // 1000, steps)}
    for name, prec in (("fp32_inner", P.DG_FP32_INNER), ("fp64", P.DG_FP64)):
        r = serve.Server(max_active=64, precision=prec).run(reqs, realtime=True)
        r.pop("members")
        out[name] = {k: r[k] for k in ("done", "failed", "rounds", "wall_s", "dof_updates_per_s",
                                       "step_ms_p50", "step_ms_p99", "e2e_s_p50", "e2e_s_p99")}
        print("[bench] serving %s: %s" % (name, out[name]), file=sys.stderr, flush=True)
    out["gain_fp32_inner_vs_fp64"] = round(out["fp32_inner"]["dof_updates_per_s"] / out["fp64"]["dof_updates_per_s"], 3)
    # throughput of the shared launches: every request present from the start, served together
    # (up to 64 members in flight) and one at a time (a batch of one per round: the same per-member
    # arithmetic, so the same bits and the same accuracy), FP64; admission, setup and release
    # included in both
    thr = {}
    for name, act in (("served", 64), ("one_at_a_time", 1)):
        r = serve.Server(max_active=act, precision=P.DG_FP64).run(reqs, realtime=False)
        r.pop("members")
        thr[name] = {k: r[k] for k in ("done", "failed", "rounds", "wall_s", "dof_updates_per_s",
                                       "step_ms_p50", "step_ms_p99")}
        print("[bench] serving fp64 %s, all requests present: %s" % (name, thr[name]), file=sys.stderr, flush=True)
    thr["gain_served_vs_one_at_a_time"] = round(thr["served"]["dof_updates_per_s"] / thr["one_at_a_time"]["dof_updates_per_s"], 3)
    out["fp64_all_present"] = thr
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(workload, ncols):
    """FP64 oracle: one IMEX-RK2 step of an ncols x ncols base-column sample of the workload (same
    cell sizes, refinement and height); returns the figures as a dict."""
    from oracle import oracle as O
    from paper_2408_08129_amd import cases
    from tests import _common as C

    w = dict(cases.WORKLOADS[workload])
    ws = cases.column_sample(w, ncols, ncols)
    o = O.Oracle(C.oracle_case(ws))
    U = o.initial_state(w["ubar"])
    t0 = time.perf_counter()
    st = {}
    o.step(U, w["dt"], rtol=1e-8, stats=st)
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(o.nf * o.N / t, 1), "unit": "DoF-updates/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "one FP64 IMEX-RK2 step of a %dx%d-column sample of the workload (%d cells, %d DoFs, "
                      "full height, same refinement), %.1f s, GMRES its %s (diagonal preconditioner, "
                      "restart 30)" % (ncols, ncols, o.ncell, o.nf * o.N, t, st.get("gmres_iters"))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the leg with the enthalpy-split energy flux (the stable long-run form)")
    ap.add_argument("--gmres-restart", type=int, default=0,
                    help="GMRES restart length of the FP64 solve (0: the library default)")
    ap.add_argument("--inner-restart", type=int, default=0,
                    help="restart length of the FP32 inner GMRES of the mixed form (0: the library default)")
    ap.add_argument("--quad-extra", type=int, default=0,
                    help="over-integrate the explicit flux with degree + 1 + Q points per direction")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--cpu-leg", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_leg:
        # child process of the one-core baseline (started with OMP_NUM_THREADS=1)
        print(json.dumps(cpu_leg(args.workload, args.cpu_leg)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    one_core = None
    if not args.no_cpu_baseline:
        # the one-core oracle leg runs beside the GPU legs on a host core of its own
        env = dict(os.environ, OMP_NUM_THREADS="1")
        one_core = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-leg", "1",
                                     "--workload", args.workload], env=env, stdout=subprocess.PIPE,
                                    text=True)

    import torch

    import paper_2408_08129_amd as P
    from paper_2408_08129_amd import cases

    P.lib()  # fails loudly if the HIP library is not built
    assert torch.cuda.is_available(), "needs a ROCm GPU"
    w = dict(cases.WORKLOADS[args.workload])
    w["rtol"] = 1e-8
    w["quad_extra"] = args.quad_extra
    if args.gmres_restart:
        w["gmres_restart"] = args.gmres_restart
    if args.inner_restart:
        w["inner_restart"] = args.inner_restart

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
                   "precision": "fp64", "quad_extra": args.quad_extra, "gmres_restart": args.gmres_restart or 15},
        "p50_step_ms": round(percentile(r64["lat"], 50), 3),
        "p99_step_ms": round(percentile(r64["lat"], 99), 3),
        "gmres_iters": [s["gmres_iters"] for s in r64["stats"]],
    }
    line["roofline"] = roofline(r64, args.workload)
    if not args.no_mixed:
        U64 = r64["U"]
        ref = U64.clone()
        r64["solver"].close()
        del r64, U64
        torch.cuda.empty_cache()
        r32 = run_gpu(w, P.DG_FP32_INNER, args.steps, args.warmup)
        v32 = r32["dofs"] * args.steps / r32["total"]
        # same number of steps from the same initial state: per-field difference to FP64;
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
            "inner_restart": args.inner_restart or 30,
            "inner_iters": [s["gmres_iters"] for s in r32["stats"]],
            "outer_iters": [s["outer_iters"] for s in r32["stats"]],
        }
        r32["solver"].close()
        del r32, ref
        torch.cuda.empty_cache()
    if not args.no_split:
        # the stable long-run form (enthalpy split of the implicit energy flux, no pressure-jump
        # penalty), FP64, same workload, a few steps
        ws = dict(w, enthalpy_split=1, penalty_beta=0.0)
        ks = min(args.steps, 3)
        rs = run_gpu(ws, P.DG_FP64, ks, 1)
        vs = rs["dofs"] * ks / rs["total"]
        st = rs["stats"]
        n1 = sum(x["n_kernel"]["helmholtz_pass1"] for x in st)
        t12 = sum(x["t_kernel_ms"]["helmholtz_pass1"] + x["t_kernel_ms"]["helmholtz_pass2"] for x in st)
        line["enthalpy_split"] = {
            "value": round(vs, 1), "unit": "DoF-updates/s", "steps": ks,
            "ms_per_step": round(rs["total"] / ks * 1e3, 3), "vs_plain_fp64": round(vs / value, 3),
            "helmholtz_apply_ms": round(t12 / max(1, n1), 4),
            "gmres_iters": [x["gmres_iters"] for x in st],
            "form": "FP64, enthalpy split of the implicit energy flux in one column pass, penalty_beta 0"}
        rs["solver"].close()
        del rs
        torch.cuda.empty_cache()
    if not args.no_accuracy:
        acc = accuracy_vs_oracle(args.workload)
        if acc is not None:
            line["accuracy_vs_oracle"] = acc
    if not args.no_serving:
        line["serving"] = serving_leg()
    if args.calibrate_copy:
        a = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_leg(args.workload, 1)
        out, _ = one_core.communicate()
        if one_core.returncode == 0:
            line["cpu_baseline"]["one_core"] = json.loads(out.strip().splitlines()[-1])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
