"""The 3D bell-hill benchmark of Section 3.1 on one GPU: a uniform and a non-conforming mesh.

Section 3.1 runs a stratified flow (N = 0.01 1/s, u = 10 m/s) over the bell of Eq. (3)
(h_c = 400 m, a_c = 1 km, centred at (30, 20) km) in a 60 x 40 x 16 km box at degree 4 with
dt = 2 s for one hour, on a uniform mesh of 60 x 40 x 16 hexahedra (1 km cells, 250 m between
nodes) and on a non-conforming mesh of 1958 cells whose finest cells match the uniform ones.  It
shows the vertical velocity on an x-z slice at y = 20 km and an x-y slice at z = 800 m for both
meshes and reports the wall-clock times 2560 s (non-conforming) and 36500 s (uniform), a 93 %
saving.

The paper's non-conforming mesh exists only as a figure.  The one re-created here
(``bell3d_r4_nonconforming``) has 4 km base cells, one level over the lowest 4 km and a second
level (1 km cells, as in the uniform mesh) over the lowest 2 km within 10 km of the hill in x and
4 km in y: 1930 cells.  The non-reflecting top and lateral boundaries are absorbing layers
(Rayleigh friction towards the background wind) below the lid and along the periodic sides.

``python -m paper_2408_08129_amd.bellhill`` runs both meshes and prints one JSON line: wall-clock
per mesh and the saving, GMRES iterations, and the two slices of w compared between the meshes
(evaluated from the DG polynomials at common points).

Both meshes run with the enthalpy split of the implicit energy flux and without the
pressure-jump penalty: with the plain flux (and with the penalty) grid-scale buoyancy modes grow
in a stratified atmosphere, with e-folding times of 20-60 s, and end the run after about 300 s.
``--plain`` runs the plain flux with the penalty instead; ``--seconds`` sets the final time (the
paper's hour by default); a run that fails reports the step it failed at.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import cases

PAPER_WALL_S = {"uniform": 36500.0, "nonconforming": 2560.0}


def terrain_height(w: dict, x, y):
    """Orography height at horizontal positions (the five profiles of the case description)."""
    kind = w["orography"]
    h0, a, xc, yc = w["oro"]
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if kind == cases.ORO_FLAT:
        return np.zeros_like(x)
    if kind == cases.ORO_AGNESI:
        return h0 * a * a / (a * a + (x - xc) ** 2)
    if kind == cases.ORO_BELL:
        r2 = ((x - xc) / a) ** 2 + (((y - yc) / a) ** 2 if w["dim"] == 3 else 0.0)
        return h0 / (1.0 + r2) ** 1.5
    if kind == cases.ORO_GAUSS_HILL:
        r2 = (x - xc) ** 2 + ((y - yc) ** 2 if w["dim"] == 3 else 0.0)
        return h0 * np.exp(-r2 / (2.0 * a * a))
    if kind == cases.ORO_GAUSS_RIDGE:
        return h0 * np.exp(-((x - xc) / a) ** 2)
    raise ValueError("unknown orography kind %r" % kind)


class PointEvaluator:
    """Evaluates a nodal DG field of a mesh at physical points.

    A point (x, y, z) is mapped to its logical height zeta by inverting the terrain-following map
    z = zeta + h (1 - zeta / H), located in the leaf cell that contains (x, y, zeta) (finest level
    first), and the cell's tensor Lagrange polynomial through its Gauss-Legendre nodes (x fastest)
    is evaluated there.  Points below the ground or outside the box give NaN."""

    def __init__(self, cells: np.ndarray, degree: int, w: dict):
        self.w = w
        self.d = w["dim"]
        self.np1 = degree + 1
        self.xi = np.polynomial.legendre.leggauss(self.np1)[0]
        self.L = [float(w["length"][a]) for a in (0, 1, 2)]
        nb = w["nbase"]
        self.nb = [int(nb[0]), int(nb[2])] if self.d == 2 else [int(v) for v in nb]
        self.Ld = [self.L[0], self.L[2]] if self.d == 2 else self.L
        cells = np.asarray(cells, dtype=np.int64)
        self.maxlev = int(cells[:, 0].max())
        self.index = []
        for lev in range(self.maxlev + 1):
            n = [b << lev for b in self.nb]
            tab = np.full(int(np.prod(n)), -1, dtype=np.int64)
            sel = np.nonzero(cells[:, 0] == lev)[0]
            key = np.zeros(len(sel), dtype=np.int64)
            for a in range(self.d - 1, -1, -1):
                key = key * n[a] + cells[sel, 1 + a]
            tab[key] = sel
            self.index.append((n, tab))

    def lagrange(self, t: np.ndarray) -> np.ndarray:
        """Values of the NP 1D Lagrange polynomials at t: shape (len(t), NP)."""
        out = np.ones((len(t), self.np1))
        for j in range(self.np1):
            for k in range(self.np1):
                if k != j:
                    out[:, j] *= (t - self.xi[k]) / (self.xi[j] - self.xi[k])
        return out

    def locate(self, x, y, z):
        """Leaf cell and reference coordinates (n, d) of each point; cell -1 outside."""
        x = np.asarray(x, dtype=np.float64).ravel()
        z = np.asarray(z, dtype=np.float64).ravel()
        y = np.zeros_like(x) if self.d == 2 else np.asarray(y, dtype=np.float64).ravel()
        H = self.Ld[-1]
        h = terrain_height(self.w, x, y)
        zeta = (z - h) / (1.0 - h / H)
        X = [x, zeta] if self.d == 2 else [x, y, zeta]
        inside = np.ones(len(x), dtype=bool)
        for a in range(self.d):
            inside &= (X[a] >= 0.0) & (X[a] <= self.Ld[a])
        cell = np.full(len(x), -1, dtype=np.int64)
        ref = np.zeros((len(x), self.d))
        for lev in range(self.maxlev, -1, -1):
            n, tab = self.index[lev]
            todo = np.nonzero(inside & (cell < 0))[0]
            if len(todo) == 0:
                break
            key = np.zeros(len(todo), dtype=np.int64)
            idx = []
            for a in range(self.d):
                s = X[a][todo] * n[a] / self.Ld[a]
                i = np.clip(np.floor(s).astype(np.int64), 0, n[a] - 1)
                idx.append((i, s))
            for a in range(self.d - 1, -1, -1):
                key = key * n[a] + idx[a][0]
            c = tab[key]
            hit = c >= 0
            cell[todo[hit]] = c[hit]
            for a in range(self.d):
                i, s = idx[a]
                ref[todo[hit], a] = 2.0 * (s[hit] - i[hit]) - 1.0
        return cell, ref

    def __call__(self, nodal: np.ndarray, x, y, z) -> np.ndarray:
        """nodal: (ncell, NL) values; returns the field at the points (NaN outside)."""
        cell, ref = self.locate(x, y, z)
        out = np.full(len(cell), np.nan)
        ok = cell >= 0
        if not np.any(ok):
            return out
        P = self.np1
        vals = nodal[cell[ok]]
        lx = self.lagrange(ref[ok, 0])
        if self.d == 2:
            lz = self.lagrange(ref[ok, 1])
            out[ok] = np.einsum("nzx,nx,nz->n", vals.reshape(-1, P, P), lx, lz)
        else:
            ly = self.lagrange(ref[ok, 1])
            lz = self.lagrange(ref[ok, 2])
            out[ok] = np.einsum("nzyx,nx,ny,nz->n", vals.reshape(-1, P, P, P), lx, ly, lz)
        return out


def slice_points(w: dict, spacing: float = 250.0):
    """The paper's two slices: x-z at y = Ly / 2 and x-y at z = 800 m, on a grid of the given
    spacing (the uniform mesh's node distance)."""
    Lx, Ly, H = (float(v) for v in w["length"])
    xs = np.arange(0.0, Lx + 0.5 * spacing, spacing)
    ys = np.arange(0.0, Ly + 0.5 * spacing, spacing)
    zs = np.arange(0.0, H + 0.5 * spacing, spacing)
    X, Z = np.meshgrid(xs, zs, indexing="ij")
    xz = (X.ravel(), np.full(X.size, 0.5 * Ly), Z.ravel())
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    xy = (X.ravel(), Y.ravel(), np.full(X.size, 800.0))
    return {"xz_y20km": xz, "xy_z800m": xy}


def interior_mask(w: dict, pts) -> np.ndarray:
    """Points outside every absorbing layer."""
    x, y, z = pts
    depth, rt, width, rl, _ = w.get("sponge", (0.0,) * 5)
    Lx, Ly, H = (float(v) for v in w["length"])
    m = np.ones(len(x), dtype=bool)
    if rt > 0.0:
        m &= z < H - depth
    if rl > 0.0:
        m &= (np.minimum(x, Lx - x) >= width) & (np.minimum(y, Ly - y) >= width)
    return m


def run_case(w: dict, steps: int, precision: int, label: str) -> dict:
    """Steps one workload on the GPU; returns wall-clock, iterations, diagnostics and w at the
    nodes (host, (ncell, NL))."""
    import torch

    import paper_2408_08129_amd as P

    opt = P.options(precision=precision, gmres_rtol=w.get("rtol", 1e-8),
                    enthalpy_split=w.get("enthalpy_split", 0), penalty_beta=w.get("penalty_beta", 1.0))
    s = P.Solver(cases.product_case(w), w["degree"], opt)
    U = s.init_state(w["ubar"])
    mass0, _ = s.diagnostics(U)
    torch.cuda.synchronize()
    iters = []
    trace = []
    failed = None
    t0 = time.perf_counter()
    last = t0
    for i in range(steps):
        try:
            st = s.step(U, w["dt"])
        except P.DGError as e:
            failed = {"step": i + 1, "error": str(e)}
            print("[bellhill] %s failed at step %d: %s" % (label, i + 1, e), file=sys.stderr, flush=True)
            break
        iters.extend(v for stage in st.as_dict(opt.fp_iters)["gmres_iters"] for v in stage)
        if (i + 1) % 20 == 0 or i + 1 == steps:
            mass, max_w = s.diagnostics(U)  # synchronises
            now = time.perf_counter()
            trace.append({"step": i + 1, "max_w": max_w, "mass_drift": (mass - mass0) / mass0})
            print("[bellhill] %s step %d/%d  %.1f ms/step  max|w| %.3f m/s" %
                  (label, i + 1, steps, (now - last) * 1e3 / 20.0 if (i + 1) % 20 == 0 else 0.0,
                   max_w), file=sys.stderr, flush=True)
            last = now
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    done = failed["step"] - 1 if failed else steps
    Uh = U.cpu().numpy()
    nl = s.nloc
    wvel = (Uh[s.dim] / Uh[0]).reshape(-1, nl)
    out = {"cells": s.ncell, "dofs": s.nf * s.N, "steps": done, "wall_s": round(wall, 3),
           "ms_per_step": round(wall / max(done, 1) * 1e3, 3), "failed": failed,
           "max_w_trace": [(t["step"], round(t["max_w"], 4)) for t in trace],
           "gmres_iters_mean": round(float(np.mean(iters)), 2) if iters else None,
           "gmres_iters_max": int(np.max(iters)) if iters else None,
           "mass_drift": trace[-1]["mass_drift"] if trace else 0.0,
           "max_w": trace[-1]["max_w"] if trace else 0.0}
    cells = s.cell_table()
    s.close()
    del U
    torch.cuda.empty_cache()
    return out, cells, wvel


def compare_slices(w_u, cells_u, wv_u, w_n, cells_n, wv_n) -> dict:
    eu = PointEvaluator(cells_u, w_u["degree"], w_u)
    en = PointEvaluator(cells_n, w_n["degree"], w_n)
    res = {}
    for name, pts in slice_points(w_u).items():
        a = eu(wv_u, *pts)
        b = en(wv_n, *pts)
        ok = np.isfinite(a) & np.isfinite(b)
        core = ok & interior_mask(w_u, pts)
        d = np.abs(a - b)
        res[name] = {
            "points": int(ok.sum()),
            "w_uniform_range": [round(float(np.min(a[ok])), 4), round(float(np.max(a[ok])), 4)],
            "w_nonconforming_range": [round(float(np.min(b[ok])), 4), round(float(np.max(b[ok])), 4)],
            "max_abs_diff": round(float(np.max(d[ok])), 5),
            "rms_diff": round(float(np.sqrt(np.mean(d[ok] ** 2))), 5),
            "max_abs_diff_outside_layers": round(float(np.max(d[core])), 5) if core.any() else None,
            "max_abs_w_outside_layers": round(float(np.max(np.abs(a[core]))), 4) if core.any() else None,
        }
    return res


def main():
    import paper_2408_08129_amd as P

    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=3600.0, help="simulated time (the paper: 3600 s)")
    ap.add_argument("--plain", action="store_true",
                    help="plain energy flux with the pressure-jump penalty (unstable after ~300 s)")
    ap.add_argument("--steps", type=int, default=None, help="override the step count")
    ap.add_argument("--fp32-inner", action="store_true")
    ap.add_argument("--save", default=None, help="also write the slices to this .npz file")
    args = ap.parse_args()

    P.lib()  # fails loudly if the HIP library is not built
    wu = dict(cases.WORKLOADS["bell3d_r4_uniform"])
    wn = dict(cases.WORKLOADS["bell3d_r4_nonconforming"])
    if args.plain:
        for w in (wu, wn):
            w["enthalpy_split"], w["penalty_beta"] = 0, 1.0
    steps = args.steps if args.steps is not None else int(round(args.seconds / wu["dt"]))
    prec = P.DG_FP32_INNER if args.fp32_inner else P.DG_FP64
    ru, cu, vu = run_case(wu, steps, prec, "uniform")
    rn, cn, vn = run_case(wn, steps, prec, "nonconforming")
    both = ru["failed"] is None and rn["failed"] is None
    out = {
        "benchmark": "3D bell-hill, Section 3.1: uniform vs non-conforming mesh on one MI355X",
        "t_final_s": steps * wu["dt"], "dt": wu["dt"], "degree": wu["degree"],
        "precision": "fp32-inner" if args.fp32_inner else "fp64",
        "energy_flux": "plain, penalty 1" if args.plain else "enthalpy split, penalty 0",
        "uniform": ru, "nonconforming": rn,
        # per step, so that a run cut short by a failure still compares like with like
        "saving": round(1.0 - rn["ms_per_step"] / ru["ms_per_step"], 4),
        "speedup": round(ru["ms_per_step"] / rn["ms_per_step"], 2),
        "paper": {"wall_s": PAPER_WALL_S,
                  "saving": round(1.0 - PAPER_WALL_S["nonconforming"] / PAPER_WALL_S["uniform"], 4),
                  "cells_nonconforming": 1958, "cells_uniform": 38400},
        "w_slices": compare_slices(wu, cu, vu, wn, cn, vn) if both else None,
    }
    if args.save and both:
        eu, en = PointEvaluator(cu, wu["degree"], wu), PointEvaluator(cn, wn["degree"], wn)
        arrays = {}
        for name, pts in slice_points(wu).items():
            arrays[name + "_points"] = np.stack(pts)
            arrays[name + "_uniform"] = eu(vu, *pts)
            arrays[name + "_nonconforming"] = en(vn, *pts)
        np.savez_compressed(args.save, **arrays)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
