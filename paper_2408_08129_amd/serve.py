"""Continuous-batching service for ensemble members on one GPU.

Requests (ensemble-forecast members over orography, of different mesh sizes and degrees) arrive
over time.  The server admits a request as soon as it has arrived and its exact device footprint
(``dg_footprint`` plus its state) fits in the HBM budget and an execution slot is free; admitted
members keep their state resident and advance step by step.  Each round is one batched step:
members of one class (dimension, degree, precision) share every kernel launch through segment
tables and every host round trip of the Krylov iteration, and each class runs on its own stream
from its own host thread.  When a member finishes (or fails) its memory and slot are released and
waiting requests are admitted.

Reported: throughput (DoF-updates/s over the run), per member-step latency p50/p99, request
end-to-end latency (arrival -> last step done) and admission wait.

The work per member follows the paper's bell-hill configuration family (Section 3.1): a
stratified atmosphere (N = 0.01 1/s) over an Agnesi ridge (2D) or the bell of Eq. (3) (3D) with
h = 400 m, u = 10 m/s, one refinement level near the hill, the time step from an acoustic Courant
number of 2.75 (Section 3), and a seeded Gaussian temperature perturbation.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import cases

GAMMA, RGAS = 1.4, 287.0


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    work: dict                # workload description (see cases.WORKLOADS)
    steps: int
    noise_seed: int
    noise_sigma: float = 0.1  # K


@dataclass
class MemberResult:
    rid: int
    dofs: int
    ncell: int
    status: str = "pending"
    error: str = ""
    admitted: float = float("nan")
    finished: float = float("nan")
    step_ms: list = field(default_factory=list)
    state: object = None      # final state (host numpy) when keep_states


def member_work(dim: int, degree: int, target_cells: int, mesh_info) -> dict:
    """A member workload of about target_cells cells: square base cells of size H / nz with nx = 2 nz
    (and ny = nx in 3D), one refinement level below H/4 within the central quarter of x (and y)."""
    H = 16000.0
    best = None
    nz0 = (target_cells / (2.0 * 1.19)) ** 0.5 if dim == 2 else (target_cells / (4.0 * 1.11)) ** (1.0 / 3.0)
    for nz in range(max(2, int(nz0) - 2), int(nz0) + 3):
        for nx in range(2 * nz - 2, 2 * nz + 3):
            if nx < 4:
                continue
            d = nz * 1.0
            dx = H / d
            Lx = nx * dx
            w = dict(dim=dim, degree=degree, nbase=(nx, nx if dim == 3 else 1, nz),
                     length=(Lx, Lx if dim == 3 else 1.0, H), periodic=(1, 1),
                     rules=[(H / 4.0, Lx / 2.0, Lx / 8.0, Lx / 2.0 if dim == 3 else 0.0,
                             Lx / 8.0 if dim == 3 else 0.0)],
                     orography=cases.ORO_AGNESI if dim == 2 else cases.ORO_BELL,
                     oro=(400.0, 1000.0, Lx / 2.0, Lx / 2.0 if dim == 3 else 0.0),
                     atmosphere=cases.ATM_STRATIFIED, atm=cases.STRAT, ubar=10.0)
            n = mesh_info(w)
            if best is None or abs(n - target_cells) < abs(best[0] - target_cells):
                best = (n, w)
    n, w = best
    # dt from the acoustic Courant number 2.75 on the finest cells (r c dt / dx_min)
    c = math.sqrt(GAMMA * RGAS * cases.STRAT[1])
    dxmin = (H / w["nbase"][2]) / 2.0
    w["dt"] = 2.75 * dxmin / (degree * c)
    w["cells"] = n
    return w


def draw_requests(n: int = 64, seed: int = 2408, mean_interarrival: float = 0.25, steps: int = 20,
                  min_cells: int = 2000, max_cells: int = 200000, mesh_info=None) -> list:
    """Poisson arrivals (exponential inter-arrival times), members drawn uniformly: dimension 2 or
    3, degree 3 or 4, cells in [min_cells, max_cells]; member k uses noise seed seed + k."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n):
        t += float(rng.exponential(mean_interarrival))
        dim = int(rng.integers(2, 4))
        degree = int(rng.integers(3, 5))
        target = int(rng.integers(min_cells, max_cells + 1))
        w = member_work(dim, degree, target, mesh_info)
        out.append(Request(rid=k, arrival=t, work=w, steps=steps, noise_seed=seed + k))
    return out


@dataclass
class _Member:
    req: Request
    res: MemberResult
    solver: object
    U: object
    stream: object
    done_steps: int = 0


class Server:
    """Iteration-level continuous batching: every round advances each admitted member by one step
    in one batched call, in which the members of one class (dimension, degree, precision) share
    every launch of the step and every host round trip of the Krylov iteration; requests that
    have arrived are admitted at round boundaries while their footprint fits the budget."""

    def __init__(self, budget_bytes: int | None = None, max_active: int = 16, precision: int = 1,
                 gmres_rtol: float = 1e-8, keep_states: bool = False):
        import torch

        import paper_2408_08129_amd as P
        self.P = P
        self.torch = torch
        if budget_bytes is None:
            free, _total = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = budget_bytes
        self.max_active = max_active
        self.opt = P.options(precision=precision, gmres_rtol=gmres_rtol)
        self.keep_states = keep_states
        self.used = 0

    def _case(self, w):
        return cases.product_case(w)

    def member_bytes(self, req: Request) -> int:
        w = req.work
        ctx_bytes = self.P.dg_footprint(self._case(w), w["degree"], self.opt)
        n = w["cells"] * (w["degree"] + 1) ** w["dim"]
        return ctx_bytes + (w["dim"] + 2) * n * 8  # + state

    # -- device side (replaceable in tests) --------------------------------------------------
    def _admit(self, req: Request, res: MemberResult) -> _Member:
        torch, P = self.torch, self.P
        w = req.work
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            solver = P.Solver(self._case(w), w["degree"], self.opt, stream=stream)
            # the temperature noise is drawn in the library (seeded, per node)
            U = solver.init_state(w["ubar"], req.noise_seed, req.noise_sigma)
        stream.synchronize()
        res.dofs = solver.nf * solver.N
        res.ncell = solver.ncell
        return _Member(req=req, res=res, solver=solver, U=U, stream=stream)

    def _step_batch(self, members: list):
        P = self.P
        stats, status = P.imex_rk2_step_batched([m.solver.ctx for m in members], [m.U for m in members],
                                                [m.req.work["dt"] for m in members], raise_on_error=False)
        return [s.t_step_ms for s in stats], status

    def _release(self, m: _Member):
        if self.keep_states and m.res.status == "done":
            m.stream.synchronize()
            m.res.state = m.U.cpu().numpy()
        m.solver.close()
        m.U = None
        m.solver = None

    def _inject_nan(self, m: _Member):
        with self.torch.cuda.stream(m.stream):
            m.U[0, 0] = float("nan")
        m.stream.synchronize()

    # -- scheduling ----------------------------------------------------------------------------
    def run(self, requests: list, realtime: bool = True, fail: dict | None = None) -> dict:
        """Serve the requests; fail maps rid -> step at which a NaN is injected (tests)."""
        fail = fail or {}
        results = {r.rid: MemberResult(rid=r.rid, dofs=0, ncell=0) for r in requests}
        need = {r.rid: self.member_bytes(r) for r in requests}
        for r in requests:
            if need[r.rid] > self.budget:
                results[r.rid].status = "rejected"
                results[r.rid].error = "footprint %d B exceeds the HBM budget %d B" % (need[r.rid], self.budget)
        pending = [r for r in sorted(requests, key=lambda r: r.arrival) if results[r.rid].status != "rejected"]
        active = []
        t0 = time.perf_counter()
        peak_used = 0
        rounds = 0
        while pending or active:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now) and len(active) < self.max_active:
                r = pending[0]
                if self.used + need[r.rid] > self.budget:
                    break
                pending.pop(0)
                res = results[r.rid]
                res.admitted = time.perf_counter() - t0
                try:
                    m = self._admit(r, res)
                except Exception as e:
                    res.status = "failed"
                    res.error = str(e)
                    res.finished = time.perf_counter() - t0
                    continue
                self.used += need[r.rid]
                peak_used = max(peak_used, self.used)
                active.append(m)
            if not active:
                if pending and realtime:
                    time.sleep(max(0.0, min(0.05, pending[0].arrival - (time.perf_counter() - t0))))
                continue
            for m in active:
                if fail.get(m.req.rid) == m.done_steps:
                    self._inject_nan(m)
            lat, status = self._step_batch(active)
            rounds += 1
            still = []
            for m, ms, st in zip(active, lat, status):
                if st != 0:
                    m.res.status = "failed"
                    m.res.error = "imexdg error %d at step %d" % (st, m.done_steps)
                else:
                    m.res.step_ms.append(ms)
                    m.done_steps += 1
                    if m.done_steps >= m.req.steps:
                        m.res.status = "done"
                if m.res.status in ("done", "failed"):
                    m.res.finished = time.perf_counter() - t0
                    self._release(m)
                    self.used -= need[m.req.rid]
                else:
                    still.append(m)
            active = still
        wall = time.perf_counter() - t0
        done = [results[r.rid] for r in requests if results[r.rid].status == "done"]
        steps = [s for m in done for s in m.step_ms]
        total_updates = sum(m.dofs * len(m.step_ms) for m in done)
        arrival = {r.rid: r.arrival for r in requests}
        e2e = [m.finished - arrival[m.rid] for m in done]
        wait = [m.admitted - arrival[m.rid] for m in done]
        pct = lambda xs, q: float(np.percentile(xs, q)) if xs else float("nan")
        return {
            "requests": len(requests), "done": len(done),
            "failed": sum(1 for m in results.values() if m.status == "failed"),
            "rejected": sum(1 for m in results.values() if m.status == "rejected"),
            "rounds": rounds, "wall_s": round(wall, 3),
            "dof_updates_per_s": round(total_updates / wall, 1),
            "step_ms_p50": round(pct(steps, 50), 3), "step_ms_p99": round(pct(steps, 99), 3),
            "e2e_s_p50": round(pct(e2e, 50), 3), "e2e_s_p99": round(pct(e2e, 99), 3),
            "admit_wait_s_p50": round(pct(wait, 50), 3), "admit_wait_s_p99": round(pct(wait, 99), 3),
            "budget_bytes": self.budget, "peak_admitted_bytes": peak_used,
            "members": results,
        }


def main():
    import paper_2408_08129_amd as P

    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--seed", type=int, default=2408)
    ap.add_argument("--rate", type=float, default=4.0, help="mean arrivals per second")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--max-cells", type=int, default=200000)
    ap.add_argument("--max-active", type=int, default=64)
    ap.add_argument("--budget-gb", type=float, default=None)
    args = ap.parse_args()

    def info(w):
        c = P.Case(dim=w["dim"], nbase=tuple(w["nbase"]), length=tuple(w["length"]),
                   periodic=tuple(w["periodic"]), rules=list(w["rules"]), orography=w["orography"],
                   oro=tuple(w["oro"]), atmosphere=w["atmosphere"], atm=tuple(w["atm"]))
        return P.dg_mesh_info(c, w["degree"], with_cells=False)[0]

    reqs = draw_requests(args.requests, args.seed, 1.0 / args.rate, args.steps,
                         max_cells=args.max_cells, mesh_info=info)
    budget = int(args.budget_gb * 1e9) if args.budget_gb else None
    srv = Server(budget_bytes=budget, max_active=args.max_active)
    out = srv.run(reqs)
    out.pop("members")
    out["workload"] = ("%d requests, Poisson arrivals at %.1f/s, 2D/3D orography members of "
                       "2k-%dk cells at degree 3-4, %d steps each, FP32-inner/FP64-outer"
                       % (args.requests, args.rate, args.max_cells // 1000, args.steps))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
