"""Serving: request generation and admission by footprint (CPU), isolation on the GPU."""
import time

import numpy as np
import pytest

import paper_2408_08129_amd as P
from paper_2408_08129_amd import serve
from tests import _common as C


def mesh_info(w):
    return P.dg_mesh_info(C.product_case(w), w["degree"], with_cells=False)[0]


def test_member_sizes_and_timestep():
    for dim in (2, 3):
        for target in (2000, 50000, 200000):
            w = serve.member_work(dim, 4, target, mesh_info)
            assert abs(w["cells"] - target) <= 0.15 * target, (dim, target, w["cells"])
            c = np.sqrt(1.4 * 287.0 * 293.15)
            dxmin = w["length"][2] / w["nbase"][2] / 2
            assert abs(4 * c * w["dt"] / dxmin - 2.75) < 1e-12


def test_request_stream_is_seeded_poisson():
    r1 = serve.draw_requests(64, 2408, 0.25, 20, max_cells=20000, mesh_info=mesh_info)
    r2 = serve.draw_requests(64, 2408, 0.25, 20, max_cells=20000, mesh_info=mesh_info)
    assert [r.arrival for r in r1] == [r.arrival for r in r2]
    gaps = np.diff([0.0] + [r.arrival for r in r1])
    assert 0.15 < gaps.mean() < 0.4
    assert {r.work["dim"] for r in r1} == {2, 3}
    assert {r.work["degree"] for r in r1} == {3, 4}
    assert [r.noise_seed for r in r1] == [2408 + k for k in range(64)]


def test_admission_respects_budget_without_gpu(monkeypatch):
    """Members are admitted in arrival order only while their exact footprint fits; the device
    side is replaced by a stub that records what is resident."""
    reqs = serve.draw_requests(12, 7, 0.01, 3, max_cells=5000, mesh_info=mesh_info)
    srv = serve.Server.__new__(serve.Server)
    srv.P = P
    srv.opt = P.options(precision=P.DG_FP32_INNER)
    srv.keep_states = False
    srv.max_active = 16
    need = {r.rid: srv.member_bytes(r) for r in reqs}
    srv.budget = int(2.5 * max(need.values()))
    srv.used = 0
    live = {}
    peak = [0]

    def admit(req, res):
        live[req.rid] = need[req.rid]
        peak[0] = max(peak[0], sum(live.values()))
        res.dofs = 10
        return serve._Member(req=req, res=res, solver=None, U=None, stream=None)

    def step_batch(members):
        time.sleep(0.005)
        return [1.0] * len(members), [0] * len(members)

    def release(m):
        live.pop(m.req.rid)

    monkeypatch.setattr(srv, "_admit", admit)
    monkeypatch.setattr(srv, "_step_batch", step_batch)
    monkeypatch.setattr(srv, "_release", release)
    out = srv.run(reqs, realtime=True)
    assert out["done"] == 12 and out["failed"] == 0
    assert peak[0] <= srv.budget
    assert out["peak_admitted_bytes"] <= srv.budget
    assert all(len(m.step_ms) == 3 for m in out["members"].values())
    assert not live


@pytest.mark.gpu
def test_served_members_match_alone_and_fail_in_isolation():
    import torch
    assert torch.cuda.is_available()
    reqs = serve.draw_requests(5, 11, 0.05, 3, min_cells=200, max_cells=1500, mesh_info=mesh_info)
    print("[case] serving isolation, members", [(r.work["dim"], r.work["degree"], r.work["cells"]) for r in reqs], flush=True)
    srv = serve.Server(budget_bytes=8 << 30, max_active=4, keep_states=True)
    mix = srv.run(reqs, realtime=True, fail={2: 1})
    assert mix["failed"] == 1 and mix["done"] == 4
    assert mix["members"][2].status == "failed" and "-5" in mix["members"][2].error
    for r in reqs:
        if r.rid == 2:
            continue
        alone = serve.Server(budget_bytes=8 << 30, max_active=1, keep_states=True).run([r], realtime=False)
        a = alone["members"][r.rid].state
        b = mix["members"][r.rid].state
        assert a is not None and b is not None
        assert np.array_equal(a, b), r.rid
    assert mix["step_ms_p99"] >= mix["step_ms_p50"] > 0
