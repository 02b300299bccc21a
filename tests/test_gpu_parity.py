"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_08129_amd import cases, inputs
from tests import _common as C

pytestmark = pytest.mark.gpu

TOL64 = 1e-12      # single operator applications, FP64
TOL_STEP = 1e-10   # time stepping, FP64
TOL_MIXED = 1e-8   # FP32-inner / FP64-outer after refinement


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a ROCm device"
    return torch


def pair(w, **opt):
    import paper_2408_08129_amd as P
    print("[case] %s %s" % ({k: w[k] for k in ("dim", "degree", "nbase")}, opt), flush=True)
    o = O.Oracle(C.oracle_case(w), beta=opt.get("penalty_beta", 1.0))
    s = P.Solver(C.product_case(w), w["degree"], P.options(**opt) if opt else None)
    perm = C.cell_perm(s.cell_table(), o.cells)
    return o, s, perm


def dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    _torch().cuda.synchronize()
    return t.cpu().numpy()


MESHES = [(C.tiny2d, r) for r in (1, 2, 3, 4, 5)] + [(C.tiny3d, r) for r in (1, 2, 3, 4, 5)] + \
         [(C.twolevel2d, 4), (C.twolevel3d, 3), (C.walls2d, 2)]


@pytest.mark.parametrize("mk,r", [(C.twolevel2d, 3), (C.twolevel3d, 2), (C.tiny3d, 4)])
def test_geometry_background_and_initial_state(mk, r):
    o, s, perm = pair(mk(r))
    x, y, z, wJ = (host(t) for t in s.node_geometry())
    for a, ref in ((x, o.x), (y, o.y), (z, o.z), (wJ, o.wJ)):
        assert C.rel_err(a, C.to_product_order(ref, perm, o.nloc)) < 1e-13
    U = host(s.init_state(10.0))
    Uo = C.to_product_order(o.initial_state(10.0), perm, o.nloc)
    for f in range(o.nf):
        assert C.rel_err(U[f], Uo[f]) < 1e-13, f


@pytest.mark.parametrize("mk,r", MESHES)
def test_explicit_residual(mk, r):
    o, s, perm = pair(mk(r))
    Uo = inputs.random_state(o.nf, o.N, seed=11 + r)
    Ro = o.explicit_residual(Uo)
    R = host(s.explicit_residual(dev(C.to_product_order(Uo, perm, o.nloc))))
    R = C.to_oracle_order(R, perm, o.nloc)
    for f in range(o.nf):
        assert C.rel_err(R[f], Ro[f]) < TOL64, (f, C.rel_err(R[f], Ro[f]))


@pytest.mark.parametrize("mk,r", [(C.tiny2d, 2), (C.tiny3d, 3), (C.twolevel2d, 4), (C.twolevel3d, 2), (C.walls2d, 3)])
def test_implicit_term(mk, r):
    o, s, perm = pair(mk(r))
    Uo = inputs.random_state(o.nf, o.N, seed=21 + r)
    Fo = o.implicit_term(Uo)
    F = C.to_oracle_order(host(s.implicit_term(dev(C.to_product_order(Uo, perm, o.nloc)))), perm, o.nloc)
    for f in range(1, o.nf):
        assert C.rel_err(F[f], Fo[f]) < TOL64, (f, C.rel_err(F[f], Fo[f]))


@pytest.mark.parametrize("mk,r", MESHES)
def test_helmholtz_fp64(mk, r):
    import paper_2408_08129_amd as P
    o, s, perm = pair(mk(r))
    h = inputs.random_positive(o.N, 31 + r, 2.5e5, 3.5e5)
    p = inputs.random_normal(o.N, 41 + r, 100.0)
    dta = 0.37
    ref = o.helmholtz(dta, h, o.cell_sound_speed(h), p)
    Ap = host(s.apply_helmholtz(dta, dev(C.to_product_order(h, perm, o.nloc)),
                                dev(C.to_product_order(p, perm, o.nloc)), P.DG_FP64))
    assert C.rel_err(C.to_oracle_order(Ap, perm, o.nloc), ref) < TOL64


@pytest.mark.parametrize("mk,r", [(C.tiny2d, 3), (C.tiny3d, 4), (C.twolevel2d, 4)])
def test_helmholtz_fp32(mk, r):
    import paper_2408_08129_amd as P
    torch = _torch()
    o, s, perm = pair(mk(r), precision=P.DG_FP32_INNER)
    h = inputs.random_positive(o.N, 51 + r, 2.5e5, 3.5e5)
    p = inputs.random_normal(o.N, 61 + r, 100.0)
    dta = 0.37
    # the oracle sees the FP32-rounded inputs
    h32 = h.astype(np.float32)
    p32 = p.astype(np.float32)
    ref = o.helmholtz(dta, h32.astype(np.float64), o.cell_sound_speed(h32.astype(np.float64)), p32.astype(np.float64))
    Ap = s.apply_helmholtz(dta, dev(C.to_product_order(h32, perm, o.nloc)),
                           dev(C.to_product_order(p32, perm, o.nloc)), P.DG_FP32_INNER)
    assert Ap.dtype == torch.float32
    Ap = C.to_oracle_order(host(Ap).astype(np.float64), perm, o.nloc)
    assert C.rel_err(Ap, ref) < 2e-5


def _run_pair(w, steps, ubar, dt, precision=0, tol=TOL_STEP, **opt):
    import paper_2408_08129_amd as P
    o, s, perm = pair(w, precision=precision, **opt)
    Uo = o.initial_state(ubar)
    U = dev(C.to_product_order(Uo, perm, o.nloc))
    for n in range(steps):
        st = {}
        Uo = o.step(Uo, dt, stats=st)
        gst = s.step(U, dt)
        print("step %d oracle its %s gpu its %s" % (n, st["gmres_iters"], gst.as_dict(2)["gmres_iters"]), flush=True)
    Ug = C.to_oracle_order(host(U), perm, o.nloc)
    errs = [C.rel_err(Ug[f], Uo[f]) for f in range(o.nf)]
    print("per-field max rel err", errs, flush=True)
    l2 = [math.sqrt(np.sum(o.wJ * (Ug[f] - Uo[f]) ** 2) / np.sum(o.wJ * Uo[f] ** 2)) for f in range(o.nf)]
    print("per-field L2 rel err", l2, flush=True)
    for f in range(o.nf):
        assert errs[f] < tol, (f, errs)
        assert l2[f] < tol, (f, l2)
    return o, s, Ug


def test_step_slice2d_r2_conforming_10_steps():
    w = cases.WORKLOADS["slice2d_r2_conforming"]
    _run_pair(w, 10, w["ubar"], w["dt"])


def test_step_twolevel2d_hanging():
    w = C.twolevel2d(4)
    _run_pair(w, 4, 10.0, 0.5)


def test_step_twolevel3d_hanging():
    w = C.twolevel3d(2)
    _run_pair(w, 3, 10.0, 1.0)


def test_step_slice2d_r4_twolevel_2_steps():
    w = cases.WORKLOADS["slice2d_r4_twolevel"]
    _run_pair(w, 2, w["ubar"], w["dt"])


@pytest.mark.parametrize("mk,r,steps,dt", [(C.twolevel2d, 1, 3, 0.5), (C.twolevel2d, 5, 2, 0.3),
                                            (C.twolevel3d, 1, 2, 1.0), (C.twolevel3d, 3, 2, 0.5),
                                            (C.tiny3d, 5, 2, 0.5), (C.walls2d, 3, 3, 0.5),
                                            (C.walls3d, 2, 2, 0.5)])
def test_step_every_degree_with_2to1_faces(mk, r, steps, dt):
    """Whole steps at the degrees the other step tests leave out (1, 3 and the largest, 5), and
    with lateral walls in 2D and 3D, on meshes with 2:1 faces, FP64."""
    _run_pair(mk(r), steps, 10.0, dt)


def test_step_diagonal_preconditioner():
    """The GPU's Jacobi-preconditioned Krylov path (general cell kernels) against the oracle."""
    _run_pair(C.twolevel3d(2), 2, 10.0, 1.0, preconditioner=0)


def test_step_plain_flux_without_penalty():
    """The plain implicit energy flux with penalty_beta = 0 on both sides."""
    _run_pair(C.twolevel2d(3), 3, 10.0, 0.5, penalty_beta=0.0)


@pytest.mark.parametrize("mk,r,dt", [(C.twolevel2d, 1, 0.5), (C.tiny3d, 5, 0.5)])
def test_step_mixed_precision_lowest_and_highest_degree(mk, r, dt):
    import paper_2408_08129_amd as P
    _run_pair(mk(r), 2, 10.0, dt, precision=P.DG_FP32_INNER, tol=TOL_MIXED)


def test_step_mixed_precision_degree3():
    import paper_2408_08129_amd as P
    _run_pair(C.twolevel3d(3), 2, 10.0, 0.5, precision=P.DG_FP32_INNER, tol=TOL_MIXED)


def test_step_mixed_precision():
    import paper_2408_08129_amd as P
    _run_pair(C.twolevel3d(2), 3, 10.0, 1.0, precision=P.DG_FP32_INNER, tol=TOL_MIXED)
    _run_pair(C.twolevel2d(4), 3, 10.0, 0.5, precision=P.DG_FP32_INNER, tol=TOL_MIXED)


def test_rest_state_stays_at_rest_on_gpu():
    w = C.twolevel3d(3, oro=3, h0=300.0)
    o, s, perm = pair(w)
    U = s.init_state(0.0)
    for _ in range(5):
        s.step(U, 2.0)
    Uh = host(U)
    umax = np.max(np.abs(Uh[1:1 + o.d] / Uh[0]))
    print("max |u| after 5 steps", umax, flush=True)
    assert umax < 1e-10


def test_mass_conservation_and_determinism():
    w = C.twolevel2d(3)
    o, s, perm = pair(w)
    U1 = s.init_state(10.0)
    U2 = s.init_state(10.0)
    m0, _ = s.diagnostics(U1)
    for _ in range(3):
        s.step(U1, 0.7)
        s.step(U2, 0.7)
    m1, _ = s.diagnostics(U1)
    assert abs(m1 - m0) < 1e-13 * m0
    assert np.array_equal(host(U1), host(U2))


def test_batched_equals_alone():
    import paper_2408_08129_amd as P
    torch = _torch()
    ws = [C.twolevel2d(3), C.tiny3d(2), C.twolevel2d(2)]
    solvers, states, alone = [], [], []
    for i, w in enumerate(ws):
        st = torch.cuda.Stream()
        s = P.Solver(C.product_case(w), w["degree"], stream=st)
        with torch.cuda.stream(st):
            U = s.init_state(10.0)
            Ua = U.clone()
        st.synchronize()
        solvers.append(s)
        states.append(U)
        for _ in range(2):
            s.step(Ua, 0.5)
        st.synchronize()
        alone.append(host(Ua))
    for _ in range(2):
        P.imex_rk2_step_batched([s.ctx for s in solvers], states, [0.5] * len(ws))
    torch.cuda.synchronize()
    for U, Ua in zip(states, alone):
        assert np.array_equal(host(U), Ua)


def test_errors_leave_state_unchanged():
    import paper_2408_08129_amd as P
    w = C.twolevel2d(2)
    o, s, perm = pair(w, gmres_maxit=1)
    U = s.init_state(10.0)
    before = host(U).copy()
    with pytest.raises(P.DGError) as e:
        s.step(U, 0.5)
    assert e.value.status == P.DG_ENOCONV
    assert np.array_equal(host(U), before)
    o, s, perm = pair(w)
    U = s.init_state(10.0)
    U[0, 5] = float("nan")
    before = host(U).copy()
    with pytest.raises(P.DGError) as e:
        s.step(U, 0.5)
    assert e.value.status == P.DG_ENAN
    after = host(U)
    assert np.array_equal(np.isnan(after), np.isnan(before))
    assert np.array_equal(after[~np.isnan(after)], before[~np.isnan(before)])
