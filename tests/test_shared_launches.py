"""Shared launches of ensemble members (imex_rk2_step_batched): members of one class (dimension,
degree, precision, preconditioner, energy-flux form) advance in lockstep through segment-table
launches.  Each member's step must be the same bits alone (a batch of one) and in any mix, and
agree with the single-context step; a member that fails leaves the others untouched."""
import numpy as np
import pytest

from tests import _common as C


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def host(U):
    return U.detach().cpu().numpy().copy()


def make(ws, **opt):
    import paper_2408_08129_amd as P
    _torch()
    out = []
    for w in ws:
        s = P.Solver(C.product_case(w), w["degree"], P.options(**opt) if opt else None)
        out.append(s)
    return out


def batched(P, solvers, states, dts, steps):
    status = None
    for _ in range(steps):
        _, status = P.imex_rk2_step_batched([s.ctx for s in solvers], states, dts, raise_on_error=False)
    _torch().cuda.synchronize()
    return status


def check_alone_equals_mix(ws, dts, steps=2, **opt):
    import paper_2408_08129_amd as P
    print("[case] shared launches", [(w["dim"], w["degree"], w["nbase"]) for w in ws], opt, flush=True)
    solvers = make(ws, **opt)
    init = [s.init_state(10.0, noise_seed=7 + i, noise_sigma_K=0.05) for i, s in enumerate(solvers)]
    alone = []
    for s, U0, dt in zip(solvers, init, dts):
        U = U0.clone()
        st = batched(P, [s], [U], [dt], steps)
        assert st == [0]
        alone.append(host(U))
    mix = [U0.clone() for U0 in init]
    st = batched(P, solvers, mix, dts, steps)
    assert st == [0] * len(ws)
    for i, (U, a) in enumerate(zip(mix, alone)):
        assert np.array_equal(host(U), a), i
    # the single-context step (direct launches) computes the same arithmetic
    for i, (s, U0, dt) in enumerate(zip(solvers, init, dts)):
        U = U0.clone()
        for _ in range(steps):
            s.step(U, dt)
        d = host(U)
        err = max(C.rel_err(d[f], alone[i][f]) for f in range(d.shape[0]))
        print("member %d: shared vs direct max rel diff %.3e" % (i, err), flush=True)
        assert err <= 1e-13
    return solvers


@pytest.mark.gpu
def test_shared_2d_members_of_different_sizes():
    ws = [C.twolevel2d(3), C.tiny2d(3), C.walls2d(3), C.tiny2d(3, oro=1, h0=80.0)]
    check_alone_equals_mix(ws, [0.5, 0.4, 0.5, 0.3])


@pytest.mark.gpu
def test_shared_3d_members_fp64_and_mixed_precision():
    ws = [C.tiny3d(2), C.twolevel3d(2), C.tiny3d(2, oro=2, h0=90.0)]
    check_alone_equals_mix(ws, [0.5, 0.5, 0.4])
    check_alone_equals_mix(ws, [0.5, 0.5, 0.4], precision=1)


@pytest.mark.gpu
def test_shared_enthalpy_split_members():
    ws = [C.tiny3d(3), C.twolevel3d(3)]
    check_alone_equals_mix(ws, [0.5, 0.5], enthalpy_split=1, penalty_beta=0.0)
    check_alone_equals_mix(ws, [0.5, 0.5], enthalpy_split=1, penalty_beta=0.0, precision=1)


@pytest.mark.gpu
def test_shared_chunked_launches_and_failure_isolation():
    """More members than one segment table holds (several launches per step), one of them failing."""
    import paper_2408_08129_amd as P
    torch = _torch()
    ws = [C.tiny2d(2, h0=60.0 + 10.0 * i) for i in range(11)]
    print("[case] shared launches, 11 members, member 4 poisoned", flush=True)
    solvers = make(ws)
    init = [s.init_state(10.0) for s in solvers]
    alone = []
    for s, U0 in zip(solvers, init):
        U = U0.clone()
        assert batched(P, [s], [U], [0.5], 2) == [0]
        alone.append(host(U))
    mix = [U0.clone() for U0 in init]
    mix[4][0, 3] = float("nan")
    before = host(mix[4])
    _, st = P.imex_rk2_step_batched([s.ctx for s in solvers], mix, [0.5] * 11, raise_on_error=False)
    torch.cuda.synchronize()
    assert st[4] == P.DG_ENAN and all(v == 0 for i, v in enumerate(st) if i != 4)
    after = host(mix[4])
    assert np.array_equal(np.isnan(after), np.isnan(before))
    assert np.array_equal(after[~np.isnan(after)], before[~np.isnan(before)])
    # the survivors take a second step together and match their alone runs
    rest = [i for i in range(11) if i != 4]
    st = batched(P, [solvers[i] for i in rest], [mix[i] for i in rest], [0.5] * len(rest), 1)
    assert st == [0] * len(rest)
    for i in rest:
        assert np.array_equal(host(mix[i]), alone[i]), i


@pytest.mark.gpu
def test_shared_members_of_several_classes():
    """One call with three classes (2D r=3, 3D r=2, 2D r=2): each class shares its launches."""
    import paper_2408_08129_amd as P
    ws = [C.tiny2d(3), C.tiny3d(2), C.twolevel2d(3), C.tiny2d(2), C.twolevel3d(2), C.twolevel2d(2)]
    print("[case] shared launches, three classes", flush=True)
    solvers = make(ws)
    init = [s.init_state(10.0) for s in solvers]
    alone = []
    for s, U0 in zip(solvers, init):
        U = U0.clone()
        assert batched(P, [s], [U], [0.5], 2) == [0]
        alone.append(host(U))
    mix = [U0.clone() for U0 in init]
    assert batched(P, solvers, mix, [0.5] * len(ws), 2) == [0] * len(ws)
    for i in range(len(ws)):
        assert np.array_equal(host(mix[i]), alone[i]), i


@pytest.mark.gpu
def test_shared_fallback_paths():
    """Members whose launches the team makes one per member: the Jacobi-preconditioned operator
    (general cell kernel) and the over-integrated explicit residual."""
    check_alone_equals_mix([C.tiny2d(3), C.twolevel2d(3)], [0.5, 0.5], preconditioner=0)
    check_alone_equals_mix([C.tiny3d(2), C.twolevel3d(2)], [0.5, 0.5], quad_extra=1)


@pytest.mark.gpu
def test_shared_team_with_a_two_round_trip_member():
    """A member above 2^23 nodes per field keeps two host round trips per Krylov iteration; in a
    team with a small member (one round trip) both keep their own arithmetic."""
    from paper_2408_08129_amd import cases
    big = dict(cases.WORKLOADS["box3d_r4_hill"])
    small = C.tiny3d(4)
    check_alone_equals_mix([big, small], [big["dt"], 0.5], steps=1)


@pytest.mark.gpu
def test_shared_rejects_a_repeated_member():
    import paper_2408_08129_amd as P
    print("[case] shared launches, one context twice", flush=True)
    s, = make([C.tiny2d(2)])
    U = s.init_state(10.0)
    Ua = U.clone()
    assert batched(P, [s], [Ua], [0.5], 1) == [0]
    V = U.clone()
    _, st = P.imex_rk2_step_batched([s.ctx, s.ctx], [U, V], [0.5, 0.5], raise_on_error=False)
    _torch().cuda.synchronize()
    assert st == [0, P.DG_EINVAL]
    assert np.array_equal(host(U), host(Ua))
    assert np.array_equal(host(V), host(s.init_state(10.0)))


@pytest.mark.gpu
def test_shared_team_members_match_the_oracle():
    """Members stepped together in shared launches end where the FP64 oracle ends."""
    import math
    import paper_2408_08129_amd as P
    from oracle import oracle as O
    from tests.test_gpu_parity import TOL_STEP
    ws = [C.twolevel2d(3), C.tiny2d(3), C.walls2d(3)]
    print("[case] shared team vs oracle", [(w["dim"], w["degree"], w["nbase"]) for w in ws], flush=True)
    solvers = make(ws)
    oracles = [O.Oracle(C.oracle_case(w)) for w in ws]
    perms = [C.cell_perm(s.cell_table(), o.cells) for s, o in zip(solvers, oracles)]
    Uo = [o.initial_state(10.0) for o in oracles]
    torch = _torch()
    U = [torch.from_numpy(C.to_product_order(u, p, o.nloc)).cuda() for u, p, o in zip(Uo, perms, oracles)]
    dts = [0.5, 0.4, 0.5]
    assert batched(P, solvers, U, dts, 2) == [0, 0, 0]
    for i, (o, p) in enumerate(zip(oracles, perms)):
        ref = Uo[i]
        for _ in range(2):
            ref = o.step(ref, dts[i])
        Ug = C.to_oracle_order(host(U[i]), p, o.nloc)
        for f in range(o.nf):
            err = C.rel_err(Ug[f], ref[f])
            l2 = math.sqrt(np.sum(o.wJ * (Ug[f] - ref[f]) ** 2) / max(np.sum(o.wJ * ref[f] ** 2), 1e-300))
            print("member %d field %d max rel %.2e L2 rel %.2e" % (i, f, err, l2), flush=True)
            assert err < TOL_STEP, (i, f, err)
