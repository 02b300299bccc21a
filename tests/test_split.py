"""The enthalpy split of the implicit energy flux (an option; the reading that keeps long runs in a
stratified atmosphere stable).

The plain flux C(h m) makes the discrete buoyancy balance of grid-scale modes depend on the
commutator C(hbar m) - hbar C(m), which stands for M m . grad(hbar); since d hbar/dz + g =
c_p T N^2 / g is a small difference of large terms, an O(1) error in it turns the effective N^2
of those modes negative and they grow (e-folding 20-60 s).  The split writes the background part
as hbar C(m) + M (d hbar/dz) m_z, with the continuity equation's divergence and the exact
gradient.

Oracle pins (CPU): d hbar/dz is the derivative of the closed-form background; in an isothermal
atmosphere (hbar constant) the split is the plain flux; the rest state stays at rest; a stratified
column seeded with 1e-3 K noise (pressure-jump penalty off) grows without the split and stays at
the noise level with it.  GPU: operators and steps with the split against the oracle."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from tests import _common as C


def _column(atm, nx=2, nz=16, r=4):
    atm_kind, atm_par = (O.STRATIFIED, (1e5, 293.15, 0.01)) if atm == "strat" else (O.ISOTHERMAL, (1e5, 250.0))
    return O.Case(dim=2, degree=r, nbase=(nx, 1, nz), length=(1000.0 * nx, 1.0, 1000.0 * nz), periodic=(1, 1),
                  atm_kind=atm_kind, atm=atm_par)


def test_background_enthalpy_derivative():
    o = O.Oracle(C.oracle_case(C.twolevel2d(3)))
    L = O.lib()
    atm = (ctypes.c_double * 3)(*[float(v) for v in o.case.atm] + [0.0] * (3 - len(o.case.atm)))
    p, r = ctypes.c_double(), ctypes.c_double()

    def hbar(z):
        L.oc_background(o.case.atm_kind, atm, z, ctypes.byref(p), ctypes.byref(r))
        return O.GAMMA * p.value / ((O.GAMMA - 1.0) * r.value)

    for k in range(0, o.N, max(1, o.N // 50)):
        z, dz = float(o.z[k]), 1.0
        fd = (hbar(z + dz) - hbar(z - dz)) / (2 * dz)
        assert abs(o.hbar[k] - hbar(z)) < 1e-9 * o.hbar[k]
        assert abs(o.dhbar[k] - fd) < 1e-6 * abs(fd)
    # stratified: d hbar/dz + g = c_p T N^2 / g > 0 (stable stratification)
    assert np.all(o.dhbar + O.G > 0)


def test_split_is_plain_flux_in_isothermal_atmosphere():
    c = _column("iso", 3, 4, 3)
    o0, o1 = O.Oracle(c), O.Oracle(c, enthalpy_split=True)
    assert np.all(o1.dhbar == 0.0)
    rng = np.random.default_rng(3)
    h = 3e5 * (1.0 + 0.1 * rng.standard_normal(o0.N))
    m = rng.standard_normal((o0.d, o0.N))
    a, b = o0.enthalpy_flux_div(h, m), o1.enthalpy_flux_div(h, m)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_split_keeps_rest_state():
    o = O.Oracle(C.oracle_case(C.twolevel2d(3)), enthalpy_split=True)
    U = o.initial_state(0.0)
    for _ in range(3):
        U = o.step(U, 2.0)
    assert np.max(np.abs(U[1:1 + o.d] / U[0])) < 1e-10


@pytest.mark.parametrize("split,bound", [(False, None), (True, 0.05)])
def test_stratified_column_stability(split, bound):
    o = O.Oracle(_column("strat"), beta=0.0, enthalpy_split=split)
    rng = np.random.default_rng(1)
    U = o.initial_state(0.0, dT=1e-3 * rng.standard_normal(o.N))
    for _ in range(160):  # 320 s
        U = o.step(U, 2.0, rtol=1e-10)
    w = float(np.max(np.abs(U[o.d] / U[0])))
    if split:
        assert w < bound, w
    else:
        assert w > 0.1, w  # the plain flux: grid-scale buoyancy modes have grown from 1e-3 K noise


# ------------------------------------------------------------------------------- library / GPU
def test_split_option_validated():
    import paper_2408_08129_amd as P
    assert P.options().enthalpy_split == 0
    with pytest.raises(P.DGError) as e:
        P.dg_footprint(C.product_case(C.tiny2d(2)), 2, P.options(enthalpy_split=2))
    assert e.value.status == P.DG_EINVAL
    assert P.dg_footprint(C.product_case(C.tiny2d(2)), 2, P.options(enthalpy_split=1)) > \
        P.dg_footprint(C.product_case(C.tiny2d(2)), 2)


def _gpu_pair(w, beta=1.0, **opt):
    import paper_2408_08129_amd as P
    print("[case] %s split beta %g %s" % ({k: w[k] for k in ("dim", "degree", "nbase")}, beta, opt), flush=True)
    o = O.Oracle(C.oracle_case(w), beta=beta, enthalpy_split=True)
    s = P.Solver(C.product_case(w), w["degree"], P.options(enthalpy_split=1, penalty_beta=beta, **opt))
    perm = C.cell_perm(s.cell_table(), o.cells)
    return o, s, perm


@pytest.mark.gpu
@pytest.mark.parametrize("mk,r", [(C.tiny3d, 3), (C.twolevel2d, 4), (C.twolevel3d, 2), (C.walls2d, 3)])
def test_gpu_split_operators(mk, r):
    import paper_2408_08129_amd as P
    from paper_2408_08129_amd import inputs
    from tests.test_gpu_parity import TOL64, dev, host
    o, s, perm = _gpu_pair(mk(r))
    U = inputs.random_state(o.nf, o.N, seed=91 + r)
    Fo = o.implicit_term(U)
    F = C.to_oracle_order(host(s.implicit_term(dev(C.to_product_order(U, perm, o.nloc)))), perm, o.nloc)
    for f in range(1, o.nf):
        assert C.rel_err(F[f], Fo[f]) < TOL64, (f, C.rel_err(F[f], Fo[f]))
    h = inputs.random_positive(o.N, 92 + r, 2.5e5, 3.5e5)
    p = inputs.random_normal(o.N, 93 + r, 100.0)
    dta = 0.37
    ref = o.helmholtz(dta, h, o.cell_sound_speed(h), p)
    Ap = host(s.apply_helmholtz(dta, dev(C.to_product_order(h, perm, o.nloc)),
                                dev(C.to_product_order(p, perm, o.nloc)), P.DG_FP64))
    assert C.rel_err(C.to_oracle_order(Ap, perm, o.nloc), ref) < TOL64
    # the split differs from the plain flux here (stratified background)
    o0 = O.Oracle(C.oracle_case(mk(r)))
    assert C.rel_err(o0.helmholtz(dta, h, o0.cell_sound_speed(h), p), ref) > 1e-8
    # FP32 operator with the oracle fed the FP32-rounded inputs
    o32, s32, perm = _gpu_pair(mk(r), precision=P.DG_FP32_INNER)
    h32, p32 = h.astype(np.float32), p.astype(np.float32)
    ref = o32.helmholtz(dta, h32.astype(np.float64), o32.cell_sound_speed(h32.astype(np.float64)),
                        p32.astype(np.float64))
    Ap = s32.apply_helmholtz(dta, dev(C.to_product_order(h32, perm, o.nloc)),
                             dev(C.to_product_order(p32, perm, o.nloc)), P.DG_FP32_INNER)
    assert C.rel_err(C.to_oracle_order(host(Ap).astype(np.float64), perm, o.nloc), ref) < 2e-5


@pytest.mark.gpu
@pytest.mark.parametrize("mk,r,beta,steps,dt,prec", [(C.twolevel3d, 2, 1.0, 3, 1.0, 0), (C.twolevel2d, 4, 0.0, 4, 0.5, 0),
                                                     (C.twolevel3d, 2, 0.0, 3, 1.0, 1)])
def test_gpu_split_steps(mk, r, beta, steps, dt, prec):
    import math
    from tests.test_gpu_parity import TOL_MIXED, TOL_STEP, dev, host
    o, s, perm = _gpu_pair(mk(r), beta=beta, precision=prec)
    Uo = o.initial_state(10.0)
    U = dev(C.to_product_order(Uo, perm, o.nloc))
    for _ in range(steps):
        Uo = o.step(Uo, dt)
        s.step(U, dt)
    Ug = C.to_oracle_order(host(U), perm, o.nloc)
    tol = TOL_MIXED if prec else TOL_STEP
    for f in range(o.nf):
        err = C.rel_err(Ug[f], Uo[f])
        l2 = math.sqrt(np.sum(o.wJ * (Ug[f] - Uo[f]) ** 2) / np.sum(o.wJ * Uo[f] ** 2))
        print("field %d max rel %.2e L2 rel %.2e" % (f, err, l2), flush=True)
        assert err < tol and l2 < tol, (f, err, l2)
