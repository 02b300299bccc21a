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
