"""Absorbing layers (Section 3.1 defers the non-reflecting boundaries to cited work).

Reading: Rayleigh friction on the momentum, d m/dt = -tau (m - rho u_ref e_x), in the explicit
part of the IMEX split, with the sin^2 rate profile of Klemp and Lilly (1978) below the lid and
along the lateral sides, walled or periodic (at a periodic seam the layer absorbs what leaves one
side before it re-enters on the other).

Oracle pins (CPU): a uniform wind over flat ground is a steady state of the undamped equations, and
stays one under a top layer (its rate varies across the wind only), so inside that layer every
node's momentum must decay by exactly the explicit ARK2 amplification factor of d m/dt = -tau m
per step (computed here from the Butcher tableau, independently of the DG code) and stay
unchanged outside it; every layer leaves the wind alone when u_ref equals it; the rate profile
integrates to rate * thickness / 2 over each boundary.  (Lateral layers vary along the wind, so
the damped wind is no longer steady and has no closed form.)  GPU parity: explicit residual and whole steps with layers against the oracle."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def ark2_explicit_factor(o, z):
    """Amplification of y' = lam y over one step of the explicit tableau, z = lam dt."""
    A, b = o.A, o.b
    Y = []
    for i in range(3):
        Y.append(1.0 + z * sum(A[i, j] * Y[j] for j in range(i)))
    return 1.0 + z * sum(b[j] * Y[j] for j in range(3))


def layered_case(dim, sponge, periodic):
    if dim == 2:
        return O.Case(dim=2, degree=3, nbase=(4, 1, 4), length=(4000.0, 1.0, 4000.0), periodic=periodic,
                      atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0), sponge=sponge)
    return O.Case(dim=3, degree=2, nbase=(2, 4, 2), length=(2000.0, 4000.0, 2000.0), periodic=periodic,
                  atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0), sponge=sponge)


@pytest.mark.parametrize("dim,sponge,periodic", [
    (2, (2000.0, 0.02, 0.0, 0.0, 0.0), (1, 1)),      # top layer, 2D
    (3, (800.0, 0.03, 0.0, 0.0, 0.0), (1, 0)),       # top layer, 3D, y walls
])
def test_layer_damps_uniform_wind_at_the_explicit_rk_rate(dim, sponge, periodic):
    o = O.Oracle(layered_case(dim, sponge, periodic))
    u0, dt, K = 1.0, 2.0, 10
    U = o.initial_state(u0)
    m0 = U[1].copy()
    for _ in range(K):
        U = o.step(U, dt)
    tau = o.tau
    assert np.any(tau > 0.0) and np.any(tau == 0.0)
    expect = m0 * np.array([ark2_explicit_factor(o, -t * dt) for t in tau]) ** K
    inside = tau > 0.0
    assert np.max(np.abs(U[1] - expect) / np.abs(m0)) < 2e-5
    assert np.max(np.abs(U[1][~inside] - m0[~inside]) / np.abs(m0[~inside])) < 2e-5
    # the strongest node has really decayed (the test would pass trivially otherwise)
    assert np.min(U[1] / m0) < 0.75


@pytest.mark.parametrize("dim,sponge,periodic", [
    (2, (2000.0, 0.02, 0.0, 0.0, 3.0), (1, 1)),
    (2, (2000.0, 0.02, 1000.0, 0.03, 3.0), (1, 1)),   # layers at the periodic x seam
    (3, (800.0, 0.03, 600.0, 0.02, 3.0), (1, 0)),
])
def test_layer_leaves_the_reference_wind_alone(dim, sponge, periodic):
    o = O.Oracle(layered_case(dim, sponge, periodic))
    U = o.initial_state(3.0)
    U0 = U.copy()
    for _ in range(3):
        U = o.step(U, 2.0)
    assert np.max(np.abs(U[1] - U0[1])) < 1e-10 * np.max(np.abs(U0[1]))


@pytest.mark.parametrize("dim,sponge,periodic,expect", [
    # integral of the rate over the domain: each layer contributes rate * (its depth or width) / 2
    # times the area of its boundary (the mean of sin^2 over a quarter period is 1/2); in 3D the
    # four lateral sides of the 2 x 4 x 2 km box: two of 4 x 2 km^2 (x = 0, the periodic seam
    # x = Lx) and two of 2 x 2 km^2 (the y walls)
    (2, (2000.0, 0.05, 0.0, 0.0, 0.0), (1, 1), 0.05 * 2000.0 / 2 * 4000.0),
    (3, (0.0, 0.0, 1000.0, 0.02, 0.0), (1, 0),
     2 * 0.02 * 1000.0 / 2 * (4000.0 * 2000.0 + 2000.0 * 2000.0)),
])
def test_layer_rate_integrates_to_half_rate_times_thickness(dim, sponge, periodic, expect):
    c = layered_case(dim, sponge, periodic)
    c.degree = 5  # Gauss quadrature of the smooth profile on cells aligned with the layer
    o = O.Oracle(c)
    total = float(np.sum(o.wJ * o.tau))
    assert abs(total - expect) < 1e-6 * expect
    # non-negative, and below the sum of the rates that can meet at one node (the top and one
    # layer per lateral axis), reached only on the boundary itself
    assert np.all(o.tau >= 0.0) and np.max(o.tau) < sponge[1] + (dim - 1) * sponge[3]


# ------------------------------------------------------------------------------- GPU parity
def _sponged(w, sponge, periodic=None):
    w = dict(w)
    w["sponge"] = sponge
    if periodic is not None:
        w["periodic"] = periodic
    return w


def _layer_cases():
    from tests import _common as C
    return [
        _sponged(C.walls2d(3), (1500.0, 0.03, 2000.0, 0.02, 4.0)),
        _sponged(C.twolevel3d(2), (800.0, 0.05, 1200.0, 0.02, -3.0), periodic=(1, 0)),
        _sponged(C.tiny3d(4), (400.0, 0.1, 0.0, 0.0, 2.0)),
    ]


@pytest.mark.gpu
@pytest.mark.parametrize("i", [0, 1, 2])
def test_gpu_explicit_residual_with_layers(i):
    from paper_2408_08129_amd import inputs
    from tests import _common as C
    from tests.test_gpu_parity import TOL64, dev, host, pair
    w = _layer_cases()[i]
    o, s, perm = pair(w)
    assert np.any(o.tau > 0.0)
    Uo = inputs.random_state(o.nf, o.N, seed=71 + i)
    Ro = o.explicit_residual(Uo)
    R = C.to_oracle_order(host(s.explicit_residual(dev(C.to_product_order(Uo, perm, o.nloc)))), perm, o.nloc)
    for f in range(o.nf):
        assert C.rel_err(R[f], Ro[f]) < TOL64, (f, C.rel_err(R[f], Ro[f]))


@pytest.mark.gpu
@pytest.mark.parametrize("i", [0, 1])
def test_gpu_steps_with_layers(i):
    from tests.test_gpu_parity import _run_pair
    _run_pair(_layer_cases()[i], 3, 6.0, 0.5)


@pytest.mark.gpu
def test_gpu_steps_with_layers_fp32_inner():
    import paper_2408_08129_amd as P
    from tests.test_gpu_parity import TOL_MIXED, _run_pair
    _run_pair(_layer_cases()[0], 3, 6.0, 0.5, precision=P.DG_FP32_INNER, tol=TOL_MIXED)


def test_invalid_layer_parameters_rejected():
    import paper_2408_08129_amd as P
    from tests import _common as C
    for sp in [(-1.0, 0.01, 0.0, 0.0, 0.0), (0.0, 0.01, 0.0, 0.0, 0.0), (5000.0, 0.01, 0.0, 0.0, 0.0),
               (100.0, 0.01, 0.0, -0.5, 0.0), (100.0, 0.01, 0.0, 0.0, float("nan"))]:
        w = dict(C.walls2d(2))
        w["sponge"] = sp
        with pytest.raises(P.DGError) as e:
            P.dg_footprint(C.product_case(w), 2)
        assert e.value.status == P.DG_EINVAL, sp
    w = dict(C.walls2d(2))
    w["sponge"] = (1000.0, 0.01, 500.0, 0.02, 3.0)
    assert P.dg_footprint(C.product_case(w), 2) > 0
