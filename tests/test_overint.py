"""Over-integration of the explicit flux (volume and face integrals with r + 1 + e Gauss points per
direction; mass matrix and gravity work unchanged).

Oracle pins (CPU): with r + 1 points the over-integrated routine is the nodal (collocated) residual
already pinned elsewhere, on meshes with walls and 2:1 faces; for a polynomial state whose fluxes
are polynomials the over-integrated weak form equals a brute-force evaluation with a 10-point rule
written here in numpy (while the nodal rule does not); mass is conserved across 2:1 faces; a free
stream stays steady.  GPU: the over-integrated residual and whole steps against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from tests import _common as C


def _oracle(mk, r, e=0, **kw):
    return O.Oracle(C.oracle_case(dict(mk(r), **kw)), quad_extra=e)


@pytest.mark.parametrize("mk,r", [(C.tiny2d, 2), (C.tiny3d, 3), (C.twolevel2d, 3), (C.twolevel3d, 2),
                                  (C.walls2d, 2)])
def test_nodal_rule_reproduces_collocation(mk, r):
    import ctypes
    o = _oracle(mk, r)
    L = O.lib()
    assert L.oc_set_quadrature(o._m, r + 1) == 0
    rng = np.random.default_rng(5)
    U = o.initial_state(3.0)
    U = U * (1.0 + 0.01 * rng.standard_normal(U.shape))
    U[1:1 + o.d] += 0.5 * rng.standard_normal((o.d, o.N)) * U[0]
    R0 = o.explicit_residual(U)
    R1 = np.zeros_like(U)
    Uc = np.ascontiguousarray(U)
    L.oc_explicit_residual_oi(o._m, Uc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              R1.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    for f in range(o.nf):
        scale = np.abs(R0[f]).max() + 1e-300
        assert np.abs(R1[f] - R0[f]).max() / scale < 1e-12, f


def _lagrange(xs, j, t):
    v = np.ones_like(t)
    for k, xk in enumerate(xs):
        if k != j:
            v = v * (t - xk) / (xs[j] - xs[k])
    return v


def _dlagrange(xs, j, t):
    out = np.zeros_like(t)
    for m_, xm in enumerate(xs):
        if m_ == j:
            continue
        term = np.ones_like(t) / (xs[j] - xm)
        for k, xk in enumerate(xs):
            if k != j and k != m_:
                term = term * (t - xk) / (xs[j] - xk)
        out = out + term
    return out


def _flux(d, X):
    """rho = 1 and a momentum polynomial of degree 2 per coordinate: the explicit fluxes
    (rho u, rho u (x) u, rho k u) are polynomials (degrees 2, 4, 6)."""
    x, z = X[0] / 1000.0, X[-1] / 1000.0
    y = X[1] / 1000.0 if d == 3 else 0.0
    m = [0.8 + 0.3 * x * z - 0.2 * z * z, 0.1 + 0.2 * x * x - 0.3 * x * z]
    if d == 3:
        m.insert(1, -0.4 + 0.25 * y * z + 0.1 * x * y)
        m[0] = m[0] + 0.15 * y * y
    m = np.array(m)
    rk = 0.5 * np.sum(m * m, axis=0)
    F = np.zeros((d + 2, d) + np.shape(x))
    for k in range(d):
        F[0, k] = m[k]
        for a in range(d):
            F[1 + a, k] = m[a] * m[k]
        F[1 + d, k] = rk * m[k]
    return m, F


def _brute_weak_form(o, cell_ids, dx):
    """sum over the cell of F . grad(phi_i) minus the boundary integral of (F . n) phi_i, with a
    10-point Gauss rule per direction (exact for these polynomials)."""
    d, r = o.d, o.r
    xs = np.polynomial.legendre.leggauss(r + 1)[0]
    g, gw = np.polynomial.legendre.leggauss(10)
    out = {}
    for c in cell_ids:
        lev, ix, iy, iz = o.cells[c]
        lo = np.array([ix * dx[0], iz * dx[-1]] if d == 2 else [ix * dx[0], iy * dx[1], iz * dx[2]])
        W = np.zeros((d + 2, o.nloc))
        # volume
        grids = np.meshgrid(*([g] * d), indexing="ij")
        wts = np.ones_like(grids[0])
        for a in range(d):
            wts = wts * gw[np.indices(grids[0].shape)[a]]
        X = [lo[a] + 0.5 * dx[a] * (1 + grids[a]) for a in range(d)]
        jac = np.prod([0.5 * dx[a] for a in range(d)])
        _, F = _flux(d, X)
        for i in range(o.nloc):
            ia = [(i // (r + 1) ** a) % (r + 1) for a in range(d)]
            for k in range(d):
                gphi = np.ones_like(grids[0])
                for a in range(d):
                    gphi = gphi * (_dlagrange(xs, ia[a], grids[a]) * 2.0 / dx[a] if a == k else
                                   _lagrange(xs, ia[a], grids[a]))
                for f in range(d + 2):
                    W[f, i] += np.sum(wts * F[f, k] * gphi) * jac
        # faces
        for k in range(d):
            for s in (0, 1):
                tg = [a for a in range(d) if a != k]
                fg = np.meshgrid(*([g] * (d - 1)), indexing="ij") if d == 3 else [g]
                fw = np.ones_like(fg[0])
                for t in range(d - 1):
                    fw = fw * gw[np.indices(fg[0].shape)[t]]
                Xf = [None] * d
                Xf[k] = np.full(fg[0].shape, lo[k] + s * dx[k])
                for t, a in enumerate(tg):
                    Xf[a] = lo[a] + 0.5 * dx[a] * (1 + fg[t])
                fjac = np.prod([0.5 * dx[a] for a in tg])
                _, Ff = _flux(d, Xf)
                sign = 1.0 if s else -1.0
                for i in range(o.nloc):
                    ia = [(i // (r + 1) ** a) % (r + 1) for a in range(d)]
                    phi = _lagrange(xs, ia[k], np.array(1.0 if s else -1.0)) * np.ones_like(fg[0])
                    for t, a in enumerate(tg):
                        phi = phi * _lagrange(xs, ia[a], fg[t])
                    for f in range(d + 2):
                        W[f, i] -= sign * np.sum(fw * Ff[f, k] * phi) * fjac
        out[c] = W
    return out


@pytest.mark.parametrize("d", [2, 3])
def test_overintegration_exact_for_polynomial_fluxes(d):
    r = 2
    if d == 2:
        case = O.Case(dim=2, degree=r, nbase=(4, 1, 4), length=(4000.0, 1.0, 4000.0), periodic=(1, 1),
                      atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0))
    else:
        case = O.Case(dim=3, degree=r, nbase=(4, 4, 4), length=(4000.0, 4000.0, 4000.0), periodic=(1, 1),
                      atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0))
    o = O.Oracle(case, quad_extra=2)
    o0 = O.Oracle(case)
    Xn = [o.x, o.z] if d == 2 else [o.x, o.y, o.z]
    m, _ = _flux(d, Xn)
    U = np.zeros((o.nf, o.N))
    U[0] = 1.0
    U[1:1 + d] = m
    # the explicit fluxes do not involve the energy; a small constant keeps the rounding of its
    # traces (which the Rusanov jump term sees) below the tolerance
    U[1 + d] = 2.0
    dx = [1000.0] * d
    # interior cells: away from the walls and from the periodic seams (the polynomial is not
    # periodic), so every face sees a continuous state and the numerical flux is F(U).n
    inner = [c for c in range(o.ncell) if all(1 <= v <= 2 for v in (list(o.cells[c][1:3]) if d == 3 else
                                                                    [o.cells[c][1], o.cells[c][3]]))
             and (d == 2 or 1 <= o.cells[c][3] <= 2)]
    assert len(inner) == (4 if d == 2 else 8)
    ref = _brute_weak_form(o, inner, dx)

    def weak(oo):
        R = oo.explicit_residual(U)
        R[1 + d] += O.G * U[d]  # the pointwise gravity work is not part of the flux weak form
        return (R * oo.wJ[None, :]).reshape(o.nf, o.ncell, o.nloc)

    Woi, W0 = weak(o), weak(o0)
    err_oi = max(np.abs(Woi[:, c] - ref[c]).max() / np.abs(ref[c]).max() for c in inner)
    err_0 = max(np.abs(W0[:, c] - ref[c]).max() / np.abs(ref[c]).max() for c in inner)
    assert err_oi < 1e-11, err_oi
    assert err_0 > 1e-6, err_0  # the nodal rule is not exact here: the test sees the quadrature


@pytest.mark.parametrize("mk,r,e", [(C.twolevel2d, 3, 1), (C.twolevel3d, 2, 2)])
def test_overintegrated_mass_conserved_across_hanging_faces(mk, r, e):
    o = _oracle(mk, r, e)
    assert o.nhang > 0
    rng = np.random.default_rng(9)
    U = o.initial_state(5.0)
    U[0] *= 1.0 + 0.02 * rng.standard_normal(o.N)
    U[1:1 + o.d] += 2.0 * rng.standard_normal((o.d, o.N))
    R = o.explicit_residual(U)
    total = float(np.sum(o.wJ * R[0]))
    scale = float(np.sum(o.wJ * np.abs(R[0])))
    assert abs(total) < 1e-12 * scale


def test_overintegrated_free_stream():
    case = O.Case(dim=3, degree=3, nbase=(2, 2, 2), length=(2000.0, 2000.0, 2000.0), periodic=(1, 1),
                  atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0))
    o = O.Oracle(case, quad_extra=2)
    U = np.zeros((o.nf, o.N))
    U[0] = 1.2
    U[1] = 1.2 * 7.0
    U[2] = -1.2 * 3.0
    U[4] = 2.5e5
    R = o.explicit_residual(U)
    assert np.abs(R).max() < 1e-9 * np.abs(U[1]).max()


def test_quad_extra_out_of_range():
    with pytest.raises(ValueError):
        _oracle(C.tiny2d, 2, 20)


# ------------------------------------------------------------------------------- library / GPU
def test_quad_extra_option_validated():
    import paper_2408_08129_amd as P
    assert P.options().quad_extra == 0
    w = C.tiny3d(2)
    base = P.dg_footprint(C.product_case(w), 2)
    assert P.dg_footprint(C.product_case(w), 2, P.options(quad_extra=3)) >= base
    with pytest.raises(P.DGError) as e:
        P.dg_footprint(C.product_case(w), 2, P.options(quad_extra=-1))
    assert e.value.status == P.DG_EINVAL
    for deg, ex in [(5, 3), (2, 4)]:
        with pytest.raises(P.DGError) as e:
            P.dg_footprint(C.product_case(C.tiny3d(deg)), deg, P.options(quad_extra=ex))
        assert e.value.status == P.DG_EUNSUPPORTED


def _gpu_pair(w, e, **opt):
    import paper_2408_08129_amd as P
    print("[case] %s quad_extra %d" % ({k: w[k] for k in ("dim", "degree", "nbase")}, e), flush=True)
    o = O.Oracle(C.oracle_case(w), quad_extra=e)
    s = P.Solver(C.product_case(w), w["degree"], P.options(quad_extra=e, **opt))
    perm = C.cell_perm(s.cell_table(), o.cells)
    return o, s, perm


@pytest.mark.gpu
@pytest.mark.parametrize("mk,r,e", [(C.tiny2d, 2, 1), (C.tiny2d, 1, 3), (C.tiny3d, 3, 1), (C.tiny3d, 2, 3),
                                    (C.tiny3d, 5, 2), (C.twolevel2d, 4, 1), (C.twolevel2d, 3, 2),
                                    (C.twolevel3d, 2, 2), (C.twolevel3d, 4, 1), (C.walls2d, 2, 1)])
def test_gpu_overintegrated_residual(mk, r, e):
    from paper_2408_08129_amd import inputs
    from tests.test_gpu_parity import TOL64, dev, host
    o, s, perm = _gpu_pair(mk(r), e)
    Uo = inputs.random_state(o.nf, o.N, seed=31 + r + 7 * e)
    Ro = o.explicit_residual(Uo)
    R = C.to_oracle_order(host(s.explicit_residual(dev(C.to_product_order(Uo, perm, o.nloc)))), perm, o.nloc)
    for f in range(o.nf):
        assert C.rel_err(R[f], Ro[f]) < TOL64, (f, C.rel_err(R[f], Ro[f]))
    # over-integration changes the result (the test is not passing on the nodal kernel)
    o0 = O.Oracle(C.oracle_case(mk(r)))
    assert max(C.rel_err(o0.explicit_residual(Uo)[f], Ro[f]) for f in range(o.nf)) > 1e-8


@pytest.mark.gpu
@pytest.mark.parametrize("mk,r,e,steps,dt,prec", [(C.twolevel3d, 2, 1, 3, 1.0, 0), (C.twolevel2d, 4, 2, 4, 0.5, 0),
                                                 (C.twolevel2d, 3, 1, 2, 0.5, 1)])
def test_gpu_overintegrated_steps(mk, r, e, steps, dt, prec):
    """Steps with the over-integrated explicit flux against the oracle; the last case with the
    FP32-inner / FP64-outer solve (tolerance of the mixed form)."""
    import math
    from tests.test_gpu_parity import TOL_MIXED, TOL_STEP, dev, host
    if prec:
        TOL_STEP = TOL_MIXED
    o, s, perm = _gpu_pair(mk(r), e, precision=prec)
    Uo = o.initial_state(10.0)
    U = dev(C.to_product_order(Uo, perm, o.nloc))
    for n in range(steps):
        Uo = o.step(Uo, dt)
        s.step(U, dt)
    Ug = C.to_oracle_order(host(U), perm, o.nloc)
    for f in range(o.nf):
        err = C.rel_err(Ug[f], Uo[f])
        l2 = math.sqrt(np.sum(o.wJ * (Ug[f] - Uo[f]) ** 2) / np.sum(o.wJ * Uo[f] ** 2))
        print("field %d max rel %.2e L2 rel %.2e" % (f, err, l2), flush=True)
        assert err < TOL_STEP and l2 < TOL_STEP, (f, err, l2)
