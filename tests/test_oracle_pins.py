"""Pins of the FP64 oracle against what the paper and the mathematics fix (no GPU needed)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def tiny2d(r, oro=O.FLAT, h0=0.0, periodic=(0, 0)):
    """2x2 base quads with the lower-left cell refined once: 7 cells, hanging faces in x and z."""
    return O.Case(dim=2, degree=r, nbase=(2, 1, 2), length=(1000.0, 1.0, 1000.0), periodic=periodic,
                  rules=[(500.0, 250.0, 250.0, 0, 0)], oro_kind=oro, oro=(h0, 300.0, 500.0, 0.0),
                  atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0))


def tiny3d(r, oro=O.FLAT, h0=0.0, periodic=(0, 0)):
    """2x2x2 base hexes with one corner cell refined once: 15 cells."""
    return O.Case(dim=3, degree=r, nbase=(2, 2, 2), length=(1000.0, 1000.0, 1000.0), periodic=periodic,
                  rules=[(500.0, 250.0, 250.0, 250.0, 250.0)], oro_kind=oro,
                  oro=(h0, 300.0, 500.0, 500.0), atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0))


def twolevel2d(r, oro=O.FLAT, h0=0.0, periodic=(0, 0)):
    """4x4 base with two nested refinement levels: hanging faces of both orientations."""
    return O.Case(dim=2, degree=r, nbase=(4, 1, 4), length=(4000.0, 1.0, 2000.0), periodic=periodic,
                  rules=[(1000.0, 2000.0, 1500.0, 0, 0), (500.0, 2000.0, 700.0, 0, 0)],
                  oro_kind=oro, oro=(h0, 500.0, 2000.0, 0.0), atm_kind=O.ISOTHERMAL,
                  atm=(1e5, 250.0))


def twolevel3d(r, oro=O.FLAT, h0=0.0, periodic=(0, 0)):
    return O.Case(dim=3, degree=r, nbase=(3, 3, 2), length=(3000.0, 3000.0, 2000.0), periodic=periodic,
                  rules=[(1000.0, 1500.0, 1000.0, 1500.0, 1000.0)], oro_kind=oro,
                  oro=(h0, 500.0, 1500.0, 1500.0), atm_kind=O.ISOTHERMAL, atm=(1e5, 250.0))


# ----------------------------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_matches_leggauss(n):
    x, w = O.gauss(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(x - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14


@pytest.mark.parametrize("n", range(1, 8))
def test_gauss_exact_to_degree_2n_minus_1(n):
    x, w = O.gauss(n)
    for k in range(2 * n):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


@pytest.mark.parametrize("r", [1, 2, 4, 6])
def test_lagrange_derivative_exact_on_polynomials(r):
    x, _ = O.gauss(r + 1)
    rng = np.random.default_rng(r)
    c = rng.standard_normal(r + 1)
    f = np.polynomial.polynomial.polyval(x, c)
    df = np.polynomial.polynomial.polyder(c)
    for t in (-1.0, -0.3, 0.77, 1.0):
        v, d = O.lagrange_eval(x, t)
        assert abs(np.dot(v, f) - np.polynomial.polynomial.polyval(t, c)) < 1e-12
        assert abs(np.dot(d, f) - np.polynomial.polynomial.polyval(t, df)) < 1e-11


# ----------------------------------------------------------------------------- paper numbers
def test_courant_worked_example():
    g = json.load(open(GOLD))
    k = g["constants"]
    ex = g["courant_example"]
    c = math.sqrt(k["gamma"] * k["R"] * k["T_ref"])
    C = O.courant(ex["degree"], c, ex["dt"], [ex["cell_size"]] * ex["dim"], ex["dim"])
    assert round(C, ex["C_decimals"]) == pytest.approx(ex["C"], abs=0.011)


def test_dof_counts_of_the_scaling_meshes():
    g = json.load(open(GOLD))["dof_counts"]
    nx, ny, nz = g["uniform_base"]
    assert nx * ny * nz == g["uniform_cells"]
    u = O.dofs_per_scalar(g["uniform_cells"], g["degree"], 3) / 1e6
    n = O.dofs_per_scalar(g["nonconforming_cells"], g["degree"], 3) / 1e6
    assert abs(u - g["uniform_millions"]) <= g["millions_tolerance"] + 1e-9
    assert abs(n - g["nonconforming_millions"]) <= g["millions_tolerance"] + 1e-9


def test_constants_match_paper():
    k = json.load(open(GOLD))["constants"]
    assert (O.G, O.RGAS, O.GAMMA) == (k["g"], k["R"], k["gamma"])


# ------------------------------------------------------------------------------- background
@pytest.mark.parametrize("kind,atm", [(O.ISOTHERMAL, (1e5, 250.0, 0.0)), (O.STRATIFIED, (1e5, 293.15, 0.01))])
def test_background_is_hydrostatic(kind, atm):
    for z in (0.0, 800.0, 5000.0, 15000.0):
        dz = 1e-3
        pp, _ = O.background(kind, atm, z + dz)
        pm, _ = O.background(kind, atm, z - dz)
        p, rho = O.background(kind, atm, z)
        dpdz = (pp - pm) / (2 * dz)
        assert abs(dpdz + rho * O.G) < 1e-6 * rho * O.G
        assert abs(p - rho * O.RGAS * (p / (rho * O.RGAS))) < 1e-9 * p


def test_stratified_potential_temperature():
    k = json.load(open(GOLD))["constants"]
    atm = (k["p_ref"], k["T_ref"], k["N"])
    Gm = (O.GAMMA - 1.0) / O.GAMMA
    for z in (0.0, 1000.0, 8000.0):
        p, rho = O.background(O.STRATIFIED, atm, z)
        T = p / (rho * O.RGAS)
        theta = T * (k["p_ref"] / p) ** Gm
        assert abs(theta - k["T_ref"] * math.exp(k["N"] ** 2 * z / k["g"])) < 1e-9 * theta


# -------------------------------------------------------------------------------------- mesh
def test_mesh_counts_c1_c2():
    c1 = O.Case(dim=2, degree=2, nbase=(32, 1, 16), length=(20000.0, 1.0, 10000.0),
                oro_kind=O.AGNESI, oro=(1.0, 1000.0, 10000.0, 0.0))
    o = O.Oracle(c1)
    assert (o.ncell, o.N, o.nhang) == (512, 4608, 0)
    c2 = O.Case(dim=2, degree=4, nbase=(64, 1, 32), length=(20000.0, 1.0, 10000.0),
                rules=[(2000.0, 10000.0, 5000.0, 0, 0), (1000.0, 10000.0, 2500.0, 0, 0)],
                oro_kind=O.AGNESI, oro=(400.0, 1000.0, 10000.0, 0.0), atm_kind=O.STRATIFIED,
                atm=(1e5, 293.15, 0.01))
    o = O.Oracle(c2)
    assert (o.ncell, o.N, o.nhang) == (3200, 80000, 176)
    assert list(np.bincount(o.cells[:, 0])) == [1856, 576, 768]


def test_mesh_counts_c3():
    c3 = O.Case(dim=3, degree=1, nbase=(64, 64, 32), length=(40000.0, 40000.0, 20000.0),
                rules=[(3000.0, 0.0, -1.0, 0.0, -1.0)], oro_kind=O.GAUSS_HILL,
                oro=(400.0, 2000.0, 20000.0, 20000.0))
    o = O.Oracle(c3)
    assert o.ncell == 274432
    assert o.nhang == 16384


def test_mesh_rejects_2to1_violation():
    bad = O.Case(dim=2, degree=1, nbase=(4, 1, 4), length=(4000.0, 1.0, 4000.0),
                 rules=[(1000.0, 500.0, 500.0, 0, 0), (500.0, 500.0, 500.0, 0, 0),
                        (400.0, 500.0, 500.0, 0, 0)])
    # three nested levels in a single base cell next to unrefined neighbours -> level jump of 2+
    with pytest.raises(O.MeshError):
        O.Oracle(bad)


def test_domain_volume_flat_and_terrain():
    o = O.Oracle(twolevel2d(3))
    assert abs(o.wJ.sum() - 4000.0 * 2000.0) < 1e-8 * 4000.0 * 2000.0
    o = O.Oracle(twolevel3d(3))
    assert abs(o.wJ.sum() - 3000.0 * 3000.0 * 2000.0) < 1e-8 * 1.8e10
    # Agnesi hill: area = H L - h0 a (atan((L - xc)/a) + atan(xc/a)); spectral accuracy in r
    c = O.Case(dim=2, degree=6, nbase=(16, 1, 4), length=(4000.0, 1.0, 2000.0), periodic=(0, 0),
               oro_kind=O.AGNESI, oro=(100.0, 500.0, 2000.0, 0.0))
    o = O.Oracle(c)
    exact = 2000.0 * 4000.0 - 100.0 * 500.0 * (math.atan(2000.0 / 500.0) * 2)
    assert abs(o.wJ.sum() - exact) < 1e-7 * exact


def test_bottom_normals_follow_terrain():
    c = O.Case(dim=3, degree=3, nbase=(4, 4, 2), length=(4000.0, 4000.0, 2000.0), periodic=(1, 1),
               oro_kind=O.GAUSS_HILL, oro=(300.0, 700.0, 2000.0, 2000.0))
    o = O.Oracle(c)
    rows = o.bottom_normals()
    x, y, h = rows[:, 0], rows[:, 1], rows[:, 2]
    n = rows[:, 3:6]
    hx = -(x - 2000.0) / 700.0 ** 2 * h
    hy = -(y - 2000.0) / 700.0 ** 2 * h
    # outward normal of the bottom boundary is parallel to (h_x, h_y, -1)
    ref = np.stack([hx, hy, -np.ones_like(hx)], axis=1)
    cos = np.sum(n * ref, axis=1) / (np.linalg.norm(n, axis=1) * np.linalg.norm(ref, axis=1))
    assert np.min(cos) > 1 - 1e-13


# --------------------------------------------------------------------------- explicit residual
def _rand_state(o, seed):
    rng = np.random.default_rng(seed)
    U = np.zeros((o.nf, o.N))
    rho = 1.0 + 0.2 * rng.uniform(-1, 1, o.N)
    U[0] = rho
    for l in range(o.d):
        U[1 + l] = rho * 10.0 * rng.uniform(-1, 1, o.N)
    p = 1e5 * (1.0 + 0.1 * rng.uniform(-1, 1, o.N))
    U[1 + o.d] = p / (O.GAMMA - 1) + 0.5 * np.sum(U[1:1 + o.d] ** 2, axis=0) / rho
    return U


@pytest.mark.parametrize("mk", [tiny2d, tiny3d, twolevel2d])
def test_explicit_rest_state_is_exactly_steady(mk):
    o = O.Oracle(mk(3, oro=O.GAUSS_HILL, h0=100.0, periodic=(1, 1)))
    U = o.initial_state(0.0)
    assert np.max(np.abs(o.explicit_residual(U))) == 0.0


@pytest.mark.parametrize("mk", [tiny2d, tiny3d, twolevel2d, twolevel3d])
@pytest.mark.parametrize("h0", [0.0, 150.0])
def test_explicit_conservation(mk, h0):
    o = O.Oracle(mk(2, oro=O.GAUSS_HILL, h0=h0, periodic=(1, 1)))
    U = _rand_state(o, 3)
    R = o.explicit_residual(U)
    # mass always; horizontal momentum only over a flat bottom (terrain exerts a wall force)
    fields = [0] + (list(range(1, o.d)) if h0 == 0.0 else [])
    for f in fields:
        tot = np.sum(o.wJ * R[f])
        scale = np.sum(np.abs(o.wJ * R[f]))
        assert abs(tot) < 1e-13 * scale, f
    # energy: only the gravity work -g rho w is not a divergence
    e = R[1 + o.d] + O.G * U[o.d]
    assert abs(np.sum(o.wJ * e)) < 1e-13 * np.sum(np.abs(o.wJ * e))


@pytest.mark.parametrize("mk,r", [(twolevel2d, 4), (twolevel3d, 4), (tiny3d, 4)])
def test_explicit_polynomial_exactness_flat(mk, r):
    """rho = 1, m vanishing at the walls, quadratic per variable: the DG divergence of the mass and
    momentum fluxes is exact at the nodes (volume, faces, hanging faces, walls)."""
    o = O.Oracle(mk(r))
    Lx = o.case.length[0]
    H = o.case.length[2]
    Ly = o.case.length[1]
    x, y, z = o.x / Lx, o.y / Ly, o.z / H
    U = np.zeros((o.nf, o.N))
    U[0] = 1.0
    ax, az, ay = 3.0, 2.0, 1.5
    mx = ax * x * (1 - x)
    mz = az * z * (1 - z)
    U[1] = mx
    U[o.d] = mz
    dmx_dx = ax * (1 - 2 * x) / Lx
    dmz_dz = az * (1 - 2 * z) / H
    if o.d == 3:
        my = ay * y * (1 - y)
        U[2] = my
        dmy_dy = ay * (1 - 2 * y) / Ly
    U[1 + o.d] = 1e5
    R = o.explicit_residual(U)
    if o.d == 2:
        div_m = dmx_dx + dmz_dz
        Rmx = -(2 * mx * dmx_dx + mx * dmz_dz)       # -(d(mx mx)/dx + d(mx mz)/dz)
        Rmz = -(mz * dmx_dx + 2 * mz * dmz_dz)
        exp = [-div_m, Rmx, Rmz]
    else:
        div_m = dmx_dx + dmy_dy + dmz_dz
        exp = [-div_m, -(mx * div_m + mx * dmx_dx), -(my * div_m + my * dmy_dy),
               -(mz * div_m + mz * dmz_dz)]
    for f, e in enumerate(exp):
        assert np.max(np.abs(R[f] - e)) < 1e-11 * (np.max(np.abs(e)) + 1e-3), f


def test_explicit_energy_flux_exact_degree6():
    """With r = 6 the kinetic-energy flux (|m|^2 / 2) m of a quadratic m is resolved exactly, so the
    energy tendency equals -div((|m|^2/2) m) - g m_z at the nodes."""
    o = O.Oracle(twolevel2d(6))
    Lx, _, H = o.case.length
    x, z = o.x / Lx, o.z / H
    mx = 3.0 * x * (1 - x)
    mz = 2.0 * z * (1 - z)
    U = np.zeros((o.nf, o.N))
    U[0] = 1.0
    U[1] = mx
    U[2] = mz
    U[3] = 1e5
    k = 0.5 * (mx ** 2 + mz ** 2)
    dk_dx = mx * 3.0 * (1 - 2 * x) / Lx
    dk_dz = mz * 2.0 * (1 - 2 * z) / H
    div_m = 3.0 * (1 - 2 * x) / Lx + 2.0 * (1 - 2 * z) / H
    expect = -(k * div_m + mx * dk_dx + mz * dk_dz) - O.G * mz
    R = o.explicit_residual(U)
    assert np.max(np.abs(R[3] - expect)) < 1e-10 * np.max(np.abs(expect))


def test_explicit_free_stream_flat():
    o = O.Oracle(twolevel2d(3, periodic=(1, 1)))
    U = np.zeros((o.nf, o.N))
    U[0] = 1.2
    U[1] = 1.2 * 10.0
    U[1 + o.d] = 1e5 / 0.4 + 0.5 * 1.2 * 100.0
    R = o.explicit_residual(U)
    assert np.max(np.abs(R[:o.d + 1])) < 1e-11
    assert np.max(np.abs(R[1 + o.d])) < 1e-7


# ----------------------------------------------------------------------------- weak operators
def _assemble(apply, n_in, n_out):
    A = np.zeros((n_out, n_in))
    for j in range(n_in):
        e = np.zeros(n_in)
        e[j] = 1.0
        A[:, j] = np.ravel(apply(e))
    return A


@pytest.mark.parametrize("mk,r", [(twolevel2d, 3), (twolevel3d, 2), (tiny3d, 4)])
def test_grad_exact_for_polynomials_flat(mk, r):
    o = O.Oracle(mk(r))
    Lx, Ly, H = o.case.length
    x, y, z = o.x / Lx, o.y / Ly, o.z / H
    if o.d == 2:
        p = x ** r + 2 * x * z ** (r - 1) + z ** r
        g = [(r * x ** (r - 1) + 2 * z ** (r - 1)) / Lx, (2 * (r - 1) * x * z ** (r - 2) + r * z ** (r - 1)) / H]
    else:
        p = x ** r + x * y * z + z ** r + y ** 2
        g = [(r * x ** (r - 1) + y * z) / Lx, (x * z + 2 * y) / Ly, (x * y + r * z ** (r - 1)) / H]
    q = o.grad(p)
    for l in range(o.d):
        assert np.max(np.abs(q[l] - g[l])) < 1e-10 * np.max(np.abs(g[l])), l


@pytest.mark.parametrize("mk,r", [(twolevel2d, 3), (twolevel3d, 2)])
def test_div_exact_for_polynomials_flat(mk, r):
    o = O.Oracle(mk(r))
    Lx, Ly, H = o.case.length
    x, y, z = o.x / Lx, o.y / Ly, o.z / H
    w = np.zeros((o.d, o.N))
    w[0] = x * (1 - x) * (1 + z)
    w[o.d - 1] = z * (1 - z) * (2 - x)
    div = (1 - 2 * x) * (1 + z) / Lx + (1 - 2 * z) * (2 - x) / H
    if o.d == 3:
        w[1] = y * (1 - y) * x
        div = div + (1 - 2 * y) * x / Ly
    v = o.div(w) / o.wJ
    assert np.max(np.abs(v - div)) < 1e-10 * np.max(np.abs(div))


@pytest.mark.parametrize("mk,r", [(tiny2d, 2), (tiny3d, 2), (twolevel2d, 1)])
def test_divergence_is_minus_gradient_transpose_flat(mk, r):
    o = O.Oracle(mk(r, periodic=(1, 1)))
    N, d = o.N, o.d
    B = _assemble(lambda e: o.wJ[None, :] * o.grad(e), N, d * N)  # weak gradient, (d N) x N
    C = _assemble(lambda e: o.div(e.reshape(d, N)), d * N, N)    # weak divergence, N x (d N)
    assert np.max(np.abs(C + B.T)) < 1e-11 * np.max(np.abs(B))


def _helm_matrix(o, dta, h, lam):
    return _assemble(lambda e: o.helmholtz(dta, h, lam, e), o.N, o.N)


def _rand_h(o, seed):
    rng = np.random.default_rng(seed)
    h = 1e5 * (3.0 + rng.uniform(0, 1, o.N))
    return h, o.cell_sound_speed(h)


@pytest.mark.parametrize("mk", [tiny2d, tiny3d])
def test_helmholtz_symmetric_positive_on_flat_mesh(mk):
    o = O.Oracle(mk(2, periodic=(1, 0)))
    h, lam = _rand_h(o, 1)
    A = _helm_matrix(o, 0.7, h, lam)
    assert np.max(np.abs(A - A.T)) < 1e-11 * np.max(np.abs(A))
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() > 0


@pytest.mark.parametrize("mk", [tiny2d, tiny3d])
def test_helmholtz_nonsymmetric_over_terrain(mk):
    o = O.Oracle(mk(2, oro=O.GAUSS_HILL, h0=200.0, periodic=(1, 1)))
    h, lam = _rand_h(o, 2)
    A = _helm_matrix(o, 0.7, h, lam)
    asym = np.max(np.abs(A - A.T)) / np.max(np.abs(A))
    assert asym > 1e-6


def test_helmholtz_small_dt_limit_is_mass():
    o = O.Oracle(tiny2d(3, oro=O.GAUSS_HILL, h0=100.0))
    h, lam = _rand_h(o, 4)
    rng = np.random.default_rng(5)
    p = rng.standard_normal(o.N)
    assert np.array_equal(o.helmholtz(0.0, h, lam, p), o.wJ * p / (O.GAMMA - 1.0))
    for dta in (1e-2, 1e-3):
        diff = o.helmholtz(dta, h, lam, p) - o.wJ * p / (O.GAMMA - 1.0)
        assert np.max(np.abs(diff)) < 50 * dta * np.max(np.abs(o.wJ * p))


def test_helmholtz_matches_assembled_composition():
    """matrix-free A p == M/(g-1) + dt a beta/(2(g-1)) P - (dt a)^2 C H M^{-1} B built from the
    separately assembled operators."""
    for mk in (tiny2d, tiny3d):
        o = O.Oracle(mk(2, oro=O.GAUSS_HILL, h0=100.0, periodic=(1, 1)))
        N, d = o.N, o.d
        h, lam = _rand_h(o, 6)
        B = _assemble(lambda e: o.wJ[None, :] * o.grad(e), N, d * N)
        C = _assemble(lambda e: o.div(e.reshape(d, N)), d * N, N)
        P = _assemble(lambda e: o.penalty(lam, e), N, N)
        Minv = np.tile(1.0 / o.wJ, d)
        Hd = np.tile(h, d)
        dta = 0.9
        Aref = (np.diag(o.wJ) / (O.GAMMA - 1) + dta * o.beta / (2 * (O.GAMMA - 1)) * P
                - dta ** 2 * C @ (Hd[:, None] * Minv[:, None] * B))
        A = _helm_matrix(o, dta, h, lam)
        assert np.max(np.abs(A - Aref)) < 1e-12 * np.max(np.abs(Aref))
        # penalty: symmetric, positive semi-definite, annihilates constants
        assert np.max(np.abs(P - P.T)) < 1e-12 * np.max(np.abs(P))
        assert np.linalg.eigvalsh(P).min() > -1e-9 * np.max(np.abs(P))
        assert np.max(np.abs(P @ np.ones(N))) < 1e-10 * np.max(np.abs(P))


def test_grad_converges_over_terrain():
    """M^{-1} B p -> grad p in physical coordinates on a terrain-following mesh, order ~ r."""
    errs = []
    r = 3
    for n in (4, 8):
        c = O.Case(dim=2, degree=r, nbase=(n, 1, n // 2), length=(4000.0, 1.0, 2000.0),
                   periodic=(1, 1), oro_kind=O.AGNESI, oro=(200.0, 600.0, 2000.0, 0.0))
        o = O.Oracle(c)
        kx = 2 * math.pi / 4000.0
        kz = math.pi / 4000.0
        p = np.sin(kx * o.x) * np.cos(kz * o.z)
        gx = kx * np.cos(kx * o.x) * np.cos(kz * o.z)
        gz = -kz * np.sin(kx * o.x) * np.sin(kz * o.z)
        q = o.grad(p)
        errs.append(math.sqrt(np.sum(o.wJ * ((q[0] - gx) ** 2 + (q[1] - gz) ** 2))))
    assert errs[0] / errs[1] > 2 ** (r - 0.5)


# ------------------------------------------------------------------------------------- GMRES
def test_gmres_solves_nonsymmetric_system():
    rng = np.random.default_rng(7)
    n = 80
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    x, its, res, ok = O.Oracle.gmres(lambda v: A @ v, b, np.ones(n), 1e-12, 0.0, 10, 1000)
    assert ok and its > 10  # restarts exercised
    assert np.max(np.abs(x - np.linalg.solve(A, b))) < 1e-10


# -------------------------------------------------------------------------------- time stepping
def test_ark2_tableau_order_conditions():
    o = O.Oracle(tiny2d(1))
    A, At, b, bt = o.A, o.At, o.b, o.bt
    c = A.sum(axis=1)
    ct = At.sum(axis=1)
    assert np.allclose(c, ct, atol=1e-15)
    assert abs(b.sum() - 1) < 1e-15 and abs(bt.sum() - 1) < 1e-15
    for x in (b, bt):
        for y in (c, ct):
            assert abs(x @ y - 0.5) < 1e-15
    assert np.allclose(bt, At[2])  # stiffly accurate implicit part


@pytest.mark.parametrize("mk", [twolevel2d, tiny3d])
def test_rest_state_stays_at_rest(mk):
    c = mk(3, oro=O.GAUSS_HILL, h0=200.0, periodic=(1, 1))
    c.atm_kind = O.STRATIFIED
    c.atm = (1e5, 293.15, 0.01)
    o = O.Oracle(c)
    U = o.initial_state(0.0)
    for _ in range(3):
        U = o.step(U, 2.0)
    umax = np.max(np.abs(U[1:1 + o.d] / U[0]))
    assert umax < 1e-10


def test_mass_conserved_to_roundoff():
    c = twolevel2d(3, oro=O.AGNESI, h0=100.0, periodic=(1, 1))
    o = O.Oracle(c)
    U = o.initial_state(10.0)
    m0 = o.mass(U)
    for _ in range(3):
        U = o.step(U, 1.0)
    assert abs(o.mass(U) - m0) < 1e-13 * m0


def test_time_order_two():
    c = O.Case(dim=2, degree=2, nbase=(8, 1, 4), length=(8000.0, 1.0, 4000.0), periodic=(1, 1),
               oro_kind=O.AGNESI, oro=(200.0, 1000.0, 4000.0, 0.0), atm_kind=O.STRATIFIED,
               atm=(1e5, 293.15, 0.01))
    o = O.Oracle(c)
    U0 = o.initial_state(10.0)
    T = 2.0

    def run(dt):
        U = U0
        for _ in range(int(round(T / dt))):
            U = o.step(U, dt)
        return U

    ref = run(1.0 / 32)
    errs = [np.max(np.abs(run(dt)[1:] - ref[1:])) for dt in (0.5, 0.25, 0.125)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)


def test_acoustic_standing_wave_sign_and_speed():
    """Flat, shallow, periodic box at rest with p' = eps sin(k x): the horizontal momentum first
    follows -dt dp'/dx, and after half an acoustic period (speed c = sqrt(gamma R T)) the pressure
    perturbation is inverted."""
    L, T0 = 4000.0, 250.0
    c = O.Case(dim=2, degree=3, nbase=(8, 1, 1), length=(L, 1.0, 200.0), periodic=(1, 1),
               atm_kind=O.ISOTHERMAL, atm=(1e5, T0))
    o = O.Oracle(c)
    k = 2 * math.pi / L
    eps = 10.0
    pp0 = eps * np.sin(k * o.x)
    U = o.initial_state(0.0)
    U[1 + o.d] = (o.pbar + pp0) / (O.GAMMA - 1.0)
    dt = 0.25
    U1 = o.step(U, dt, fp_iters=3)
    expect = -dt * eps * k * np.cos(k * o.x)
    corr = np.dot(U1[1], expect) / (np.linalg.norm(U1[1]) * np.linalg.norm(expect))
    assert corr > 0.99
    cs = math.sqrt(O.GAMMA * O.RGAS * T0)
    half = L / cs / 2
    n = int(round(half / dt))
    Un = U
    for _ in range(n):
        Un = o.step(Un, dt, fp_iters=3)
    ppn = o.pressure(Un) - o.pbar
    corr = np.dot(ppn, pp0) / (np.linalg.norm(ppn) * np.linalg.norm(pp0))
    assert corr < -0.95


def test_gravity_pulls_heavier_air_down():
    c = twolevel2d(2, periodic=(1, 1))
    o = O.Oracle(c)
    U = o.initial_state(0.0)
    bump = np.exp(-((o.x - 2000.0) ** 2 + (o.z - 1000.0) ** 2) / (300.0 ** 2))
    U[0] = o.rbar * (1 + 0.01 * bump)
    U1 = o.step(U, 0.5)
    i = np.argmax(bump)
    assert U1[o.d][i] < 0
    assert U1[o.d][i] / U1[0][i] == pytest.approx(-0.5 * O.G * 0.01 * bump[i] / (1 + 0.01 * bump[i]), rel=0.1)
