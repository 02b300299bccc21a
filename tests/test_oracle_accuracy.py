"""Accuracy pins of the FP64 oracle (no GPU): what the high-order DG discretisation of Section 2
must achieve on smooth exact solutions, the terrain of Section 3.1 against its closed forms, and the
slip-wall flux against the Rusanov flux with the mirror state.

The exact fields come from tests/_exact.py, which never calls the oracle.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import _exact as E


def _l2_rel(o, a, b):
    return math.sqrt(np.sum(o.wJ * (a - b) ** 2) / np.sum(o.wJ * b * b))


def _rates(e0, e1):
    """log2 of the error ratio per field; a field that is exact on both meshes (the vertical
    momentum of a flow over flat ground, identically zero) counts as converged."""
    out = np.full(len(e0), np.inf)
    nz = e0 > 0
    assert np.all(e1[~nz] == 0.0)
    out[nz] = np.log2(e0[nz] / e1[nz])
    return out


# ------------------------------------------------------------ spatial order: explicit residual
def _tangent_case(dim, r, n, oro_kind, h0, refine):
    if dim == 2:
        L, nb, oro = (20000.0, 1.0, 10000.0), (2 * n, 1, n), (h0, 3000.0, 10000.0, 0.0)
        rules = [(5000.0, 10000.0, 5000.0, 0.0, 0.0)] if refine else []
    else:
        L, nb, oro = (20000.0, 20000.0, 10000.0), (2 * n, 2 * n, n), (h0, 3000.0, 10000.0, 10000.0)
        rules = [(5000.0, 10000.0, 5000.0, 10000.0, 5000.0)] if refine else []
    return O.Case(dim=dim, degree=r, nbase=nb, length=L, periodic=(0, 0), rules=rules,
                  oro_kind=oro_kind, oro=oro)


def _explicit_errors(case):
    o = O.Oracle(case)
    st = E.TangentState(case.dim, case.length, case.oro_kind, case.oro)
    U = np.array(st.conserved(o.x, o.y, o.z))
    R = o.explicit_residual(U)
    Rx = st.explicit_tendency(o.x, o.y, o.z, O.G)
    # a field whose exact tendency vanishes (vertical momentum over flat ground) is measured
    # against the largest momentum tendency
    mscale = max(math.sqrt(np.sum(o.wJ * Rx[f] ** 2)) for f in range(1, 1 + o.d))
    errs = []
    for f in range(o.nf):
        nrm = math.sqrt(np.sum(o.wJ * Rx[f] ** 2))
        if 1 <= f <= o.d and nrm < 1e-3 * mscale:
            nrm = mscale
        errs.append(math.sqrt(np.sum(o.wJ * (R[f] - Rx[f]) ** 2)) / nrm)
    return np.array(errs)


CASES_2D = [(2, (8, 16)), (3, (16, 32))]


@pytest.mark.parametrize("r,ns", CASES_2D)
@pytest.mark.parametrize("oro_kind,h0", [(O.FLAT, 0.0), (O.AGNESI, 800.0), (O.BELL, 800.0)])
@pytest.mark.parametrize("refine", [0, 1])
def test_explicit_residual_order_2d(r, ns, oro_kind, h0, refine):
    """A smooth state tangent to the coordinate surfaces (walls at the sides, ground and lid): the
    nodal residual M^-1 (explicit weak form) converges to the exact tendency -div F - g rho w in
    L2 at order >= r - 1/2 per field, uniform and with 2:1 faces, flat and over terrain.  A
    transposed metric in the contravariant fluxes makes the error O(1)."""
    e0 = _explicit_errors(_tangent_case(2, r, ns[0], oro_kind, h0, refine))
    e1 = _explicit_errors(_tangent_case(2, r, ns[1], oro_kind, h0, refine))
    rates = _rates(e0, e1)
    assert np.all(rates > r - 0.5), (e0, e1, rates)
    assert np.all(e1 < 5e-2), e1


@pytest.mark.parametrize("oro_kind", [O.BELL, O.GAUSS_HILL])
def test_explicit_residual_order_3d(oro_kind):
    """The same in 3D at r = 2 over a hill with a 2:1 level around it."""
    r = 2
    e0 = _explicit_errors(_tangent_case(3, r, 4, oro_kind, 800.0, 1))
    e1 = _explicit_errors(_tangent_case(3, r, 8, oro_kind, 800.0, 1))
    rates = _rates(e0, e1)
    assert np.all(rates > r - 0.5), (e0, e1, rates)


# ------------------------------------------------------------ spatial order: the whole step
VORTEX_R = 2000.0
VORTEX_L = 12 * VORTEX_R
VORTEX_U = 50.0
VORTEX_P = 1e5


def _vortex_error(r, n, dt, T):
    """Isentropic vortex (strength 1, radius 2 km, Mach 0.13) translating at 50 m/s through a
    periodic 24 x 24 km slice with slip walls 6 radii away, gravity off (Eq. (1) without the
    gravity terms): L2 error per field after time T."""
    c = O.Case(dim=2, degree=r, nbase=(n, 1, n), length=(VORTEX_L, 1.0, VORTEX_L), periodic=(1, 1),
               atm_kind=O.ISOTHERMAL, atm=(VORTEX_P, VORTEX_P / O.RGAS), gravity=0.0)
    o = O.Oracle(c)
    args = (VORTEX_L / 2, VORTEX_L / 2, VORTEX_R, 1.0, VORTEX_U, 1.0, VORTEX_P)
    U = E.isentropic_vortex(o.x, o.z, 0.0, *args)
    for _ in range(int(round(T / dt))):
        U = o.step(U, dt)
    ex = E.isentropic_vortex(o.x, o.z, T, *args)
    return np.array([_l2_rel(o, U[f], ex[f]) for f in range(o.nf)])


@pytest.mark.parametrize("r,ns,order", [(2, (8, 16), 2.5), (3, (8, 16), 2.5), (4, (8, 16), 3.5)])
def test_step_spatial_order_isentropic_vortex(r, ns, order):
    """The whole IMEX-RK2 step (explicit residual, implicit pressure stages, fixed point, GMRES)
    on an exact solution: after 8 s the L2 error of every field falls under mesh refinement at
    order >= r + 1/2 for r = 2 and >= r - 1/2 for r = 3, 4 (measured: 2.7-3.1 at r = 2, 2.6-3.7 at
    r = 3, 4.0-4.2 at r = 4; the implicit pressure gradient and energy flux are central, with a
    jump penalty on the pressure only, and central fluxes for the acoustic subsystem are known to
    cost up to one order).  Halving the time step changes the errors by < 1 % except the energy
    at r = 4 (25 %), whose rate it raises."""
    T = 8.0
    e0 = _vortex_error(r, ns[0], 0.25, T)
    e1 = _vortex_error(r, ns[1], 0.25, T)
    rates = _rates(e0, e1)
    assert np.all(rates > order), (e0, e1, rates)
    assert np.all(e1 < 1e-2), e1


# --------------------------------------------------------------------- terrain of Section 3.1
TERRAINS = [
    (2, O.AGNESI, (400.0, 1000.0, 10000.0, 0.0)),
    (2, O.BELL, (400.0, 1000.0, 10000.0, 0.0)),
    (2, O.GAUSS_HILL, (400.0, 2000.0, 10000.0, 0.0)),
    (2, O.GAUSS_RIDGE, (1000.0, 5000.0, 10000.0, 0.0)),
    (2, O.FLAT, (0.0, 1.0, 0.0, 0.0)),
    (3, O.BELL, (400.0, 1000.0, 30000.0, 20000.0)),        # Section 3.1, Eq. (3)
    (3, O.GAUSS_HILL, (400.0, 2000.0, 30000.0, 20000.0)),
    (3, O.GAUSS_RIDGE, (1000.0, 5000.0, 30000.0, 0.0)),
    (3, O.AGNESI, (400.0, 1000.0, 30000.0, 0.0)),
    (3, O.FLAT, (0.0, 1.0, 0.0, 0.0)),
]


def _terrain_case(dim, kind, oro):
    if dim == 2:
        return O.Case(dim=2, degree=3, nbase=(20, 1, 4), length=(20000.0, 1.0, 16000.0),
                      periodic=(1, 1), rules=[(4000.0, 10000.0, 3000.0, 0.0, 0.0)],
                      oro_kind=kind, oro=oro)
    return O.Case(dim=3, degree=2, nbase=(12, 8, 2), length=(60000.0, 40000.0, 16000.0),
                  periodic=(1, 1), rules=[(4000.0, 30000.0, 6000.0, 20000.0, 6000.0)],
                  oro_kind=kind, oro=oro)


@pytest.mark.parametrize("dim,kind,oro", TERRAINS)
def test_terrain_heights_and_slopes_closed_form(dim, kind, oro):
    """Node heights z = zeta + h(x, y)(1 - zeta/H) and the bottom boundary's area-weighted outward
    normal (h_x, h_y, -1) times the face's logical half-widths, against the closed forms of the
    five orographies (Eq. (3) for the bell), with slopes by the complex step."""
    c = _terrain_case(dim, kind, oro)
    o = O.Oracle(c)
    H = c.length[2]
    # logical height of every node from the cell table and the Gauss points (numpy's)
    xi = np.polynomial.legendre.leggauss(c.degree + 1)[0]
    lev = o.cells[:, 0].astype(np.float64)
    kz = o.cells[:, 3].astype(np.float64)
    dz = H / (c.nbase[2] * 2.0 ** lev)
    nz_axis = np.repeat(xi, (c.degree + 1) ** (dim - 1))          # the vertical axis is slowest
    zeta = (dz[:, None] * (kz[:, None] + 0.5 * (1.0 + nz_axis[None, :]))).reshape(-1)
    h = E.terrain(kind, oro, dim, o.x, o.y)
    zexp = zeta + h * (1.0 - zeta / H)
    assert np.max(np.abs(o.z - zexp)) < 1e-9 * H
    rows = o.bottom_normals()
    x, y, hb, N = rows[:, 0], rows[:, 1], rows[:, 2], rows[:, 3:6]
    assert np.max(np.abs(hb - E.terrain(kind, oro, dim, x, y))) < 1e-12 * max(oro[0], 1.0)
    hx, hy = E.terrain_slopes(kind, oro, dim, x, y)
    if kind != O.FLAT:
        assert np.max(np.abs(hx)) > 0.01
    # the bottom cells are unrefined at the edges of the domain and refined near the centre:
    # the normal's vertical component is minus the product of the face's half-widths
    area = -N[:, 2]
    assert np.all(area > 0)
    assert np.max(np.abs(N[:, 0] / area - hx)) < 1e-12
    assert np.max(np.abs(N[:, 1] / area - (hy if dim == 3 else 0.0))) < 1e-12
    halfw = np.unique(np.round(area, 6))
    dx = c.length[0] / c.nbase[0]
    dy = c.length[1] / c.nbase[1] if dim == 3 else 2.0
    expect = {round(0.25 * dx * dy / 4 ** l, 6) for l in (0, 1)} if dim == 3 else {round(0.5 * dx / 2 ** l, 6) for l in (0, 1)}
    assert set(halfw.tolist()) <= expect


# -------------------------------------------------------------------------------- slip walls
def _mirror_rusanov(d, U, N):
    """Rusanov flux of the explicit part between U and its mirror image across the wall with
    outward area-weighted normal N (Section 2's explicit advective fluxes; advective speed)."""
    n = N / np.linalg.norm(N)
    rho, m, E_ = U[0], U[1:1 + d], U[1 + d]
    mm = m - 2.0 * np.dot(m, n) * n
    Um = np.concatenate([[rho], mm, [E_]])

    def flux(V):
        r, mv, e = V[0], V[1:1 + d], V[1 + d]
        k = 0.5 * np.dot(mv, mv) / r
        un = np.dot(mv, N) / r
        return np.concatenate([[r * un], mv * un, [k * un]])

    lam = max(abs(np.dot(m, N) / rho), abs(np.dot(mm, N) / rho))
    return 0.5 * (flux(U) + flux(Um)) - 0.5 * lam * (Um - U)


@pytest.mark.parametrize("d", [2, 3])
def test_wall_flux_is_mirror_state_rusanov(d):
    """With m . n != 0 (inflow and outflow through the wall), the oracle's closed form equals
    the Rusanov flux against the mirror state (rho, m - 2 (m.n) n, rho E)."""
    rng = np.random.default_rng(11 + d)
    for _ in range(50):
        U = np.concatenate([[rng.uniform(0.5, 1.5)], rng.uniform(-20, 20, d), [rng.uniform(2e5, 3e5)]])
        N = rng.uniform(-3, 3, d)
        ref = _mirror_rusanov(d, U, N)
        got = O.wall_flux(d, U, N)
        # scale: the one-sided momentum flux |m| |m . N| / rho (the energy and mass components of
        # the reference cancel to rounding of that size)
        scale = np.linalg.norm(U[1:1 + d]) * abs(np.dot(U[1:1 + d], N)) / U[0] * (1.0 + 0.5 * np.linalg.norm(U[1:1 + d]) / U[0])
        assert np.max(np.abs(got - ref)) < 1e-13 * scale
        assert got[0] == 0.0 and got[1 + d] == 0.0


def test_wall_flux_enters_the_residual():
    """Flat, laterally periodic slice with vertical momentum through the ground and the lid:
    the domain total of the vertical-momentum tendency equals minus the wall fluxes integrated
    over both walls, evaluated here from the nodal traces (numpy Lagrange basis) and the
    mirror-state Rusanov flux; horizontal momentum and mass see no wall force."""
    r = 3
    c = O.Case(dim=2, degree=r, nbase=(6, 1, 3), length=(6000.0, 1.0, 3000.0), periodic=(1, 1))
    o = O.Oracle(c)
    Lx, _, H = c.length
    rho = 1.0 + 0.1 * np.cos(2 * np.pi * o.x / Lx)
    u = 5.0 + 2.0 * np.sin(2 * np.pi * o.x / Lx)
    w = 3.0 * np.cos(2 * np.pi * o.x / Lx) * (1.0 - 2.0 * o.z / H) + 1.0   # through both walls
    U = np.stack([rho, rho * u, rho * w, 2.5e5 + 0.5 * rho * (u * u + w * w)])
    R = o.explicit_residual(U)
    xi, wq = np.polynomial.legendre.leggauss(r + 1)
    V = np.vander(xi, r + 1, increasing=True)
    lo = np.linalg.solve(V.T, np.array([(-1.0) ** k for k in range(r + 1)]))   # l_j(-1)
    hi = np.linalg.solve(V.T, np.ones(r + 1))                                   # l_j(+1)
    np1 = r + 1
    dx = Lx / c.nbase[0]
    total = np.zeros(4)
    for cell in range(o.ncell):
        lev, ix, _, iz = o.cells[cell]
        Uc = U[:, cell * o.nloc:(cell + 1) * o.nloc].reshape(4, np1, np1)       # [f][z][x]
        for side, lz, N in ((iz == 0, lo, np.array([0.0, -0.5 * dx])),
                            (iz == c.nbase[2] - 1, hi, np.array([0.0, 0.5 * dx]))):
            if not side:
                continue
            tr = np.einsum("k,fkx->fx", lz, Uc)
            for j in range(np1):
                total -= wq[j] * _mirror_rusanov(2, tr[:, j], N)
    got = np.array([np.sum(o.wJ * R[f]) for f in range(4)])
    got[3] += np.sum(o.wJ * O.G * U[2])            # the gravity work is not a flux
    scale = np.sum(np.abs(o.wJ * R[2]))
    assert abs(total[2]) > 1e-3 * scale
    assert abs(got[2] - total[2]) < 1e-12 * scale
    assert abs(got[0]) < 1e-12 * np.sum(np.abs(o.wJ * R[0]))
    assert abs(got[1]) < 1e-12 * np.sum(np.abs(o.wJ * R[1]))


# ------------------------------------------------------------------- initial-state noise
def test_noise_generator_is_splitmix64():
    """The oracle's temperature noise follows SplitMix64's published definition: its output mix of
    the state G = 0x9e3779b97f4a7c15 (seed 0, first draw) is 0xe220a8397b1dcdaf.  A one-node,
    one-cell mesh pins the key chain: the first deviate equals the Box-Muller transform of the two
    draws that follow the chain, written out here from the definition."""
    def mix(z):
        m = (1 << 64) - 1
        z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & m
        z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & m
        return z ^ (z >> 31)
    G_ = 0x9e3779b97f4a7c15
    m64 = (1 << 64) - 1
    assert mix(G_) == 0xe220a8397b1dcdaf
    o = O.Oracle(O.Case(dim=2, degree=1, nbase=(3, 1, 2), length=(3000.0, 1.0, 2000.0)))
    seed = 2408
    n = o.temperature_noise(seed, 1.0)
    for cell in (0, 4):
        lev, ix, iy, iz = (int(v) for v in o.cells[cell])
        for q in range(o.nloc):
            k = mix((seed + G_ * (lev + 1)) & m64)
            for v in (ix, iy, iz, q):
                k = mix((k + G_ * (v + 1)) & m64)
            u1 = (mix((k + G_) & m64) >> 11) * 2.0 ** -53
            u2 = (mix((k + 2 * G_) & m64) >> 11) * 2.0 ** -53
            ref = math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2.0 * math.pi * u2)
            assert abs(n[cell * o.nloc + q] - ref) < 1e-15


def test_noise_is_standard_normal_and_seeded():
    from scipy import stats
    o = O.Oracle(O.Case(dim=3, degree=3, nbase=(12, 12, 6), length=(1e4, 1e4, 5e3)))
    n = o.temperature_noise(2408, 1.0)
    assert abs(n.mean()) < 5.0 / math.sqrt(len(n))
    assert abs(n.std() - 1.0) < 0.01
    assert stats.kstest(n, "norm").pvalue > 1e-3
    assert np.array_equal(n, o.temperature_noise(2408, 1.0))
    assert abs(np.corrcoef(n, o.temperature_noise(2409, 1.0))[0, 1]) < 0.02
    assert np.allclose(o.temperature_noise(2408, 0.1), 0.1 * n, rtol=1e-15, atol=0)
