"""The 3D bell-hill benchmark (Section 3.1): meshes, the slice evaluator, GPU parity.

CPU: the two meshes have the stated sizes and the non-conforming one equals the oracle's mesh; the
point evaluator reproduces a field that is polynomial of degree <= r in each logical coordinate
(so every cell's nodal interpolant is the field itself) at points placed with the forward
terrain-following map, which pins the inverse map, the leaf search and the Lagrange evaluation.
GPU: two steps of the non-conforming bell-hill case with its absorbing layers (degree 2, dt = 2 s)
against the oracle, and the evaluator at the library's own node positions returns the nodal
values."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_08129_amd import bellhill as B
from paper_2408_08129_amd import cases
from tests import _common as C


def _bell(name, degree=None):
    w = dict(cases.WORKLOADS[name])
    if degree is not None:
        w["degree"] = degree
    return w


@pytest.mark.parametrize("name,ncell,nhang", [("bell3d_r4_uniform", 38400, 0),
                                              ("bell3d_r4_nonconforming", 1930, 872)])
def test_bell_meshes(name, ncell, nhang):
    import paper_2408_08129_amd as P
    w = _bell(name)
    n, nh, cells = P.dg_mesh_info(C.product_case(w), w["degree"])
    assert (n, nh) == (ncell, nhang)
    if name.endswith("nonconforming"):
        assert np.bincount(cells[:, 0]).tolist() == [450, 1160, 320]
        o = O.Oracle(C.oracle_case(_bell(name, 1)))
        assert o.ncell == n and o.nhang == nh
        C.cell_perm(cells, o.cells)
        # the finest cells are the uniform mesh's 1 km cells
        assert w["length"][0] / (w["nbase"][0] << 2) == 1000.0


def _logical_poly(w, r):
    Lx, Ly, H = (float(v) for v in w["length"])

    def f(x, y, zeta):
        a, b, c = x / Lx, y / Ly, zeta / H
        return 0.3 + a - 2.0 * b ** r + c * a ** (r - 1) * b + 0.7 * c ** r - a * b * c

    return f


@pytest.mark.parametrize("degree", [2, 4])
def test_point_evaluator_reproduces_cell_polynomials(degree):
    w = _bell("bell3d_r4_nonconforming", degree)
    o = O.Oracle(C.oracle_case(w))
    f = _logical_poly(w, degree)
    H = float(w["length"][2])
    h = B.terrain_height(w, o.x, o.y)
    zeta = (o.z - h) / (1.0 - h / H)  # logical height of the oracle's nodes
    # product cell order: the evaluator takes (ncell, NL) arrays in the library's cell order,
    # which is the host mesh query's order
    import paper_2408_08129_amd as P
    _, _, cells = P.dg_mesh_info(C.product_case(w), degree)
    perm = C.cell_perm(cells, o.cells)
    nodal = C.to_product_order(f(o.x, o.y, zeta), perm, o.nloc).reshape(-1, o.nloc)
    ev = B.PointEvaluator(cells, degree, w)
    rng = np.random.default_rng(2408)
    n = 4000
    x = rng.uniform(0.0, w["length"][0], n)
    y = rng.uniform(0.0, w["length"][1], n)
    zt = rng.uniform(0.0, H, n)
    hz = B.terrain_height(w, x, y)
    z = zt + hz * (1.0 - zt / H)  # forward terrain-following map
    got = ev(nodal, x, y, z)
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - f(x, y, zt))) < 1e-12
    # below the ground and above the lid: outside
    assert np.all(np.isnan(ev(nodal, np.array([30000.0, 100.0]), np.array([20000.0, 100.0]),
                              np.array([100.0, 16000.5]))))


def test_slices_and_layers():
    w = _bell("bell3d_r4_uniform")
    s = B.slice_points(w)
    assert set(s) == {"xz_y20km", "xy_z800m"}
    x, y, z = s["xz_y20km"]
    assert np.all(y == 20000.0) and x.max() == 60000.0 and z.max() == 16000.0
    x, y, z = s["xy_z800m"]
    assert np.all(z == 800.0) and len(x) == 241 * 161
    m = B.interior_mask(w, s["xy_z800m"])
    # interior of the side layers: 40 km x 20 km
    assert abs(m.mean() - (161 * 81) / (241 * 161)) < 0.01


@pytest.mark.gpu
def test_gpu_bell_nonconforming_two_steps():
    """In the benchmark's configuration: enthalpy split, no pressure-jump penalty."""
    import math
    from tests.test_gpu_parity import TOL_STEP, dev, host
    from tests.test_split import _gpu_pair
    w = _bell("bell3d_r4_nonconforming", 2)
    assert w["enthalpy_split"] == 1 and w["penalty_beta"] == 0.0
    o, s, perm = _gpu_pair(w, beta=0.0)
    Uo = o.initial_state(w["ubar"])
    U = dev(C.to_product_order(Uo, perm, o.nloc))
    for _ in range(2):
        Uo = o.step(Uo, w["dt"])
        s.step(U, w["dt"])
    Ug = C.to_oracle_order(host(U), perm, o.nloc)
    for f in range(o.nf):
        err = C.rel_err(Ug[f], Uo[f])
        l2 = math.sqrt(np.sum(o.wJ * (Ug[f] - Uo[f]) ** 2) / np.sum(o.wJ * Uo[f] ** 2))
        assert err < TOL_STEP and l2 < TOL_STEP, (f, err, l2)


@pytest.mark.gpu
def test_gpu_evaluator_at_library_nodes():
    import torch

    import paper_2408_08129_amd as P
    w = _bell("bell3d_r4_nonconforming", 3)
    s = P.Solver(C.product_case(w), w["degree"])
    x, y, z, _ = (t.cpu().numpy() for t in s.node_geometry())
    cells = s.cell_table()
    rng = np.random.default_rng(7)
    vals = rng.standard_normal(s.N)
    ev = B.PointEvaluator(cells, w["degree"], w)
    sel = rng.choice(s.N, 5000, replace=False)
    got = ev(vals.reshape(-1, s.nloc), x[sel], y[sel], z[sel])
    assert np.max(np.abs(got - vals[sel])) < 1e-10
    s.close()
    torch.cuda.empty_cache()
