"""Parity at the full size of the benchmarked 3D workload (274,432 cells, degree 4, 34.3 M nodes
per field, 171.5 M DoFs), on the mesh and in the launch configuration the benchmark times: every
node of the explicit residual and of the Helmholtz operator (FP64, and FP32 with the oracle fed
the FP32-rounded inputs) against the oracle."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2408_08129_amd import cases, inputs
from tests import _common as C


@pytest.mark.gpu
def test_full_size_box3d_hill_operators():
    import paper_2408_08129_amd as P
    from tests.test_gpu_parity import TOL64, dev, host
    w = dict(cases.WORKLOADS["box3d_r4_hill"])
    t0 = time.time()
    o = O.Oracle(C.oracle_case(w))
    s = P.Solver(C.product_case(w), w["degree"])
    perm = C.cell_perm(s.cell_table(), o.cells)
    assert o.ncell == 274432 and s.N == o.N == 34304000
    print("[full] setup %.1f s" % (time.time() - t0), flush=True)

    # the background state with the workload's wind and 1 % seeded noise per node and field (the
    # uniform +-20 % density of the small-mesh tests, extrapolated to the 34 M nodes' sub-face
    # points, reaches near-zero densities at a few 2:1 faces, where rounding is amplified 1e4-fold)
    U = o.initial_state(w["ubar"])
    for f in range(o.nf):
        U[f] *= 1.0 + 0.01 * inputs.random_normal(o.N, 2408 + f)
    t0 = time.time()
    Ro = o.explicit_residual(U)
    print("[full] oracle explicit residual %.1f s" % (time.time() - t0), flush=True)
    R = C.to_oracle_order(host(s.explicit_residual(dev(C.to_product_order(U, perm, o.nloc)))), perm, o.nloc)
    for f in range(o.nf):
        e = C.rel_err(R[f], Ro[f])
        print("[full] explicit residual field %d rel err %.2e" % (f, e), flush=True)
        assert e < TOL64
    del U, Ro, R

    h = inputs.random_positive(o.N, 2409, 2.5e5, 3.5e5)
    p = inputs.random_normal(o.N, 2410, 100.0)
    dta = 0.6 * 0.2928932188134525
    t0 = time.time()
    ref = o.helmholtz(dta, h, o.cell_sound_speed(h), p)
    print("[full] oracle Helmholtz %.1f s" % (time.time() - t0), flush=True)
    Ap = host(s.apply_helmholtz(dta, dev(C.to_product_order(h, perm, o.nloc)),
                                dev(C.to_product_order(p, perm, o.nloc)), P.DG_FP64))
    e = C.rel_err(C.to_oracle_order(Ap, perm, o.nloc), ref)
    print("[full] Helmholtz FP64 rel err %.2e" % e, flush=True)
    assert e < TOL64
    s.close()

    s32 = P.Solver(C.product_case(w), w["degree"], P.options(precision=P.DG_FP32_INNER))
    h32 = h.astype(np.float32)
    p32 = p.astype(np.float32)
    ref = o.helmholtz(dta, h32.astype(np.float64), o.cell_sound_speed(h32.astype(np.float64)),
                      p32.astype(np.float64))
    Ap = s32.apply_helmholtz(dta, dev(C.to_product_order(h32, perm, o.nloc)),
                             dev(C.to_product_order(p32, perm, o.nloc)), P.DG_FP32_INNER)
    e = C.rel_err(C.to_oracle_order(host(Ap).astype(np.float64), perm, o.nloc), ref)
    print("[full] Helmholtz FP32 rel err %.2e" % e, flush=True)
    assert e < 2e-5
    s32.close()


@pytest.mark.gpu
def test_full_size_ridge_large_step_properties():
    """The headline workload at full size (2,183,168 cells, degree 4, 272.9 M nodes per field,
    1.36e9 DoFs) in the configuration the benchmark times (FP64, GMRES rtol 1e-8), through
    properties that hold at any size: the hydrostatic rest state over the ridge stays at rest (the
    scheme in perturbation form is well balanced), a step with the wind and seeded temperature
    noise conserves mass to rounding (the continuity equation is explicit and in flux form), and
    the step is deterministic (the same bits twice).  The oracle covers this workload through its
    one-column sample (test_gpu_oracle_configs)."""
    import math

    import torch

    import paper_2408_08129_amd as P
    w = dict(cases.WORKLOADS["box3d_r4_ridge_large"])
    t0 = time.time()
    s = P.Solver(cases.product_case(w), w["degree"], P.options(gmres_rtol=1e-8))
    assert s.ncell == 2183168 and s.N == 272896000
    print("[full ridge] setup %.1f s" % (time.time() - t0), flush=True)

    U = s.init_state(0.0)
    st = s.step(U, w["dt"])
    _, max_w = s.diagnostics(U)
    print("[full ridge] rest: max |w| after one step %.3e m/s, GMRES its %s" % (max_w, st.as_dict(2)["gmres_iters"]),
          flush=True)
    assert max_w < 1e-10
    del U
    torch.cuda.empty_cache()

    U1 = s.init_state(w["ubar"], noise_seed=11, noise_sigma_K=0.05)
    U2 = U1.clone()
    m0, _ = s.diagnostics(U1)
    st = s.step(U1, w["dt"])
    s.step(U2, w["dt"])
    m1, w1 = s.diagnostics(U1)
    print("[full ridge] wind + noise: mass drift %.3e, max |w| %.3f m/s, GMRES its %s" %
          ((m1 - m0) / m0, w1, st.as_dict(2)["gmres_iters"]), flush=True)
    assert abs(m1 - m0) < 1e-13 * m0
    assert math.isfinite(w1) and w1 < 50.0
    assert torch.equal(U1, U2)
    s.close()
