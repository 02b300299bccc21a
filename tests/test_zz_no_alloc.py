"""The allocation-free diagnostics entry point against dg_diagnostics, through the C ABI."""
import numpy as np
import pytest

from paper_2408_08129_amd import inputs
from tests import _common as C

pytestmark = pytest.mark.gpu


def test_diagnostics_noalloc_equals_diagnostics_twice_second_smaller():
    import torch

    import paper_2408_08129_amd as P
    assert torch.cuda.is_available()
    results = []
    # a larger mesh first, then a smaller one: the second call must not see the first's partials
    for w, seed in ((C.twolevel3d(4), 5), (C.tiny2d(2), 6)):
        print("[case] no-alloc diagnostics %s" % ({k: w[k] for k in ("dim", "degree", "nbase")},), flush=True)
        s = P.Solver(C.product_case(w), w["degree"])
        U = torch.from_numpy(inputs.random_state(s.nf, s.N, seed=seed)).cuda()
        ref = P.dg_diagnostics(s.ctx, U)
        got = P.dg_diagnostics_noalloc(s.ctx, U)
        print("  dg_diagnostics %r  noalloc %r" % (ref, got), flush=True)
        assert got[0] == ref[0] and got[1] == ref[1]
        assert np.isfinite(got[0]) and got[0] > 0 and got[1] > 0
        results.append(got)
        s.close()
    assert results[0] != results[1]
