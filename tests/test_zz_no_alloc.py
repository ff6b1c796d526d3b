"""lbm_invariants_static, the variant of lbm_invariants that keeps its reduction scratch in
a static device array instead of the context's workspace, called through the C ABI: two
calls in a row on contexts of different sizes (the second smaller), each against
lbm_invariants on the same state. Both run the same kernels in the same order, so the totals
must agree bit for bit; they are also checked against FP64 sums of the exported populations,
and a non-finite population must be reported the same way."""
import numpy as np
import pytest

import lbm_inputs as inp
from tests.gpu_util import gpu_sim

pytestmark = pytest.mark.gpu


def _totals_of(f):
    """sum rho, sum rho u_x, sum rho u_y of dense [9, ny, nx] populations (paper numbering)."""
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
    return np.array([f.sum(), (cx[:, None, None] * f).sum(), (cy[:, None, None] * f).sum()])


@pytest.mark.parametrize("pattern", ["ab", "aa"])
def test_static_scratch_invariants_equal_workspace_invariants(pattern):
    from paper_2602_21242_amd import capi
    # The second call is on a smaller grid than the first, with another storage type.
    for nx, ny, storage, seed in ((96, 40, "f64", 1), (33, 7, "f32", 2)):
        print(f"static-scratch invariants: {nx}x{ny} {storage} {pattern}", flush=True)
        f0 = inp.random_populations(nx, ny, seed=seed)
        f0[1] *= 1.3  # net momentum along +x
        f0[4] *= 0.8  # and along +y
        sim = gpu_sim(nx, ny, 0.4, 0.02, "complete", storage, pattern, f0=f0)
        sim.step(3)
        s1, a = capi.lbm_invariants(sim._ctx)
        s2, b = capi.lbm_invariants_static(sim._ctx)
        assert s1 == capi.LBM_OK and s2 == capi.LBM_OK, capi.last_error()
        assert a == b, (a, b)
        ref = _totals_of(sim.populations().cpu().numpy())
        assert np.allclose(a, ref, rtol=1e-12, atol=1e-12 * ref[0]), (a, ref)


def test_static_scratch_reports_nonfinite_populations():
    from paper_2602_21242_amd import capi
    f0 = inp.random_populations(9, 6, seed=2)
    f0[3, 2, 4] = np.nan
    sim = gpu_sim(9, 6, 0.4, 0.02, "complete", "f32", f0=f0)
    s1, _ = capi.lbm_invariants(sim._ctx)
    s2, _ = capi.lbm_invariants_static(sim._ctx)
    assert s1 == s2 == capi.LBM_ERR_NONFINITE
    assert "non-finite" in capi.last_error()


def test_static_scratch_null_arguments():
    from paper_2602_21242_amd import capi
    assert capi.lib().lbm_invariants_static(None, None) == capi.LBM_ERR_INVALID_ARGUMENT
