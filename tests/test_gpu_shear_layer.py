"""The double shear layer at the paper's parameters (u0 = 0.04, kappa = 80, delta = 0.05,
Re = 30000, theta 0.4 and 0.6) on small boxes: the GPU step against the oracle, and the
package's shear-layer diagnostics against the same quantities computed here in numpy on
the oracle's fields."""
import math

import numpy as np
import pytest
from scipy import ndimage

import lbm_inputs as inp
import oracle
from tests.gpu_util import gpu_sim
from tests.lbm_diag import eps_f, field_moments

pytestmark = pytest.mark.gpu

U0, KAPPA, DELTA, RE = 0.04, 80.0, 0.05, 30000.0


@pytest.mark.parametrize("model", ["bgk", "uc", "partial", "complete"])
@pytest.mark.parametrize("theta", [0.4, 0.6])
def test_paper_shear_layer_parity_fp64(model, theta):
    n, steps = 64, 300
    fields = inp.double_shear_layer(n, n, U0, KAPPA, DELTA)
    nu = U0 * n / RE
    sim = gpu_sim(n, n, theta, nu, model, "f64", "ab", fields=fields)
    sim.step(steps)
    ref = oracle.run(oracle.init_equilibrium(*fields, theta), theta, nu, model, steps)
    assert eps_f(sim.populations().cpu().numpy(), ref) <= 1e-12


def _numpy_thickness(ux):
    prof = ux.mean(axis=1)
    d = 0.5 * np.abs(np.roll(prof, -1) - np.roll(prof, 1))
    ny = prof.size
    return 0.5 * (2 * U0 / d[: ny // 2].max() + 2 * U0 / d[ny // 2:].max()) / ny


def _numpy_cores(ux, uy, frac=0.3, window=5):
    w = 0.5 * (np.roll(uy, -1, 1) - np.roll(uy, 1, 1)) - 0.5 * (np.roll(ux, -1, 0) - np.roll(ux, 1, 0))
    a = np.abs(w)
    m = ndimage.maximum_filter(a, size=window, mode="wrap")
    return int(np.sum((a == m) & (a > frac * a.max())))


@pytest.mark.parametrize("model", ["bgk", "complete"])
def test_shear_layer_diagnostics_match_numpy_on_oracle_fields(model):
    """n = 64, one tenth of a convective time (160 steps), theta = 0.4."""
    from paper_2602_21242_amd.diagnostics import double_shear_layer_run
    n, theta = 64, 0.4
    got = double_shear_layer_run(model, theta, n, t_conv=0.1)
    fields = inp.double_shear_layer(n, n, U0, KAPPA, DELTA)
    f = oracle.run(oracle.init_equilibrium(*fields, theta), theta, U0 * n / RE, model, got["steps"])
    _, ux, uy = field_moments(f)
    assert got["stable"]
    assert got["thickness"] == pytest.approx(_numpy_thickness(ux), rel=1e-9)
    assert got["vortex_cores"] == _numpy_cores(ux, uy)
