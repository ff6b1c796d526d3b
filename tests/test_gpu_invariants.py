"""lbm_invariants (the FP64 mass and momentum totals, Sec. 1 and eq:density-momentum) against
the oracle's totals of the same state: the populations the GPU holds, exported exactly
(every storage type converts to FP64 without rounding; the export adds the storage shift
w_i rho0 in FP64), are summed by oracle.invariants, and the two must agree to FP64
rounding, for every storage type, the A-B pattern and both AA parities, and a state that
lives in a checkpoint slot of a recorded run. rho0 = 1.3 and a state with a net momentum of
different size along +x and -y, so that a wrong mass offset rho0 nx ny, a swapped or
sign-flipped momentum component would show. Beside it, conservation: the totals after the
steps equal the oracle's totals of the FP64 initial state to within the storage type's
rounding of the stored populations (complete model: mass and momentum conserved)."""
import numpy as np
import pytest

import lbm_inputs as inp
import oracle
from tests.gpu_util import gpu_sim

pytestmark = pytest.mark.gpu

RHO0 = 1.3
UNIT_ROUNDOFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def _state(nx, ny, seed):
    f = RHO0 * inp.random_populations(nx, ny, seed=seed, amp=0.05)
    f[1] *= 1.04   # net momentum along +x ...
    f[4] *= 1.015  # ... and a smaller one along -y
    return f


def _check(sim, f0, storage, steps):
    got = np.array(sim.invariants())
    f = sim.populations().cpu().numpy()
    ref = oracle.invariants(f)
    mass = ref[0]
    assert ref[1] > 0 and ref[2] < 0
    assert np.all(np.abs(got - ref) <= 1e-13 * mass), (got, ref)
    # Conservation against the FP64 initial state: each stored (shifted) population is off by at
    # most half an ulp of the storage type per rounding, once at the import and once per step.
    # |g| = |f - w rho0| <= rho0 for these states (0 < f < rho0, 0 < w < 1)
    bound = (steps + 1) * UNIT_ROUNDOFF[storage] * 9 * f0[0].size * RHO0 + 1e-12 * mass
    ini = oracle.invariants(f0)
    assert np.all(np.abs(got - ini) <= bound), (got, ini, bound)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("pattern,steps", [("ab", 0), ("ab", 3), ("aa", 0), ("aa", 1), ("aa", 2), ("aa", 3)])
def test_invariants_equal_oracle_totals(storage, pattern, steps):
    nx, ny = 70, 13
    f0 = _state(nx, ny, seed=7)
    sim = gpu_sim(nx, ny, 0.4, 0.02, "complete", storage, pattern, f0=f0, rho0=RHO0)
    sim.step(steps)
    _check(sim, f0, storage, steps)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
@pytest.mark.parametrize("pattern", ["ab", "aa"])
def test_invariants_of_a_state_in_a_checkpoint_slot(storage, pattern):
    """A recorded run (checkpoints every 2 steps) stepped to t = 2 and t = 4: the state then
    lives in a checkpoint slot; at t = 5 in a population buffer again."""
    nx, ny = 40, 9
    f0 = _state(nx, ny, seed=8)
    sim = gpu_sim(nx, ny, 0.4, 0.02, "complete", storage, pattern, f0=f0, rho0=RHO0, record_steps=6,
                  ckpt_stride=2)
    done = 0
    for t in (2, 4, 5):
        sim.step(t - done)
        done = t
        _check(sim, f0, storage, t)


def test_invariants_of_a_uniform_flow():
    """Closed form: the guided equilibrium of a uniform flow carries N rho0 (1, u_x, u_y)."""
    nx, ny, u = 64, 20, (0.05, -0.02)
    rho = np.full((ny, nx), RHO0)
    sim = gpu_sim(nx, ny, 0.35, 0.01, "complete", "f64", fields=(rho, np.full((ny, nx), u[0]),
                                                                  np.full((ny, nx), u[1])), rho0=RHO0)
    sim.step(5)
    got = np.array(sim.invariants())
    n = nx * ny
    assert np.allclose(got, [n * RHO0, n * RHO0 * u[0], n * RHO0 * u[1]], rtol=1e-13, atol=0)
