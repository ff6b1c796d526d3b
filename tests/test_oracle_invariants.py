"""Pins of the oracle's moments and FP64 totals (oracle.moments, oracle.invariants) against
results the definitions fix in closed form (Sec. 1: rho = sum_i f_i, rho u = sum_i c_i f_i;
eq:density-momentum), independent of the oracle's own code:

* a state with a single population occupied, f_k = a(x, y), has rho = a and u = c_k at every
  node and totals (sum a, c_kx sum a, c_ky sum a) -- the lattice vectors are read off the
  paper's D2Q9 figure (Fig. 1a) below, so a swapped or sign-flipped component, a wrong
  population order or a missing population fails;
* on a random state with a net momentum along both axes, the totals equal exactly rounded
  sums (math.fsum) of the populations weighted by those vectors to FP64 rounding (the
  oracle's compensated sums must not lose the small momentum to the large mass);
* the total of a state at the guided equilibrium of a uniform flow is N rho (1, u_x, u_y).
"""
import math

import numpy as np
import pytest

import lbm_inputs as inp
import oracle

# D2Q9 velocities in the numbering of the paper's figure: rest, E, N, W, S, NE, NW, SW, SE.
CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)


@pytest.mark.parametrize("k", range(9))
def test_single_population_states(k):
    nx, ny = 13, 7
    a = 0.25 + np.random.default_rng(k).uniform(0.0, 1.0, size=(ny, nx))
    f = np.zeros((9, ny, nx))
    f[k] = a
    rho, ux, uy = oracle.moments(f)
    assert np.array_equal(rho, a)
    assert np.all(ux == CX[k]) and np.all(uy == CY[k])
    tot = oracle.invariants(f)
    s = math.fsum(a.ravel())
    assert tot[0] == pytest.approx(s, rel=1e-15)
    assert tot[1] == pytest.approx(CX[k] * s, rel=1e-15, abs=0.0)
    assert tot[2] == pytest.approx(CY[k] * s, rel=1e-15, abs=0.0)


def test_totals_of_random_asymmetric_state():
    nx, ny = 37, 23
    f = inp.random_populations(nx, ny, seed=21, amp=0.002)
    f[1] *= 1.002      # a small net momentum along +x ...
    f[8] *= 1.003      # ... and +x, -y
    f[6] *= 0.999      # less along -x, +y
    tot = oracle.invariants(f)
    m = math.fsum(f.ravel())
    jx = math.fsum((np.array(CX, dtype=float)[:, None, None] * f).ravel())
    jy = math.fsum((np.array(CY, dtype=float)[:, None, None] * f).ravel())
    assert jx > 0 and jy < 0 and abs(jx) != abs(jy)
    assert abs(tot[0] - m) <= 4e-16 * m
    # the momenta are 1e-4 of the mass: a plain FP64 sum would be good to ~1e-12 of them,
    # the compensated sums to the last bits
    assert abs(tot[1] - jx) <= 4e-16 * m
    assert abs(tot[2] - jy) <= 4e-16 * m
    rho, ux, uy = oracle.moments(f)
    r = f.sum(axis=0)
    assert np.allclose(rho, r, rtol=1e-15, atol=0)
    assert np.allclose(ux * rho, np.tensordot(np.array(CX, float), f, axes=1), rtol=1e-14, atol=1e-16)
    assert np.allclose(uy * rho, np.tensordot(np.array(CY, float), f, axes=1), rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("theta", [0.3, 1.0 / 3.0, 0.45])
def test_totals_of_uniform_equilibrium(theta):
    nx, ny, rho0, u = 11, 9, 1.3, (0.07, -0.031)
    rho = np.full((ny, nx), rho0)
    f = oracle.init_equilibrium(rho, np.full((ny, nx), u[0]), np.full((ny, nx), u[1]), theta)
    tot = oracle.invariants(f)
    n = nx * ny
    assert tot[0] == pytest.approx(n * rho0, rel=1e-14)
    assert tot[1] == pytest.approx(n * rho0 * u[0], rel=1e-13)
    assert tot[2] == pytest.approx(n * rho0 * u[1], rel=1e-13)
