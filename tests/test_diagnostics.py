"""The package's flow diagnostics (torch, run here on CPU tensors) against closed forms:
mode amplitude and decay viscosity, vorticity of a sine field, thickness of a tanh layer,
vortex-core count of separated Gaussian vortices."""
import math

import numpy as np

import pytest
import torch

from paper_2602_21242_amd import diagnostics as d


def _grid(n):
    x = torch.arange(n, dtype=torch.float64)[None, :]
    y = torch.arange(n, dtype=torch.float64)[:, None]
    return x, y


def test_mode_amplitude_and_decay_viscosity():
    n, A, U = 48, 1e-3, 0.1
    x, y = _grid(n)
    u = U / math.sqrt(2) + A * torch.sin(2 * math.pi * (-x + y) / n)
    a = d.mode_amplitude(u, u.clone(), -1, 1)
    # u_x + u_y = sqrt(2) U + 2 A sin(phi): the coefficient at +k is 2A/(2i) = -iA
    assert abs(a - (-1j * A)) < 1e-15
    k2 = 2 * (2 * math.pi / n) ** 2
    assert d.decay_viscosity(a, a * math.exp(-0.01 * k2 * 300), k2, 300) == pytest.approx(0.01, rel=1e-12)


def test_vorticity_of_sine_fields():
    n = 64
    x, y = _grid(n)
    k = 2 * math.pi / n
    ux = torch.sin(k * y) + 0 * x
    uy = torch.sin(k * x) + 0 * y
    # central differences of sin(k s) give sin(k) cos(k s)
    w = d.vorticity(ux, uy)
    ref = math.sin(k) * (torch.cos(k * x) - torch.cos(k * y))
    assert float((w - ref).abs().max()) < 1e-14


def test_thickness_of_tanh_layers():
    n, u0, kappa = 1024, 0.04, 80.0
    x, y = _grid(n)
    s = y / n
    ux = torch.where(y <= n / 2, u0 * torch.tanh(kappa * (s - 0.25)), u0 * torch.tanh(kappa * (0.75 - s))) + 0 * x
    # vorticity thickness 2 u0 / max dU/dy; the steepest point y = n/4 is a grid node, where
    # the central difference of u0 tanh(kappa (y/n - 1/4)) is u0 tanh(kappa/n) (2/kappa of the
    # box height in the continuum limit)
    assert d.shear_layer_thickness(ux, u0) == pytest.approx(2 / (n * math.tanh(kappa / n)), rel=1e-12)


def test_vortex_cores_counts_separated_vortices_across_the_wrap():
    n = 128
    x, y = _grid(n)
    wrap = lambda a: (a + n / 2) % n - n / 2
    g = lambda cx, cy, s: torch.exp(-(wrap(x - cx) ** 2 + wrap(y - cy) ** 2) / (2 * s * s))
    om = g(0, 0, 4) - g(64, 70, 5) + 0.1 * g(30, 100, 3)    # the weak one is below 30 %
    assert d.vortex_cores(om) == 2
    assert d.vortex_cores(om, frac=0.05) == 3


@pytest.mark.parametrize("c", [math.sqrt(1 / 3), math.sqrt(0.4), math.sqrt(0.55)])
def test_isothermal_riemann_solution_satisfies_jump_conditions(c):
    """The test-side exact shocktube solution: mass and momentum Rankine-Hugoniot conditions
    at the shock, the rarefaction joining the left state to the plateau continuously, and
    mass conservation of the whole profile (x in [0, 800], jump at 399.5, t = 400)."""
    from tests.lbm_diag import isothermal_riemann
    rl, rr = 1.0, 0.5
    _, _, rm, um, s = isothermal_riemann(np.array([0.0]), 400.0, 399.5, rl, rr, c)
    assert rr < rm < rl and um > 0 and s > um
    assert abs(s * (rm - rr) - rm * um) <= 1e-12
    assert abs(s * rm * um - (rm * um * um + c * c * rm - c * c * rr)) <= 1e-12
    assert abs(rl * math.exp(-um / c) - rm) <= 1e-12
    x = np.linspace(0.0, 800.0, 800001)
    rho, u, *_ = isothermal_riemann(x, 400.0, 399.5, rl, rr, c)
    mass = np.trapezoid(rho, x)
    assert abs(mass - (rl * 399.5 + rr * 400.5)) <= 1e-3
    assert rho[0] == rl and rho[-1] == rr and u[0] == 0.0 and u[-1] == 0.0


@pytest.mark.parametrize("c", [math.sqrt(0.4), math.sqrt(0.55)])
def test_package_riemann_solution_matches_test_side(c):
    """The package's exact shocktube solution (torch) against the test-side one (numpy)."""
    from tests.lbm_diag import isothermal_riemann
    x = np.arange(800, dtype=np.float64)
    r0, u0, rm0, um0, s0 = isothermal_riemann(x, 400.0, 399.5, 1.0, 0.5, c)
    r1, u1, rm1, um1, s1 = d.isothermal_riemann(torch.from_numpy(x), 400.0, 399.5, 1.0, 0.5, c)
    assert abs(rm1 - rm0) <= 1e-14 and abs(um1 - um0) <= 1e-14 and abs(s1 - s0) <= 1e-14
    np.testing.assert_allclose(r1.numpy(), r0, rtol=1e-14, atol=0)
    np.testing.assert_allclose(u1.numpy(), u0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("geometry", ["column", "diagonal"])
def test_rotated_wave_fields_match_inputs(geometry):
    """The package's rotated-wave initial fields (torch, on the CPU here) equal the test-side
    generators: mean flow Uc in each component plus the sine along y (column, shape
    (n, 1)) or along -x + y (n x n box)."""
    import lbm_inputs as inp
    n, A, Uc = 40, 1e-3, 0.3 / math.sqrt(6.0)
    rho, ux, uy = d.rotated_wave_fields(n, A, Uc, device="cpu", geometry=geometry)
    ref = inp.shear_wave_column(n, A, Uc=Uc) if geometry == "column" else inp.rotated_shear_wave(n, A, U=Uc * math.sqrt(2))
    for a, b in zip((rho, ux, uy), ref):
        assert tuple(a.shape) == b.shape
        np.testing.assert_allclose(a.numpy(), b, rtol=0, atol=1e-15)
    with pytest.raises(ValueError):
        d.rotated_wave_fields(n, A, Uc, device="cpu", geometry="spiral")
