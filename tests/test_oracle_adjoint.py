"""Pins of the oracle's discrete adjoint (complex-step Jacobians) against central finite
differences of the oracle's forward map and the adjoint (dot-product) identity."""
import numpy as np
import pytest

import lbm_inputs as inp
import oracle


def _objective_and_seed(rho, ux, uy):
    """Kinetic energy E = 1/2 sum rho |u|^2 and its partial derivatives."""
    E = 0.5 * np.sum(rho * (ux * ux + uy * uy))
    return E, 0.5 * (ux * ux + uy * uy), rho * ux, rho * uy


@pytest.mark.parametrize("model", ["bgk", "uc", "partial", "complete"])
def test_gradient_matches_central_differences(model):
    nx, ny, theta, nu, steps = 8, 6, 0.4, 0.02, 12
    rho0, ux0, uy0 = inp.shear_wave(nx, ny, 0.05, (0.1, 0.0), noise=1e-2, seed=5)
    rhoN, uxN, uyN = oracle.forward_fields(rho0, ux0, uy0, theta, nu, model, steps)
    _, rb, uxb, uyb = _objective_and_seed(rhoN, uxN, uyN)
    gx, gy = oracle.gradient(rho0, ux0, uy0, rb, uxb, uyb, theta, nu, model, steps)
    for seed in range(3):
        vx, vy = inp.random_direction((2, ny, nx), 100 + seed)
        h = 1e-5
        Ep = _objective_and_seed(*oracle.forward_fields(rho0, ux0 + h * vx, uy0 + h * vy, theta, nu, model, steps))[0]
        Em = _objective_and_seed(*oracle.forward_fields(rho0, ux0 - h * vx, uy0 - h * vy, theta, nu, model, steps))[0]
        fd = (Ep - Em) / (2 * h)
        ad = np.sum(gx * vx) + np.sum(gy * vy)
        assert abs(ad - fd) <= 1e-8 * abs(fd), (ad, fd)


@pytest.mark.parametrize("model", ["bgk", "complete"])
def test_adjoint_step_dot_product(model):
    """<J v, w> = <v, J^T w> for one time step, J v by central differences."""
    nx, ny, theta, nu = 7, 5, 1 / 3, 0.01
    f = oracle.init_equilibrium(*inp.random_fields(nx, ny, seed=6), theta) + 1e-3 * inp.random_populations(nx, ny, 7)
    v = inp.random_direction(f.shape, 8)
    w = inp.random_direction(f.shape, 9)
    h = 1e-6
    Jv = (oracle.run(f + h * v, theta, nu, model, 1) - oracle.run(f - h * v, theta, nu, model, 1)) / (2 * h)
    JTw = oracle.adjoint_step(f, w, theta, nu, model)
    assert abs(np.sum(Jv * w) - np.sum(v * JTw)) < 1e-9 * np.linalg.norm(JTw)
