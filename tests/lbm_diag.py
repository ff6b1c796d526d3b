"""Test-side diagnostics: the D2Q9 velocity table typed from the paper's lattice figure,
population moments, decay-rate extraction and parity metrics. Independent of both the
oracle's and the HIP path's code.
"""
import math

import numpy as np

# D2Q9 numbering of Fig. 1(a): 0 rest; 1 (+1,0); 2 (0,+1); 3 (-1,0); 4 (0,-1);
# 5 (+1,+1); 6 (-1,+1); 7 (-1,-1); 8 (+1,-1).
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]


def node_moments(f):
    """(rho, j_x, j_y, P_xx, P_yy, P_xy) of populations f[9, ...]."""
    f = np.asarray(f)
    s = lambda w: np.tensordot(w, f, axes=(0, 0))
    return s(np.ones(9)), s(CX), s(CY), s(CX * CX), s(CY * CY), s(CX * CY)


def field_moments(f):
    rho, jx, jy, *_ = node_moments(f)
    return rho, jx / rho, jy / rho


def mode_amplitude(field, kx, ky):
    """Complex Fourier coefficient of `field` at integer wave numbers (kx, ky)."""
    ny, nx = field.shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.mean(field * np.exp(-2j * math.pi * (kx * x / nx + ky * y / ny)))


def decay_viscosity(a1, a2, k2, dt):
    """nu such that |a| decays as exp(-nu k2 t) between two samples dt apart."""
    return -math.log(abs(a2) / abs(a1)) / (k2 * dt)


def eps_f(f, fref):
    """max |f - fref| / max |fref| over all populations and nodes."""
    return float(np.max(np.abs(f - fref)) / np.max(np.abs(fref)))


def isothermal_riemann(x, t, x0, rho_l, rho_r, c):
    """Exact solution (rho, u) at positions x and time t > 0 of the isothermal Euler equations
    rho_t + (rho u)_x = 0, (rho u)_t + (rho u^2 + c^2 rho)_x = 0 for a fluid at rest with
    density rho_l left of x0 and rho_r < rho_l right of it: a left rarefaction, a plateau
    (rho_m, u_m) and a right-moving shock. Along the rarefaction u + c ln rho is constant;
    across the shock the jump conditions give u_m = c (rho_m - rho_r) / sqrt(rho_m rho_r).
    rho_m solves c ln(rho_l / rho_m) = c (rho_m - rho_r) / sqrt(rho_m rho_r) (bisection).
    Returns (rho, u, rho_m, u_m, shock speed)."""
    assert rho_l > rho_r > 0 and t > 0
    g = lambda r: math.log(rho_l / r) - (r - rho_r) / math.sqrt(r * rho_r)
    lo, hi = rho_r, rho_l
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    rho_m = 0.5 * (lo + hi)
    u_m = c * math.log(rho_l / rho_m)
    s = rho_m * u_m / (rho_m - rho_r)
    xi = (np.asarray(x, dtype=np.float64) - x0) / t
    u_fan = xi + c
    rho = np.where(xi < -c, rho_l, np.where(xi < u_m - c, rho_l * np.exp(-u_fan / c), np.where(xi < s, rho_m, rho_r)))
    u = np.where(xi < -c, 0.0, np.where(xi < u_m - c, u_fan, np.where(xi < s, u_m, 0.0)))
    return rho, u, rho_m, u_m, s


def eps_u(u, uref):
    return float(np.max(np.abs(u - uref)) / np.max(np.abs(uref)))
