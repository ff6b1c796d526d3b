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


def eps_u(u, uref):
    return float(np.max(np.abs(u - uref)) / np.max(np.abs(uref)))
