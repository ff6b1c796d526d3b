"""Seeded synthetic inputs for the D2Q9 lattice Boltzmann workloads.

This module serves both the CPU oracle (oracle/) and the HIP path
(paper_2602_21242_amd/). It holds none of the method's arithmetic: it only builds
initial density/velocity fields, random populations and perturbation directions in FP64
on the host, plus the workload definitions. Every random draw uses numpy's PCG64
generator with an explicit seed.

Coordinates are node indices x = 0..nx-1, y = 0..ny-1; every field is a float64 array of
shape (ny, nx) (x fastest). The paper's own workloads are analytic initial conditions
(rotated shear wave, doubly periodic shear layer); the remaining ones (Taylor-Green
vortex, random-phase turbulence) are standard periodic test flows.
"""
from dataclasses import dataclass, field
import math

import numpy as np


def _grid(nx, ny):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y


def gaussian_noise(shape, sigma, seed):
    """i.i.d. N(0, sigma^2) samples, float64."""
    return np.random.default_rng(seed).normal(0.0, sigma, size=shape)


def taylor_green(nx, ny, U0, theta, rho0=1.0, noise=0.0, seed=0):
    """Taylor-Green vortex with one wavelength per box side.

    u_x = -U0 cos(kx x) sin(ky y), u_y = U0 sin(kx x) cos(ky y), kx = 2 pi/nx, ky = 2 pi/ny,
    density from the ideal-gas pressure p = theta rho of the vortex (square boxes):
    rho = rho0 [1 - U0^2/(4 theta) (cos 2 kx x + cos 2 ky y)].
    Optional i.i.d. Gaussian noise of standard deviation `noise` on each velocity component.
    """
    x, y = _grid(nx, ny)
    kx, ky = 2 * math.pi / nx, 2 * math.pi / ny
    ux = -U0 * np.cos(kx * x) * np.sin(ky * y)
    uy = U0 * np.sin(kx * x) * np.cos(ky * y)
    rho = rho0 * (1.0 - U0 * U0 / (4.0 * theta) * (np.cos(2 * kx * x) + np.cos(2 * ky * y)))
    if noise > 0.0:
        n = gaussian_noise((2, ny, nx), noise, seed)
        ux = ux + n[0]
        uy = uy + n[1]
    return rho, ux, uy


def shear_wave(nx, ny, A, U=(0.0, 0.0), rho0=1.0, noise=0.0, seed=0):
    """Axis-aligned shear wave u_x = U_x + A sin(2 pi y/ny), u_y = U_y, rho = rho0."""
    x, y = _grid(nx, ny)
    ux = U[0] + A * np.sin(2 * math.pi * y / ny)
    uy = U[1] + 0.0 * x
    rho = rho0 + 0.0 * x
    if noise > 0.0:
        n = gaussian_noise((2, ny, nx), noise, seed)
        ux = ux + n[0]
        uy = uy + n[1]
    return rho, ux, uy


def rotated_shear_wave(n, A, U=0.0, rho0=1.0):
    """Shear wave rotated by pi/4 on a doubly periodic n x n box.

    u_x = u_y = U/sqrt(2) + A sin(2 pi (-x + y)/n): the velocity perturbation lies along
    (1, 1) and the wave vector along (-1, 1) (the rotated decaying shear wave of the
    paper's first benchmark, on a doubly periodic box).
    """
    x, y = _grid(n, n)
    ux = U / math.sqrt(2.0) + A * np.sin(2 * math.pi * (-x + y) / n)
    uy = ux.copy()
    rho = rho0 + 0.0 * x
    return rho, ux, uy


def shear_wave_column(n, A, Uc=0.0, rho0=1.0):
    """The rotated shear wave on a 1 x n column (nx = 1, ny = n, both periodic):
    u_x = u_y = Uc + A sin(2 pi y/n), so u_x is a shear wave and u_y a longitudinal wave
    along y, both advected by the mean flow (Uc, Uc). Fields have shape (n, 1)."""
    y = np.arange(n, dtype=np.float64)[:, None]
    ux = Uc + A * np.sin(2 * math.pi * y / n)
    return rho0 + 0.0 * y, ux, ux.copy()


def random_phase_turbulence(n, kmin, kmax, u_rms, seed=0, rho0=1.0):
    """Solenoidal random-phase velocity field with an E(K) ~ K^(-5/3) shell spectrum.

    Stream-function modes at integer wave vectors with shell K = round(|k|) in
    [kmin, kmax], amplitude |psi_hat| ~ K^(-7/3), uniform random phases; u = d psi/dy,
    v = -d psi/dx (spectral derivatives); one common scale factor (which keeps the field
    divergence-free) sets the rms over both components, sqrt(<u^2 + v^2>/2), to u_rms.
    """
    rng = np.random.default_rng(seed)
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    ky, kx = np.meshgrid(k1, k1, indexing="ij")
    K = np.rint(np.sqrt(kx * kx + ky * ky))
    mask = (K >= kmin) & (K <= kmax)
    amp = np.zeros((n, n))
    amp[mask] = K[mask] ** (-7.0 / 3.0)
    phase = rng.uniform(0.0, 2 * math.pi, size=(n, n))
    psi_hat = amp * np.exp(1j * phase)
    psi = np.fft.ifft2(psi_hat).real
    psi_hat = np.fft.fft2(psi)  # Hermitian-symmetric spectrum of the real field
    two_pi_over_n = 2 * math.pi / n
    ux = np.fft.ifft2(1j * ky * two_pi_over_n * psi_hat).real
    uy = np.fft.ifft2(-1j * kx * two_pi_over_n * psi_hat).real
    scale = u_rms / np.sqrt(0.5 * np.mean(ux * ux + uy * uy))
    ux *= scale
    uy *= scale
    rho = np.full((n, n), rho0)
    return rho, ux, uy


def double_shear_layer(nx, ny, u0, kappa, delta, rho0=1.0):
    """Doubly periodic shear layer (the paper's third benchmark), on an nx x ny box.

    u_x = u0 tanh[kappa (y/ny - 1/4)] for y <= ny/2, u0 tanh[kappa (3/4 - y/ny)] otherwise;
    u_y = delta u0 sin[2 pi (x/nx + 1/4)]; rho = rho0.
    """
    x, y = _grid(nx, ny)
    s = y / ny
    ux = np.where(y <= ny / 2, u0 * np.tanh(kappa * (s - 0.25)), u0 * np.tanh(kappa * (0.75 - s)))
    uy = delta * u0 * np.sin(2 * math.pi * (x / nx + 0.25))
    rho = rho0 + 0.0 * x
    return rho, ux, uy


def shocktube(nx, rho_l=1.0, rho_r=0.5, ny=1):
    """Isothermal shocktube on an nx x ny box with wall columns x = 0 and x = nx - 1: fluid at
    rest, rho = rho_l for x < nx/2 and rho_r for x >= nx/2 (the jump between nodes nx/2 - 1
    and nx/2); the wall nodes take the density of their side."""
    x, y = _grid(nx, ny)
    rho = np.where(x < nx // 2, rho_l, rho_r) + 0.0 * y
    return rho, 0.0 * rho, 0.0 * rho


def random_fields(nx, ny, seed, rho_spread=0.1, u_max=0.2, rho0=1.0):
    """Independent uniform random rho in rho0*[1-spread, 1+spread] and |u_a| <= u_max."""
    rng = np.random.default_rng(seed)
    rho = rho0 * (1.0 + rho_spread * rng.uniform(-1, 1, size=(ny, nx)))
    ux = u_max * rng.uniform(-1, 1, size=(ny, nx))
    uy = u_max * rng.uniform(-1, 1, size=(ny, nx))
    return rho, ux, uy


def random_populations(nx, ny, seed, amp=0.2, scale=1.0 / 9.0):
    """Positive random populations f[9, ny, nx] = scale (1 + amp r), r ~ U(-1, 1).

    Far from any equilibrium on purpose: the collision is exercised on arbitrary states.
    """
    rng = np.random.default_rng(seed)
    return scale * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(9, ny, nx)))


def random_direction(shape, seed):
    """Unit-norm (Frobenius) random direction for directional-derivative checks."""
    v = np.random.default_rng(seed).normal(size=shape)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------------------------------
# Workloads. Model names: "bgk", "uc" (uncorrected OReg), "partial", "complete".

@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    theta: float
    nu: float
    steps: int
    models: tuple
    storages: tuple
    rho0: float = 1.0
    extra: dict = field(default_factory=dict)

    def fields(self, seed=0):
        e = self.extra
        kind = e["kind"]
        if kind == "taylor_green":
            return taylor_green(self.nx, self.ny, e["U0"], self.theta, self.rho0, e.get("noise", 0.0), seed)
        if kind == "turbulence":
            return random_phase_turbulence(self.nx, e["kmin"], e["kmax"], e["u_rms"], seed, self.rho0)
        if kind == "shear_wave":
            return shear_wave(self.nx, self.ny, e["A"], (e["U"], 0.0), self.rho0, e.get("noise", 0.0), seed)
        if kind == "double_shear_layer":
            return double_shear_layer(self.nx, self.ny, e["u0"], e["kappa"], e["delta"], self.rho0)
        raise ValueError(kind)


WORKLOADS = {
    # Taylor-Green vortex 64^2, FP64, 1000 steps (oracle scale).
    "tg64": Workload("tg64", 64, 64, 1.0 / 3.0, 0.01, 1000, ("complete", "bgk", "partial", "uc"), ("f64",),
                     extra={"kind": "taylor_green", "U0": 0.05}),
    # Taylor-Green vortex 4096^2 + Gaussian velocity noise 1e-3, FP32, 2000 steps.
    "tg4096": Workload("tg4096", 4096, 4096, 0.3, 0.005, 2000, ("complete", "bgk", "partial"), ("f32",),
                       extra={"kind": "taylor_green", "U0": 0.1, "noise": 1e-3}),
    # Decaying random-phase turbulence 8192^2, k^-5/3 on k in [4, 64], u_rms 0.05, 5000 steps.
    "turb8192": Workload("turb8192", 8192, 8192, 1.0 / 3.0, 1e-4, 5000, ("complete", "bgk"),
                         ("f64", "f32", "bf16", "f16"),
                         extra={"kind": "turbulence", "kmin": 4, "kmax": 64, "u_rms": 0.05}),
    # Advected shear wave 1024^2 for the adjoint: u_x = 0.1 + 0.05 sin(2 pi y/L) + noise 1e-3.
    "shear1024": Workload("shear1024", 1024, 1024, 0.4, 0.01, 500, ("complete",), ("f32",),
                          extra={"kind": "shear_wave", "A": 0.05, "U": 0.1, "noise": 1e-3}),
    # Double shear layer 16384 x 4096, u0 0.2, kappa 80, delta 0.05, 3000 steps.
    "dsl16384": Workload("dsl16384", 16384, 4096, 1.0 / 3.0, 2e-4, 3000, ("complete",), ("f32",),
                         extra={"kind": "double_shear_layer", "u0": 0.2, "kappa": 80.0, "delta": 0.05}),
}
