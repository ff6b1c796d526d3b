"""Flow diagnostics on the fields a Simulation returns (torch, FP64; any device):

* the Fourier amplitude of a velocity mode and the effective viscosity from its decay,
  with the rotated shear-wave measurement of the paper's first benchmark (Sec. 5, the
  pi/4-rotated decaying shear wave), read on a doubly periodic n x n box:
  u_x = u_y = U/sqrt(2) + A sin(2 pi (-x + y)/n), wave vector k = (2 pi/n)(-1, 1),
  perturbation along (1, 1), so the mean flow U (along (1, 1)) advects the wave parallel
  to its crests;
* vorticity, the vorticity thickness of the x-averaged profile and a count of vortex cores
  for the double shear layer of the paper's third benchmark (Sec. 5).

These are post-processing of the library's outputs, not steps of the method.
"""
import math

import torch
import torch.nn.functional as F

from .simulation import Simulation


def mode_amplitude(ux, uy, kx, ky):
    """Complex Fourier coefficient (1/N) sum (u_x + u_y) exp(-i 2 pi (kx x/nx + ky y/ny)) of
    [ny, nx] periodic fields at the integer wave vector (kx, ky), in FP64."""
    ny, nx = ux.shape
    dev = ux.device
    x = torch.arange(nx, device=dev, dtype=torch.float64)[None, :]
    y = torch.arange(ny, device=dev, dtype=torch.float64)[:, None]
    phase = 2.0 * math.pi * (kx * x / nx + ky * y / ny)
    s = ux.double() + uy.double()
    re = float((s * torch.cos(phase)).sum())
    im = -float((s * torch.sin(phase)).sum())
    return complex(re, im) / (nx * ny)


def decay_viscosity(a0, a1, k2, steps):
    """Effective viscosity from a mode's amplitude decay |a1| = |a0| exp(-nu k^2 steps)."""
    return -math.log(abs(a1) / abs(a0)) / (k2 * steps)


def rotated_wave_fields(n, A, U, rho0=1.0, device=None):
    """FP64 device fields (rho, u_x, u_y) of the rotated shear wave on an n x n box."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    x = torch.arange(n, device=dev, dtype=torch.float64)[None, :]
    y = torch.arange(n, device=dev, dtype=torch.float64)[:, None]
    ux = U / math.sqrt(2.0) + A * torch.sin(2.0 * math.pi * (-x + y) / n)
    return torch.full((n, n), rho0, device=dev, dtype=torch.float64), ux, ux.clone()


def rotated_wave_viscosity(model, theta, nu, mach, n=200, A=1e-3, skip=200, steps=1000, storage="f64",
                           pattern="ab"):
    """nu~/nu of the rotated shear wave advected at U = mach sqrt(theta) (the lattice sound
    speed is sqrt(theta)): the decay of the (-1, 1) mode between step `skip` and step
    `skip + steps`, which leaves out the initial transient of the non-equilibrium modes.
    Returns None when the run is unstable: not finite, the mode grows, or the velocity
    deviates from the mean flow by more than 1.5 A anywhere (energy has gone into other
    modes, so the decay of this one no longer measures a viscosity)."""
    rho, ux, uy = rotated_wave_fields(n, A, mach * math.sqrt(theta))
    sim = Simulation(n, n, theta, nu, ux, uy, rho=rho, model=model, storage=storage, pattern=pattern)
    sim.step(skip)
    _, u0, v0 = sim.moments()
    a0 = mode_amplitude(u0, v0, -1, 1)
    sim.step(steps)
    _, u1, v1 = sim.moments()
    a1 = mode_amplitude(u1, v1, -1, 1)
    dev = max(float((u1 - u1.mean()).abs().max()), float((v1 - v1.mean()).abs().max()))
    sim.close()
    if not (math.isfinite(abs(a0)) and math.isfinite(abs(a1)) and math.isfinite(dev)):
        return None
    if abs(a1) == 0 or abs(a1) > abs(a0) or dev > 1.5 * A:
        return None
    return decay_viscosity(a0, a1, 2.0 * (2.0 * math.pi / n) ** 2, steps) / nu


def vorticity(ux, uy):
    """omega = d u_y/dx - d u_x/dy by periodic central differences, fields [ny, nx]."""
    dvdx = 0.5 * (torch.roll(uy, -1, dims=1) - torch.roll(uy, 1, dims=1))
    dudy = 0.5 * (torch.roll(ux, -1, dims=0) - torch.roll(ux, 1, dims=0))
    return dvdx.double() - dudy.double()


def shear_layer_thickness(ux, u0):
    """Vorticity thickness 2 u0 / max |d<u_x>/dy| of the x-averaged profile, averaged over the
    lower (y < ny/2) and upper layer, in units of the box height ny."""
    prof = ux.double().mean(dim=1)
    ny = prof.numel()
    d = 0.5 * (torch.roll(prof, -1) - torch.roll(prof, 1)).abs()
    lower, upper = float(d[: ny // 2].max()), float(d[ny // 2:].max())
    return 0.5 * (2.0 * u0 / lower + 2.0 * u0 / upper) / ny


def vortex_cores(omega, frac=0.3, window=5):
    """Number of local maxima of |omega| over a periodic window x window neighbourhood that
    exceed frac times the global maximum."""
    a = omega.abs()[None, None]
    h = window // 2
    m = F.max_pool2d(F.pad(a, (h, h, h, h), mode="circular"), window, stride=1)
    return int(((a == m) & (a > frac * a.max())).sum())


def double_shear_layer_run(model, theta, n, u0=0.04, kappa=80.0, delta=0.05, re=30000.0, t_conv=1.0,
                           storage="f64", pattern="ab"):
    """The double shear layer of the paper's third benchmark on an n x n periodic box
    (the 2 pi x 2 pi domain), nu = u0 n / Re, run for t_conv convective times n / u0.
    Returns a dict: steps, stable (finite and max |u| < 5 u0), thickness (box units),
    vortex cores, max |omega| (lattice units)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    x = torch.arange(n, device=dev, dtype=torch.float64)[None, :]
    y = torch.arange(n, device=dev, dtype=torch.float64)[:, None]
    s = y / n
    ux = torch.where(y <= n / 2, u0 * torch.tanh(kappa * (s - 0.25)), u0 * torch.tanh(kappa * (0.75 - s))) + 0.0 * x
    uy = delta * u0 * torch.sin(2.0 * math.pi * (x / n + 0.25)) + 0.0 * y
    nu = u0 * n / re
    steps = int(round(t_conv * n / u0))
    sim = Simulation(n, n, theta, nu, ux, uy, model=model, storage=storage, pattern=pattern)
    sim.step(steps)
    _, u, v = sim.moments()
    sim.close()
    umax = float(torch.maximum(u.abs().max(), v.abs().max()))
    out = {"steps": steps, "nu": nu, "stable": bool(math.isfinite(umax) and umax < 5.0 * u0)}
    if out["stable"]:
        w = vorticity(u, v)
        out.update(thickness=shear_layer_thickness(u, u0), vortex_cores=vortex_cores(w),
                   max_vorticity=float(w.abs().max()))
    return out
