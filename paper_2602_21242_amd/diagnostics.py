"""Flow diagnostics on the fields a Simulation returns (torch, FP64; any device):

* the Fourier amplitude of a velocity mode and the effective viscosity from its decay,
  with the rotated shear-wave measurement of the paper's first benchmark (Sec. 5, the
  pi/4-rotated decaying shear wave, mean flow Ma/sqrt(6) in each component), in two
  geometries: "diagonal", a doubly periodic n x n box with
  u_x = u_y = Ma/sqrt(6) + A sin(2 pi (-x + y)/n) (wave vector along (-1, 1), perturbation
  and mean flow along (1, 1)), and "column", the paper's 1 x n grid, where the wave can only
  vary along y: u_x = u_y = Ma/sqrt(6) + A sin(2 pi y/n), u_x being the shear wave;
* the isothermal shocktube of the paper's second benchmark (Sec. 5) between two bounce-back
  walls, against the exact solution of the isothermal Riemann problem;
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


def rotated_wave_fields(n, A, Uc, rho0=1.0, device=None, geometry="diagonal"):
    """FP64 device fields (rho, u_x, u_y) of the rotated shear wave with mean flow Uc in each
    component: an n x n box ("diagonal") or an n x 1 column ("column")."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    y = torch.arange(n, device=dev, dtype=torch.float64)[:, None]
    if geometry == "column":
        ux = Uc + A * torch.sin(2.0 * math.pi * y / n)
        return torch.full((n, 1), rho0, device=dev, dtype=torch.float64), ux, ux.clone()
    if geometry != "diagonal":
        raise ValueError(f"unknown geometry {geometry!r}")
    x = torch.arange(n, device=dev, dtype=torch.float64)[None, :]
    ux = Uc + A * torch.sin(2.0 * math.pi * (-x + y) / n)
    return torch.full((n, n), rho0, device=dev, dtype=torch.float64), ux, ux.clone()


def rotated_wave_viscosity(model, theta, nu, mach, n=200, A=1e-3, skip=200, steps=1000, storage="f64",
                           pattern="ab", geometry="diagonal"):
    """nu~/nu of the rotated shear wave advected by the mean flow Ma/sqrt(6) in each
    component (the paper's initial condition): the decay between step `skip` and step
    `skip + steps` (which leaves out the initial transient of the non-equilibrium modes) of
    the (-1, 1) mode of u_x + u_y on the n x n box ("diagonal"), or of the first mode of
    u_x along the 1 x n column ("column"). Returns None when the run is unstable: not finite,
    the mode grows, or the velocity deviates from the mean flow by more than 1.5 A anywhere
    (energy has gone into other modes, so the decay of this one no longer measures a
    viscosity)."""
    rho, ux, uy = rotated_wave_fields(n, A, mach / math.sqrt(6.0), geometry=geometry)
    ny, nx = ux.shape
    sim = Simulation(nx, ny, theta, nu, ux, uy, rho=rho, model=model, storage=storage, pattern=pattern)
    if geometry == "column":
        amp = lambda u, v: mode_amplitude(u, 0.0 * u, 0, 1)
        k2 = (2.0 * math.pi / n) ** 2
    else:
        amp = lambda u, v: mode_amplitude(u, v, -1, 1)
        k2 = 2.0 * (2.0 * math.pi / n) ** 2
    sim.step(skip)
    _, u0, v0 = sim.moments()
    a0 = amp(u0, v0)
    sim.step(steps)
    _, u1, v1 = sim.moments()
    a1 = amp(u1, v1)
    dev = max(float((u1 - u1.mean()).abs().max()), float((v1 - v1.mean()).abs().max()))
    sim.close()
    if not (math.isfinite(abs(a0)) and math.isfinite(abs(a1)) and math.isfinite(dev)):
        return None
    if abs(a1) == 0 or abs(a1) > abs(a0) or dev > 1.5 * A:
        return None
    return decay_viscosity(a0, a1, k2, steps) / nu


def isothermal_riemann(x, t, x0, rho_l, rho_r, c):
    """Exact solution of the isothermal Euler equations (sound speed c) for a fluid at rest
    with density rho_l left of x0 and rho_r < rho_l right of it, at positions x (tensor) and
    time t > 0: a left rarefaction along which u + c ln rho is constant, a plateau
    (rho_m, u_m), and a shock whose jump conditions give u_m = c (rho_m - rho_r) /
    sqrt(rho_m rho_r). Returns (rho, u, rho_m, u_m, shock speed); rho_m by bisection."""
    if not (rho_l > rho_r > 0 and t > 0):
        raise ValueError("need rho_l > rho_r > 0 and t > 0")
    lo, hi = rho_r, rho_l
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if math.log(rho_l / mid) > (mid - rho_r) / math.sqrt(mid * rho_r):
            lo = mid
        else:
            hi = mid
    rho_m = 0.5 * (lo + hi)
    u_m = c * math.log(rho_l / rho_m)
    s = rho_m * u_m / (rho_m - rho_r)
    xi = (x.double() - x0) / t
    fan = (xi >= -c) & (xi < u_m - c)
    plateau = (xi >= u_m - c) & (xi < s)
    rho = torch.where(xi < -c, torch.full_like(xi, rho_l), torch.full_like(xi, rho_r))
    rho = torch.where(fan, rho_l * torch.exp(-(xi + c) / c), rho)
    rho = torch.where(plateau, torch.full_like(xi, rho_m), rho)
    u = torch.where(fan, xi + c, torch.zeros_like(xi))
    u = torch.where(plateau, torch.full_like(xi, u_m), u)
    return rho, u, rho_m, u_m, s


def shocktube_run(model, theta, nu, nx=800, steps=400, rho_l=1.0, rho_r=0.5, storage="f64"):
    """The isothermal shocktube of the paper's second benchmark: an nx x 1 box whose columns
    x = 0 and nx - 1 are bounce-back walls, fluid at rest with rho = rho_l for x < nx/2 and
    rho_r beyond, run for `steps` steps. Returns a dict with the fluid profiles (x = 1 ..
    nx - 2), `stable` (finite, 0 < rho < 2 rho_l and |u| < 2 sqrt(theta) everywhere) and, when
    stable: the plateau density and velocity (mean of the 21 nodes around
    the middle of the exact plateau) and their errors relative to the exact solution
    (sound speed sqrt(theta), jump at x = nx/2 - 1/2), the mean absolute density error over
    the fluid, and the total variation of the density relative to the exact one (spurious
    oscillations raise it above 1)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    x = torch.arange(nx, device=dev, dtype=torch.float64)[None, :]
    rho0 = torch.where(x < nx // 2, rho_l, rho_r).double()
    sim = Simulation(nx, 1, theta, nu, 0.0 * x, 0.0 * x, rho=rho0, model=model, storage=storage, walls=True)
    sim.step(steps)
    r, u, _ = sim.moments()
    sim.close()
    r, u = r[0, 1:-1].double(), u[0, 1:-1].double()
    xf = x[0, 1:-1]
    c = math.sqrt(theta)
    stable = bool(torch.isfinite(r).all() and torch.isfinite(u).all())
    stable = stable and bool(((r > 0) & (r < 2 * rho_l) & (u.abs() < 2 * c)).all())
    out = {"steps": steps, "rho": r, "u": u, "stable": stable}
    re, ue, rho_m, u_m, s = isothermal_riemann(xf, float(steps), nx / 2 - 0.5, rho_l, rho_r, c)
    out.update(rho_exact=re, u_exact=ue, rho_plateau_exact=rho_m, u_plateau_exact=u_m)
    if out["stable"]:
        xm = int(round(nx / 2 - 0.5 + steps * 0.5 * (u_m - c + s))) - 1  # index into the fluid
        pl = slice(xm - 10, xm + 11)
        rp, up = float(r[pl].mean()), float(u[pl].mean())
        tv = float((r[1:] - r[:-1]).abs().sum()) / float((re[1:] - re[:-1]).abs().sum())
        out.update(rho_plateau=rp, u_plateau=up, rho_plateau_err=rp / rho_m - 1, u_plateau_err=up / u_m - 1,
                   l1_rho=float((r - re).abs().mean()), tv_ratio=tv)
    return out


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
