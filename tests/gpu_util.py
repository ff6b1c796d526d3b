"""Helpers for the GPU parity tests (test-side only)."""
import numpy as np

import oracle


def gpu_sim(nx, ny, theta, nu, model, storage, pattern="ab", fields=None, f0=None, **kw):
    """Simulation initialised from FP64 host fields (rho, ux, uy) or from populations f0."""
    import torch
    from paper_2602_21242_amd import Simulation
    if fields is None:
        fields = (None, np.zeros((ny, nx)), np.zeros((ny, nx)))
    rho, ux, uy = fields
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64, device="cuda")
    sim = Simulation(nx, ny, theta, nu, t(ux), t(uy), rho=t(rho), model=model, storage=storage, pattern=pattern, **kw)
    if f0 is not None:
        sim.set_populations(t(f0))
    return sim


def sample_nodes(nx, ny, n, seed):
    """Corner and edge nodes plus seeded random nodes."""
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, ny // 2)}
    while len(pts) < n:
        pts.add((int(rng.integers(nx)), int(rng.integers(ny))))
    return sorted(pts)


def oracle_light_cone(fields, theta, nu, model, k, nodes):
    """Oracle populations at each sampled node after k steps, computed on a periodic patch of
    (2k+3)^2 nodes centred on it: after k steps the centre depends only on nodes within
    distance k, so the patch's artificial wrap never reaches it."""
    rho, ux, uy = fields
    ny, nx = ux.shape
    h = k + 1
    out = {}
    for (x, y) in nodes:
        xs = (x + np.arange(-h, h + 1)) % nx
        ys = (y + np.arange(-h, h + 1)) % ny
        sub = lambda a: a[np.ix_(ys, xs)]
        r = sub(rho) if rho is not None else np.ones((2 * h + 1, 2 * h + 1))
        f = oracle.init_equilibrium(r, sub(ux), sub(uy), theta)
        f = oracle.run(f, theta, nu, model, k)
        out[(x, y)] = f[:, h, h]
    return out


def gather_nodes(f_gpu, nodes):
    """Populations of the sampled nodes from a torch [9, ny, nx] tensor (host numpy)."""
    import torch
    xs = torch.tensor([p[0] for p in nodes], device=f_gpu.device)
    ys = torch.tensor([p[1] for p in nodes], device=f_gpu.device)
    vals = f_gpu[:, ys, xs].double().cpu().numpy()
    return {p: vals[:, j] for j, p in enumerate(nodes)}
