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


def seam_nodes(nx, ny):
    """Nodes on both sides of the places where the kernels' work is split: with lane-strided
    rows (S = ceil(nx/64) groups, node x in group x mod S of lane x div S) the seam between
    the two-step kernel's block columns of 8 groups (x mod S = 7 | 8), the wrap of the rotated
    lanes at the end of a row (x = S - 1 | S), and row-block boundaries at multiples of 64
    rows (y = 63 | 64), plus the last row."""
    S = (nx + 63) // 64
    xs = sorted({x for x in (7, 8, S - 1, S, 5 * S + 7, 5 * S + 8, nx - 1) if 0 <= x < nx})
    ys = sorted({y for y in (0, 63, 64, ny // 2 - 1, ny // 2, ny - 1) if 0 <= y < ny})
    return [(x, y) for x in xs for y in ys]


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
