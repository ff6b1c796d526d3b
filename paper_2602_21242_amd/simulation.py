"""PyTorch-facing wrapper of liblbm.so: torch supplies the device workspace and the stream;
every step of the method runs in the library's HIP kernels.
"""
import torch

from . import capi

_TORCH_DTYPE = {capi.LBM_F64: torch.float64, capi.LBM_F32: torch.float32}


def _ptr(t):
    return None if t is None else t.data_ptr()


class Simulation:
    """One D2Q9 OReg-GEq lattice Boltzmann run on a periodic nx x ny box (lbm_init ...
    lbm_destroy). Fields are [ny, nx] tensors; populations [9, ny, nx].

    model: "bgk" | "uc" | "partial" | "complete"; storage: "f64" | "f32" | "bf16" | "f16";
    pattern: "ab" | "aa". record_steps > 0 checkpoints the first record_steps steps for
    adjoint() (sqrt(N) checkpoints by default, or every ckpt_stride steps; the forward run
    keeps the last segment's moments, so ckpt_stride >= record_steps needs no recomputation
    at record_steps x 5 x 4 (FP64: x 8) bytes per node). two_step: 0 runs
    two steps per launch where the grid is large enough for it to pay, 1 wherever the layout
    allows, -1 never (results are bit-identical). walls: solid bounce-back columns at x = 0
    and x = nx - 1 (A-B pattern, no recording).
    """

    def __init__(self, nx, ny, theta, nu, ux, uy, rho=None, rho0=1.0, model="complete", storage="f32",
                 pattern="ab", record_steps=0, ckpt_stride=0, two_step=0, walls=False, device=None):
        self.params = capi.make_params(nx, ny, theta, nu, rho0, model, storage, pattern, record_steps, ckpt_stride,
                                       two_step, walls)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        s, nbytes = capi.lbm_workspace_bytes(self.params)
        capi.check(s, "lbm_workspace_bytes")
        self.workspace_bytes = nbytes
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.compute_dtype = torch.float64 if self.params.storage == capi.LBM_F64 else torch.float32
        f64 = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
        rho_t, ux_t, uy_t = f64(rho), f64(ux), f64(uy)
        for a in (rho_t, ux_t, uy_t):
            if a is not None and tuple(a.shape) != (ny, nx):
                raise ValueError(f"fields must have shape ({ny}, {nx}), got {tuple(a.shape)}")
        self.stream = torch.cuda.current_stream(self.device)
        self._ctx = None
        with torch.cuda.device(self.device):
            s, ctx = capi.lbm_init(self.params, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream,
                                   _ptr(rho_t), _ptr(ux_t), _ptr(uy_t))
        capi.check(s, "lbm_init")
        self._ctx = ctx
        # The init kernel reads the FP64 fields asynchronously; wait once so the caller may
        # free or reuse them on any stream.
        self.stream.synchronize()

    # -- lifecycle ------------------------------------------------------------------------------
    def close(self):
        """Destroy the context and release the workspace (its memory returns to torch's
        allocator, which orders reuse after the work already queued on this stream)."""
        if self._ctx is not None:
            capi.lbm_destroy(self._ctx)
            self._ctx = None
        self.workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def time(self):
        return capi.lbm_time(self._ctx)

    @property
    def steps_per_launch(self):
        """Time steps one step-kernel launch advances (2 on the two-step kernel's grids)."""
        return capi.lbm_steps_per_launch(self._ctx)

    @property
    def shape(self):
        return self.params.ny, self.params.nx

    # -- forward --------------------------------------------------------------------------------
    def step(self, n=1):
        capi.check(capi.lbm_step(self._ctx, n), "lbm_step")
        return self

    def moments(self, dtype=torch.float64):
        code = capi.LBM_F64 if dtype == torch.float64 else capi.LBM_F32
        rho, ux, uy = (torch.empty(self.shape, dtype=dtype, device=self.device) for _ in range(3))
        capi.check(capi.lbm_moments(self._ctx, code, rho.data_ptr(), ux.data_ptr(), uy.data_ptr()), "lbm_moments")
        return rho, ux, uy

    def populations(self, dtype=torch.float64):
        code = capi.LBM_F64 if dtype == torch.float64 else capi.LBM_F32
        f = torch.empty((9,) + self.shape, dtype=dtype, device=self.device)
        capi.check(capi.lbm_get_populations(self._ctx, code, f.data_ptr()), "lbm_get_populations")
        return f

    def set_populations(self, f):
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        if tuple(f.shape) != (9,) + self.shape:
            raise ValueError("populations must have shape (9, ny, nx)")
        capi.check(capi.lbm_set_populations(self._ctx, f.data_ptr()), "lbm_set_populations")
        self.stream.synchronize()
        return self

    def invariants(self, allow_nonfinite=False):
        """(sum rho, sum rho u_x, sum rho u_y) in FP64; raises on non-finite populations."""
        s, out = capi.lbm_invariants(self._ctx)
        if s == capi.LBM_ERR_NONFINITE and allow_nonfinite:
            return None
        capi.check(s, "lbm_invariants")
        return out

    # -- adjoint --------------------------------------------------------------------------------
    def adjoint(self, rho_bar, ux_bar, uy_bar):
        """dJ/du_x(0), dJ/du_y(0) from dJ/drho, dJ/du at t = record_steps (compute dtype)."""
        cast = lambda a: None if a is None else a.to(device=self.device, dtype=self.compute_dtype).contiguous()
        rb, uxb, uyb = cast(rho_bar), cast(ux_bar), cast(uy_bar)
        gx = torch.empty(self.shape, dtype=self.compute_dtype, device=self.device)
        gy = torch.empty_like(gx)
        capi.check(capi.lbm_adjoint(self._ctx, _ptr(rb), _ptr(uxb), _ptr(uyb), gx.data_ptr(), gy.data_ptr()),
                   "lbm_adjoint")
        return gx, gy

    def adjoint_populations(self, fbar_N):
        fb = fbar_N.to(device=self.device, dtype=self.compute_dtype).contiguous()
        out = torch.empty_like(fb)
        capi.check(capi.lbm_adjoint_populations(self._ctx, fb.data_ptr(), out.data_ptr()), "lbm_adjoint_populations")
        return out


class LBMFunction(torch.autograd.Function):
    """(u_x0, u_y0) -> (rho, u_x, u_y) after `steps` steps, differentiable through the
    library's discrete adjoint (sqrt(N) checkpointing by default; ckpt_stride=steps keeps the
    moments of every step instead and skips recomputation). The initial density is held fixed.

    Usage: rho, ux, uy = LBMFunction.apply(ux0, uy0, config) with
    config = dict(nx=..., ny=..., theta=..., nu=..., steps=..., model=..., storage=...,
    pattern=..., rho=None, rho0=1.0, ckpt_stride=0, two_step=0).
    """

    @staticmethod
    def forward(ctx, ux0, uy0, config):
        c = dict(config)
        steps = int(c.pop("steps"))
        sim = Simulation(c.pop("nx"), c.pop("ny"), c.pop("theta"), c.pop("nu"), ux0.detach(), uy0.detach(),
                         record_steps=steps, **c)
        sim.step(steps)
        rho, ux, uy = sim.moments(dtype=sim.compute_dtype)
        ctx.sim = sim
        ctx.in_dtypes = (ux0.dtype, uy0.dtype)
        return rho, ux, uy

    @staticmethod
    def backward(ctx, rho_bar, ux_bar, uy_bar):
        sim = ctx.sim
        z = lambda a: a if a is not None else torch.zeros(sim.shape, dtype=sim.compute_dtype, device=sim.device)
        gx, gy = sim.adjoint(rho_bar, z(ux_bar), z(uy_bar))
        return gx.to(ctx.in_dtypes[0]), gy.to(ctx.in_dtypes[1]), None
