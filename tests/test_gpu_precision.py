"""Precision sweep at full size: the 8192^2 decaying-turbulence workload (random-phase velocity
field with a k^-5/3 spectrum over 4 <= |k| <= 64, u_rms = 0.05, theta = 1/3, nu = 1e-4),
5000 steps, with shifted populations f_i - w_i rho0 stored in FP32, FP16 and BF16 (FP32
arithmetic) against the FP64 run on the same grid, element by element over every population
of every node (eps_f = max |f - f64| / max |f64|), in the launch configuration lbm_step uses
by default.

The 16-bit error is rounding noise that the flow carries: each step stores every population
with a relative error of up to 2^-11 (FP16) or 2^-8 (BF16), and at tau = 0.5003 the momentum
and shear modes are hardly damped, so the stored noise walks. With FP16 storage the OReg
collision returns populations whose stored values keep the node's mass and momentum: the axis
populations are rounded first and the momentum they miss goes to the four diagonal ones, a
combination that leaves mass, D and P_xy alone, so a node's stored momentum carries the
rounding of the node's four smallest populations instead of seven. Measured on MI355X
(complete model) after 100 / 1000 / 2000 / 3000 / 5000 steps: FP16 3.4e-4 / 3.9e-4 / 4.3e-4 /
4.7e-4 / 5.3e-4 (with the residual split over the axis pairs instead, diagonals rounded first:
4.5e-4 / 6.8e-4 / 9.4e-4 / 1.08e-3 / 1.27e-3; with the direct form 4.8e-4 / 1.06e-3 / - / - /
2.04e-3); BF16 (direct form) 4.5e-3 / 1.36e-2 / 2.2e-2 / 3.3e-2 / 5.6e-2; FP32 2.3e-7 / 3.4e-7
/ 3.9e-7 / 4.7e-7 / 4.9e-7. LBGK with FP16 storage (direct form, which neither split
improves: its error is carried by the non-equilibrium moments it keeps): 1.4e-3 / 2.8e-3 /
2.9e-3 / 3.1e-3 / 3.3e-3.

FP32 is held to its bar (1e-5) at every mark; FP16 to its measured curve, which lies below its
bar (1e-3) at every mark (bounds about 1.3 x the measurements: 3.4e-4 / 3.8e-4 / 3.9e-4 /
4.3e-4 / 4.7e-4 / 5.3e-4 after 100 / 700 / 1000 / 2000 / 3000 / 5000 steps); BF16 and LBGK
with FP16 storage, which do not meet 1e-3, to their measured curves as well."""
import pytest

import lbm_inputs as inp

pytestmark = pytest.mark.gpu

MARKS = (100, 700, 1000, 2000, 3000, 5000)
BOUNDS = {
    ("complete", "f32"): {n: 1e-5 for n in MARKS},
    ("complete", "f16"): {100: 4.5e-4, 700: 5e-4, 1000: 5.2e-4, 2000: 5.7e-4, 3000: 6.2e-4, 5000: 7e-4},
    ("complete", "bf16"): {100: 6e-3, 700: 1.35e-2, 1000: 1.7e-2, 2000: 2.8e-2, 3000: 4.1e-2, 5000: 7e-2},
    ("bgk", "f16"): {100: 1.9e-3, 700: 3.5e-3, 1000: 3.8e-3, 2000: 3.8e-3, 3000: 3.9e-3, 5000: 4.1e-3},
    ("partial", "f16"): {n: 4.5e-4 for n in MARKS},
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
    """FP32 within 1e-5 over the whole run; FP16 on its measured curve, within 1e-3 over the
    whole run; BF16 on its measured curve."""
    res = _sweep("complete", ("f32", "f16", "bf16"))
    for s, by_step in res.items():
        for n, e in by_step.items():
            assert e <= BOUNDS[("complete", s)][n], (s, n, e)
    assert max(res["f16"].values()) <= 1e-3


def test_precision_sweep_bgk_fp16():
    """LBGK with FP16 storage on the same workload, on its measured curve."""
    res = _sweep("bgk", ("f16",))["f16"]
    for n, e in res.items():
        assert e <= BOUNDS[("bgk", "f16")][n], (n, e)


def test_precision_sweep_partial_fp16():
    """The partially corrected model with FP16 storage (the same stored-precision conservation):
    measured 3.3e-4 / 2.9e-4 / 3.2e-4 / 3.1e-4 / 3.3e-4 after 100 / 1000 / 2000 / 3000 / 5000
    steps, held within about 1.35 x the largest of them, below the 1e-3 bar."""
    res = _sweep("partial", ("f16",))["f16"]
    for n, e in res.items():
        assert e <= BOUNDS[("partial", "f16")][n], (n, e)
