"""Benchmark of the D2Q9 OReg-GEq lattice Boltzmann step on one MI355X.

Headline: GLUPS (10^9 lattice-node updates per second) of the FP32 completely corrected
OReg-GEq step on the 4096^2 Taylor-Green workload (theta = 0.3, nu = 0.005, U0 = 0.1 plus
Gaussian velocity noise 1e-3), with the fraction of the HBM roofline at 72 algorithmic
bytes per node update. Beside it: LBGK and partial models, the AA pattern, FP16/BF16/FP64
storage on the 8192^2 turbulence workload (with the error against the FP64 run), the
adjoint step and the end-to-end gradient, a device-to-device copy, and the FP64 CPU oracle
timed on the host cores.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak (vendor figure)
ALG_BYTES = {"f64": 144, "f32": 72, "f16": 36, "bf16": 36}   # one read + one write of 9 populations
ADJ_BYTES = {"f64": 184, "f32": 92, "f16": 92, "bf16": 92}   # fbar read + write, 5 recorded moments
METRIC = "GLUPS & %HBM peak, D2Q9 OReg-GEq step FP32 vs FP16-store; adjoint GLUPS"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _strip_comments(text):
    """C++ source without // and /* */ comments, trailing blanks and empty lines."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


# Host-only source of the library (the C ABI's orchestration: no kernel, no launch geometry).
HOST_ONLY_SOURCES = ("lbm_api.hip",)


def kernel_source_hash():
    """sha256 (first 16 hex digits) of the library's device code and launch configuration
    (every file under csrc/ but the host-only C ABI), comments and blank lines removed, so
    that counters taken on the same kernels stay valid across comment and host-side edits."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2602_21242_amd", "csrc", "*"))):
        if os.path.basename(p) in HOST_ONLY_SOURCES:
            continue
        with open(p, encoding="utf-8") as fh:
            h.update(os.path.basename(p).encode())
            h.update(_strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload, model, storage, pattern):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    if data.get("kernel_source_hash") != kernel_source_hash():
        return None
    key = f"{workload}/{model}/{storage}/{pattern}"
    ent = data.get("entries", {}).get(key)
    return None if ent is None else ent.get("hbm_bytes_per_launch")


def section(var, name, fn):
    """Run one optional section of the benchmark and merge its dict into `var`. An exception
    (for instance a device allocation that does not fit next to another process's memory) is
    recorded under "<name>_error" and the run goes on, so that the headline line is still
    printed; device memory cached by torch is released either way."""
    try:
        var.update(fn())
    except Exception as e:  # noqa: BLE001 - recorded in the output, not hidden
        log(f"[bench] {name} failed: {e!r}")
        var[f"{name}_error"] = repr(e)
    finally:
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
        except Exception:  # noqa: BLE001
            pass


def make_sim(w, model, storage, pattern, fields, **kw):
    import torch
    from paper_2602_21242_amd import Simulation
    t = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64, device="cuda")
    rho, ux, uy = fields
    return Simulation(w.nx, w.ny, w.theta, w.nu, t(ux), t(uy), rho=t(rho), model=model, storage=storage,
                      pattern=pattern, **kw)


def spin_up(sim, seconds):
    """Keep the GPU busy with steps of `sim` (a throwaway context) for about `seconds`, and
    return with a last chunk still queued, so that work enqueued next starts without an idle
    gap. The GPU's clocks change after every idle period: the first milliseconds of a burst of
    two-step launches run fast, the next 15-20 ms up to 1.5x slower, then the launches settle
    (measured per launch on MI355X), and only the steady state says what a long run gets."""
    import torch
    chunk = 16 * sim.steps_per_launch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        sim.step(chunk)
        torch.cuda.synchronize()
    sim.step(chunk)


def time_steps(sim, steps, warmup, spin=None, spin_s=0.0):
    """Average milliseconds per step over `steps` steps after `warmup` untimed ones, bracketed
    by torch.cuda.synchronize() on both sides and timed with HIP events recorded on the stream
    the library launches on. With `spin` (another context on the same stream) the GPU first
    runs that context for about spin_s seconds and the warm-up follows without a pause. (The
    synchronize before the timed steps idles the GPU for microseconds, which the clocks do not
    react to: 214-220 us per 4096^2 pair launch with it, 216-218 without, on MI355X.)"""
    import torch
    if spin is not None:
        spin_up(spin, spin_s)
    else:
        torch.cuda.synchronize()
    sim.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    sim.step(steps)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def time_steady(sim, steps, spin_s=0.2):
    """Milliseconds per step of `sim` in the steady state: its own steps for about spin_s
    seconds, then `steps` timed steps without a pause (the variants, which have no fixed
    warm-up count)."""
    return time_steps(sim, steps, 0, spin=sim, spin_s=spin_s)


def time_single_steps(sim, steps, warmup, spin=None, spin_s=0.0):
    """Like time_steps, with one lbm_step(1) call per step (always the single-step kernel)."""
    import torch
    if spin is not None:
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < spin_s:
            for _ in range(16):
                spin.step(1)
            torch.cuda.synchronize()
        for _ in range(16):
            spin.step(1)
    else:
        torch.cuda.synchronize()
    for _ in range(warmup):
        sim.step(1)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    for _ in range(steps):
        sim.step(1)
    stop.record(sim.stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def copy_bandwidth(nbytes=2 << 30, reps=20):
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(w, model, budget_s=15.0):
    """The FP64 CPU oracle on the same workload (full grid), timed for a bounded number of
    steps on all host cores; plus every model for 2 warm-up + 10 timed steps, and the
    chosen model on one thread for one step (MLUPS)."""
    import oracle
    rho, ux, uy = w.fields(seed=0)
    f0 = oracle.init_equilibrium(rho, ux, uy, w.theta)
    nodes = w.nx * w.ny
    t0 = time.perf_counter()
    f = oracle.run(f0, w.theta, w.nu, model, 1)
    one = time.perf_counter() - t0
    n = max(1, min(50, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(f, w.theta, w.nu, model, n)
    dt = time.perf_counter() - t0
    cores = oracle.num_threads()
    per_model = {}
    for m in ("bgk", "uc", "partial", "complete"):
        g = oracle.run(f0, w.theta, w.nu, m, 2)
        t0 = time.perf_counter()
        oracle.run(g, w.theta, w.nu, m, 10)
        per_model[m] = nodes * 10 / (time.perf_counter() - t0) / 1e6
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.run(f0, w.theta, w.nu, model, 1)
        single = nodes / (time.perf_counter() - t0) / 1e6
    finally:
        oracle.set_num_threads(cores)
    return {"value": nodes * n / dt / 1e9, "unit": "GLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{w.name} {w.nx}x{w.ny} {model} model, {n} steps after 1 warm-up step, "
                      f"{dt:.1f} s, host cpu_count={os.cpu_count()}",
            "mlups_per_model": per_model, "mlups_single_thread": single}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="tg4096")
    ap.add_argument("--model", default="complete")
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--pattern", default="ab")
    ap.add_argument("--quick", action="store_true", help="headline only: no variants, no CPU baseline")
    ap.add_argument("--single-step", action="store_true",
                    help="time the headline with one lbm_step(1) call per step (the single-step kernel)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-dsl", action="store_true", help="skip the 16384 x 4096 double-shear-layer gradient")
    ap.add_argument("--spin-up", type=float, default=0.25,
                    help="seconds of steps on a throwaway context right before the headline's warm-up steps")
    ap.add_argument("--precision-steps", type=int, default=5000,
                    help="last step of the 8192^2 storage-precision table (also taken at 100 and 1000; 0: skip)")
    ap.add_argument("--only", choices=["adjoint", "precision", "viscosity", "shear-layer", "shocktube"], default=None,
                    help="run only one section and print its JSON (adjoint: sweep and end-to-end gradient; "
                         "precision: storage types on the 8192^2 turbulence workload against the FP64 run; "
                         "viscosity: rotated shear-wave nu~/nu over theta, Mach number and model; "
                         "shear-layer: the double shear layer at the paper's parameters over n, theta and model; "
                         "shocktube: the isothermal shocktube between bounce-back walls against the exact solution)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes (counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"slab decomposition is a design, not a built path", file=sys.stderr)
        sys.exit(2)

    import torch
    import lbm_inputs as inp
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.copy_probe:
        a = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: 3 x {args.copy_probe} bytes")
        return

    if args.only == "adjoint":
        print(json.dumps(bench_adjoint(inp)), flush=True)
        return
    if args.only == "precision":
        print(json.dumps(bench_precision(inp)), flush=True)
        return
    if args.only == "viscosity":
        print(json.dumps(bench_viscosity()), flush=True)
        return
    if args.only == "shear-layer":
        print(json.dumps(bench_shear_layer()), flush=True)
        return
    if args.only == "shocktube":
        print(json.dumps(bench_shocktube()), flush=True)
        return

    w = inp.WORKLOADS[args.workload]
    nodes = w.nx * w.ny
    log(f"[bench] headline: {w.name} {w.nx}x{w.ny} {args.model} {args.storage} {args.pattern}, "
        f"{args.warmup} warm-up + {args.steps} timed steps")
    fields = w.fields(seed=0)
    timer = time_single_steps if args.single_step else time_steps
    # Cold: a fresh context, the warm-up steps and the timed steps right after its creation,
    # with the clocks wherever the preceding idle period left them.
    sim = make_sim(w, args.model, args.storage, args.pattern, fields)
    cold_ms = timer(sim, args.steps, args.warmup)
    del sim
    # Steady state: the same on a new context after a spin-up of a throwaway context of the
    # same configuration, with no pause between the spin-up, the warm-up and the timed steps.
    sim = make_sim(w, args.model, args.storage, args.pattern, fields)
    spin = make_sim(w, args.model, args.storage, args.pattern, fields)
    spl = 1 if args.single_step else sim.steps_per_launch
    ms = timer(sim, args.steps, args.warmup, spin=spin, spin_s=args.spin_up)
    del spin
    inv = sim.invariants(allow_nonfinite=True)
    del sim
    glups = nodes / (ms * 1e-3) / 1e9
    launch_s = spl * ms * 1e-3
    # Roofline: one read and one write of the nine populations per node update (72 B in FP32)
    # times the updates of one launch, over the launch time. A launch of the two-step kernel
    # performs two updates and keeps the intermediate state in LDS, so its own floor is one
    # read and one write per launch (36 B per update in FP32), reported as pair_floor.
    achieved = ALG_BYTES[args.storage] * spl * nodes / launch_s / 1e9
    log(f"[bench] {ms:.4f} ms/step ({spl} step(s) per launch), {glups:.2f} GLUPS "
        f"(cold {cold_ms:.4f} ms/step, {nodes / (cold_ms * 1e-3) / 1e9:.2f} GLUPS), "
        f"{achieved:.0f} GB/s algorithmic at {ALG_BYTES[args.storage]} B per node update")
    traffic = load_traffic(w.name, args.model, args.storage, args.pattern)
    kernel = (f"k_step2<{args.storage},{args.model}>" if spl == 2 else f"k_step<{args.storage},{args.model},{args.pattern}>")
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel, "steps_per_launch": spl,
                "alg_bytes_per_node_update": ALG_BYTES[args.storage], "launch_us": launch_s * 1e6,
                "traffic_frac": None if traffic is None else traffic / launch_s / 1e9 / HBM_PEAK_GBS}
    if spl == 2:
        floor = ALG_BYTES[args.storage] * nodes / launch_s / 1e9
        roofline["pair_floor"] = {"bytes_per_node_update": ALG_BYTES[args.storage] // 2, "achieved": floor,
                                  "frac": floor / HBM_PEAK_GBS}

    out = {
        "metric": METRIC, "value": glups, "unit": "GLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if args.storage != "f64" else "f64", "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "theta": w.theta, "nu": w.nu,
                   "model": args.model, "storage": args.storage, "pattern": args.pattern,
                   "initial_field": "Taylor-Green U0=0.1 + N(0,1e-3^2) velocity noise, seed 0"
                   if w.name == "tg4096" else w.extra},
        "roofline": roofline,
        "clock": {"spin_up_s": args.spin_up, "cold_ms_per_step": cold_ms,
                  "cold_GLUPS": nodes / (cold_ms * 1e-3) / 1e9,
                  "note": "value: timed steps after a spin-up of a throwaway context of the same configuration "
                          "(steady clocks); cold: the same warm-up and timed steps on a fresh context right "
                          "after its creation"},
        "mass_after_run": inv[0] if inv else None,
    }

    if not args.quick:
        var = {}
        log("[bench] copy bandwidth")
        section(var, "d2d_copy", lambda: {"d2d_copy_GBs": copy_bandwidth()})
        steps_v = max(100, min(args.steps, 500))

        def tg4096_variants():
            res = {}
            for model, pattern in (("complete", "ab"), ("complete", "aa"), ("bgk", "ab"), ("bgk", "aa"),
                                   ("uc", "aa"), ("partial", "aa")):
                log(f"[bench] variant tg4096 {model} f32 {pattern}")
                s = make_sim(w, model, "f32", pattern, fields)
                sp = s.steps_per_launch
                m = time_steady(s, steps_v)
                res[f"tg4096/{model}/f32/{pattern}"] = {
                    "ms_per_step": m, "GLUPS": nodes / (m * 1e-3) / 1e9, "steps_per_launch": sp,
                    "hbm_frac_per_update": 72 * nodes / (m * 1e-3) / 1e9 / HBM_PEAK_GBS}
                del s
            # The single-step kernel on the headline workload (one lbm_step(1) call per step).
            log("[bench] variant tg4096 complete f32 ab, one step per launch")
            s = make_sim(w, "complete", "f32", "ab", fields)
            m = time_single_steps(s, steps_v, 0, spin=s, spin_s=0.2)
            res["tg4096/complete/f32/ab/single-step-kernel"] = {
                "ms_per_step": m, "GLUPS": nodes / (m * 1e-3) / 1e9, "steps_per_launch": 1,
                "hbm_frac_per_update": 72 * nodes / (m * 1e-3) / 1e9 / HBM_PEAK_GBS}
            return res

        section(var, "tg4096_variants", tg4096_variants)
        del fields

        # Storage types on the 8192^2 turbulence workload: throughput, and the error table against
        # the FP64 run after 100, 1000 and 5000 steps.
        def turb8192_storage():
            res = {}
            wt = inp.WORKLOADS["turb8192"]
            log("[bench] generating turb8192 fields")
            tf = wt.fields(seed=0)
            nt = wt.nx * wt.ny
            for storage in ("f64", "f32", "f16", "bf16"):
                log(f"[bench] variant turb8192 complete {storage} ab")
                s = make_sim(wt, "complete", storage, "ab", tf)
                sp = s.steps_per_launch
                m = time_steady(s, 200)
                ent = {"ms_per_step": m, "GLUPS": nt / (m * 1e-3) / 1e9, "steps_per_launch": sp,
                       "hbm_frac_per_update": ALG_BYTES[storage] * nt / (m * 1e-3) / 1e9 / HBM_PEAK_GBS}
                if sp == 2:
                    ent["pair_floor_frac"] = ALG_BYTES[storage] * nt / (sp * m * 1e-3) / 1e9 / HBM_PEAK_GBS
                del s
                res[f"turb8192/complete/{storage}/ab"] = ent
            return res

        section(var, "turb8192_storage", turb8192_storage)
        if args.precision_steps:
            log("[bench] storage precision on turb8192")
            section(var, "precision_turb8192", lambda: {
                "precision_turb8192": bench_precision(inp, checkpoints=(100, 1000, args.precision_steps))})
        # Adjoint: the adjoint kernels at 4096^2 (HBM-sized), the end-to-end gradient on the
        # 1024^2 advected shear wave (500 steps, sqrt(N) checkpoints) and on the 16384 x 4096
        # double shear layer (3000 steps, enstrophy gradient).
        log("[bench] adjoint")
        section(var, "adjoint", lambda: bench_adjoint(inp))
        if not args.no_dsl:
            log("[bench] double shear layer gradient")
            section(var, "gradient_dsl16384", lambda: bench_gradient_dsl(inp))
        out["variants"] = var
        if not args.no_cpu:
            log("[bench] CPU oracle baseline")
            cpu = {}
            section(cpu, "cpu_baseline", lambda: {"cpu_baseline": cpu_baseline(w, args.model)})
            out.update(cpu)
    out["kernel_source_hash"] = kernel_source_hash()
    print(json.dumps(out), flush=True)


def shell_spectrum(ux, uy):
    """Kinetic-energy spectrum E(K) = 1/2 sum over |k| in [K - 1/2, K + 1/2) of |u_hat|^2 of a
    square periodic field (FP64 FFT on the device; a diagnostic, not part of the step)."""
    import torch
    n = ux.shape[0]
    fx = torch.fft.fft2(ux.double()) / ux.numel()
    fy = torch.fft.fft2(uy.double()) / uy.numel()
    e = 0.5 * (fx.abs() ** 2 + fy.abs() ** 2)
    k = torch.fft.fftfreq(n, d=1.0 / n, device=ux.device, dtype=torch.float64)
    K = torch.round(torch.sqrt(k[:, None] ** 2 + k[None, :] ** 2)).long()
    return torch.bincount(K.flatten(), weights=e.flatten()).cpu()


def bench_precision(inp, checkpoints=(100, 1000, 5000), storages=("f32", "f16", "bf16")):
    """Storage precision on the 8192^2 decaying-turbulence workload (complete model): errors
    of FP32, FP16 and BF16 storage against the FP64-storage run at the given steps
    (populations, velocity, density, kinetic energy and the shell energy spectrum), all on
    the device. eps_f = max |f - f_ref| / max |f_ref| over populations and nodes."""
    import torch
    w = inp.WORKLOADS["turb8192"]
    fields = w.fields(seed=0)
    ref = {}
    log("[precision] FP64 reference")
    s = make_sim(w, "complete", "f64", "ab", fields)
    done = 0
    for n in checkpoints:
        s.step(n - done)
        done = n
        r, ux, uy = s.moments()
        ref[n] = dict(f=s.populations(dtype=torch.float64), rho=r, ux=ux, uy=uy,
                      ke=float(0.5 * (r * (ux * ux + uy * uy)).sum()), spec=shell_spectrum(ux, uy))
    del s
    out = {"workload": w.name, "model": "complete", "reference": "FP64 storage, FP64 arithmetic",
           "ke_reference": {str(n): ref[n]["ke"] for n in checkpoints}}
    for storage in storages:
        log(f"[precision] {storage}")
        s = make_sim(w, "complete", storage, "ab", fields)
        done = 0
        res = {}
        for n in checkpoints:
            s.step(n - done)
            done = n
            r, ux, uy = s.moments()
            f = s.populations(dtype=torch.float64)
            R = ref[n]
            ke = float(0.5 * (r * (ux * ux + uy * uy)).sum())
            umax = max(float(R["ux"].abs().max()), float(R["uy"].abs().max()))
            spec = shell_spectrum(ux, uy)
            nk = min(len(spec), len(R["spec"]))
            rel = (spec[:nk] - R["spec"][:nk]).abs() / R["spec"][:nk]
            res[str(n)] = {
                "eps_f": float((f - R["f"]).abs().max() / R["f"].abs().max()),
                "eps_u_inf": max(float((ux - R["ux"]).abs().max()), float((uy - R["uy"]).abs().max())) / umax,
                "eps_u_l2": float(torch.sqrt(((ux - R["ux"]) ** 2 + (uy - R["uy"]) ** 2).sum()
                                             / (R["ux"] ** 2 + R["uy"] ** 2).sum())),
                "eps_rho": float((r - R["rho"]).abs().max() / (R["rho"] - w.rho0).abs().max()),
                "ke_rel": ke / R["ke"] - 1.0,
                "spectrum_max_rel_K4_64": float(rel[4:65].max()),
                "spectrum_rel_l1": float((spec[:nk] - R["spec"][:nk]).abs().sum() / R["spec"][:nk].sum()),
            }
            del f
        out[storage] = res
        del s
    return out


def bench_viscosity(thetas=(0.25, 1.0 / 3.0, 0.4, 0.5), machs=tuple(i / 10 for i in range(11)),
                    models=("bgk", "uc", "partial", "complete"), n=200, nu=1e-3, amp=1e-3, skip=200, steps=1000):
    """Effective viscosity nu~/nu of the pi/4-rotated decaying shear wave (the paper's first
    benchmark: nu = 1e-3, amplitude 1e-3, 1200 iterations, mean flow Ma/sqrt(6) in each
    component) over theta, Ma and the model, FP64 storage, in both geometries: the paper's
    1 x n column (u_x the shear wave along y) and a doubly periodic n x n box with the wave
    along (-1, 1). null = the wave blew up or grew."""
    from paper_2602_21242_amd.diagnostics import rotated_wave_viscosity
    t0 = time.perf_counter()
    out = {"workload": f"rotated shear wave, n={n}, nu={nu}, A={amp}, decay over steps {skip}..{skip + steps}, "
                       f"mean flow Ma/sqrt(6) per component, FP64 storage", "mach": list(machs)}
    for geometry in ("column", "diagonal"):
        table = {}
        for th in thetas:
            log(f"[viscosity] {geometry} theta {th:.4f}")
            table[f"{th:.4f}"] = {m: [rotated_wave_viscosity(m, th, nu, ma, n=n, A=amp, skip=skip, steps=steps,
                                                             geometry=geometry)
                                      for ma in machs] for m in models}
        out[f"nu_ratio_{geometry}"] = table
    out["seconds"] = time.perf_counter() - t0
    return out


def bench_shear_layer(grids=(128, 256, 512), thetas=(0.4, 0.6), models=("bgk", "uc", "partial", "complete"),
                      extra=((0.6, 1024), (0.6, 2048))):
    """The double shear layer at the paper's parameters (u0 = 0.04, kappa = 80, delta = 0.05,
    Re = 30000, one convective time n/u0, FP64 storage): stability, vorticity thickness of
    the x-averaged profile (box units; 2/kappa = 0.025 initially), vortex cores above 30 % of
    the peak vorticity, per model, grid and theta; LBGK and the complete model also at the
    larger grids for theta = 0.6."""
    import torch
    from paper_2602_21242_amd.diagnostics import double_shear_layer_run
    t0 = time.perf_counter()
    runs = []
    cases = [(th, n, m) for th in thetas for n in grids for m in models]
    cases += [(th, n, m) for th, n in extra for m in ("bgk", "complete")]
    for th, n, m in cases:
        log(f"[shear-layer] theta {th} n {n} {m}")
        t1 = time.perf_counter()
        r = double_shear_layer_run(m, th, n)
        torch.cuda.synchronize()
        r.update(theta=th, n=n, model=m, seconds=time.perf_counter() - t1)
        runs.append(r)
    return {"workload": "double shear layer, u0=0.04, kappa=80, delta=0.05, Re=30000, 1 convective time, FP64",
            "runs": runs, "seconds": time.perf_counter() - t0}


def bench_shocktube(cases=((0.4, 1e-12), (0.55, 1e-9)), models=("bgk", "uc", "partial", "complete"),
                    storages=("f64", "f32")):
    """The isothermal shocktube of the paper's second benchmark: 800 x 1 between bounce-back
    wall columns, rho = 1 | 0.5 at rest, 400 steps, per (theta, nu), model and storage type:
    stability, plateau density and velocity against the exact isothermal Riemann solution,
    mean absolute density error, and the density's total variation relative to the exact
    one (spurious oscillations raise it above 1)."""
    from paper_2602_21242_amd.diagnostics import shocktube_run
    t0 = time.perf_counter()
    runs = []
    for th, nu in cases:
        for st in storages:
            for m in models:
                log(f"[shocktube] theta {th} nu {nu:g} {m} {st}")
                r = shocktube_run(m, th, nu, storage=st)
                runs.append({"theta": th, "nu": nu, "model": m, "storage": st,
                             **{k: v for k, v in r.items() if isinstance(v, (bool, int, float))}})
    return {"workload": "isothermal shocktube 800x1, walls at x=0 and 799, rho 1|0.5, 400 steps",
            "runs": runs, "seconds": time.perf_counter() - t0}


def _time_adjoint(sim, z, spin_s=0.2, reps=3):
    """Milliseconds of one sim.adjoint call in the steady state (calls for about spin_s seconds
    first, then `reps` timed calls without a pause)."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < spin_s:
        sim.adjoint(None, z + 1e-3, z)
        torch.cuda.synchronize()
    sim.adjoint(None, z + 1e-3, z)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(sim.stream)
    for _ in range(reps):
        sim.adjoint(None, z + 1e-3, z)
    e.record(sim.stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def bench_adjoint(inp):
    import torch
    res = {}
    # Reverse sweep of a recorded 64-step run at 4096^2: recomputation from each checkpoint
    # (spacing 8) with moment recording, then the adjoint steps.
    w = inp.WORKLOADS["tg4096"]
    fields = w.fields(seed=0)
    N = 64
    nodes = w.nx * w.ny
    z = torch.zeros((w.ny, w.nx), dtype=torch.float32, device="cuda")
    sim = make_sim(w, "complete", "f32", "ab", fields, record_steps=N, ckpt_stride=8)
    sim.step(N)
    ms_sweep = _time_adjoint(sim, z)
    res["adjoint/tg4096/complete/f32/sweep"] = {
        "steps": N, "ms_total": ms_sweep, "GLUPS_gradient_sweep": nodes * N / (ms_sweep * 1e-3) / 1e9,
        "note": "reverse sweep = recorded recomputation from each checkpoint + adjoint step per step"}
    del sim
    # The same sweep with one checkpoint segment: the forward run kept the moments of every
    # step (64 x 20 B per node), so the sweep is the adjoint kernels alone (92 B per node and
    # reverse step: fbar read and written, five recorded moments read).
    sim = make_sim(w, "complete", "f32", "ab", fields, record_steps=N, ckpt_stride=N)
    sim.step(N)
    ms_one = _time_adjoint(sim, z)
    res["adjoint/tg4096/complete/f32/sweep_one_segment"] = {
        "steps": N, "ms_total": ms_one, "GLUPS_gradient_sweep": nodes * N / (ms_one * 1e-3) / 1e9,
        "hbm_frac_at_92B_per_update": 92 * nodes * N / (ms_one * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "note": "ckpt_stride = N: moments of every step kept from the forward run, no recomputation"}
    del sim, z
    # End-to-end gradient of the final kinetic energy on the 1024^2 shear wave.
    from paper_2602_21242_amd import LBMFunction
    wa = inp.WORKLOADS["shear1024"]
    rho, ux, uy = wa.fields(seed=0)
    cfg = dict(nx=wa.nx, ny=wa.ny, theta=wa.theta, nu=wa.nu, steps=wa.steps, model="complete", storage="f32",
               pattern="ab")
    t = lambda a: torch.as_tensor(a, dtype=torch.float32, device="cuda")
    for key, c, note in (("gradient/shear1024/complete/f32/ab", cfg,
                          "forward with checkpoints + recomputation + adjoint, cache-resident size"),
                         ("gradient/shear1024/complete/f32/ab/one_segment", dict(cfg, ckpt_stride=wa.steps),
                          "ckpt_stride = steps: forward keeps every step's moments (10.5 GB), sweep without "
                          "recomputation")):
        for rep in range(3):
            ux0 = t(ux).requires_grad_(True)
            uy0 = t(uy).requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r, vx, vy = LBMFunction.apply(ux0, uy0, c)
            E = 0.5 * (r * (vx * vx + vy * vy)).sum()
            E.backward()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        res[key] = {"steps": wa.steps, "s_total": dt, "GLUPS_end_to_end": wa.nx * wa.ny * wa.steps / dt / 1e9,
                    "note": note}
    return res


def _enstrophy(ux, uy):
    """Half the sum of the squared central-difference vorticity (periodic), in FP64."""
    import torch
    wz = 0.5 * (torch.roll(uy, -1, 1) - torch.roll(uy, 1, 1)) - 0.5 * (torch.roll(ux, -1, 0) - torch.roll(ux, 1, 0))
    return 0.5 * (wz.double() * wz.double()).sum()


def bench_gradient_dsl(inp):
    """End-to-end gradient on the 16384 x 4096 double shear layer: the 3000-step FP32 forward
    with sqrt(N) checkpoints (55-step spacing), the final enstrophy, and its gradient with
    respect to the initial velocity (recomputation of every checkpoint segment but the last,
    and the adjoint sweep); about 219 GB of workspace. Skipped when the device lacks the
    memory."""
    import torch
    from paper_2602_21242_amd import LBMFunction, capi
    import gc
    w = inp.WORKLOADS["dsl16384"]
    p = capi.make_params(w.nx, w.ny, w.theta, w.nu, model="complete", storage="f32", pattern="ab",
                         record_steps=w.steps)
    need = capi.lbm_workspace_bytes(p)[1]
    gc.collect()
    torch.cuda.empty_cache()  # memory the earlier sections left in torch's cache
    free = torch.cuda.mem_get_info()[0]
    key = f"gradient/dsl16384/complete/f32/ab"
    if free < need + (2 << 30):
        return {key: {"skipped": f"needs {need / 1e9:.0f} GB of device memory, {free / 1e9:.0f} GB free"}}
    rho, ux, uy = w.fields(seed=0)
    cfg = dict(nx=w.nx, ny=w.ny, theta=w.theta, nu=w.nu, steps=w.steps, model="complete", storage="f32",
               pattern="ab")
    ux0 = torch.as_tensor(ux, dtype=torch.float32, device="cuda").requires_grad_(True)
    uy0 = torch.as_tensor(uy, dtype=torch.float32, device="cuda").requires_grad_(True)
    del rho, ux, uy
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, vx, vy = LBMFunction.apply(ux0, uy0, cfg)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _enstrophy(vx, vy).backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    nodes = w.nx * w.ny
    out = {key: {"steps": w.steps, "workspace_GB": need / 1e9, "s_forward": t1 - t0, "s_backward": t2 - t1,
                 "GLUPS_end_to_end": nodes * w.steps / (t2 - t0) / 1e9,
                 "GLUPS_forward_recorded": nodes * w.steps / (t1 - t0) / 1e9,
                 "grad_uy0_l2": float(uy0.grad.double().norm()),
                 "note": "forward with 55-step checkpoints (first launches include the context set-up), "
                         "enstrophy, recomputation + adjoint sweep + initial-condition adjoint"}}
    del r, vx, vy, ux0, uy0
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
