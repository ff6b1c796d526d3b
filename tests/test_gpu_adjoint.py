"""Parity of the HIP discrete adjoint (hand-derived vector-Jacobian product of the collision,
reverse streaming, sqrt(N) checkpointing with recomputation) with the oracle's
complex-step adjoint, and of the FP32 gradient with FP64 central finite differences."""
import numpy as np
import pytest

import lbm_inputs as inp
import oracle
from tests.gpu_util import gpu_sim

pytestmark = pytest.mark.gpu

MODELS = ["bgk", "uc", "partial", "complete"]


def _t(a, dtype=None):
    import torch
    return torch.as_tensor(a, dtype=dtype or torch.float64, device="cuda")


def _oracle_population_adjoint(f0, w, theta, nu, model, n):
    states = [f0]
    for _ in range(n - 1):
        states.append(oracle.run(states[-1], theta, nu, model, 1))
    fb = w
    for s in reversed(states):
        fb = oracle.adjoint_step(s, fb, theta, nu, model)
    return fb


@pytest.mark.parametrize("pattern", ["ab", "aa"])
@pytest.mark.parametrize("model", MODELS)
def test_population_adjoint_fp64(model, pattern):
    """dJ/df^0 from dJ/df^N through N = 7 steps, for several checkpoint spacings (including
    spacings that do not divide N, one step per segment, and a single segment)."""
    nx, ny, th, nu, N = 13, 7, 0.4, 0.02, 7
    f0 = inp.random_populations(nx, ny, seed=21, amp=0.1)
    w = inp.random_direction((9, ny, nx), seed=22)
    ref = _oracle_population_adjoint(f0, w, th, nu, model, N)
    for stride in (0, 1, 2, 3, 7, 10):
        sim = gpu_sim(nx, ny, th, nu, model, "f64", pattern, f0=f0, record_steps=N, ckpt_stride=stride)
        sim.step(N)
        got = sim.adjoint_populations(_t(w)).cpu().numpy()
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= 1e-12, (stride, err)


@pytest.mark.parametrize("model", ["bgk", "uc", "complete"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16", "bf16"])
def test_population_adjoint_with_two_step_launches(model, storage):
    """With two steps per launch asked for (512 x 100, two_step = 1) the recorded forward run
    and the recomputation in the reverse sweep take two steps per launch (every storage type,
    with moment records of both, except where a pair would pass over a checkpoint time), and
    the reverse sweep takes two adjoint steps per launch (every storage type; the adjoint
    computes in FP32 or FP64), except for a segment's last odd step. N = 7 with spacings 3
    (segments of 3, 3, 1 steps), 2 and the default: against the same run with two_step = -1
    (one step per launch everywhere) to rounding (the two adjoint kernels inline the same
    VJP, but the compiler may contract its products into FMAs differently: 1e-14 of the
    largest entry in FP64, 1e-6 in FP32), and for FP64/FP32 against the oracle's
    complex-step adjoint."""
    import torch
    nx, ny, th, nu, N = 512, 100, 0.4, 0.02, 7
    f0 = inp.random_populations(nx, ny, seed=27, amp=0.05)
    w = inp.random_direction((9, ny, nx), seed=28)
    ref = _oracle_population_adjoint(f0, w, th, nu, model, N) if storage in ("f64", "f32") else None
    dtype = torch.float64 if storage == "f64" else torch.float32
    for stride in (3, 2, 0):
        got = {}
        for ts in (1, -1):
            sim = gpu_sim(nx, ny, th, nu, model, storage, "ab", f0=f0, record_steps=N, ckpt_stride=stride,
                          two_step=ts)
            assert sim.steps_per_launch == (2 if ts == 1 else 1)
            sim.step(N)
            got[ts] = sim.adjoint_populations(_t(w, dtype)).cpu().numpy()
        scale = np.max(np.abs(got[-1]))
        assert np.max(np.abs(got[1] - got[-1])) <= (1e-14 if storage == "f64" else 1e-6) * scale, stride
        if ref is not None:
            err = np.max(np.abs(got[1] - ref)) / np.max(np.abs(ref))
            assert err <= (1e-12 if storage == "f64" else 1e-5), (stride, err)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_population_adjoint_small_grid_with_two_step_sweep(storage):
    """512 x 64 (2^15 storage positions, so lbm_step replays step graphs of single steps and
    steps_per_launch reports 1) with two_step = 1: the recorded forward run takes single
    steps while the reverse sweep's recomputation and adjoint take pairs. N = 9, spacing 4:
    against two_step = -1 to rounding and against the oracle's complex-step adjoint."""
    import torch
    nx, ny, th, nu, N = 512, 64, 0.4, 0.02, 9
    f0 = inp.random_populations(nx, ny, seed=29, amp=0.05)
    w = inp.random_direction((9, ny, nx), seed=30)
    ref = _oracle_population_adjoint(f0, w, th, nu, "complete", N)
    dtype = torch.float64 if storage == "f64" else torch.float32
    got = {}
    for ts in (1, -1):
        sim = gpu_sim(nx, ny, th, nu, "complete", storage, "ab", f0=f0, record_steps=N, ckpt_stride=4, two_step=ts)
        assert sim.steps_per_launch == 1
        sim.step(N)
        got[ts] = sim.adjoint_populations(_t(w, dtype)).cpu().numpy()
    scale = np.max(np.abs(got[-1]))
    assert np.max(np.abs(got[1] - got[-1])) <= (1e-14 if storage == "f64" else 1e-6) * scale
    err = np.max(np.abs(got[1] - ref)) / np.max(np.abs(ref))
    assert err <= (1e-12 if storage == "f64" else 1e-5), err


@pytest.mark.parametrize("pattern", ["ab", "aa"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_adjoint_uses_the_forward_runs_last_segment(storage, pattern):
    """The forward run keeps the moments of its last checkpoint segment, and the reverse
    sweep recomputes only the other segments; with a single segment (spacing >= N) it
    recomputes nothing. 512 x 80 (two steps per launch for A-B), N = 11, spacing 4
    (segments 4, 4, 3), 11 and 50 (one segment), the forward advanced in one call and in
    calls of 3, 1, 2 and 5 steps (pairs and single steps meeting the last segment's start
    and end), each adjoint taken twice (the second call recomputes the last segment when
    there are several). Every result against the oracle's complex-step adjoint and against
    the first one to rounding."""
    import torch
    nx, ny, th, nu, N = 512, 80, 0.4, 0.02, 11
    f0 = inp.random_populations(nx, ny, seed=33, amp=0.05)
    w = inp.random_direction((9, ny, nx), seed=34)
    ref = _oracle_population_adjoint(f0, w, th, nu, "complete", N)
    dtype = torch.float64 if storage == "f64" else torch.float32
    results = []
    for stride in (4, 11, 50):
        for pieces in ((N,), (3, 1, 2, 5)):
            sim = gpu_sim(nx, ny, th, nu, "complete", storage, pattern, f0=f0, record_steps=N, ckpt_stride=stride,
                          two_step=1)
            for n in pieces:
                sim.step(n)
            before = sim.populations().cpu().numpy()
            for _ in range(2):
                results.append(sim.adjoint_populations(_t(w, dtype)).cpu().numpy())
                # the state at N is kept in place (one segment) or restored
                assert np.array_equal(sim.populations().cpu().numpy(), before), stride
                assert sim.time == N
            sim.close()
    scale = np.max(np.abs(ref))
    for k, r in enumerate(results):
        err = np.max(np.abs(r - ref)) / scale
        assert err <= (1e-12 if storage == "f64" else 1e-5), (k, err)
        assert np.max(np.abs(r - results[0])) <= (1e-14 if storage == "f64" else 1e-6) * scale, k


@pytest.mark.parametrize("pattern", ["ab", "aa"])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_recorded_run_reads_like_an_unrecorded_one(storage, pattern):
    """A recorded run keeps its state in a checkpoint slot after a step that ends at a
    checkpoint time (and starts there: the initial state is checkpoint 0). Its populations,
    moments and invariants read at every stop (several of them checkpoint times) equal an
    unrecorded run's bit for bit. 512 x 80, N = 12, spacing 3, two steps per launch asked
    for; stops after 3, 1, 2, 3, 3 and 2 steps (the last one past N)."""
    import torch
    nx, ny, th, nu, N = 512, 80, 0.4, 0.02, 12
    fields = inp.random_fields(nx, ny, seed=35, u_max=0.08)
    rec = gpu_sim(nx, ny, th, nu, "complete", storage, pattern, fields=fields, record_steps=N, ckpt_stride=3,
                  two_step=1)
    ref = gpu_sim(nx, ny, th, nu, "complete", storage, pattern, fields=fields, two_step=1)
    for n in (0, 3, 1, 2, 3, 3, 2):
        rec.step(n)
        ref.step(n)
        assert np.array_equal(rec.populations().cpu().numpy(), ref.populations().cpu().numpy()), n
        for a, b in zip(rec.moments(), ref.moments()):
            assert torch.equal(a, b), n
        assert rec.invariants() == ref.invariants(), n
    rec.close()
    ref.close()


@pytest.mark.parametrize("nx,ny,pattern", [(512, 80, "ab"), (512, 80, "aa"), (64, 16, "ab")])
def test_recorded_runs_in_random_pieces(nx, ny, pattern):
    """Checkpoint slots, the kept last segment and the placement of two-step launches
    depend on how a recorded run is cut into lbm_step calls. N = 13, spacings 1, 2, 3, 5, 7
    and 13, each run cut into seeded random pieces (some of length 0, the last past N):
    populations at every stop equal an unrecorded run's bit for bit, and the population
    adjoint equals that of the same run stepped in one call to 1e-14 (FP64). 512 x 80 takes
    two steps per launch (A-B); 64 x 16 runs single steps only (rows too short for the
    two-step kernel)."""
    import torch
    th, nu, N = 0.4, 0.02, 13
    rng = np.random.default_rng(36)
    fields = inp.random_fields(nx, ny, seed=37, u_max=0.08)
    w = _t(inp.random_direction((9, ny, nx), seed=38))
    ref = gpu_sim(nx, ny, th, nu, "complete", "f64", pattern, fields=fields, two_step=1)
    ref_states = {0: ref.populations().cpu().numpy()}
    for t in range(1, N + 4):
        ref.step(1)
        ref_states[t] = ref.populations().cpu().numpy()
    ref.close()
    for stride in (1, 2, 3, 5, 7, 13):
        one = gpu_sim(nx, ny, th, nu, "complete", "f64", pattern, fields=fields, record_steps=N, ckpt_stride=stride,
                      two_step=1)
        one.step(N)
        want = one.adjoint_populations(w).cpu().numpy()
        one.close()
        sim = gpu_sim(nx, ny, th, nu, "complete", "f64", pattern, fields=fields, record_steps=N, ckpt_stride=stride,
                      two_step=1)
        t = 0
        while t < N:
            n = int(rng.integers(0, 5))
            n = min(n, N - t) if rng.random() < 0.8 else n  # now and then run past N
            sim.step(n)
            t += n
            assert np.array_equal(sim.populations().cpu().numpy(), ref_states[t]), (stride, t)
        if t == N:
            got = sim.adjoint_populations(w).cpu().numpy()
            assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want)), stride
            assert np.array_equal(sim.populations().cpu().numpy(), ref_states[N]), stride
        sim.close()


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(512, 1), (512, 5), (4096, 200)])
def test_adjoint_pair_over_row_block_heights(storage, nx, ny):
    """The two-step adjoint kernel's interior wavefronts run a prologue, a loop and an
    epilogue whose lengths follow the row-block height h: 512 x 1 has h = 1, 512 x 5 blocks
    of 2 and 3 rows, 4096 x 200 32 row blocks of 6 or 7 rows (the loop body runs). Sweep
    with pairs (two_step = 1) against single adjoint steps (two_step = -1) to rounding, the
    two small grids also against the oracle's complex-step adjoint. N = 9, spacing 4."""
    import torch
    th, nu, N = 0.4, 0.02, 9
    f0 = inp.random_populations(nx, ny, seed=31, amp=0.05)
    w = inp.random_direction((9, ny, nx), seed=32)
    dtype = torch.float64 if storage == "f64" else torch.float32
    got = {}
    for ts in (1, -1):
        sim = gpu_sim(nx, ny, th, nu, "complete", storage, "ab", f0=f0, record_steps=N, ckpt_stride=4, two_step=ts)
        sim.step(N)
        got[ts] = sim.adjoint_populations(_t(w, dtype)).cpu().numpy()
        sim.close()
    scale = np.max(np.abs(got[-1]))
    assert np.max(np.abs(got[1] - got[-1])) <= (1e-14 if storage == "f64" else 1e-6) * scale
    if nx * ny <= 4096:
        ref = _oracle_population_adjoint(f0, w, th, nu, "complete", N)
        err = np.max(np.abs(got[1] - ref)) / np.max(np.abs(ref))
        assert err <= (1e-12 if storage == "f64" else 1e-5), err


@pytest.mark.parametrize("model", MODELS)
def test_velocity_gradient_fp64_matches_oracle(model):
    """Gradient of the final kinetic energy E = 1/2 sum rho |u|^2 with respect to the initial
    velocity (rho fixed), through lbm_adjoint, against the oracle's complex-step gradient."""
    nx, ny, th, nu, N = 12, 10, 0.4, 0.02, 9
    rho0, ux0, uy0 = inp.shear_wave(nx, ny, 0.05, (0.1, 0.0), noise=1e-2, seed=3)
    rN, uxN, uyN = oracle.forward_fields(rho0, ux0, uy0, th, nu, model, N)
    gx_ref, gy_ref = oracle.gradient(rho0, ux0, uy0, 0.5 * (uxN ** 2 + uyN ** 2), rN * uxN, rN * uyN, th, nu, model, N)
    for pattern in ("ab", "aa"):
        sim = gpu_sim(nx, ny, th, nu, model, "f64", pattern, fields=(rho0, ux0, uy0), record_steps=N)
        sim.step(N)
        r, vx, vy = sim.moments()
        gx, gy = sim.adjoint(0.5 * (vx * vx + vy * vy), r * vx, r * vy)
        scale = max(np.max(np.abs(gx_ref)), np.max(np.abs(gy_ref)))
        assert np.max(np.abs(gx.cpu().numpy() - gx_ref)) <= 1e-12 * scale
        assert np.max(np.abs(gy.cpu().numpy() - gy_ref)) <= 1e-12 * scale


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f16", 3e-3)])
def test_population_adjoint_reduced_precision(storage, tol):
    nx, ny, th, nu, N = 24, 16, 0.4, 0.02, 6
    f0 = oracle.init_equilibrium(*inp.random_fields(nx, ny, seed=4, u_max=0.1), th)
    w = inp.random_direction((9, ny, nx), seed=5)
    ref = _oracle_population_adjoint(f0, w, th, nu, "complete", N)
    sim = gpu_sim(nx, ny, th, nu, "complete", storage, "aa", f0=f0, record_steps=N)
    sim.step(N)
    got = sim.adjoint_populations(_t(w)).cpu().numpy()
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= tol


def _ke(rho, ux, uy):
    return 0.5 * float((rho * (ux * ux + uy * uy)).sum())


def _fd_check(w, model, steps, ndir, pattern="aa", h=1e-5):
    """FP32 adjoint gradient of the final kinetic energy against FP64 central differences of
    the GPU FP64 forward (itself pinned to the oracle) along seeded random directions."""
    import torch
    rho, ux, uy = w.fields(seed=0)
    sim = gpu_sim(w.nx, w.ny, w.theta, w.nu, model, "f32", pattern, fields=(rho, ux, uy), record_steps=steps)
    sim.step(steps)
    r, vx, vy = sim.moments(dtype=torch.float32)
    gx, gy = sim.adjoint(0.5 * (vx * vx + vy * vy), r * vx, r * vy)
    gx, gy = gx.double().cpu().numpy(), gy.double().cpu().numpy()

    def J(dx, dy):
        s = gpu_sim(w.nx, w.ny, w.theta, w.nu, model, "f64", pattern, fields=(rho, ux + dx, uy + dy))
        s.step(steps)
        return _ke(*s.moments())

    errs = []
    for k in range(ndir):
        v = inp.random_direction((2, w.ny, w.nx), seed=100 + k)
        fd = (J(h * v[0], h * v[1]) - J(-h * v[0], -h * v[1])) / (2 * h)
        ad = float(np.sum(gx * v[0]) + np.sum(gy * v[1]))
        errs.append(abs(ad - fd) / abs(fd))
    return errs


def test_fp32_gradient_vs_fd_small():
    w = inp.Workload("shear128", 128, 128, 0.4, 0.01, 100, ("complete",), ("f32",),
                     extra={"kind": "shear_wave", "A": 0.05, "U": 0.1, "noise": 1e-3})
    errs = _fd_check(w, "complete", 100, 3)
    print("relative errors", errs)
    assert max(errs) <= 1e-4


def test_fp32_gradient_vs_fd_full_size():
    """The 1024^2 advected shear wave, 500 steps, sqrt(N) = 23-step checkpoints."""
    errs = _fd_check(inp.WORKLOADS["shear1024"], "complete", 500, 2)
    print("relative errors", errs)
    assert max(errs) <= 1e-4


def test_autograd_function_enstrophy_matches_direct_adjoint():
    """LBMFunction + a torch objective (enstrophy of the central-difference vorticity) gives
    the same gradient as finite differences of the FP64 forward."""
    import torch
    from paper_2602_21242_amd import LBMFunction
    nx, ny, th, nu, N = 64, 48, 1 / 3, 2e-3, 40
    rho, ux, uy = inp.double_shear_layer(nx, ny, 0.1, 20.0, 0.05)
    cfg = dict(nx=nx, ny=ny, theta=th, nu=nu, steps=N, model="complete", storage="f64", pattern="ab")

    def enstrophy(vx, vy):
        w = 0.5 * (torch.roll(vy, -1, 1) - torch.roll(vy, 1, 1)) - 0.5 * (torch.roll(vx, -1, 0) - torch.roll(vx, 1, 0))
        return 0.5 * (w * w).sum()

    uy0 = _t(uy).requires_grad_(True)
    r, vx, vy = LBMFunction.apply(_t(ux), uy0, cfg)
    enstrophy(vx, vy).backward()
    g = uy0.grad.cpu().numpy()
    v = inp.random_direction((ny, nx), seed=7)
    h = 1e-5  # FD round-off ~ J eps / h ~ 3e-11 absolute, about 5e-7 of the derivative

    def J(d):
        _, a, b = LBMFunction.apply(_t(ux), _t(uy + d), cfg)
        return float(enstrophy(a, b))

    fd = (J(h * v) - J(-h * v)) / (2 * h)
    assert abs(np.sum(g * v) - fd) <= 1e-5 * abs(fd)


def test_adjoint_restores_state_and_repeats():
    import torch
    nx, ny, N = 16, 9, 5
    f0 = inp.random_populations(nx, ny, seed=8)
    sim = gpu_sim(nx, ny, 0.4, 0.02, "complete", "f32", "aa", f0=f0, record_steps=N, ckpt_stride=2)
    sim.step(N)
    before = sim.populations().cpu().numpy()
    w = _t(inp.random_direction((9, ny, nx), seed=9), torch.float32)
    a = sim.adjoint_populations(w).cpu().numpy()
    assert sim.time == N
    assert np.array_equal(sim.populations().cpu().numpy(), before)
    b = sim.adjoint_populations(w).cpu().numpy()
    assert np.array_equal(a, b)


def test_adjoint_state_errors():
    import torch
    from paper_2602_21242_amd import LBMError, capi
    nx, ny = 8, 8
    w = _t(np.zeros((9, ny, nx)), torch.float32)
    sim = gpu_sim(nx, ny, 0.4, 0.02, "complete", "f32")
    sim.step(2)
    with pytest.raises(LBMError) as e:
        sim.adjoint_populations(w)
    assert e.value.status == capi.LBM_ERR_STATE
    sim = gpu_sim(nx, ny, 0.4, 0.02, "complete", "f32", record_steps=3)
    sim.step(2)
    with pytest.raises(LBMError) as e:
        sim.adjoint_populations(w)
    assert e.value.status == capi.LBM_ERR_STATE
    sim.step(1)
    sim.set_populations(np.full((9, ny, nx), 1 / 9))
    with pytest.raises(LBMError) as e:
        sim.adjoint_populations(w)
    assert e.value.status == capi.LBM_ERR_STATE
