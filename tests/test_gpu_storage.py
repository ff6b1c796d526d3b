"""Storage conversions of the HIP path: shifted populations g = f - w rho0 rounded to the
storage type with round-to-nearest-even, bit-exact against a numpy emulation (ties
included). theta = 1/2 makes the rest weights 1/4, 1/8, 1/16, so f - w rho0 is exact in
FP64 and a tie stays a tie whether the conversion rounds once or through FP32."""
import numpy as np
import pytest

from tests.gpu_util import gpu_sim

pytestmark = pytest.mark.gpu


def _rest_weights(theta):
    r = lambda c: (1.0 - theta) if c == 0 else 0.5 * theta
    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]
    return np.array([r(cx[i]) * r(cy[i]) for i in range(9)])


def _to_bf16_rne(x32):
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32)


def _shifted_values(storage, shape, seed):
    """Random magnitudes over many binades plus exact rounding ties of the 16-bit format."""
    rng = np.random.default_rng(seed)
    g = (rng.standard_normal(shape) * 10.0 ** rng.uniform(-6, -1, size=shape)).astype(np.float32)
    flat = g.reshape(-1)
    n = flat.size // 2
    if storage == "f16":
        a = rng.standard_normal(n).astype(np.float16)
        a = a[np.isfinite(a) & (a != 0)]
        b = np.nextafter(a, np.float16(np.inf))
        flat[: a.size] = (a.astype(np.float32) + b.astype(np.float32)) / 2  # exact midpoints
    elif storage == "bf16":
        hi = rng.integers(0x3000, 0x4000, size=n, dtype=np.uint32)
        flat[:n] = ((hi << 16) | 0x8000).view(np.float32) * np.where(rng.random(n) < 0.5, -1, 1).astype(np.float32)
    return flat.reshape(shape).astype(np.float64)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("pattern", ["ab", "aa"])
def test_storage_round_trip_is_rne(storage, pattern):
    nx, ny, th = 48, 10, 0.5
    w = _rest_weights(th)[:, None, None]
    g = _shifted_values(storage, (9, ny, nx), seed=1)
    f = g + w  # rho0 = 1
    sim = gpu_sim(nx, ny, th, 0.02, "complete", storage, pattern, f0=f)
    got = sim.populations().cpu().numpy()
    g32 = (f - w).astype(np.float32)
    if storage == "f16":
        gs = g32.astype(np.float16).astype(np.float64)
    elif storage == "bf16":
        gs = _to_bf16_rne(g32).astype(np.float64)
    else:
        gs = g32.astype(np.float64)
    exp = gs + w
    bad = np.argwhere(got != exp)
    for idx in bad[:8]:
        i = tuple(idx)
        print(f"mismatch at {i}: got-w {got[i] - w[i[0], 0, 0]:.9e} expected-w {gs[i]:.9e} g32 {g32[i]:.9e}")
    assert bad.shape[0] == 0, f"{bad.shape[0]} of {got.size} values differ"



def _f64_to_bf16_rne(x):
    """Correctly rounded FP64 -> BF16 (nearest, ties to even) on the FP64 bit pattern: BF16 keeps
    8 significand bits, so 45 of the 53 are rounded off (normal range only)."""
    u = np.abs(x).view(np.uint64)
    u = (u + np.uint64((1 << 44) - 1) + ((u >> np.uint64(45)) & np.uint64(1))) >> np.uint64(45) << np.uint64(45)
    return np.copysign(u.view(np.float64), x)


def _near_ties(storage, n, seed):
    """Shifted values within half an FP32 ulp of a tie between two 16-bit neighbours: rounding
    through a nearest-even FP32 first lands exactly on the tie and then on the even neighbour,
    while a single rounding of the FP64 value goes to the nearer one."""
    rng = np.random.default_rng(seed)
    if storage == "f16":
        a = (rng.standard_normal(n) * 10.0 ** rng.uniform(-3, -1, size=n)).astype(np.float16)
        a = a[np.isfinite(a) & (np.abs(a) >= np.finfo(np.float16).tiny)]  # normal range
        b = np.nextafter(a, np.float16(np.inf))
        t = (a.astype(np.float64) + b.astype(np.float64)) / 2
    else:
        hi = rng.integers(0x3C00, 0x3E00, size=n, dtype=np.uint32)   # |g| in about [0.008, 0.125)
        t = ((hi << 16) | 0x8000).view(np.float32).astype(np.float64) * np.where(rng.random(n) < 0.5, -1, 1)
    ulp32 = np.spacing(np.abs(t).astype(np.float32)).astype(np.float64)
    # short binary fractions of an FP32 ulp, so that f = g + w rho0 stays exact in FP64
    frac = rng.choice([-0.375, -0.25, 0.25, 0.375], size=t.size)
    return t + frac * ulp32


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_import_rounds_fp64_once(storage):
    """lbm_set_populations rounds g = f - w rho0 (formed in FP64) once, directly to the 16-bit
    type: on values within half an FP32 ulp of a 16-bit tie the result is the nearer neighbour,
    which rounding through FP32 would miss. theta = 1/2 keeps f - w rho0 exact in FP64."""
    nx, ny, th = 48, 10, 0.5
    w = _rest_weights(th)[:, None, None]
    vals = _near_ties(storage, 9 * nx * ny, seed=3)
    g = np.resize(vals, (9, ny, nx))
    f = g + w
    assert np.array_equal(f - w, g)
    sim = gpu_sim(nx, ny, th, 0.02, "complete", storage, "ab", f0=f)
    got = sim.populations().cpu().numpy() - w
    exp = g.astype(np.float16).astype(np.float64) if storage == "f16" else _f64_to_bf16_rne(g)
    twice = (g.astype(np.float32).astype(np.float16).astype(np.float64) if storage == "f16"
             else _to_bf16_rne(g.astype(np.float32)).astype(np.float64))
    assert np.count_nonzero(twice != exp) > g.size // 4  # the inputs do separate the two roundings
    bad = np.argwhere(got != exp)
    assert bad.shape[0] == 0, f"{bad.shape[0]} of {got.size} values differ, e.g. {tuple(bad[0])}"


def _moments64(f):
    """Exact-enough FP64 mass and momentum of one node's nine populations."""
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=np.float64)
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=np.float64)
    return np.sum(f), np.sum(cx * f), np.sum(cy * f)


@pytest.mark.parametrize("model", ["complete", "partial", "uc"])
def test_fp16_collision_keeps_mass_and_momentum_of_stored_values(model):
    """With FP16 storage the OReg collision's stored populations keep the node's mass and
    momentum up to the rounding of g*_0 (mass) and of the four diagonal populations, which take
    the momentum the rounded axis populations miss (momentum), instead of up to the rounding of
    every population. A spatially
    uniform state is unchanged by streaming, so one step maps each node's stored populations
    to its next stored populations: their FP64 moments are compared directly, over many
    random non-equilibrium states. The uncorrected model keeps only the mass (Sec. 3)."""
    nx, ny, th = 64, 2, 0.4
    w = _rest_weights(th)
    rng = np.random.default_rng(23)
    eps32 = np.finfo(np.float32).eps
    for trial in range(24):
        g = rng.standard_normal(9) * 10.0 ** rng.uniform(-3, -1.3)
        f = np.broadcast_to((g + w)[:, None, None], (9, ny, nx)).copy()
        sim = gpu_sim(nx, ny, th, 0.02, model, "f16", "ab", f0=f)
        f0 = sim.populations().cpu().numpy()
        sim.step(1)
        f1 = sim.populations().cpu().numpy()
        assert np.array_equal(f1, np.broadcast_to(f1[:, :1, :1], f1.shape))  # still uniform
        a, b = f0[:, 0, 0], f1[:, 0, 0]
        g1 = b - w
        assert np.max(np.abs(b - a)) > 0  # the collision changed the state
        half_ulp = lambda i: 0.5 * float(np.spacing(np.abs(np.float16(g1[i]))))
        slack = 64 * eps32 * np.max(np.abs(np.concatenate([a - w, g1])))  # FP32 sums
        (m0, jx0, jy0), (m1, jx1, jy1) = _moments64(a), _moments64(b)
        assert abs(m1 - m0) <= half_ulp(0) + slack, (trial, m1 - m0)
        if model != "uc":
            diag = sum(half_ulp(i) for i in (5, 6, 7, 8))
            assert abs(jx1 - jx0) <= diag + slack, (trial, jx1 - jx0)
            assert abs(jy1 - jy0) <= diag + slack, (trial, jy1 - jy0)
