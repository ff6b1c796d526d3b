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

