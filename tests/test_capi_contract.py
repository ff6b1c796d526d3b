"""C-ABI contract of liblbm.so, checked on the host without a GPU: every symbol include/lbm.h
declares is exported, the workspace plan, and argument validation (which happens before any
HIP call)."""
import ctypes
import math
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def capi():
    from paper_2602_21242_amd import build, capi as c
    if not os.path.exists(c.LIB_PATH):
        build.build()
    c.lib()
    return c


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("lbm_init", "lbm_step", "lbm_moments", "lbm_adjoint", "lbm_workspace_bytes",
                     "lbm_invariants", "lbm_destroy", "lbm_time", "lbm_status_string", "lbm_last_error",
                     "lbm_get_populations", "lbm_set_populations", "lbm_adjoint_populations",
                     "lbm_steps_per_launch"):
        assert required in names


def test_every_declared_symbol_is_exported(capi):
    lib = ctypes.CDLL(capi.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def _params(capi, **kw):
    base = dict(nx=64, ny=32, theta=0.4, nu=0.02, rho0=1.0, model="complete", storage="f32", pattern="ab")
    base.update(kw)
    return capi.make_params(**base)


def _round_up(v, a):
    return (v + a - 1) // a * a


@pytest.mark.parametrize("storage,esize,tsize", [("f64", 8, 8), ("f32", 4, 4), ("f16", 2, 4), ("bf16", 2, 4)])
@pytest.mark.parametrize("pattern,nbuf", [("ab", 2), ("aa", 1)])
def test_workspace_plan(capi, storage, esize, tsize, pattern, nbuf):
    nx, ny = 37, 11
    pitch = _round_up(nx, 64)  # rows of whole 64-node groups
    pop = _round_up(9 * pitch * ny * esize, 4096)
    s, n = capi.lbm_workspace_bytes(_params(capi, nx=nx, ny=ny, storage=storage, pattern=pattern))
    assert s == capi.LBM_OK
    assert n == nbuf * pop + 1024 * 4 * 8 + 256
    N = 500
    s, m = capi.lbm_workspace_bytes(_params(capi, nx=nx, ny=ny, storage=storage, pattern=pattern, record_steps=N))
    stride = math.ceil(math.sqrt(N))
    nck = -(-N // stride)
    rec = _round_up(5 * pitch * ny * tsize, 4096)
    fbar = _round_up(9 * pitch * ny * tsize, 4096)
    assert m == n + (nck + 1) * pop + stride * rec + 2 * fbar
    s, m2 = capi.lbm_workspace_bytes(_params(capi, nx=nx, ny=ny, storage=storage, pattern=pattern, record_steps=N,
                                             ckpt_stride=100))
    assert m2 == n + (5 + 1) * pop + 100 * rec + 2 * fbar
    # One segment: a spacing of N or more keeps the moments of all N steps (N record slots,
    # one checkpoint plus the slot of the final state), larger spacings count as N.
    for big in (N, N + 1, 4 * N):
        s, m3 = capi.lbm_workspace_bytes(_params(capi, nx=nx, ny=ny, storage=storage, pattern=pattern,
                                                 record_steps=N, ckpt_stride=big))
        assert s == capi.LBM_OK
        assert m3 == n + (1 + 1) * pop + N * rec + 2 * fbar, big


BAD = [dict(nx=0), dict(ny=0), dict(nx=-3), dict(theta=0.0), dict(theta=1.0), dict(theta=float("nan")),
       dict(nu=0.0), dict(nu=-1e-3), dict(nu=float("inf")), dict(rho0=0.0), dict(model=4), dict(model=-1),
       dict(storage=4), dict(pattern=2), dict(record_steps=-1), dict(ckpt_stride=-2), dict(two_step=2), dict(two_step=-2),
       dict(walls=True, nx=2),
       dict(nx=65536, ny=32768), dict(nx=65537, ny=32767), dict(nx=2 ** 31 - 63, ny=1)]


@pytest.mark.parametrize("nx,ny", [(65536, 32767), (59652288, 1), (1, 2 ** 25 - 1)])
def test_largest_accepted_grids(capi, nx, ny):
    """The padded plane (nx rounded up to 64) * ny must stay below 2^31."""
    s, n = capi.lbm_workspace_bytes(_params(capi, nx=nx, ny=ny, storage="f16", pattern="aa"))
    assert s == capi.LBM_OK
    assert n >= 9 * 2 * _round_up(nx, 64) * ny


@pytest.mark.parametrize("storage,elem", [("f64", 8), ("f32", 4), ("f16", 4), ("bf16", 4)])
def test_row_width_limit(capi, storage, elem):
    """Byte offsets within one lattice row are 32-bit: 9 * pitch * (larger of the storage and
    compute element sizes) must stay below 2^31. Accepted at the widest such row (and nx one
    node short of it), rejected one node wider, for plain and recorded runs."""
    widest = (2 ** 31 - 1) // (9 * elem) // 64 * 64
    assert 9 * widest * elem < 2 ** 31 <= 9 * (widest + 64) * elem
    for rec in (0, 3):
        for nx in (widest, widest - 1):
            s, _ = capi.lbm_workspace_bytes(_params(capi, nx=nx, ny=1, storage=storage, record_steps=rec))
            assert s == capi.LBM_OK, (nx, rec)
        s, _ = capi.lbm_workspace_bytes(_params(capi, nx=widest + 1, ny=1, storage=storage, record_steps=rec))
        assert s == capi.LBM_ERR_INVALID_ARGUMENT
        assert "too wide" in capi.last_error()


@pytest.mark.parametrize("bad", BAD)
def test_invalid_parameters_rejected(capi, bad):
    s, _ = capi.lbm_workspace_bytes(_params(capi, **bad))
    assert s == capi.LBM_ERR_INVALID_ARGUMENT
    assert capi.last_error()
    s, ctx = capi.lbm_init(_params(capi, **bad), 4096, 1 << 30, None, None, 4096, 4096)
    assert s == capi.LBM_ERR_INVALID_ARGUMENT and not ctx


def test_init_argument_errors_before_any_device_work(capi):
    p = _params(capi)
    _, need = capi.lbm_workspace_bytes(p)
    s, ctx = capi.lbm_init(p, None, need, None, None, 4096, 4096)
    assert s == capi.LBM_ERR_INVALID_ARGUMENT and "workspace" in capi.last_error()
    s, ctx = capi.lbm_init(p, 4096 + 8, need, None, None, 4096, 4096)
    assert s == capi.LBM_ERR_INVALID_ARGUMENT and "aligned" in capi.last_error()
    s, ctx = capi.lbm_init(p, 4096, need - 1, None, None, 4096, 4096)
    assert s == capi.LBM_ERR_WORKSPACE_TOO_SMALL
    s, ctx = capi.lbm_init(p, 4096, need, None, None, None, 4096)
    assert s == capi.LBM_ERR_INVALID_ARGUMENT and "velocity" in capi.last_error()


def test_null_context(capi):
    assert capi.lbm_step(None, 1) == capi.LBM_ERR_INVALID_ARGUMENT
    assert capi.lbm_moments(None, capi.LBM_F64, None, None, None) == capi.LBM_ERR_INVALID_ARGUMENT
    assert capi.lbm_get_populations(None, capi.LBM_F64, 4096) == capi.LBM_ERR_INVALID_ARGUMENT
    assert capi.lbm_invariants(None)[0] == capi.LBM_ERR_INVALID_ARGUMENT
    assert capi.lbm_adjoint(None, None, 1, 1, 1, 1) == capi.LBM_ERR_INVALID_ARGUMENT
    assert capi.lbm_time(None) == -1
    assert capi.lbm_steps_per_launch(None) == -1
    capi.lbm_destroy(None)


def test_status_strings(capi):
    names = ["LBM_OK", "LBM_ERR_INVALID_ARGUMENT", "LBM_ERR_UNSUPPORTED", "LBM_ERR_WORKSPACE_TOO_SMALL",
             "LBM_ERR_HIP", "LBM_ERR_NONFINITE", "LBM_ERR_STATE"]
    for code, name in enumerate(names):
        assert capi.status_string(code) == name
    assert capi.status_string(99) == "LBM_ERR_UNKNOWN"


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_wall_parameters(capi):
    """walls: 0 or 1 (else invalid); nx >= 3; A-B without recording (else unsupported); the
    workspace does not depend on it."""
    s0, n0 = capi.lbm_workspace_bytes(_params(capi))
    s1, n1 = capi.lbm_workspace_bytes(_params(capi, walls=True))
    assert s0 == s1 == capi.LBM_OK and n0 == n1
    p = _params(capi)
    p.walls = 2
    assert capi.lbm_workspace_bytes(p)[0] == capi.LBM_ERR_INVALID_ARGUMENT
    s, _ = capi.lbm_workspace_bytes(_params(capi, walls=True, pattern="aa"))
    assert s == capi.LBM_ERR_UNSUPPORTED and "A-B" in capi.last_error()
    s, _ = capi.lbm_workspace_bytes(_params(capi, walls=True, record_steps=5))
    assert s == capi.LBM_ERR_UNSUPPORTED and "recorded" in capi.last_error()
