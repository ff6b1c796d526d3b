"""FP64 CPU oracle of the D2Q9 OReg-GEq lattice Boltzmann step (ctypes binding).

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
leg may import this package. It shares no code with the HIP path in
paper_2602_21242_amd/, and that package never imports it.

Arrays are numpy float64, C-contiguous. Populations: f[9, ny, nx] in the numbering of the
paper's D2Q9 figure; fields: [ny, nx]. Models: 0 LBGK, 1 uncorrected OReg, 2 partially
corrected, 3 completely corrected (Sec. 4 of the paper).
"""
import ctypes

import numpy as np

from .build import ensure_built

BGK, OREG_UC, OREG_PARTIAL, OREG_COMPLETE = 0, 1, 2, 3
MODELS = {"bgk": BGK, "uc": OREG_UC, "partial": OREG_PARTIAL, "complete": OREG_COMPLETE}

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(ensure_built())
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_relaxation_time.restype = ctypes.c_double
        lib.oracle_relaxation_time.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.oracle_lattice.argtypes = [ctypes.POINTER(ctypes.c_int)] * 2
        lib.oracle_guided_equilibrium.argtypes = [ctypes.c_double] * 4 + [_dp]
        lib.oracle_collide_node.argtypes = [_dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
        lib.oracle_init_equilibrium.argtypes = [_i64, _i64, ctypes.c_double, _dp, _dp, _dp, _dp]
        lib.oracle_run.argtypes = [_i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_int, _i64, _dp]
        lib.oracle_run_walls.argtypes = [_i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_int, _i64, _dp]
        lib.oracle_moments.argtypes = [_i64, _i64, _dp, _dp, _dp, _dp]
        lib.oracle_invariants.argtypes = [_i64, _i64, _dp, _dp]
        lib.oracle_forward_fields.argtypes = [_i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              _i64, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_adjoint_step.argtypes = [_i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            _dp, _dp, _dp]
        lib.oracle_gradient.argtypes = [_i64, _i64, ctypes.c_double, ctypes.c_double, ctypes.c_int, _i64,
                                        _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib = lib
    return _lib


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _model(m):
    return MODELS[m] if isinstance(m, str) else int(m)


def num_threads():
    return _load().oracle_num_threads()


def set_num_threads(n):
    _load().oracle_set_num_threads(int(n))


def relaxation_time(theta, nu):
    return _load().oracle_relaxation_time(theta, nu)


def lattice():
    cx = (ctypes.c_int * 9)()
    cy = (ctypes.c_int * 9)()
    _load().oracle_lattice(cx, cy)
    return np.array(cx[:]), np.array(cy[:])


def guided_equilibrium(rho, ux, uy, theta):
    out = np.zeros(9)
    _load().oracle_guided_equilibrium(rho, ux, uy, theta, _ptr(out))
    return out


def collide_node(f, model, theta, tau):
    """All intermediate quantities of one collision (dict of numpy arrays)."""
    f = _f64(f).reshape(9)
    p = np.zeros(45)
    _load().oracle_collide_node(_ptr(f), _model(model), theta, tau, _ptr(p))
    return {
        "rho": p[0], "u": p[1:3], "feq": p[3:12], "fo": p[12:21], "psi": p[21:23],
        "pref": p[23], "Pi": np.array([[p[24], p[26]], [p[26], p[25]]]),
        "Psi": p[27:36], "fstar": p[36:45],
    }


def init_equilibrium(rho, ux, uy, theta):
    rho, ux, uy = _f64(rho), _f64(ux), _f64(uy)
    ny, nx = rho.shape
    f = np.zeros((9, ny, nx))
    _load().oracle_init_equilibrium(nx, ny, theta, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(f))
    return f


def run(f, theta, nu, model, nsteps, walls=False):
    """Return f after nsteps time steps (input left unchanged). walls: the columns x = 0 and
    x = nx - 1 are solid nodes with fullway bounce-back (nx >= 3)."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    _, ny, nx = f.shape
    if walls:
        assert nx >= 3
        _load().oracle_run_walls(nx, ny, theta, nu, _model(model), int(nsteps), _ptr(f))
    else:
        _load().oracle_run(nx, ny, theta, nu, _model(model), int(nsteps), _ptr(f))
    return f


def moments(f):
    f = _f64(f)
    _, ny, nx = f.shape
    rho, ux, uy = (np.zeros((ny, nx)) for _ in range(3))
    _load().oracle_moments(nx, ny, _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy))
    return rho, ux, uy


def invariants(f):
    f = _f64(f)
    _, ny, nx = f.shape
    out = np.zeros(3)
    _load().oracle_invariants(nx, ny, _ptr(f), _ptr(out))
    return out


def forward_fields(rho0, ux0, uy0, theta, nu, model, nsteps):
    rho0, ux0, uy0 = _f64(rho0), _f64(ux0), _f64(uy0)
    ny, nx = rho0.shape
    rho, ux, uy = (np.zeros((ny, nx)) for _ in range(3))
    _load().oracle_forward_fields(nx, ny, theta, nu, _model(model), int(nsteps), _ptr(rho0), _ptr(ux0),
                                  _ptr(uy0), _ptr(rho), _ptr(ux), _ptr(uy))
    return rho, ux, uy


def adjoint_step(f, fbar_next, theta, nu, model):
    f, fbar_next = _f64(f), _f64(fbar_next)
    _, ny, nx = f.shape
    out = np.zeros_like(f)
    _load().oracle_adjoint_step(nx, ny, theta, nu, _model(model), _ptr(f), _ptr(fbar_next), _ptr(out))
    return out


def gradient(rho0, ux0, uy0, rho_bar, ux_bar, uy_bar, theta, nu, model, nsteps):
    """(dJ/dux0, dJ/duy0) for J depending on the moments after nsteps steps."""
    args = [_f64(a) for a in (rho0, ux0, uy0, rho_bar, ux_bar, uy_bar)]
    ny, nx = args[0].shape
    gx, gy = np.zeros((ny, nx)), np.zeros((ny, nx))
    _load().oracle_gradient(nx, ny, theta, nu, _model(model), int(nsteps), *[_ptr(a) for a in args],
                            _ptr(gx), _ptr(gy))
    return gx, gy
