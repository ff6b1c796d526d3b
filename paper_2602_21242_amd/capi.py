"""ctypes binding of liblbm.so (include/lbm.h). Argument marshalling only.

Loads the in-tree library built by paper_2602_21242_amd/build.py and fails loudly when it
is missing: there is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_ERR_INVALID_ARGUMENT, LBM_ERR_UNSUPPORTED, LBM_ERR_WORKSPACE_TOO_SMALL = 0, 1, 2, 3
LBM_ERR_HIP, LBM_ERR_NONFINITE, LBM_ERR_STATE = 4, 5, 6
LBM_BGK, LBM_OREG_UC, LBM_OREG_PARTIAL, LBM_OREG_COMPLETE = 0, 1, 2, 3
LBM_F64, LBM_F32, LBM_BF16, LBM_F16 = 0, 1, 2, 3
LBM_AB, LBM_AA = 0, 1

MODELS = {"bgk": LBM_BGK, "uc": LBM_OREG_UC, "partial": LBM_OREG_PARTIAL, "complete": LBM_OREG_COMPLETE}
DTYPES = {"f64": LBM_F64, "f32": LBM_F32, "bf16": LBM_BF16, "f16": LBM_F16}
PATTERNS = {"ab": LBM_AB, "aa": LBM_AA}


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("theta", ctypes.c_double), ("nu", ctypes.c_double), ("rho0", ctypes.c_double),
        ("model", ctypes.c_int32), ("storage", ctypes.c_int32), ("pattern", ctypes.c_int32),
        ("ckpt_stride", ctypes.c_int32), ("record_steps", ctypes.c_int64),
        ("two_step", ctypes.c_int32), ("walls", ctypes.c_int32),
    ]


class LBMError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}: {detail}")


_lib = None
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"liblbm.so not found at {LIB_PATH}; build it with "
                              f"`python -m paper_2602_21242_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int
        L.lbm_workspace_bytes.restype = st
        L.lbm_workspace_bytes.argtypes = [ctypes.POINTER(lbm_params), ctypes.POINTER(ctypes.c_size_t)]
        L.lbm_init.restype = st
        L.lbm_init.argtypes = [ctypes.POINTER(lbm_params), _vp, ctypes.c_size_t, _vp, _vp, _vp, _vp,
                               ctypes.POINTER(_vp)]
        L.lbm_step.restype = st
        L.lbm_step.argtypes = [_vp, ctypes.c_int64]
        L.lbm_moments.restype = st
        L.lbm_moments.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]
        L.lbm_get_populations.restype = st
        L.lbm_get_populations.argtypes = [_vp, ctypes.c_int, _vp]
        L.lbm_set_populations.restype = st
        L.lbm_set_populations.argtypes = [_vp, _vp]
        L.lbm_invariants.restype = st
        L.lbm_invariants.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
        L.lbm_invariants_static.restype = st
        L.lbm_invariants_static.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
        L.lbm_adjoint.restype = st
        L.lbm_adjoint.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
        L.lbm_adjoint_populations.restype = st
        L.lbm_adjoint_populations.argtypes = [_vp, _vp, _vp]
        L.lbm_time.restype = ctypes.c_int64
        L.lbm_time.argtypes = [_vp]
        L.lbm_steps_per_launch.restype = ctypes.c_int32
        L.lbm_steps_per_launch.argtypes = [_vp]
        L.lbm_status_string.restype = ctypes.c_char_p
        L.lbm_status_string.argtypes = [ctypes.c_int]
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_last_error.argtypes = []
        L.lbm_destroy.restype = None
        L.lbm_destroy.argtypes = [_vp]
        _lib = L
    return _lib


def status_string(s):
    return lib().lbm_status_string(int(s)).decode()


def last_error():
    return lib().lbm_last_error().decode()


def check(status, where):
    if status != LBM_OK:
        raise LBMError(status, where, last_error())


def make_params(nx, ny, theta, nu, rho0=1.0, model="complete", storage="f32", pattern="ab",
                record_steps=0, ckpt_stride=0, two_step=0, walls=False):
    return lbm_params(int(nx), int(ny), float(theta), float(nu), float(rho0),
                      MODELS[model] if isinstance(model, str) else int(model),
                      DTYPES[storage] if isinstance(storage, str) else int(storage),
                      PATTERNS[pattern] if isinstance(pattern, str) else int(pattern),
                      int(ckpt_stride), int(record_steps), int(two_step), int(bool(walls)))


# Thin wrappers with the C names (raw status returned; pointers as ints or None).

def lbm_workspace_bytes(params):
    n = ctypes.c_size_t(0)
    s = lib().lbm_workspace_bytes(ctypes.byref(params), ctypes.byref(n))
    return s, n.value


def lbm_init(params, d_workspace, workspace_bytes, stream, d_rho, d_ux, d_uy):
    ctx = _vp()
    s = lib().lbm_init(ctypes.byref(params), d_workspace, workspace_bytes, stream, d_rho, d_ux, d_uy,
                       ctypes.byref(ctx))
    return s, ctx.value


def lbm_step(ctx, n):
    return lib().lbm_step(ctx, int(n))


def lbm_moments(ctx, out_dtype, d_rho, d_ux, d_uy):
    return lib().lbm_moments(ctx, int(out_dtype), d_rho, d_ux, d_uy)


def lbm_get_populations(ctx, out_dtype, d_f):
    return lib().lbm_get_populations(ctx, int(out_dtype), d_f)


def lbm_set_populations(ctx, d_f):
    return lib().lbm_set_populations(ctx, d_f)


def lbm_invariants(ctx):
    out = (ctypes.c_double * 3)()
    s = lib().lbm_invariants(ctx, out)
    return s, tuple(out)


def lbm_invariants_static(ctx):
    out = (ctypes.c_double * 3)()
    s = lib().lbm_invariants_static(ctx, out)
    return s, tuple(out)


def lbm_adjoint(ctx, d_rho_bar, d_ux_bar, d_uy_bar, d_ux0_bar, d_uy0_bar):
    return lib().lbm_adjoint(ctx, d_rho_bar, d_ux_bar, d_uy_bar, d_ux0_bar, d_uy0_bar)


def lbm_adjoint_populations(ctx, d_fbarN, d_fbar0):
    return lib().lbm_adjoint_populations(ctx, d_fbarN, d_fbar0)


def lbm_time(ctx):
    return lib().lbm_time(ctx)


def lbm_steps_per_launch(ctx):
    return lib().lbm_steps_per_launch(ctx)


def lbm_status_string(s):
    return status_string(s)


def lbm_last_error():
    return last_error()


def lbm_destroy(ctx):
    lib().lbm_destroy(ctx)
