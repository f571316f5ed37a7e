"""ctypes declarations of the C ABI in include/lbm_mc.h (argument marshalling
only).  Importing this module loads liblbm_mc.so from this package directory
and raises ImportError if it has not been built: there is no fallback."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_mc.so")

c_int32, c_int64, c_double, c_float = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
P = ctypes.POINTER

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_HIP, ERR_UNSTABLE, ERR_NONFINITE = range(6)
STATUS_NAMES = {0: "OK", 1: "ERR_INVALID", 2: "ERR_UNSUPPORTED", 3: "ERR_HIP",
                4: "ERR_UNSTABLE", 5: "ERR_NONFINITE"}
D2Q9, D3Q19 = 0, 1
PERIODIC, WALL, WALL_EQ = 0, 1, 2


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", c_int32), ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
        ("n_species", c_int32), ("bc", c_int32 * 3),
        ("molar_mass", c_double * 4), ("diff", (c_double * 4) * 4), ("tau1", c_double),
        ("g", c_double * 3), ("n0", c_double), ("forcing", c_int32), ("reserved", c_int32),
        ("wall_velocity", (c_double * 3) * 2),
    ]


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2504_07059_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    sig = {
        "lbm_mc_layout": [P(Params), c_int32, P(c_int64), P(c_int64), P(c_int32), P(c_int64)],
        "lbm_mc_check": [P(Params), c_int32, P(c_double), P(c_double)],
        "lbm_mc_init": [P(Params), c_int32, P(c_double), vp, vp, c_int64, vp, P(vp)],
        "lbm_mc_init_field": [P(Params), c_int32, P(c_double), vp, vp, vp, c_int64, vp, P(vp)],
        "lbm_mc_step": [vp, c_int64],
        "lbm_mc_prepare": [vp, c_int64],
        "lbm_mc_sync": [vp],
        "lbm_mc_moments": [vp, vp, vp, vp, vp, vp, P(c_double), P(c_double)],
        "lbm_mc_state": [vp, P(vp), P(vp), P(c_int64)],
        "lbm_mc_restore": [vp, vp, vp, c_int64],
        "lbm_mc_adjoint_step": [vp, vp, vp, vp, vp],
        "lbm_mc_adjoint_init": [vp, vp, vp],
        "lbm_mc_replay": [vp, vp, c_int64, vp, c_int64],
        "lbm_mc_adjoint_run": [vp, vp, c_int64, c_int64, vp, vp, vp],
        "lbm_mc_profile": [vp, vp, vp],
        "lbm_mc_profile_static": [vp, vp, vp],
        "lbm_mc_profile_vjp": [vp, vp, vp, vp],
        "lbm_mc_set_tuning": [vp, c_int32, c_int32, c_int32, c_int32, c_int32],
        "lbm_mc_get_tuning": [vp, P(c_int32), P(c_int32), P(c_int32), P(c_int32), P(c_int32)],
        "lbm_mc_autotune": [vp, c_int32, P(c_double)],
        "lbm_mc_set_batched_mode": [vp, c_int32],
        "lbm_mc_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_int32
    lib.lbm_mc_last_error.argtypes = []
    lib.lbm_mc_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def check(status):
    if status != OK:
        raise LbmError(status, lib.lbm_mc_last_error().decode())
    return status


lib.lbm_mc_stream_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, c_int64, c_int32,
                                   ctypes.c_void_p]
lib.lbm_mc_stream_copy.restype = c_int32
