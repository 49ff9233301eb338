"""ctypes loader of the HIP library ``libsve.so`` and mirrors of its C
structs (declarations in include/sve.h).  Argument marshalling only: every
step of the solver runs in the library's kernels."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the library built in the package directory, unless SVE_LIBRARY names another build
LIB_PATH = os.environ.get("SVE_LIBRARY") or os.path.join(HERE, "libsve.so")

# error codes
SVE_OK = 0
SVE_ERR_ARG = -1
SVE_ERR_HIP = -2
SVE_ERR_POSITIVITY = -3
SVE_ERR_ORDER = -4
SVE_ERR_NONFINITE = -5
SVE_ERR_STATE = -6

LAW_GRASS, LAW_MPM, LAW_FLVB, LAW_NIELSEN, LAW_RIBBERINK, LAW_CAMENEN = range(6)
FRIC_STRICKLER, FRIC_MANNING, FRIC_DARCY = range(3)
BC_PERIODIC, BC_FREE, BC_INFLOW = range(3)
FP64, FP32 = 0, 1
PATH_FUSED, PATH_SPLIT, PATH_RESIDENT, PATH_RESIDUAL = 0, 1, 2, 3


class SveParams(ctypes.Structure):
    _fields_ = [("law", ctypes.c_int), ("g", ctypes.c_double), ("A_g", ctypes.c_double),
                ("m_g", ctypes.c_double), ("friction", ctypes.c_int),
                ("fric_coef", ctypes.c_double), ("d_s", ctypes.c_double),
                ("s", ctypes.c_double), ("tau_cr", ctypes.c_double),
                ("momentum_friction", ctypes.c_int), ("reconstruction", ctypes.c_int),
                ("order", ctypes.c_int)]


class SveBC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("h", ctypes.c_double), ("hu", ctypes.c_double),
                ("hv", ctypes.c_double)]


class SveMember(ctypes.Structure):
    """Ensemble member description (include/sve_ensemble.h)."""
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("Lx", ctypes.c_double),
                ("Ly", ctypes.c_double), ("A_g", ctypes.c_double), ("m_g", ctypes.c_double),
                ("h", ctypes.c_void_p), ("hu", ctypes.c_void_p), ("hv", ctypes.c_void_p),
                ("zb", ctypes.c_void_p)]


class SveError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = _LIB.sve_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})")


_LIB = None
_LOAD_ERROR = None

P = ctypes.c_void_p
D = ctypes.c_double
I = ctypes.c_int
LL = ctypes.c_longlong
DP = ctypes.POINTER(ctypes.c_double)

SIGNATURES = {
    "sve_init_state": (I, [ctypes.POINTER(P), I, I, D, D, P, P, P, P, P,
                           ctypes.POINTER(SveParams), ctypes.POINTER(SveBC), I, P]),
    "sve_init_state_dev": (I, [ctypes.POINTER(P), I, I, D, D, P, P, P, P, P,
                               ctypes.POINTER(SveParams), ctypes.POINTER(SveBC), I, P]),
    "sve_step": (I, [P, I, D, D, DP]),
    "sve_step_fixed_dt": (I, [P, I, D]),
    "sve_get_state": (I, [P, P, P, P, P, DP, DP, ctypes.POINTER(LL)]),
    "sve_get_state_dev": (I, [P, P, P, P, P, DP, DP, ctypes.POINTER(LL)]),
    "sve_destroy": (I, [P]),
    "sve_strerror": (ctypes.c_char_p, [I]),
    "sve_set_path": (I, [P, I]),
    "sve_set_tile_rows": (I, [P, I]),
    "sve_debug_poke": (I, [P, I, LL, D]),
    "sve_last_elapsed_ms": (I, [P, DP]),
    "sve_step_dev_noalloc": (I, [I, I, D, D, ctypes.POINTER(SveParams), ctypes.POINTER(SveBC),
                                 P, P, P, P, P, P, P, P, I, D, D, DP, DP, P]),
    "sve_adj_forward": (I, [P, I, D, I]),
    "sve_adj_backward": (I, [P, P, P, P]),
    "sve_adj_step_vjp": (I, [P, D, P, P, P]),
    "sve_adj_set_tile_rows": (I, [P, I]),
    "sve_ens_create": (I, [ctypes.POINTER(P), I, ctypes.POINTER(SveMember),
                           ctypes.POINTER(SveParams), P]),
    "sve_ens_step": (I, [P, I, D]),
    "sve_ens_step_sequential": (I, [P, I, D]),
    "sve_ens_get": (I, [P, I, P, P, P, P, DP, ctypes.POINTER(LL)]),
    "sve_ens_autotune": (I, [P, I, D, ctypes.POINTER(I), ctypes.POINTER(I)]),
    "sve_ens_set_schedule": (I, [P, I, I]),
    "sve_ens_last_elapsed_ms": (I, [P, DP]),
    "sve_ens_destroy": (I, [P]),
}


def load(path: str = LIB_PATH):
    """Load the library once; raise if it is not built."""
    global _LIB, _LOAD_ERROR
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        _LOAD_ERROR = f"HIP library not built: {path} (run __graft_entry__.build())"
        raise RuntimeError(_LOAD_ERROR)
    # torch brings its own HIP runtime (same soname as the system one): load
    # it first so that the library binds to that single runtime instance and
    # device pointers and streams from torch are valid in the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def exported_symbols():
    return list(SIGNATURES)


def check(code: int, what: str):
    if code != SVE_OK:
        raise SveError(code, what)
