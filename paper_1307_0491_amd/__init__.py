"""MI355X-native relaxation solver for the Saint-Venant--Exner system.

The HIP library ``libsve.so`` (C ABI: include/sve.h) holds every step of the
method; this package is its Python binding.  Nothing here falls back to a
CPU implementation: using the solver without the built library, or without
a HIP device, raises.
"""
from . import _lib
from ._lib import (LAW_GRASS, LAW_MPM, LAW_FLVB, LAW_NIELSEN, LAW_RIBBERINK,
                   LAW_CAMENEN, FRIC_STRICKLER, FRIC_MANNING, FRIC_DARCY,
                   BC_PERIODIC, BC_FREE, BC_INFLOW, FP64, FP32, PATH_FUSED,
                   PATH_SPLIT, PATH_RESIDENT, PATH_RESIDUAL, SveError)
from .solver import Params, BC, Solver, current_stream_handle


def require_device():
    """Load the library and check that a HIP device is present."""
    _lib.load()
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible: the solver runs on the GPU only")
    return True


__all__ = [
    "LAW_GRASS", "LAW_MPM", "LAW_FLVB", "LAW_NIELSEN", "LAW_RIBBERINK",
    "LAW_CAMENEN", "FRIC_STRICKLER", "FRIC_MANNING", "FRIC_DARCY",
    "BC_PERIODIC", "BC_FREE", "BC_INFLOW", "FP64", "FP32", "PATH_FUSED",
    "PATH_SPLIT", "PATH_RESIDENT", "PATH_RESIDUAL", "SveError", "Params", "BC", "Solver",
    "current_stream_handle", "require_device",
]
