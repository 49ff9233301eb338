"""Python binding of the solver's C ABI (include/sve.h).

Argument marshalling only: the state lives in device memory owned by the
library, every step runs in its HIP kernels, and torch provides the device
memory of tensor arguments and the HIP stream the library launches on.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from . import _lib
from ._lib import check


@dataclasses.dataclass
class Params:
    """Model parameters (sve_params)."""
    law: int = _lib.LAW_GRASS
    g: float = 9.81
    A_g: float = 1e-3
    m_g: float = 3.0
    friction: int = _lib.FRIC_STRICKLER
    fric_coef: float = 40.0
    d_s: float = 1e-3
    s: float = 2.65
    tau_cr: float = 0.05
    momentum_friction: int = 0
    reconstruction: int = 0
    order: int = 1

    def to_c(self) -> _lib.SveParams:
        return _lib.SveParams(self.law, self.g, self.A_g, self.m_g, self.friction,
                              self.fric_coef, self.d_s, self.s, self.tau_cr,
                              self.momentum_friction, self.reconstruction,
                              self.order)


@dataclasses.dataclass
class BC:
    """Boundary condition of one side (sve_bc)."""
    kind: int = _lib.BC_PERIODIC
    h: float = 0.0
    hu: float = 0.0
    hv: float = 0.0


def _bcs_to_c(bcs):
    arr = (_lib.SveBC * 4)()
    for s in range(4):
        b = bcs[s] if s < len(bcs) else BC()
        arr[s] = _lib.SveBC(b.kind, b.h, b.hu, b.hv)
    return arr


def _torch():
    import torch
    return torch


def current_stream_handle():
    """HIP stream of torch's current stream on the current device."""
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _host_ptr(a):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(t):
    if t is None:
        return None, None
    torch = _torch()
    tt = t.to(dtype=torch.float64).contiguous()
    return tt, ctypes.c_void_p(tt.data_ptr())


class Solver:
    """One solver context: state (h, hu, [hv,] z_b) on an nx x ny grid.

    Arrays are (ny, nx) for 2D and (nx,) for 1D (hv omitted).  Inputs may be
    numpy arrays (copied from host memory) or torch HIP tensors (copied on
    the device, on torch's current stream)."""

    def __init__(self, h, hu, zb, hv=None, *, lx: float, ly: float = 1.0,
                 params: Params | None = None, bcs=None, Ag=None,
                 storage: str = "fp64", stream=None):
        lib = _lib.load()
        params = params or Params()
        self.dim = 1 if hv is None else 2
        shape = tuple(np.shape(h))
        if self.dim == 1:
            if len(shape) != 1:
                raise ValueError("1D state must be a 1-D array")
            self.nx, self.ny = shape[0], 1
        else:
            if len(shape) != 2:
                raise ValueError("2D state must be (ny, nx)")
            self.ny, self.nx = shape
        for a in (hu, zb, hv, Ag):
            if a is not None and tuple(np.shape(a)) != shape:
                raise ValueError("all fields must have the same shape")
        self.shape = shape
        self.storage = storage
        bcs = bcs if bcs is not None else [BC()] * 4
        self._keep = []
        is_dev = not isinstance(h, np.ndarray) and hasattr(h, "is_cuda") and h.is_cuda
        if stream is None and is_dev:
            stream = current_stream_handle()
        self.stream = stream
        conv = _dev_ptr if is_dev else _host_ptr
        ptrs = []
        for a in (h, hu, hv, zb, Ag):
            keep, p = conv(a)
            self._keep.append(keep)
            ptrs.append(p)
        ctx = ctypes.c_void_p()
        fn = lib.sve_init_state_dev if is_dev else lib.sve_init_state
        code = fn(ctypes.byref(ctx), self.nx, self.ny, float(lx), float(ly), ptrs[0], ptrs[1],
                  ptrs[2], ptrs[3], ptrs[4], ctypes.byref(params.to_c()), _bcs_to_c(bcs),
                  _lib.FP32 if storage == "fp32" else _lib.FP64, stream)
        check(code, "sve_init_state")
        self._ctx = ctx
        self._keep = []
        self.lib = lib

    # -- stepping ---------------------------------------------------------
    def step(self, n: int, cfl: float = 0.5, t_end: float = 0.0) -> float:
        t = ctypes.c_double()
        check(self.lib.sve_step(self._ctx, int(n), float(cfl), float(t_end), ctypes.byref(t)),
              "sve_step")
        return t.value

    def step_fixed_dt(self, n: int, dt: float):
        check(self.lib.sve_step_fixed_dt(self._ctx, int(n), float(dt)), "sve_step_fixed_dt")

    def set_path(self, path: int):
        check(self.lib.sve_set_path(self._ctx, int(path)), "sve_set_path")

    def set_tile_rows(self, rows: int):
        check(self.lib.sve_set_tile_rows(self._ctx, int(rows)), "sve_set_tile_rows")

    def last_elapsed_ms(self) -> float:
        ms = ctypes.c_double()
        check(self.lib.sve_last_elapsed_ms(self._ctx, ctypes.byref(ms)), "sve_last_elapsed_ms")
        return ms.value

    def poke(self, field: int, k: int, value: float):
        check(self.lib.sve_debug_poke(self._ctx, int(field), int(k), float(value)),
              "sve_debug_poke")

    # -- state --------------------------------------------------------------
    def get_state(self):
        """(fields, t, dt_last, nsteps) with fields = (h, hu, [hv,] z_b) as
        float64 numpy arrays."""
        outs = [np.empty(self.shape) for _ in range(4)]
        t, dtl, ns = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        hv = ptr(outs[2]) if self.dim == 2 else None
        check(self.lib.sve_get_state(self._ctx, ptr(outs[0]), ptr(outs[1]), hv, ptr(outs[3]),
                                     ctypes.byref(t), ctypes.byref(dtl), ctypes.byref(ns)),
              "sve_get_state")
        fields = (outs[0], outs[1], outs[3]) if self.dim == 1 else tuple(outs)
        return fields, t.value, dtl.value, ns.value

    def times(self):
        """(t, dt_last, nsteps) without copying the state."""
        t, dtl, ns = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
        check(self.lib.sve_get_state(self._ctx, None, None, None, None, ctypes.byref(t),
                                     ctypes.byref(dtl), ctypes.byref(ns)), "sve_get_state")
        return t.value, dtl.value, ns.value

    def get_state_torch(self, device="cuda"):
        """Same as get_state with float64 torch tensors on the device."""
        torch = _torch()
        outs = [torch.empty(self.shape, dtype=torch.float64, device=device) for _ in range(4)]
        t, dtl, ns = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
        p = lambda x: ctypes.c_void_p(x.data_ptr())
        hv = p(outs[2]) if self.dim == 2 else None
        check(self.lib.sve_get_state_dev(self._ctx, p(outs[0]), p(outs[1]), hv, p(outs[3]),
                                         ctypes.byref(t), ctypes.byref(dtl), ctypes.byref(ns)),
              "sve_get_state_dev")
        fields = (outs[0], outs[1], outs[3]) if self.dim == 1 else tuple(outs)
        return fields, t.value, dtl.value, ns.value

    @property
    def handle(self):
        return self._ctx

    def close(self):
        if getattr(self, "_ctx", None):
            self.lib.sve_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
