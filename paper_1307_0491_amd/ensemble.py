"""Python binding of the batched ensemble (include/sve_ensemble.h).
Argument marshalling only: every step runs in the HIP library."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import check
from .solver import Params

ENS_QUEUE = 0
ENS_GRID = 1


class Ensemble:
    """Independent periodic 2D Grass runs advanced together.

    members: sequence of dicts with keys h, hu, hv, zb ((ny, nx) arrays),
    lx, ly, A_g, m_g."""

    def __init__(self, members, params: Params | None = None, stream=None):
        self.lib = _lib.load()
        params = params or Params()
        arr = (_lib.SveMember * len(members))()
        self._keep = []
        self.shapes = []
        for i, m in enumerate(members):
            fields = [np.ascontiguousarray(m[k], dtype=np.float64) for k in ("h", "hu", "hv", "zb")]
            self._keep.append(fields)
            ny, nx = fields[0].shape
            self.shapes.append((ny, nx))
            arr[i] = _lib.SveMember(nx, ny, float(m["lx"]), float(m["ly"]), float(m["A_g"]),
                                    float(m["m_g"]), *[f.ctypes.data for f in fields])
        h = ctypes.c_void_p()
        check(self.lib.sve_ens_create(ctypes.byref(h), len(members), arr,
                                      ctypes.byref(params.to_c()), stream), "sve_ens_create")
        self._keep = []
        self._h = h
        self.n = len(members)

    def step(self, nsteps: int, cfl: float = 0.5):
        check(self.lib.sve_ens_step(self._h, int(nsteps), float(cfl)), "sve_ens_step")

    def step_sequential(self, nsteps: int, cfl: float = 0.5):
        check(self.lib.sve_ens_step_sequential(self._h, int(nsteps), float(cfl)),
              "sve_ens_step_sequential")

    def get(self, m: int):
        ny, nx = self.shapes[m]
        outs = [np.empty((ny, nx)) for _ in range(4)]
        t, ns = ctypes.c_double(), ctypes.c_longlong()
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        check(self.lib.sve_ens_get(self._h, int(m), p(outs[0]), p(outs[1]), p(outs[2]),
                                   p(outs[3]), ctypes.byref(t), ctypes.byref(ns)), "sve_ens_get")
        return tuple(outs), t.value, ns.value

    def autotune(self, nprobe: int = 5, cfl: float = 0.5):
        rows, mode = ctypes.c_int(), ctypes.c_int()
        check(self.lib.sve_ens_autotune(self._h, int(nprobe), float(cfl), ctypes.byref(rows),
                                        ctypes.byref(mode)), "sve_ens_autotune")
        return rows.value, mode.value

    def set_schedule(self, rows: int, mode: int):
        check(self.lib.sve_ens_set_schedule(self._h, int(rows), int(mode)), "sve_ens_set_schedule")

    def last_elapsed_ms(self) -> float:
        ms = ctypes.c_double()
        check(self.lib.sve_ens_last_elapsed_ms(self._h, ctypes.byref(ms)), "sve_ens_last_elapsed_ms")
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            self.lib.sve_ens_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
