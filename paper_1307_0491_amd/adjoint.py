"""Python binding of the discrete adjoint (include/sve_adjoint.h) and a
torch.autograd.Function giving gradients of a function of the final bed
with respect to the initial bed and the per-cell Grass constant.

Argument marshalling only: the forward steps, the checkpoints, their
recomputation and the reverse steps all run in the HIP library."""
from __future__ import annotations

import ctypes

from ._lib import check
from .solver import Solver, current_stream_handle


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def state_tensor(fields):
    """Stack (h, hu, hv, z_b) (each (ny, nx)) into one contiguous float64
    state array of 4*ny*nx values."""
    import torch
    return torch.stack([f.to(torch.float64) for f in fields]).contiguous()


class AdjointRun:
    """Fixed-dt forward run with checkpoints on an existing Solver, then
    reverse sweeps.  Device tensors are float64 on the solver's device."""

    def __init__(self, solver: Solver):
        if solver.dim != 2:
            raise ValueError("the adjoint supports 2D grids")
        self.s = solver
        self.lib = solver.lib

    def forward(self, nsteps: int, dt: float, every: int = 0):
        check(self.lib.sve_adj_forward(self.s.handle, int(nsteps), float(dt), int(every)),
              "sve_adj_forward")

    def backward(self, gT, want_ag: bool = True):
        """gT: (4, ny, nx) float64 device tensor dL/dU(T).  Returns
        (g0 (4, ny, nx), gAg (ny, nx) or None)."""
        import torch
        gT = gT.to(torch.float64).contiguous()
        g0 = torch.empty_like(gT)
        gAg = torch.empty(gT.shape[1:], dtype=torch.float64, device=gT.device) if want_ag else None
        check(self.lib.sve_adj_backward(self.s.handle, _ptr(gT), _ptr(g0),
                                        _ptr(gAg) if gAg is not None else None),
              "sve_adj_backward")
        return g0, gAg

    def set_tile_rows(self, rows: int):
        """Tile height of the reverse-step kernel (8, 16, 32 or 64)."""
        check(self.lib.sve_adj_set_tile_rows(self.s.handle, int(rows)), "sve_adj_set_tile_rows")

    def step_vjp(self, dt: float, lam):
        """One reverse step at the solver's current state."""
        import torch
        lam = lam.to(torch.float64).contiguous()
        out = torch.empty_like(lam)
        gAg = torch.empty(lam.shape[1:], dtype=torch.float64, device=lam.device)
        check(self.lib.sve_adj_step_vjp(self.s.handle, float(dt), _ptr(lam), _ptr(out),
                                        _ptr(gAg)), "sve_adj_step_vjp")
        return out, gAg


def final_bed(zb0, Ag, h0, hu0, hv0, *, lx, ly, params, nsteps, dt, every=0):
    """z_b(T) after `nsteps` fixed-dt steps from (h0, hu0, hv0, zb0) with the
    per-cell Grass constant Ag, differentiable in zb0 and Ag."""
    return _FinalBed.apply(zb0, Ag, h0, hu0, hv0, lx, ly, params, nsteps, dt, every)


def _make_function():
    import torch

    class _FB(torch.autograd.Function):
        @staticmethod
        def forward(ctx, zb0, Ag, h0, hu0, hv0, lx, ly, params, nsteps, dt, every):
            from .solver import BC
            from . import _lib
            bcs = [BC(_lib.BC_PERIODIC)] * 4
            s = Solver(h0.detach(), hu0.detach(), zb0.detach(), hv0.detach(), lx=lx, ly=ly,
                       params=params, bcs=bcs, Ag=Ag.detach(),
                       stream=current_stream_handle())
            run = AdjointRun(s)
            run.forward(nsteps, dt, every)
            fields, _, _, _ = s.get_state_torch(device=zb0.device)
            ctx.run = run
            return fields[3].clone()

        @staticmethod
        def backward(ctx, g_zT):
            gT = torch.zeros((4,) + tuple(g_zT.shape), dtype=torch.float64, device=g_zT.device)
            gT[3] = g_zT
            g0, gAg = ctx.run.backward(gT)
            ctx.run.s.close()
            return g0[3], gAg, None, None, None, None, None, None, None, None, None

    return _FB


class _Lazy:
    _fn = None

    @classmethod
    def apply(cls, *args):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(*args)


_FinalBed = _Lazy
