"""Finite-volume time step of the oracle (1D and 2D structured grids).

Test infrastructure only (see the package docstring).

One explicit step (section "Numerical method": auxiliaries from the state
at t^n, one homogeneous Riemann problem per interface, cell mean of the
Riemann solutions; 2D by the method of lines on a structured mesh, section
"Parallelization", with one ghost cell because the scheme is first order):
  1. ghost ring: periodic wrap, FREE (zero-gradient copy of the adjacent
     cell) or INFLOW (Dirichlet h, hu, hv; bed copied from the adjacent
     cell);
  2. lambda = 0 projection and closure in every cell (ghosts included);
  3. relaxation Riemann problem at every x- and y-interface
     (``oracle.riemann``), normal/transverse roles swapped for y;
  4. time step (the paper prints no CFL rule; reading used here):
     dt = CFL / (S_x/dx + S_y/dy), S = largest max(|sigma1|, |sigma5|) over
     the interfaces of that direction (1D: dt = CFL dx / S_x), clipped so
     that t does not pass t_end;
  5. conservative cell update, left-to-right in the order written below,
     with the non-conservative momentum fluctuations F^L / F^R;
  6. optional semi-implicit momentum friction (off by default; the paper's
     system has no friction source in the momentum equation).
Relaxation variables are never stored: they are projected again from the
state at the start of every step.

Well-balanced variant (Params.reconstruction = 1).  The paper notes that
the scheme is not well balanced (a lake at rest over a varying bed does not
stay at rest) and names well balancing as future work, citing among others
the hydrostatic reconstruction of Audusse, Bouchut, Bristeau, Klein and
Perthame (2004).  That method, applied with the relaxation solver above as
the interface solver:
  * at each interface, z* = max(z_L, z_R) and the reconstructed depths
    h_L* = max(0, h_L + z_L - z*), h_R* = max(0, h_R + z_R - z*), the
    velocities kept: U_L* = (h_L*, h_L* u_L, h_L* v_L), likewise U_R*;
  * each reconstructed state is projected (closure at h*, U) and the
    relaxation Riemann problem is solved between them with the bed z* on
    both sides (the bed step is carried by the reconstruction; the sediment
    waves still move the bed through Omega);
  * the momentum fluxes seen by the two cells get the hydrostatic
    corrections g/2 (h_L^2 - h_L*^2) (left cell) and g/2 (h_R^2 - h_R*^2)
    (right cell); the mass, transverse-momentum and bed fluxes are those
    of the reconstructed problem.
A lake at rest (u = v = 0, h + z_b constant) gives equal reconstructed
states at every interface, hence constant Riemann solutions, zero mass and
bed fluxes and momentum fluxes g h^2/2 that cancel in each cell: it is kept
for every bedload law and exponent.  On a flat bed the variant is the
scheme itself.

Second-order variant (Params.order = 2): ``oracle.second_order`` (MUSCL
reconstruction with the minmod limiter, a cell term for the bed slope,
Heun's method); Oracle1D and Oracle2D hand their steps to it.

Storage "fp32" emulates float32 state storage with float64 arithmetic: the
state is rounded to float32 at initialisation and after every step.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .closures import Params, closure, friction_factor
from .riemann import (CellState, interface_solve, project, ERR_NONFINITE,
                      ERR_POSITIVITY, _max, _re)

BC_PERIODIC = 0
BC_FREE = 1
BC_INFLOW = 2


@dataclasses.dataclass
class BC:
    kind: int = BC_PERIODIC
    h: float = 0.0
    hu: float = 0.0
    hv: float = 0.0


class OracleError(RuntimeError):
    def __init__(self, code: int, step: int, where: str = ""):
        super().__init__(f"oracle step {step}: error mask {code} {where}")
        self.code = code
        self.step = step


# ----------------------------------------------------------------------------
# Ghost cells
# ----------------------------------------------------------------------------
def _ghost_1d(a, lo: BC, hi: BC, field: str):
    """Pad a 1D array (last axis) with one ghost cell on each side."""
    first = a[..., :1]
    last = a[..., -1:]
    if lo.kind == BC_PERIODIC:
        glo = last
    elif lo.kind == BC_FREE or field in ("z", "Ag"):
        glo = first
    else:
        glo = np.full_like(first, getattr(lo, field))
    if hi.kind == BC_PERIODIC:
        ghi = first
    elif hi.kind == BC_FREE or field in ("z", "Ag"):
        ghi = last
    else:
        ghi = np.full_like(last, getattr(hi, field))
    return np.concatenate([glo, a, ghi], axis=-1)


def pad2d(fields: dict, bcs) -> dict:
    """Ghost ring for (ny, nx) arrays.  bcs = (west, east, south, north).
    Corner ghosts are not used by the five-point stencil; they hold copies
    that keep the projection finite."""
    west, east, south, north = bcs
    out = {}
    for name, a in fields.items():
        ax = _ghost_1d(a, west, east, name)                 # (ny, nx+2)
        ay = _ghost_1d(ax.T, south, north, name).T          # (ny+2, nx+2)
        out[name] = ay
    return out


def pad1d(fields: dict, bcs) -> dict:
    west, east = bcs
    return {name: _ghost_1d(a, west, east, name) for name, a in fields.items()}


# ----------------------------------------------------------------------------
# Step helpers
# ----------------------------------------------------------------------------
def _cells(P: dict, normal: str, sl):
    """CellState of the slice `sl` of the projected padded arrays, with the
    interface normal along x ('x') or y ('y')."""
    if normal == "x":
        return CellState(P["h"][sl], P["tau"][sl], P["u"][sl], P["v"][sl],
                         P["Pi"][sl], P["z"][sl], P["qx"][sl], P["bx2"][sl],
                         P["aK"][sl])
    return CellState(P["h"][sl], P["tau"][sl], P["v"][sl], P["u"][sl],
                     P["Pi"][sl], P["z"][sl], P["qy"][sl], P["by2"][sl],
                     P["aK"][sl])


def _project_padded(Pd: dict, p: Params):
    h, hu, hv, z = Pd["h"], Pd["hu"], Pd["hv"], Pd["z"]
    tau = 1.0 / h
    u = hu * tau
    v = hv * tau
    qx, qy, bx, by = closure(h, u, v, p, Pd.get("Ag"))
    return project(h, hu, hv, z, qx, qy, bx, by, p.g)


def _reconstructed_sides(Pd: dict, p: Params, normal: str, slL, slR):
    """Hydrostatic reconstruction between the padded cells slL (left) and
    slR (right): the projected reconstructed states and the depths needed
    by the momentum corrections."""
    hL, zL = Pd["h"][slL], Pd["z"][slL]
    hR, zR = Pd["h"][slR], Pd["z"][slR]
    zs = _max(zL, zR)
    hLs = _max(hL + zL - zs, 0.0 * hL)
    hRs = _max(hR + zR - zs, 0.0 * hR)
    out = []
    for sl, hs in ((slL, hLs), (slR, hRs)):
        u = Pd["hu"][sl] / Pd["h"][sl]
        v = Pd["hv"][sl] / Pd["h"][sl]
        fields = dict(h=hs, hu=hs * u, hv=hs * v, z=zs)
        if "Ag" in Pd:
            fields["Ag"] = Pd["Ag"][sl]
        P = _project_padded(fields, p)
        out.append(_cells(P, normal, Ellipsis))
    return out[0], out[1], hL, hLs, hR, hRs


def _reconstructed_solve(Pd: dict, p: Params, normal: str, slL, slR):
    """Interface results of the well-balanced variant: the relaxation
    Riemann problem between the reconstructed states, with the hydrostatic
    corrections added to the momentum fluxes of the two cells."""
    L, R, hL, hLs, hR, hRs = _reconstructed_sides(Pd, p, normal, slL, slR)
    res = interface_solve(L, R, p.g)
    res.FhuL = res.FhuL + 0.5 * p.g * (hL * hL - hLs * hLs)
    res.FhuR = res.FhuR + 0.5 * p.g * (hR * hR - hRs * hRs)
    return res


def fluxes_2d(h, hu, hv, z, p: Params, bcs, Ag=None):
    """All x-interface results (ny, nx+1) and y-interface results (ny+1, nx).
    x-interface m of row j lies between cells m-1 and m; y-interface m of
    column i lies between rows m-1 and m."""
    fields = dict(h=h, hu=hu, hv=hv, z=z)
    if Ag is not None:
        fields["Ag"] = Ag
    Pd = pad2d(fields, bcs)
    ny, nx = h.shape
    if p.reconstruction:
        X = _reconstructed_solve(Pd, p, "x", (slice(1, ny + 1), slice(0, nx + 1)),
                                 (slice(1, ny + 1), slice(1, nx + 2)))
        Y = _reconstructed_solve(Pd, p, "y", (slice(0, ny + 1), slice(1, nx + 1)),
                                 (slice(1, ny + 2), slice(1, nx + 1)))
        return X, Y
    P = _project_padded(Pd, p)
    Lx = _cells(P, "x", (slice(1, ny + 1), slice(0, nx + 1)))
    Rx = _cells(P, "x", (slice(1, ny + 1), slice(1, nx + 2)))
    Ly = _cells(P, "y", (slice(0, ny + 1), slice(1, nx + 1)))
    Ry = _cells(P, "y", (slice(1, ny + 2), slice(1, nx + 1)))
    return interface_solve(Lx, Rx, p.g), interface_solve(Ly, Ry, p.g)


def fluxes_1d(h, hu, z, p: Params, bcs, Ag=None):
    """All interface results (nx+1); interface m lies between cells m-1, m."""
    fields = dict(h=h, hu=hu, hv=np.zeros_like(h), z=z)
    if Ag is not None:
        fields["Ag"] = Ag
    Pd = pad1d(fields, bcs)
    nx = h.shape[0]
    if p.reconstruction:
        return _reconstructed_solve(Pd, p, "x", slice(0, nx + 1), slice(1, nx + 2))
    P = _project_padded(Pd, p)
    L = _cells(P, "x", slice(0, nx + 1))
    R = _cells(P, "x", slice(1, nx + 2))
    return interface_solve(L, R, p.g)


def dt_from_speeds(Sx, Sy, dx, dy, cfl):
    """CFL time step (reading: sum of directional rates in 2D)."""
    if Sy is None:
        return cfl * dx / Sx
    return cfl / (Sx / dx + Sy / dy)


def update_2d(h, hu, hv, z, X, Y, dt, dx, dy):
    lx = dt / dx
    ly = dt / dy
    hn = h - lx * (X.Fh[:, 1:] - X.Fh[:, :-1]) - ly * (Y.Fh[1:, :] - Y.Fh[:-1, :])
    hun = (hu - lx * (X.FhuL[:, 1:] - X.FhuR[:, :-1])
           - ly * (Y.Fht[1:, :] - Y.Fht[:-1, :]))
    hvn = (hv - lx * (X.Fht[:, 1:] - X.Fht[:, :-1])
           - ly * (Y.FhuL[1:, :] - Y.FhuR[:-1, :]))
    zn = z - lx * (X.Fz[:, 1:] - X.Fz[:, :-1]) - ly * (Y.Fz[1:, :] - Y.Fz[:-1, :])
    return hn, hun, hvn, zn


def update_1d(h, hu, z, X, dt, dx):
    lx = dt / dx
    hn = h - lx * (X.Fh[1:] - X.Fh[:-1])
    hun = hu - lx * (X.FhuL[1:] - X.FhuR[:-1])
    zn = z - lx * (X.Fz[1:] - X.Fz[:-1])
    return hn, hun, zn


def momentum_friction(hn, hun, hvn, dt, p: Params):
    """Semi-implicit (hu, hv) / (1 + dt phi(h, |U|)) with phi from the
    friction slope (optional source, off unless p.momentum_friction)."""
    un = hun / hn
    vn = hvn / hn
    speed = np.sqrt(un * un + vn * vn)
    phi = friction_factor(hn, speed, p)
    den = 1.0 + dt * phi
    return hun / den, hvn / den


def _check(err_mask, step):
    if np.any(err_mask):
        raise OracleError(int(np.bitwise_or.reduce(np.ravel(err_mask))), step)


def _check_state(step, *arrays):
    for a in arrays:
        if not np.all(np.isfinite(a)):
            raise OracleError(ERR_NONFINITE, step, "non-finite state")
    if np.any(_re(arrays[0]) <= 0.0):
        raise OracleError(ERR_POSITIVITY, step, "h <= 0 after update")


def _round32(*arrays):
    return tuple(a.astype(np.float32).astype(np.float64) for a in arrays)


# ----------------------------------------------------------------------------
# Time-stepping classes
# ----------------------------------------------------------------------------
class Oracle2D:
    """2D state (h, hu, hv, z_b) on an nx x ny grid over [0,Lx] x [0,Ly]."""

    def __init__(self, h, hu, hv, zb, dx, dy, params: Params, bcs,
                 Ag=None, storage: str = "fp64"):
        self.p = params
        self.bcs = tuple(bcs)
        self.dx = float(dx)
        self.dy = float(dy)
        self.storage = storage
        self.Ag = None if Ag is None else np.asarray(Ag, dtype=np.float64)
        st = tuple(np.array(a, dtype=np.float64) for a in (h, hu, hv, zb))
        if storage == "fp32":
            st = _round32(*st)
        self.h, self.hu, self.hv, self.z = st
        self.t = 0.0
        self.nsteps = 0
        self.dt_last = 0.0

    @property
    def state(self):
        return self.h, self.hu, self.hv, self.z

    def fluxes(self):
        return fluxes_2d(self.h, self.hu, self.hv, self.z, self.p, self.bcs,
                         self.Ag)

    def cfl_dt(self, cfl: float) -> float:
        if self.p.order == 2:
            from .second_order import rates_2d
            _, X, Y = rates_2d(*self.state, self.p, self.bcs, self.dx, self.dy,
                               self.Ag)
        else:
            X, Y = self.fluxes()
        return float(dt_from_speeds(np.max(X.speed), np.max(Y.speed),
                                    self.dx, self.dy, cfl))

    def _heun(self, cfl=None, dt=None, t_end=None):
        from .second_order import heun_step_2d
        Un, dt, t_new = heun_step_2d(self.state, self.p, self.bcs, self.dx,
                                     self.dy, self.Ag, self.nsteps, cfl=cfl,
                                     dt=dt, t=self.t, t_end=t_end)
        if self.storage == "fp32":
            Un = _round32(*Un)
        self.h, self.hu, self.hv, self.z = Un
        self.nsteps += 1
        self.dt_last = dt
        self.t = t_new

    def _advance(self, dt: float, X, Y):
        _check(X.err, self.nsteps)
        _check(Y.err, self.nsteps)
        hn, hun, hvn, zn = update_2d(self.h, self.hu, self.hv, self.z, X, Y,
                                     dt, self.dx, self.dy)
        if self.p.momentum_friction:
            hun, hvn = momentum_friction(hn, hun, hvn, dt, self.p)
        _check_state(self.nsteps, hn, hun, hvn, zn)
        if self.storage == "fp32":
            hn, hun, hvn, zn = _round32(hn, hun, hvn, zn)
        self.h, self.hu, self.hv, self.z = hn, hun, hvn, zn
        self.nsteps += 1
        self.dt_last = dt

    def step(self, n: int, cfl: float, t_end: float | None = None):
        """n CFL steps; with t_end, dt is clipped to reach t_end exactly and
        the remaining steps leave the state unchanged."""
        for i in range(n):
            if t_end is not None and t_end > 0.0 and self.t >= t_end:
                self.nsteps += n - i          # remaining steps are no-ops
                self.dt_last = 0.0
                break
            if self.p.order == 2:
                self._heun(cfl=cfl, t_end=t_end)
                continue
            X, Y = self.fluxes()
            dt = float(dt_from_speeds(np.max(X.speed), np.max(Y.speed),
                                      self.dx, self.dy, cfl))
            t_new = self.t + dt
            if t_end is not None and t_end > 0.0:
                if dt >= t_end - self.t:
                    dt = t_end - self.t
                    t_new = t_end
            self._advance(dt, X, Y)
            self.t = t_new
        return self.t

    def step_fixed_dt(self, n: int, dt: float):
        for _ in range(n):
            if self.p.order == 2:
                self._heun(dt=dt)
                continue
            X, Y = self.fluxes()
            self._advance(dt, X, Y)
            self.t = self.t + dt
        return self.t


class Oracle1D:
    """1D state (h, hu, z_b) on nx cells over [0, L]; bcs = (west, east)."""

    def __init__(self, h, hu, zb, dx, params: Params, bcs, Ag=None,
                 storage: str = "fp64"):
        self.p = params
        self.bcs = tuple(bcs)
        self.dx = float(dx)
        self.storage = storage
        self.Ag = None if Ag is None else np.asarray(Ag, dtype=np.float64)
        st = tuple(np.array(a, dtype=np.float64) for a in (h, hu, zb))
        if storage == "fp32":
            st = _round32(*st)
        self.h, self.hu, self.z = st
        self.t = 0.0
        self.nsteps = 0
        self.dt_last = 0.0

    @property
    def state(self):
        return self.h, self.hu, self.z

    def fluxes(self):
        return fluxes_1d(self.h, self.hu, self.z, self.p, self.bcs, self.Ag)

    def cfl_dt(self, cfl: float) -> float:
        if self.p.order == 2:
            from .second_order import rates_1d
            _, X = rates_1d(*self.state, self.p, self.bcs, self.dx, self.Ag)
        else:
            X = self.fluxes()
        return float(dt_from_speeds(np.max(X.speed), None, self.dx, None, cfl))

    def _heun(self, cfl=None, dt=None, t_end=None):
        from .second_order import heun_step_1d
        Un, dt, t_new = heun_step_1d(self.state, self.p, self.bcs, self.dx,
                                     self.Ag, self.nsteps, cfl=cfl, dt=dt,
                                     t=self.t, t_end=t_end)
        if self.storage == "fp32":
            Un = _round32(*Un)
        self.h, self.hu, self.z = Un
        self.nsteps += 1
        self.dt_last = dt
        self.t = t_new

    def _advance(self, dt: float, X):
        _check(X.err, self.nsteps)
        hn, hun, zn = update_1d(self.h, self.hu, self.z, X, dt, self.dx)
        if self.p.momentum_friction:
            hun, _ = momentum_friction(hn, hun, np.zeros_like(hn), dt, self.p)
        _check_state(self.nsteps, hn, hun, zn)
        if self.storage == "fp32":
            hn, hun, zn = _round32(hn, hun, zn)
        self.h, self.hu, self.z = hn, hun, zn
        self.nsteps += 1
        self.dt_last = dt

    def step(self, n: int, cfl: float, t_end: float | None = None):
        for i in range(n):
            if t_end is not None and t_end > 0.0 and self.t >= t_end:
                self.nsteps += n - i          # remaining steps are no-ops
                self.dt_last = 0.0
                break
            if self.p.order == 2:
                self._heun(cfl=cfl, t_end=t_end)
                continue
            X = self.fluxes()
            dt = float(dt_from_speeds(np.max(X.speed), None, self.dx, None, cfl))
            t_new = self.t + dt
            if t_end is not None and t_end > 0.0:
                if dt >= t_end - self.t:
                    dt = t_end - self.t
                    t_new = t_end
            self._advance(dt, X)
            self.t = t_new
        return self.t

    def step_fixed_dt(self, n: int, dt: float):
        for _ in range(n):
            if self.p.order == 2:
                self._heun(dt=dt)
                continue
            self._advance(dt, self.fluxes())
            self.t = self.t + dt
        return self.t


# ----------------------------------------------------------------------------
# Pure functions (used for complex-step tangents)
# ----------------------------------------------------------------------------
def step2d_arrays(h, hu, hv, z, dt, dx, dy, p: Params, bcs, Ag=None):
    """One fixed-dt 2D step on arrays (float64 or complex128)."""
    X, Y = fluxes_2d(h, hu, hv, z, p, bcs, Ag)
    hn, hun, hvn, zn = update_2d(h, hu, hv, z, X, Y, dt, dx, dy)
    if p.momentum_friction:
        hun, hvn = momentum_friction(hn, hun, hvn, dt, p)
    return hn, hun, hvn, zn


def step1d_arrays(h, hu, z, dt, dx, p: Params, bcs, Ag=None):
    X = fluxes_1d(h, hu, z, p, bcs, Ag)
    hn, hun, zn = update_1d(h, hu, z, X, dt, dx)
    if p.momentum_friction:
        hun, _ = momentum_friction(hn, hun, np.zeros_like(hn), dt, p)
    return hn, hun, zn
