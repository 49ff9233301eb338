"""Second-order variant of the oracle's scheme (Params.order = 2).

Test infrastructure only (see the package docstring).

The paper finds the first-order relaxation scheme very diffusive, expects
a higher order to cure this, and names high order and well balancing as
the next numerical work (sections "Parallelization" and "Conclusions and
perspectives"); it prints no higher-order scheme.  The reading used here
is the classical second-order extension of a first-order Godunov-type
scheme, in the order the steps are taken:
  1. two ghost layers, each filled by the first-order ghost rule (periodic
     wrap; FREE: copies of the adjacent cell; INFLOW: the Dirichlet
     (h, hu, hv) with the adjacent cell's bed and A_g);
  2. per cell the values h, u = hu/h, v = hv/h and the free surface
     eta = h + z_b; along each direction a slope per cell, the minmod of
     the two one-sided differences (zero unless both have the same sign,
     else the one of smaller magnitude), and the face values
     q -/+ slope/2 (MUSCL reconstruction, van Leer); at a face the state
     (h_f, h_f u_f, h_f v_f, eta_f - h_f).  Reconstructing eta rather
     than z_b keeps a lake at rest flat at the faces;
  3. at each interface the first-order interface problem between the two
     face states that meet there: the relaxation Riemann problem of the
     projected face states, or, with Params.reconstruction = 1, its
     hydrostatic reconstruction (z* = max(z_L, z_R), h* = max(0, h + z -
     z*), face velocities kept, corrections g/2 (h_f^2 - h*^2) on the
     momentum fluxes the two cells see);
  4. inside each cell the bed varies from z_W to z_E, and the
     non-conservative product g h dz/dx over the cell is taken on a
     straight path with h frozen at the mean of the cell's two face
     depths, as at an interface: the cell term
     g (h_W + h_E)/2 (z_E - z_W), added to the normal momentum's flux
     difference (the centred source term of Audusse, Bouchut, Bristeau,
     Klein and Perthame, 2004);
  5. the rate of each field, D = (flux difference [+ cell term]) / dx
     + (...) / dy;
  6. Heun's method, the two-stage strong-stability-preserving Runge-Kutta
     scheme written with the Euler stage S(U) = U - dt D(U) (followed by
     the optional semi-implicit momentum friction):
     U1 = S(U^n), U2 = S(U1), U^{n+1} = (U^n + U2) / 2.
     dt comes from the outer wave speeds of the first stage's interface
     problems (those of the state U^n), with the first-order rule.
A lake at rest has zero eta slopes, equal face states at every interface
(zero mass and bed fluxes, momentum fluxes g h_f^2/2) and a cell term that
cancels the face pressures' difference exactly: it stays at rest for both
interface problems.  With every slope zero (each cell a local extremum of
every reconstructed field) the rate is the first-order scheme's.
"""
from __future__ import annotations

import numpy as np

from .closures import Params
from .riemann import interface_solve, _max
from .scheme import (BC_PERIODIC, BC_FREE, _cells, _project_padded,
                     momentum_friction, dt_from_speeds, _check, _check_state)


def minmod(a, b):
    """Zero where a and b differ in sign or one is zero, else the one of
    smaller magnitude."""
    return np.where(a * b > 0.0, np.where(np.abs(a) < np.abs(b), a, b), 0.0)


def _pad2(a, lo, hi, field: str):
    """Two ghost layers on each side of the last axis."""
    n = a.shape[-1]
    if lo.kind == BC_PERIODIC:
        glo = a[..., np.arange(-2, 0) % n]
    elif lo.kind == BC_FREE or field in ("z", "Ag"):
        glo = a[..., [0, 0]]
    else:
        glo = np.full(a.shape[:-1] + (2,), getattr(lo, field), dtype=a.dtype)
    if hi.kind == BC_PERIODIC:
        ghi = a[..., np.arange(n, n + 2) % n]
    elif hi.kind == BC_FREE or field in ("z", "Ag"):
        ghi = a[..., [n - 1, n - 1]]
    else:
        ghi = np.full(a.shape[:-1] + (2,), getattr(hi, field), dtype=a.dtype)
    return np.concatenate([glo, a, ghi], axis=-1)


def faces(q):
    """Face values along the last axis of a twice-padded array: for the
    cells -1 .. n (every cell but the outer ghosts), the values at their
    low and high faces, q -/+ minmod slope / 2."""
    s = minmod(q[..., 2:] - q[..., 1:-1], q[..., 1:-1] - q[..., :-2])
    return q[..., 1:-1] - 0.5 * s, q[..., 1:-1] + 0.5 * s


def _face_states(prim: dict):
    """Low and high face states along the last axis: dicts of h, u, v, z."""
    lo, hi = {}, {}
    for name in ("h", "u", "v", "eta"):
        lo[name], hi[name] = faces(prim[name])
    for d in (lo, hi):
        d["z"] = d["eta"] - d["h"]
    return lo, hi


def _interface(L: dict, R: dict, agL, agR, p: Params, normal: str):
    """First-order interface problem between face states L and R (dicts of
    h, u, v, z), plain or hydrostatically reconstructed."""
    if p.reconstruction:
        zs = _max(L["z"], R["z"])
        hLs = _max(L["h"] + L["z"] - zs, 0.0 * L["h"])
        hRs = _max(R["h"] + R["z"] - zs, 0.0 * R["h"])
        sides = [(hLs, L, agL, zs), (hRs, R, agR, zs)]
    else:
        sides = [(L["h"], L, agL, L["z"]), (R["h"], R, agR, R["z"])]
    cells = []
    for h, F, ag, z in sides:
        fields = dict(h=h, hu=h * F["u"], hv=h * F["v"], z=z)
        if ag is not None:
            fields["Ag"] = ag
        cells.append(_cells(_project_padded(fields, p), normal, Ellipsis))
    res = interface_solve(cells[0], cells[1], p.g)
    if p.reconstruction:
        res.FhuL = res.FhuL + 0.5 * p.g * (L["h"] * L["h"] - hLs * hLs)
        res.FhuR = res.FhuR + 0.5 * p.g * (R["h"] * R["h"] - hRs * hRs)
    return res


def _primitives(Pd: dict):
    return dict(h=Pd["h"], u=Pd["hu"] / Pd["h"], v=Pd["hv"] / Pd["h"],
                eta=Pd["h"] + Pd["z"])


def _cell_term(lo: dict, hi: dict, g: float):
    """g (h_low + h_high)/2 (z_high - z_low) of each cell."""
    return g * (0.5 * (lo["h"] + hi["h"])) * (hi["z"] - lo["z"])


def rates_2d(h, hu, hv, z, p: Params, bcs, dx, dy, Ag=None):
    """Rates (Dh, Dhu, Dhv, Dz) of the (ny, nx) state, the x- and y-interface
    results (ny, nx+1) and (ny+1, nx)."""
    west, east, south, north = bcs
    fields = dict(h=h, hu=hu, hv=hv, z=z)
    if Ag is not None:
        fields["Ag"] = Ag
    Pd = {}
    for name, a in fields.items():
        ax = _pad2(a, west, east, name)                   # (ny, nx+4)
        Pd[name] = _pad2(ax.T, south, north, name).T      # (ny+4, nx+4)
    ny, nx = h.shape
    prim = _primitives(Pd)
    ag = Pd.get("Ag")
    # x: rows of the grid, faces of the cells -1 .. nx
    lo, hi = _face_states({k: v[2:-2, :] for k, v in prim.items()})
    agx = None if ag is None else ag[2:-2, 1:-1]
    X = _interface({k: v[:, :-1] for k, v in hi.items()},
                   {k: v[:, 1:] for k, v in lo.items()},
                   None if agx is None else agx[:, :-1],
                   None if agx is None else agx[:, 1:], p, "x")
    cx = _cell_term({k: v[:, 1:-1] for k, v in lo.items()},
                    {k: v[:, 1:-1] for k, v in hi.items()}, p.g)
    # y: columns of the grid, faces of the rows -1 .. ny
    loT, hiT = _face_states({k: v[:, 2:-2].T for k, v in prim.items()})
    lo = {k: v.T for k, v in loT.items()}
    hi = {k: v.T for k, v in hiT.items()}
    agy = None if ag is None else ag[1:-1, 2:-2]
    Y = _interface({k: v[:-1, :] for k, v in hi.items()},
                   {k: v[1:, :] for k, v in lo.items()},
                   None if agy is None else agy[:-1, :],
                   None if agy is None else agy[1:, :], p, "y")
    cy = _cell_term({k: v[1:-1, :] for k, v in lo.items()},
                    {k: v[1:-1, :] for k, v in hi.items()}, p.g)
    Dh = (X.Fh[:, 1:] - X.Fh[:, :-1]) / dx + (Y.Fh[1:, :] - Y.Fh[:-1, :]) / dy
    Dhu = (((X.FhuL[:, 1:] - X.FhuR[:, :-1]) + cx) / dx
           + (Y.Fht[1:, :] - Y.Fht[:-1, :]) / dy)
    Dhv = ((X.Fht[:, 1:] - X.Fht[:, :-1]) / dx
           + ((Y.FhuL[1:, :] - Y.FhuR[:-1, :]) + cy) / dy)
    Dz = (X.Fz[:, 1:] - X.Fz[:, :-1]) / dx + (Y.Fz[1:, :] - Y.Fz[:-1, :]) / dy
    return (Dh, Dhu, Dhv, Dz), X, Y


def rates_1d(h, hu, z, p: Params, bcs, dx, Ag=None):
    """Rates (Dh, Dhu, Dz) of the (nx,) state and the interface results."""
    west, east = bcs
    fields = dict(h=h, hu=hu, hv=np.zeros_like(h), z=z)
    if Ag is not None:
        fields["Ag"] = Ag
    Pd = {name: _pad2(a, west, east, name) for name, a in fields.items()}
    prim = _primitives(Pd)
    ag = Pd.get("Ag")
    lo, hi = _face_states(prim)
    agx = None if ag is None else ag[1:-1]
    X = _interface({k: v[:-1] for k, v in hi.items()},
                   {k: v[1:] for k, v in lo.items()},
                   None if agx is None else agx[:-1],
                   None if agx is None else agx[1:], p, "x")
    cx = _cell_term({k: v[1:-1] for k, v in lo.items()},
                    {k: v[1:-1] for k, v in hi.items()}, p.g)
    Dh = (X.Fh[1:] - X.Fh[:-1]) / dx
    Dhu = ((X.FhuL[1:] - X.FhuR[:-1]) + cx) / dx
    Dz = (X.Fz[1:] - X.Fz[:-1]) / dx
    return (Dh, Dhu, Dz), X


def euler_stage(U, D, dt, p: Params):
    """S(U) = U - dt D(U), then the optional momentum friction.  U and D are
    tuples (h, hu, hv, z) or, in 1D, (h, hu, z)."""
    out = [a - dt * d for a, d in zip(U, D)]
    if p.momentum_friction:
        if len(out) == 4:
            out[1], out[2] = momentum_friction(out[0], out[1], out[2], dt, p)
        else:
            out[1], _ = momentum_friction(out[0], out[1], np.zeros_like(out[0]),
                                          dt, p)
    return tuple(out)


def heun_step_2d(U, p: Params, bcs, dx, dy, Ag, step: int, cfl: float = None,
                 dt: float = None, t: float = 0.0, t_end: float = None):
    """One second-order step of the 2D state U = (h, hu, hv, z): with cfl,
    dt from the first stage's wave speeds (clipped to t_end); else the
    given dt.  Returns (U^{n+1}, dt, t^{n+1})."""
    D0, X, Y = rates_2d(*U, p, bcs, dx, dy, Ag)
    t_new = None
    if cfl is not None:
        dt = float(dt_from_speeds(np.max(X.speed), np.max(Y.speed), dx, dy, cfl))
        t_new = t + dt
        if t_end is not None and t_end > 0.0 and dt >= t_end - t:
            dt = t_end - t
            t_new = t_end
    _check(X.err, step)
    _check(Y.err, step)
    U1 = euler_stage(U, D0, dt, p)
    _check_state(step, *U1)
    D1, X1, Y1 = rates_2d(*U1, p, bcs, dx, dy, Ag)
    _check(X1.err, step)
    _check(Y1.err, step)
    U2 = euler_stage(U1, D1, dt, p)
    Un = tuple(0.5 * (a + b) for a, b in zip(U, U2))
    _check_state(step, *Un)
    return Un, dt, (t + dt if t_new is None else t_new)


def heun_step_1d(U, p: Params, bcs, dx, Ag, step: int, cfl: float = None,
                 dt: float = None, t: float = 0.0, t_end: float = None):
    """One second-order step of the 1D state U = (h, hu, z)."""
    D0, X = rates_1d(*U, p, bcs, dx, Ag)
    t_new = None
    if cfl is not None:
        dt = float(dt_from_speeds(np.max(X.speed), None, dx, None, cfl))
        t_new = t + dt
        if t_end is not None and t_end > 0.0 and dt >= t_end - t:
            dt = t_end - t
            t_new = t_end
    _check(X.err, step)
    U1 = euler_stage(U, D0, dt, p)
    _check_state(step, *U1)
    D1, X1 = rates_1d(*U1, p, bcs, dx, Ag)
    _check(X1.err, step)
    U2 = euler_stage(U1, D1, dt, p)
    Un = tuple(0.5 * (a + b) for a, b in zip(U, U2))
    _check_state(step, *Un)
    return Un, dt, (t + dt if t_new is None else t_new)
