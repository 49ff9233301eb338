"""Pins of the oracle's second-order variant (``oracle/second_order.py``:
MUSCL reconstruction with the minmod limiter, a cell term for the bed
slope, Heun's method).  None of them re-types the module's formulas:
  * the limiter and the face values against hand values;
  * on a flat bed with A_g = 0 and uniform (h, u), the transverse velocity
    is a passive scalar carried by the contact wave, so the scheme must
    equal, step for step, the textbook MUSCL-minmod scheme for linear
    advection with Heun's method (written here with the sign/min form of
    minmod), along x and along y;
  * that scalar converges at second order to the exact translated
    profile, the first-order scheme at first order;
  * the coupled system converges at second order to a fine-grid run;
  * conservation of sum h and sum z_b on periodic grids;
  * a lake at rest stays at rest, for both interface problems, several
    closures, periodic and free boundaries;
  * with every slope zero (alternating data) the rate is the first-order
    scheme's update divided by dt;
  * a y-uniform 2D run equals the 1D run; transpose and mirror symmetry;
  * the first-order scheme is more diffusive (the paper's motivation);
  * Oracle1D / Oracle2D with order 2 take exactly these
    steps, with FP32 storage rounding after each step.
The mutation tests plant plausible slips in a copy of the module and check
that one of these pins fails.
"""
import os
import sys
import types

import numpy as np
import pytest

import oracle as O
import oracle.second_order as S2
import workloads as W

G = 9.81


# ----------------------------------------------------------------------------
# helpers: runs that use a given module's step functions
# ----------------------------------------------------------------------------
def run1d(M, U, p, bcs, dx, nsteps=None, cfl=0.5, t_end=None, dt=None, Ag=None):
    t, n = 0.0, 0
    while True:
        if nsteps is not None and n >= nsteps:
            break
        if t_end is not None and t >= t_end:
            break
        if dt is None:
            U, _, t = M.heun_step_1d(U, p, bcs, dx, Ag, n, cfl=cfl, t=t, t_end=t_end)
        else:
            U, _, t = M.heun_step_1d(U, p, bcs, dx, Ag, n, dt=dt, t=t)
        n += 1
    return U, t, n


def run2d(M, U, p, bcs, dx, dy, nsteps=None, cfl=0.5, t_end=None, dt=None, Ag=None):
    t, n = 0.0, 0
    while True:
        if nsteps is not None and n >= nsteps:
            break
        if t_end is not None and t >= t_end:
            break
        if dt is None:
            U, _, t = M.heun_step_2d(U, p, bcs, dx, dy, Ag, n, cfl=cfl, t=t, t_end=t_end)
        else:
            U, _, t = M.heun_step_2d(U, p, bcs, dx, dy, Ag, n, dt=dt, t=t)
        n += 1
    return U, t, n


def textbook_minmod(a, b):
    return 0.5 * (np.sign(a) + np.sign(b)) * np.minimum(np.abs(a), np.abs(b))


def textbook_advection(q, c, dt, dx, nsteps):
    """MUSCL (minmod) upwind scheme for q_t + c q_x = 0, c > 0, periodic,
    with Heun's method."""
    def rate(q):
        s = textbook_minmod(np.roll(q, -1) - q, q - np.roll(q, 1))
        qe = q + 0.5 * s
        return -(c / dx) * (qe - np.roll(qe, 1))
    for _ in range(nsteps):
        q1 = q + dt * rate(q)
        q2 = q1 + dt * rate(q1)
        q = 0.5 * (q + q2)
    return q


def per():
    return [O.BC(O.BC_PERIODIC)] * 4


def free():
    return [O.BC(O.BC_FREE)] * 4


# ----------------------------------------------------------------------------
# pins (each takes the module under test)
# ----------------------------------------------------------------------------
def pin_minmod_and_faces(M):
    a = np.array([1.0, -1.0, 1.0, 0.0, 2.0, -3.0])
    b = np.array([2.0, -3.0, -1.0, 5.0, 0.5, -0.25])
    assert np.array_equal(M.minmod(a, b), [1.0, -1.0, 0.0, 0.0, 0.5, -0.25])
    # padded q = [0, 1, 3, 4, 4, 2]: cells 1..4 have slopes
    # minmod(2, 1) = 1, minmod(1, 2) = 1, minmod(0, 1) = 0, minmod(-2, 0) = 0
    lo, hi = M.faces(np.array([0.0, 1.0, 3.0, 4.0, 4.0, 2.0]))
    assert np.array_equal(lo, [0.5, 2.5, 4.0, 4.0])
    assert np.array_equal(hi, [1.5, 3.5, 4.0, 4.0])


def transverse_case(nx, axis):
    """Uniform depth and normal velocity on a flat bed, A_g = 0, with a
    transverse velocity profile along `axis` (1: varies with x, carried by
    u; 0: varies with y, carried by v)."""
    L = 800.0
    dx = L / nx
    x = (np.arange(nx) + 0.5) * dx
    prof = 0.2 * (np.abs(x - 300.0) < 100.0) + 0.1 * np.sin(2 * np.pi * x / L)
    h = np.full((3, nx), 2.0)
    hu = h * 1.5
    hv = h * prof[None, :]
    z = np.zeros_like(h)
    if axis == 0:
        h, hu, hv, z = h.T.copy(), hv.T.copy(), hu.T.copy(), z.T.copy()
    return (h, hu, hv, z), prof, dx


def pin_textbook_advection(M):
    p = O.Params(order=2, A_g=0.0)
    for axis in (1, 0):
        U, prof, dx = transverse_case(80, axis)
        dt = 0.5 * dx / (1.5 + np.sqrt(G * 2.0))
        K = 30
        (h, hu, hv, z), _, _ = run2d(M, U, p, per(), dx, dx, nsteps=K, dt=dt)
        q = textbook_advection(prof, 1.5, dt, dx, K)
        if axis == 1:
            assert np.max(np.abs(h - 2.0)) == 0.0 and np.max(np.abs(hu - 3.0)) == 0.0
            assert np.max(np.abs(hv / h - q[None, :])) < 1e-14
        else:
            assert np.max(np.abs(h - 2.0)) == 0.0 and np.max(np.abs(hv - 3.0)) == 0.0
            assert np.max(np.abs(hu / h - q[:, None])) < 1e-14


def advection_error(M, nx, order, T=100.0):
    p = O.Params(order=order, A_g=0.0)
    L = 1000.0
    dx = L / nx
    x = (np.arange(nx) + 0.5) * dx
    h = np.ones((1, nx))
    U = (h, 2.0 * h, 0.3 * np.sin(2 * np.pi * x / L)[None, :], np.zeros_like(h))
    if order == 2:
        (h, hu, hv, z), t, _ = run2d(M, U, p, per(), dx, dx, cfl=0.4, t_end=T)
    else:
        o = O.Oracle2D(*U, dx, dx, p, per())
        o.step(10 ** 6, 0.4, t_end=T)
        h, hv, t = o.h, o.hv, o.t
    assert t == T
    exact = 0.3 * np.sin(2 * np.pi * (x - 2.0 * T) / L)
    return np.mean(np.abs(hv[0] / h[0] - exact))


def pin_advection_order(M):
    e = [advection_error(M, n, 2) for n in (50, 100, 200)]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(rates) > 1.7, rates


def dune1d(nx, amp=0.5):
    L = 1000.0
    dx = L / nx
    x = (np.arange(nx) + 0.5) * dx
    zb = amp + amp * np.sin(2 * np.pi * x / L)
    return (5.0 - zb, np.full(nx, 5.0), zb), dx


def pin_self_convergence(M):
    p = O.Params(order=2, A_g=1e-3)
    ref = run1d(M, dune1d(1600)[0], p, per()[:2], dune1d(1600)[1], t_end=20.0)[0]
    errs = []
    for n in (100, 200, 400):
        U0, dx = dune1d(n)
        st = run1d(M, U0, p, per()[:2], dx, t_end=20.0)[0]
        f = 1600 // n
        errs.append(sum(np.mean(np.abs(a - b.reshape(n, f).mean(1))) for a, b in zip(st, ref)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, rates


def bump2d(nx, ny):
    lx, ly = 400.0, 300.0
    x = W.cell_centres(nx, lx)[None, :]
    y = W.cell_centres(ny, ly)[:, None]
    zb = 0.4 * np.exp(-((x - 150.0) ** 2 + (y - 160.0) ** 2) / 2000.0) * np.ones((ny, 1))
    h = 3.0 - zb
    hu = np.full((ny, nx), 2.0) + 0.3 * np.sin(2 * np.pi * y / ly)
    hv = 0.4 * np.cos(2 * np.pi * x / lx) * np.ones((ny, 1))
    return (h, hu, hv, zb), lx / nx, ly / ny


LAWS = {
    "grass3": dict(law=O.LAW_GRASS, A_g=0.05, m_g=3.0),
    "grass2.2": dict(law=O.LAW_GRASS, A_g=0.05, m_g=2.2),
    "mpm": dict(law=O.LAW_MPM, friction=O.FRIC_STRICKLER, fric_coef=40.0),
}


def pin_conservation(M):
    for rec in (0, 1):
        for law in ("grass3", "mpm"):
            p = O.Params(order=2, reconstruction=rec, **LAWS[law])
            U, dx, dy = bump2d(40, 30)
            (h, hu, hv, z), _, _ = run2d(M, U, p, per(), dx, dy, nsteps=15)
            assert abs(h.sum() - U[0].sum()) < 1e-12 * U[0].sum()
            assert abs(z.sum() - U[3].sum()) < 1e-12 * U[0].sum()
            assert np.max(np.abs(z - U[3])) > 1e-6          # the bed moved


def pin_lake_at_rest(M):
    nx, ny = 36, 28
    x = W.cell_centres(nx, 360.0)[None, :]
    y = W.cell_centres(ny, 280.0)[:, None]
    zb = 0.5 * np.exp(-((x - 170.0) ** 2 + (y - 130.0) ** 2) / 1500.0) + 0.1 * np.sin(
        2 * np.pi * x / 360.0) * np.cos(2 * np.pi * y / 280.0)
    # the paper's interface problem keeps the lake for m_g >= 3 and MPM
    # only (for 1 < m_g < 3 round-off velocities seed a sediment celerity
    # far above the floor, as in the first-order scheme); the hydrostatic
    # reconstruction keeps it for every closure
    for rec, laws in ((0, ("grass3", "mpm")), (1, tuple(LAWS))):
        for law in laws:
            p = O.Params(order=2, reconstruction=rec, **LAWS[law])
            for bcs in (per(), free()):
                U = (2.0 - zb, np.zeros_like(zb), np.zeros_like(zb), zb.copy())
                (h, hu, hv, z), _, _ = run2d(M, U, p, bcs, 10.0, 7.0, nsteps=40)
                assert np.max(np.abs(hu)) < 1e-13 and np.max(np.abs(hv)) < 1e-13
                assert np.max(np.abs(h + z - 2.0)) < 1e-13
                assert np.max(np.abs(z - zb)) < 1e-13


def pin_zero_slopes_first_order(M):
    nx = 40
    i = np.arange(nx)
    sgn = (-1.0) ** i
    h = 2.0 + 0.1 * sgn
    zb = 0.3 + 0.05 * sgn                 # eta = 2.3 + 0.15 (-1)^i
    hu = h * (1.0 + 0.2 * sgn)            # u alternates
    for rec in (0, 1):
        p = O.Params(order=2, reconstruction=rec, A_g=0.01)
        (Dh, Dhu, Dz), _ = M.rates_1d(h, hu, zb, p, per()[:2], 2.0)
        p1 = O.Params(order=1, reconstruction=rec, A_g=0.01)
        o = O.Oracle1D(h, hu, zb, 2.0, p1, per()[:2])
        dt = 0.01
        o.step_fixed_dt(1, dt)
        for D, a, b in ((Dh, h, o.h), (Dhu, hu, o.hu), (Dz, zb, o.z)):
            first = (a - b) / dt
            assert np.max(np.abs(D - first)) < 1e-9 * max(1.0, np.max(np.abs(first)))
            assert np.max(np.abs(first)) > 1e-4


def pin_y_uniform_equals_1d(M):
    for rec in (0, 1):
        p = O.Params(order=2, reconstruction=rec, A_g=0.01)
        (h, hu, z), dx = dune1d(60, amp=0.3)
        U2 = tuple(np.tile(a, (5, 1)) for a in (h, hu, np.zeros_like(h), z))
        bcs = [O.BC(O.BC_INFLOW, 4.8, 5.0, 0.0), O.BC(O.BC_FREE)] + [O.BC(O.BC_PERIODIC)] * 2
        (h2, hu2, hv2, z2), t2, _ = run2d(M, U2, p, bcs, dx, 7.0, nsteps=25, cfl=0.3)
        (h1, hu1, z1), t1, _ = run1d(M, (h, hu, z), p, bcs[:2], dx, nsteps=25, cfl=0.3)
        assert np.max(np.abs(hv2)) == 0.0
        # dt differs: the 2D rule adds S_y/dy (S_y > 0 from the y-interfaces)
        assert t2 < t1


def pin_y_uniform_fixed_dt(M):
    for rec in (0, 1):
        p = O.Params(order=2, reconstruction=rec, A_g=0.01)
        (h, hu, z), dx = dune1d(60, amp=0.3)
        U2 = tuple(np.tile(a, (5, 1)) for a in (h, hu, np.zeros_like(h), z))
        bcs = [O.BC(O.BC_INFLOW, 4.8, 5.0, 0.0), O.BC(O.BC_FREE)] + [O.BC(O.BC_PERIODIC)] * 2
        (h2, hu2, hv2, z2), _, _ = run2d(M, U2, p, bcs, dx, 7.0, nsteps=25, dt=0.3)
        (h1, hu1, z1), _, _ = run1d(M, (h, hu, z), p, bcs[:2], dx, nsteps=25, dt=0.3)
        for a, b in ((h2, h1), (hu2, hu1), (z2, z1)):
            assert np.max(np.abs(a - b[None, :])) < 1e-13
        assert np.max(np.abs(hv2)) == 0.0


def pin_transpose(M):
    for rec in (0, 1):
        p = O.Params(order=2, reconstruction=rec, A_g=0.02, m_g=2.5)
        (h, hu, hv, z), _, _ = bump2d(30, 24)
        U = (h, hu, hv, z)
        UT = (h.T.copy(), hv.T.copy(), hu.T.copy(), z.T.copy())
        bcs = [O.BC(O.BC_INFLOW, 3.0, 2.0, 0.1), O.BC(O.BC_FREE),
               O.BC(O.BC_PERIODIC), O.BC(O.BC_PERIODIC)]
        bcsT = [O.BC(O.BC_PERIODIC), O.BC(O.BC_PERIODIC),
                O.BC(O.BC_INFLOW, 3.0, 0.1, 2.0), O.BC(O.BC_FREE)]
        (a, b, c, d), t, _ = run2d(M, U, p, bcs, 10.0, 10.0, nsteps=12)
        (aT, bT, cT, dT), tT, _ = run2d(M, UT, p, bcsT, 10.0, 10.0, nsteps=12)
        assert t == pytest.approx(tT, rel=1e-14)
        for x, y in ((a, aT), (b, cT), (c, bT), (d, dT)):
            assert np.max(np.abs(x - y.T)) < 1e-12 * max(1.0, np.max(np.abs(x)))


def pin_mirror(M):
    for rec in (0, 1):
        p = O.Params(order=2, reconstruction=rec, A_g=0.02)
        (h, hu, hv, z), _, _ = bump2d(32, 20)
        U = (h, hu, hv, z)
        UM = (h[:, ::-1].copy(), -hu[:, ::-1], hv[:, ::-1].copy(), z[:, ::-1].copy())
        (a, b, c, d), t, _ = run2d(M, U, p, free(), 10.0, 12.0, nsteps=12)
        (aM, bM, cM, dM), tM, _ = run2d(M, UM, p, free(), 10.0, 12.0, nsteps=12)
        assert t == pytest.approx(tM, rel=1e-14)
        for x, y, s in ((a, aM, 1), (b, bM, -1), (c, cM, 1), (d, dM, 1)):
            assert np.max(np.abs(x - s * y[:, ::-1])) < 1e-12 * max(1.0, np.max(np.abs(x)))


PINS = [pin_minmod_and_faces, pin_textbook_advection, pin_advection_order,
        pin_self_convergence, pin_conservation, pin_lake_at_rest,
        pin_zero_slopes_first_order, pin_y_uniform_equals_1d, pin_y_uniform_fixed_dt,
        pin_transpose, pin_mirror]


@pytest.mark.parametrize("pin", PINS, ids=[f.__name__ for f in PINS])
def test_pin(pin):
    pin(S2)


def test_first_order_converges_at_first_order():
    e = [advection_error(S2, n, 1) for n in (50, 100, 200)]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert max(rates) < 1.1, rates
    assert advection_error(S2, 200, 2) < 0.1 * e[2]


def test_less_diffusive_than_first_order():
    """The bump of a 1D dune keeps more of its height after 300 s with the
    second-order variant, and stays closer to a fine first-order run."""
    def crest(n, order, T=300.0):
        (h, hu, z), dx = dune1d(n, amp=0.5)
        o = O.Oracle1D(h, hu, z, dx, O.Params(order=order, A_g=1e-3), per()[:2])
        o.step(10 ** 6, 0.5, t_end=T)
        return o.z
    ref = crest(1600, 1).reshape(200, 8).mean(1)
    z1, z2 = crest(200, 1), crest(200, 2)
    assert np.max(z2) > np.max(z1)
    assert np.mean(np.abs(z2 - ref)) < 0.5 * np.mean(np.abs(z1 - ref))


def test_oracle_classes_take_these_steps():
    """Oracle2D / Oracle1D with order 2 give the same states and times as the
    step functions; FP32 storage rounds after every step."""
    p = O.Params(order=2, reconstruction=1, A_g=0.02, momentum_friction=1,
                 friction=O.FRIC_MANNING, fric_coef=0.03)
    U, dx, dy = bump2d(20, 14)
    bcs = [O.BC(O.BC_INFLOW, 3.0, 2.0, 0.1), O.BC(O.BC_FREE), O.BC(O.BC_FREE),
           O.BC(O.BC_FREE)]
    o = O.Oracle2D(*U, dx, dy, p, bcs)
    o.step(6, 0.45, t_end=3.0)
    Ur, t, n = run2d(S2, U, p, bcs, dx, dy, nsteps=6, cfl=0.45, t_end=3.0)
    assert o.t == t and o.nsteps == 6
    for a, b in zip(o.state, Ur):
        assert np.array_equal(a, b)
    o32 = O.Oracle2D(*U, dx, dy, p, bcs, storage="fp32")
    o32.step_fixed_dt(3, 0.2)
    V = tuple(a.astype(np.float32).astype(np.float64) for a in U)
    for k in range(3):
        V, _, _ = S2.heun_step_2d(V, p, bcs, dx, dy, None, k, dt=0.2)
        V = tuple(a.astype(np.float32).astype(np.float64) for a in V)
    for a, b in zip(o32.state, V):
        assert np.array_equal(a, b)
    (h, hu, z), dx1 = dune1d(50)
    o1 = O.Oracle1D(h, hu, z, dx1, p, bcs[:2])
    o1.step(5, 0.5)
    Ur, t, n = run1d(S2, (h, hu, z), p, bcs[:2], dx1, nsteps=5)
    assert o1.t == t
    for a, b in zip(o1.state, Ur):
        assert np.array_equal(a, b)
    assert o1.cfl_dt(0.5) == pytest.approx(o1.dt_last, rel=0.5)


def test_dry_first_stage_is_reported():
    """A face depth that reaches zero in the reconstruction of the well-
    balanced interface problem, or a depth that the first stage drives
    negative, raises the oracle's error at that step."""
    h = np.array([1.0, 1.0, 1e-3, 1.0, 1.0, 1.0])
    hu = np.array([0.0, 5.0, 0.0, -5.0, 0.0, 0.0])
    z = np.zeros(6)
    o = O.Oracle1D(h, hu, z, 1.0, O.Params(order=2, A_g=0.0), [O.BC(O.BC_FREE)] * 2)
    with pytest.raises(O.OracleError) as e:
        o.step_fixed_dt(1, 0.2)
    assert e.value.step == 0


# ----------------------------------------------------------------------------
# planted slips
# ----------------------------------------------------------------------------
SRC = open(S2.__file__).read()

MUTATIONS = [
    # the cell term dropped
    ("Dhu = (((X.FhuL[:, 1:] - X.FhuR[:, :-1]) + cx) / dx",
     "Dhu = (((X.FhuL[:, 1:] - X.FhuR[:, :-1]) + 0.0 * cx) / dx"),
    # the cell term with the wrong sign
    ("return g * (0.5 * (lo[\"h\"] + hi[\"h\"])) * (hi[\"z\"] - lo[\"z\"])",
     "return g * (0.5 * (lo[\"h\"] + hi[\"h\"])) * (lo[\"z\"] - hi[\"z\"])"),
    # the y cell term applied with the x spacing
    ("+ ((Y.FhuL[1:, :] - Y.FhuR[:-1, :]) + cy) / dy)",
     "+ (Y.FhuL[1:, :] - Y.FhuR[:-1, :]) / dy + cy / dx)"),
    # the bed reconstructed instead of the free surface
    ("eta=Pd[\"h\"] + Pd[\"z\"])", "eta=Pd[\"z\"])"),
    # faces meeting at an interface taken from the wrong side
    ("X = _interface({k: v[:, :-1] for k, v in hi.items()},\n"
     "                   {k: v[:, 1:] for k, v in lo.items()},",
     "X = _interface({k: v[:, :-1] for k, v in lo.items()},\n"
     "                   {k: v[:, 1:] for k, v in hi.items()},"),
    ("Y = _interface({k: v[:-1, :] for k, v in hi.items()},\n"
     "                   {k: v[1:, :] for k, v in lo.items()},",
     "Y = _interface({k: v[:-1, :] for k, v in lo.items()},\n"
     "                   {k: v[1:, :] for k, v in hi.items()},"),
    # no limiter (centred slope)
    ("s = minmod(q[..., 2:] - q[..., 1:-1], q[..., 1:-1] - q[..., :-2])",
     "s = 0.5 * (q[..., 2:] - q[..., :-2])"),
    # minmod keeping the larger difference
    ("np.where(np.abs(a) < np.abs(b), a, b)", "np.where(np.abs(a) < np.abs(b), b, a)"),
    # Heun's average replaced by the second Euler stage
    ("Un = tuple(0.5 * (a + b) for a, b in zip(U, U2))\n    _check_state(step, *Un)\n"
     "    return Un, dt, (t + dt if t_new is None else t_new)\n\n\ndef heun_step_1d",
     "Un = U2\n    _check_state(step, *Un)\n"
     "    return Un, dt, (t + dt if t_new is None else t_new)\n\n\ndef heun_step_1d"),
    # the second stage started from U^n
    ("D1, X1, Y1 = rates_2d(*U1, p, bcs, dx, dy, Ag)",
     "D1, X1, Y1 = rates_2d(*U, p, bcs, dx, dy, Ag)"),
    # one ghost layer of a periodic side taken from the wrong end
    ("glo = a[..., np.arange(-2, 0) % n]", "glo = a[..., np.arange(0, 2) % n]"),
    # hydrostatic corrections with the reconstructed depth of the other side
    ("res.FhuR = res.FhuR + 0.5 * p.g * (R[\"h\"] * R[\"h\"] - hRs * hRs)",
     "res.FhuR = res.FhuR + 0.5 * p.g * (R[\"h\"] * R[\"h\"] - hLs * hLs)"),
    # the face depth of the high face
    ("return q[..., 1:-1] - 0.5 * s, q[..., 1:-1] + 0.5 * s",
     "return q[..., 1:-1] - 0.5 * s, q[..., 1:-1] + 0.25 * s"),
]


def load_variant(old, new):
    assert SRC.count(old) == 1, old
    name = "oracle.second_order_mutant"
    mod = types.ModuleType(name)
    mod.__package__ = "oracle"
    sys.modules[name] = mod
    try:
        exec(compile(SRC.replace(old, new), "second_order_mutant.py", "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


@pytest.mark.parametrize("k", range(len(MUTATIONS)))
def test_mutation_is_caught(k):
    M = load_variant(*MUTATIONS[k])
    caught = []
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(M)
        except (AssertionError, O.OracleError, FloatingPointError, ValueError):
            caught.append(pin.__name__)
    assert caught, "mutation %d passed every pin" % k
