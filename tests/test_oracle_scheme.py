"""Pins of the oracle's full time step against properties the paper and the
mathematics fix:
  * conservation of water and sediment volume on periodic domains (flux
    form of eq. "bedload system");
  * lake at rest (u = 0, flat free surface) kept to round-off where the
    celerity reading makes it exact (Grass with m_g >= 3, threshold laws),
    bitwise on a flat bed;
  * no bedload on a flat bed: the scheme is the Suliciu shallow-water scheme
    (remark after eq. "relaxqs"); over a varying bed the relaxation's
    sediment waves still move the bed, by an amount that vanishes with dx;
  * a y-uniform 2D field evolves as the 1D scheme; transposed and mirrored
    data give transposed and mirrored results;
  * first-order grid convergence on a smooth case (one ghost cell, first
    order: section "Parallelization");
  * dunes move downstream at Fr < 1 and antidunes upstream at Fr > 1, at
    the speed of the sediment root of the characteristic polynomial p_A
    (section "Bedload modelling");
  * complex-step tangent of a step against central differences.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle.scheme import step1d_arrays, step2d_arrays

PER2 = (O.BC(), O.BC(), O.BC(), O.BC())
PER1 = (O.BC(), O.BC())


def grass(Ag=1e-3, mg=3.0, **kw):
    return O.Params(law=O.LAW_GRASS, A_g=Ag, m_g=mg, **kw)


def mpm(**kw):
    return O.Params(law=O.LAW_MPM, friction=O.FRIC_STRICKLER, fric_coef=40.0,
                    d_s=1e-3, s=2.65, tau_cr=0.05, **kw)


@pytest.mark.parametrize("params", [grass(), grass(Ag=0.5, mg=1.7), mpm()])
def test_mass_conservation_periodic_2d(params):
    h, hu, hv, zb, dx, dy = W.dune2d(48, 40)
    if params.law == O.LAW_MPM:
        h = 0.5 + 0.0 * h + 0.1 * zb
        hu = 2.0 + 0.3 * zb
        hv = 0.2 * zb
    o = O.Oracle2D(h, hu, hv, zb, dx, dy, params, PER2)
    m0, s0 = h.sum(), zb.sum()
    o.step(300, 0.5)
    assert abs(o.h.sum() - m0) / m0 < 1e-14
    assert abs(o.z.sum() - s0) / s0 < 1e-13
    assert np.max(np.abs(o.z - zb)) > 1e-6   # the bed did move


def test_mass_conservation_periodic_1d():
    h, hu, zb, dx = W.dune1d(500, base=0.1)
    o = O.Oracle1D(h, hu, zb, dx, grass(Ag=0.2), PER1)
    m0, s0 = h.sum(), zb.sum()
    o.step(1000, 0.5)
    assert abs(o.h.sum() - m0) / m0 < 1e-14
    assert abs(o.z.sum() - s0) / s0 < 1e-14


def _lake(nx, ny=None, bump=0.4):
    x = W.cell_centres(nx, 100.0)
    if ny is None:
        z = bump * np.exp(-((x - 50.0) / 10.0) ** 2)
        return 2.0 - z, np.zeros(nx), z, 100.0 / nx
    y = W.cell_centres(ny, 100.0)
    z = bump * np.exp(-((x[None, :] - 50.0) ** 2 + (y[:, None] - 40.0) ** 2) / 150.0)
    return 2.0 - z, np.zeros((ny, nx)), np.zeros((ny, nx)), z, 100.0 / nx, 100.0 / ny


@pytest.mark.parametrize("params", [grass(), grass(mg=4.0), mpm()])
def test_lake_at_rest_preserved_2d(params):
    # exact to round-off where b vanishes at least linearly with |U| at rest
    # (Grass m_g >= 3, threshold laws); for 1 < m_g < 3, b ~ |U|^((m_g-1)/2)
    # amplifies round-off velocities.
    h, hu, hv, z, dx, dy = _lake(40, 32)
    o = O.Oracle2D(h, hu, hv, z, dx, dy, params, PER2)
    o.step(1000, 0.5)
    # round-off accumulates over 1000 steps (about 1e-16 per step)
    assert np.max(np.abs(o.hu)) < 1e-12
    assert np.max(np.abs(o.hv)) < 1e-12
    assert np.max(np.abs(o.h + o.z - 2.0)) < 1e-12
    assert np.max(np.abs(o.z - z)) < 1e-12


def test_lake_at_rest_preserved_1d_free_bc():
    h, hu, z, dx = _lake(200)
    o = O.Oracle1D(h, hu, z, dx, mpm(), (O.BC(O.BC_FREE), O.BC(O.BC_FREE)))
    o.step(1000, 0.5)
    assert np.max(np.abs(o.hu)) < 1e-12
    assert np.max(np.abs(o.h - h)) < 1e-12


def test_flat_lake_at_rest_bitwise():
    h = np.full((16, 20), 1.5)
    z = np.full((16, 20), 0.25)
    o = O.Oracle2D(h, 0 * h, 0 * h, z, 1.0, 1.0, grass(), PER2)
    o.step(50, 0.5)
    assert np.array_equal(o.h, h) and np.array_equal(o.z, z)
    assert np.array_equal(o.hu, 0 * h) and np.array_equal(o.hv, 0 * h)


def test_grass_m1_at_rest_bed_creeps_as_the_paper_warns():
    # beta = A_g > 0 at rest for m_g = 1 gives b > 0 and moving sediment
    # waves: the scheme is not well balanced (section "Parallelization").
    h, hu, z, dx = _lake(100)
    o = O.Oracle1D(h, hu, z, dx, grass(Ag=0.05, mg=1.0), PER1)
    o.step(200, 0.5)
    assert np.max(np.abs(o.hu)) > 1e-6


def _suliciu_sw_step(h, hu, dx, cfl, a_of):
    """Independent textbook Suliciu scheme, periodic 1D, flat bed."""
    g = 9.81
    hl, hr = np.roll(h, 1), h            # interface i-1/2 between i-1 and i
    ql, qr = np.roll(hu, 1), hu
    ul, ur = ql / hl, qr / hr
    pl, pr = 0.5 * g * hl * hl, 0.5 * g * hr * hr
    a = a_of
    us = 0.5 * (ul + ur) - (pr - pl) / (2 * a)
    ps = 0.5 * (pl + pr) - 0.5 * a * (ur - ul)
    tl, tr = 1 / hl + (us - ul) / a, 1 / hr - (us - ur) / a
    s1, s3 = ul - a / hl, ur + a / hr
    tau0 = np.where(s1 >= 0, 1 / hl, np.where(us >= 0, tl, np.where(s3 > 0, tr, 1 / hr)))
    u0 = np.where(s1 >= 0, ul, np.where(s3 > 0, us, ur))
    p0 = np.where(s1 >= 0, pl, np.where(s3 > 0, ps, pr))
    F = u0 / tau0
    M = F * u0 + p0
    S = np.max(np.maximum(np.abs(s1), np.abs(s3)))
    dt = cfl * dx / S
    Fr, Mr = np.roll(F, -1), np.roll(M, -1)
    return h - dt / dx * (Fr - F), hu - dt / dx * (Mr - M)


def test_no_bedload_flat_bed_is_suliciu_scheme():
    nx = 200
    x = W.cell_centres(nx, 200.0)
    h = 1.0 + 0.5 * np.exp(-((x - 80) / 15) ** 2)
    hu = 0.3 * np.sin(2 * np.pi * x / 200.0)
    z = np.zeros(nx)
    p = grass(Ag=0.0)
    o = O.Oracle1D(h, hu, z, 1.0, p, PER1)
    hs, qs = h.copy(), hu.copy()
    for _ in range(100):
        X = o.fluxes()
        a_periodic = X.a[:-1]             # interfaces -1/2 .. nx-3/2
        hs, qs = _suliciu_sw_step(hs, qs, 1.0, 0.5, a_periodic)
        o.step(1, 0.5)
    assert np.allclose(o.h, hs, rtol=1e-12, atol=0)
    assert np.allclose(o.hu, qs, rtol=0, atol=1e-12)
    assert np.all(o.z == 0.0)


def test_no_bedload_varying_bed_moves_by_O_dx():
    changes = []
    for nx in (100, 200, 400):
        h, hu, z, dx = W.smooth_periodic1d(nx, amp=0.1)
        o = O.Oracle1D(h, hu, z, dx, grass(Ag=0.0), PER1)
        o.step(10 ** 6, 0.5, t_end=50.0)
        changes.append(np.max(np.abs(o.z - z)))
    r1, r2 = changes[0] / changes[1], changes[1] / changes[2]
    # at least first order in dx (second order is observed on this smooth bed)
    assert r1 > 1.6 and r2 > 1.6, changes
    assert changes[0] > 1e-9


def test_y_uniform_2d_equals_1d():
    h1, hu1, z1, dx = W.dune1d(120, length=1000.0)
    ny = 6
    rep = lambda a: np.repeat(a[None, :], ny, axis=0)
    p = grass(Ag=0.3)
    o2 = O.Oracle2D(rep(h1), rep(hu1), np.zeros((ny, 120)), rep(z1), dx, 3.0, p, PER2)
    o1 = O.Oracle1D(h1, hu1, z1, dx, p, PER1)
    dt = 0.5 * o1.cfl_dt(1.0)
    o1.step_fixed_dt(40, dt)
    o2.step_fixed_dt(40, dt)
    for j in range(ny):
        assert np.allclose(o2.h[j], o1.h, rtol=1e-15, atol=0)
        assert np.allclose(o2.hu[j], o1.hu, rtol=1e-15, atol=1e-15)
        assert np.allclose(o2.z[j], o1.z, rtol=1e-15, atol=1e-15)
    assert np.max(np.abs(o2.hv)) == 0.0


def _asym_field(nx, ny):
    h, hu, hv, zb, dx, dy = W.dune2d(nx, ny, lx=1000.0, ly=1000.0)
    hu = hu + 0.5 * zb
    hv = 1.5 * zb
    return h, hu, hv, zb, dx


def test_transpose_symmetry():
    h, hu, hv, zb, dx = _asym_field(40, 40)
    p = grass(Ag=0.2, mg=2.5)
    a = O.Oracle2D(h, hu, hv, zb, dx, dx, p, PER2)
    b = O.Oracle2D(h.T, hv.T, hu.T, zb.T, dx, dx, p, PER2)
    a.step(30, 0.5)
    b.step(30, 0.5)
    assert a.t == pytest.approx(b.t, rel=1e-14)
    assert np.allclose(a.h, b.h.T, rtol=1e-13, atol=0)
    assert np.allclose(a.hu, b.hv.T, rtol=0, atol=1e-12)
    assert np.allclose(a.hv, b.hu.T, rtol=0, atol=1e-12)
    assert np.allclose(a.z, b.z.T, rtol=0, atol=1e-13)


def test_mirror_symmetry():
    h, hu, hv, zb, dx = _asym_field(40, 36)
    p = mpm()
    h = 0.5 + 0.2 * zb
    a = O.Oracle2D(h, hu * 0.2, hv * 0.2, zb, dx, dx, p, PER2)
    b = O.Oracle2D(h[:, ::-1], -hu[:, ::-1] * 0.2, hv[:, ::-1] * 0.2, zb[:, ::-1],
                   dx, dx, p, PER2)
    a.step(30, 0.5)
    b.step(30, 0.5)
    assert np.allclose(a.h, b.h[:, ::-1], rtol=1e-13, atol=0)
    assert np.allclose(a.hu, -b.hu[:, ::-1], rtol=0, atol=1e-12)
    assert np.allclose(a.hv, b.hv[:, ::-1], rtol=0, atol=1e-12)
    assert np.allclose(a.z, b.z[:, ::-1], rtol=0, atol=1e-13)


def _coarsen(a, f):
    return a.reshape(-1, f).mean(axis=1)


def test_first_order_grid_convergence():
    T = 40.0
    p = grass(Ag=5e-3)
    ref_n = 3200
    h, hu, z, dx = W.smooth_periodic1d(ref_n)
    r = O.Oracle1D(h, hu, z, dx, p, PER1)
    r.step(10 ** 7, 0.5, t_end=T)
    errs = []
    ns = (100, 200, 400)
    for n in ns:
        h, hu, z, dx = W.smooth_periodic1d(n)
        o = O.Oracle1D(h, hu, z, dx, p, PER1)
        o.step(10 ** 7, 0.5, t_end=T)
        assert o.t == T
        zr = _coarsen(r.z, ref_n // n)
        qr = _coarsen(r.hu, ref_n // n)
        errs.append(np.mean(np.abs(o.z - zr)) + np.mean(np.abs(o.hu - qr)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 0.75) and np.all(orders < 1.35), (errs, orders)


def _sediment_root(h, u, beta, g=9.81):
    # p_A(lambda) = -lambda [(u - lambda)^2 - g h] + g h (beta lambda + alpha),
    # alpha = -u beta (Grass / Darcy-type laws)
    alpha = -u * beta
    coeffs = [-1.0, 2 * u, -(u * u - g * h) + g * h * beta, g * h * alpha]
    roots = np.roots(coeffs)
    roots = np.real(roots[np.abs(np.imag(roots)) < 1e-12])
    return roots[np.argmin(np.abs(roots))], roots


@pytest.mark.parametrize("regime", ["dune", "antidune"])
def test_bed_wave_moves_at_linear_sediment_celerity(regime):
    if regime == "dune":
        h0, q0, Ag, L = 10.0, 10.0, 0.5, 2000.0        # Fr = 0.1
    else:
        h0, q0, Ag, L = 0.5, 2.0, 1e-3, 400.0          # Fr = 1.8
    nx = 1000
    x = W.cell_centres(nx, L)
    dz = 1e-3 * np.exp(-((x - 0.5 * L) / (0.04 * L)) ** 2)
    z = dz.copy()
    if regime == "dune":
        h = h0 - dz             # free surface flat, discharge uniform
    else:                       # steady supercritical flow over the bump
        h = W.bernoulli_supercritical(q0, q0 * q0 / (2 * 9.81 * h0 * h0) + h0,
                                      dz, h0)
    hu = np.full(nx, q0)
    u = q0 / h0
    beta = 3.0 * Ag * u * u / h0                # d q_b / d(hu) for m_g = 3
    lam, roots = _sediment_root(h0, u, beta)
    o = O.Oracle1D(h, hu, z, L / nx, grass(Ag=Ag), PER1)
    T = 0.02 * L / abs(lam)
    o.step(10 ** 7, 0.5, t_end=T)
    c0 = np.sum(x * dz) / np.sum(dz)
    pert = o.z - np.mean(o.z[:50])
    c1 = np.sum(x * pert) / np.sum(pert)
    speed = (c1 - c0) / T
    if regime == "dune":
        assert lam > 0 and speed > 0       # downstream
    else:
        assert lam < 0 and speed < 0       # upstream (antidune)
    assert speed == pytest.approx(lam, rel=0.1), (speed, lam, roots)


def test_paper_dune_moves_downstream():
    # 1D dune of the paper (q0 = 10, A_g = 1, m_g = 3), periodic, 60 s
    h, hu, zb, dx = W.dune1d(1000)
    o = O.Oracle1D(h, hu, zb, dx, grass(Ag=1.0), PER1)
    x = W.cell_centres(1000, 1000.0)
    c0 = np.sum(x * (zb - 0.1)) / np.sum(zb - 0.1)
    o.step(10 ** 6, 0.5, t_end=60.0)
    c1 = np.sum(x * (o.z - 0.1)) / np.sum(o.z - 0.1)
    assert c1 > c0 + 5.0


def test_paper_antidune_moves_upstream():
    # 1D antidune of the paper: supercritical inflow (h0 = 0.5, q0 = 1.7)
    # at x = 0, free outflow, A_g = 1e-3, m_g = 3.
    h, hu, zb, dx = W.antidune1d(1200)
    bcs = (O.BC(O.BC_INFLOW, h=0.5, hu=1.7), O.BC(O.BC_FREE))
    o = O.Oracle1D(h, hu, zb, dx, grass(Ag=1e-3), bcs)
    x = W.cell_centres(1200, 24.0)
    c0 = np.sum(x * zb) / np.sum(zb)
    o.step(10 ** 6, 0.5, t_end=10.0)
    m = (x > 4.0) & (x < 16.0)
    pert = np.clip(o.z[m], 0.0, None)
    c1 = np.sum(x[m] * pert) / np.sum(pert)
    assert c1 < c0 - 0.05, (c0, c1)


def test_t_end_is_reached_exactly():
    h, hu, zb, dx = W.dune1d(200)
    o = O.Oracle1D(h, hu, zb, dx, grass(), PER1)
    o.step(10 ** 5, 0.5, t_end=3.3)
    assert o.t == 3.3
    z = o.z.copy()
    o.step(5, 0.5, t_end=3.3)
    assert np.array_equal(o.z, z)


def test_fp32_storage_emulation_rounds_state():
    h, hu, hv, zb, dx, dy = W.dune2d(32, 32)
    o = O.Oracle2D(h, hu, hv, zb, dx, dy, grass(), PER2, storage="fp32")
    o.step(5, 0.5)
    for a in o.state:
        assert np.array_equal(a, a.astype(np.float32).astype(np.float64))
    ref = O.Oracle2D(h, hu, hv, zb, dx, dy, grass(), PER2)
    ref.step(5, 0.5)
    assert np.max(np.abs(o.h - ref.h)) / np.max(ref.h) < 1e-6


def test_momentum_friction_hand_value():
    # uniform flow on a flat periodic bed: the hyperbolic update is exact,
    # the semi-implicit Manning source gives hu / (1 + dt g n^2 |u| / h^(4/3))
    h0, q0, n = 8.0, 4.0, 0.5
    p = O.Params(law=O.LAW_GRASS, A_g=0.0, friction=O.FRIC_MANNING, fric_coef=n,
                 momentum_friction=1)
    o = O.Oracle1D(np.full(10, h0), np.full(10, q0), np.zeros(10), 1.0, p, PER1)
    o.step_fixed_dt(1, 0.1)
    expected = q0 / (1.0 + 0.1 * 9.81 * 0.25 * 0.5 / 16.0)   # 8^(4/3) = 16
    assert np.allclose(o.hu, expected, rtol=1e-15)


def test_momentum_friction_darcy_hand_value():
    # Darcy-Weisbach slope S_f = f |U|^2 / (8 g h) (section "Bedload
    # modelling"): -g h S_f = -(f |u| / (8 h)) hu, semi-implicit:
    # hu / (1 + dt f |u| / (8 h)) on uniform flow over a flat bed
    h0, q0, f = 8.0, 4.0, 0.1
    p = O.Params(law=O.LAW_GRASS, A_g=0.0, friction=O.FRIC_DARCY, fric_coef=f,
                 momentum_friction=1)
    o = O.Oracle1D(np.full(10, h0), np.full(10, q0), np.zeros(10), 1.0, p, PER1)
    o.step_fixed_dt(1, 0.1)
    expected = q0 / (1.0 + 0.1 * f * 0.5 / (8.0 * h0))
    assert np.allclose(o.hu, expected, rtol=1e-15)
    assert expected != q0


@pytest.mark.parametrize("fric,coef,phi", [
    # |U| = 0.5 (u = 0.3, v = 0.4), h = 8 (h^(4/3) = 16), dt = 0.1
    ("DARCY", 0.1, 0.1 * 0.5 / (8.0 * 8.0)),
    ("MANNING", 0.5, 9.81 * 0.25 * 0.5 / 16.0),
    ("STRICKLER", 2.0, 9.81 * 0.5 / (4.0 * 16.0)),
])
def test_momentum_friction_2d_hand_values(fric, coef, phi):
    # both components are divided by 1 + dt phi(h, |U|), with the speed of
    # the full velocity vector
    h0 = 8.0
    p = O.Params(law=O.LAW_GRASS, A_g=0.0, friction=getattr(O, "FRIC_" + fric),
                 fric_coef=coef, momentum_friction=1)
    h = np.full((6, 7), h0)
    o = O.Oracle2D(h, 0.3 * h, 0.4 * h, np.zeros_like(h), 1.0, 2.0, p, PER2)
    o.step_fixed_dt(1, 0.1)
    den = 1.0 + 0.1 * phi
    assert np.allclose(o.hu, 0.3 * h0 / den, rtol=1e-15)
    assert np.allclose(o.hv, 0.4 * h0 / den, rtol=1e-15)


@pytest.mark.parametrize("transpose", [False, True])
def test_cfl_dt_hand_value_anisotropic_grid(transpose):
    # Uniform flow (h, u, 0) over a flat bed without bedload on a grid with
    # dx != dy.  The celerities of eq. "ab" with the reading's b: across an
    # x-interface b = |h u| (cell bound, beta = 0), a^2 = g h^3 + (h u)^2, so
    # the outer speed is S_x = |u| + sqrt(g h + u^2); across a y-interface
    # the normal velocity is 0, b is the floor and S_y = sqrt(g h) (the floor
    # changes it by 1e-28 relative).  dt = CFL / (S_x/dx + S_y/dy): each
    # direction's speed is paired with its own spacing.
    g, h0, u0, cfl, dx, dy = 9.81, 4.0, 2.0, 0.5, 1.0, 3.0
    Sx = u0 + np.sqrt(g * h0 + u0 * u0)
    Sy = np.sqrt(g * h0)
    expected = cfl / (Sx / dx + Sy / dy)
    h = np.full((9, 11), h0)
    p = grass(Ag=0.0)
    if transpose:
        o = O.Oracle2D(h.T, 0 * h.T, u0 * h.T, 0 * h.T, dy, dx, p, PER2)
    else:
        o = O.Oracle2D(h, u0 * h, 0 * h, 0 * h, dx, dy, p, PER2)
    assert o.cfl_dt(cfl) == pytest.approx(expected, rel=1e-14)
    o.step(1, cfl)
    assert o.t == pytest.approx(expected, rel=1e-14)
    # the swapped pairing differs by far more than rounding
    assert abs(cfl / (Sx / dy + Sy / dx) - expected) > 0.1 * expected


def test_complex_step_tangent_matches_central_differences():
    rng = np.random.default_rng(4)
    h, hu, hv, zb, dx, dy = W.dune2d(12, 10, lx=100.0, ly=100.0)
    zb = zb + 0.05 * rng.standard_normal(zb.shape)
    hv = hv + 0.1 * rng.standard_normal(zb.shape)
    Ag = 1e-2 * (1 + 0.3 * rng.standard_normal(zb.shape))
    p = grass(Ag=1e-2)
    dt = 0.05
    dz = rng.standard_normal(zb.shape)
    dA = rng.standard_normal(zb.shape) * 1e-3

    def run(z, A, nsteps=3):
        s = (h.astype(z.dtype), hu.astype(z.dtype), hv.astype(z.dtype), z)
        for _ in range(nsteps):
            s = step2d_arrays(*s, dt, dx, dy, p, PER2, A)
        return s[3]

    eps = 1e-30
    tan = np.imag(run(zb + 1j * eps * dz, Ag + 1j * eps * dA)) / eps
    e = 1e-6
    fd = (run(zb + e * dz, Ag + e * dA) - run(zb - e * dz, Ag - e * dA)) / (2 * e)
    assert np.allclose(tan, fd, rtol=1e-6, atol=1e-8 * np.max(np.abs(tan)))
