"""GPU path of the second-order variant (Params.order = 2: MUSCL-minmod
reconstruction, cell term for the bed slope, Heun's method; two kernels per
step) against the oracle's variant, element by element on the same seeded
inputs: relative L-infinity per field <= 1e-12 in FP64, <= 1e-5 with float32
storage against the oracle's float32-storage emulation; the time to 1e-12.

  * the periodic 2D dune (Grass m_g = 3) at several tile heights, on a grid
    that leaves a ragged last tile column; the paper's 2D bump (inflow /
    free) and the MPM channel, both interface problems;
  * the general exponent with a per-cell A_g field; momentum friction;
    float32 storage; a fixed dt; t_end; several calls in a row;
  * 1D: the dune (periodic) and the antidune (inflow / free);
  * tiny and ragged grids around the 60-column tile width;
  * a lake at rest over a bump stays at rest on the GPU;
  * the full 2000 x 2000 dune, 2 steps, on the full grid;
  * a dry first stage fails the first step and keeps the state; the entry
    points without the variant refuse it.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_helpers import assert_fields_close, rel_linf, to_oracle_bcs, to_oracle_params

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def grass(sve, Ag=1e-3, mg=3.0, rec=0, **kw):
    return sve.Params(law=sve.LAW_GRASS, A_g=Ag, m_g=mg, reconstruction=rec, order=2, **kw)


def mpm(sve, rec=0, **kw):
    return sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3,
                      s=2.65, tau_cr=0.05, reconstruction=rec, order=2, **kw)


def per(sve):
    return [sve.BC(sve.BC_PERIODIC)] * 4


def inflow_free(sve, h, hu):
    free = sve.BC(sve.BC_FREE)
    return [sve.BC(sve.BC_INFLOW, h, hu, 0.0), free, free, free]


def pair2d(sve, case, p, bcs, Ag=None, storage="fp64", rows=None):
    h, hu, hv, zb, lx, ly = case
    ny, nx = h.shape
    s = sve.Solver(h, hu, zb, hv, lx=lx, ly=ly, params=p, bcs=bcs, Ag=Ag, storage=storage)
    if rows is not None:
        s.set_tile_rows(rows)
    o = O.Oracle2D(h, hu, hv, zb, lx / nx, ly / ny, to_oracle_params(p), to_oracle_bcs(bcs),
                   Ag=Ag, storage=storage)
    return s, o


def check(s, o, tol=TOL64, close=True):
    f, t, dtl, ns = s.get_state()
    if close:
        s.close()
    assert ns == o.nsteps
    assert t == pytest.approx(o.t, rel=1e-12)
    assert dtl == pytest.approx(o.dt_last, rel=1e-12)
    names = ("h", "hu", "hv", "z") if len(o.state) == 4 else ("h", "hu", "z")
    assert_fields_close(f, o.state, tol, names=names)
    return f


def dune(nx, ny, base=0.0):
    h, hu, hv, zb, dx, dy = W.dune2d(nx, ny, base=base)
    return h, hu, hv, zb, 1000.0, 1000.0


@pytest.mark.parametrize("rows", [1, 2, 3, 5, 0])
def test_periodic_dune_tile_heights(sve, rows):
    s, o = pair2d(sve, dune(131, 70), grass(sve, Ag=0.05), per(sve), rows=rows)
    s.step(30, 0.5)
    o.step(30, 0.5)
    check(s, o)
    assert np.max(np.abs(o.z - W.dune2d(131, 70)[3])) > 1e-6


@pytest.mark.parametrize("rec", [0, 1])
@pytest.mark.parametrize("Ag,mg", [(1.0, 3.0), (0.3, 1.5)])
def test_paper_bump_inflow_free(sve, rec, Ag, mg):
    s, o = pair2d(sve, dune(130, 75, base=0.1), grass(sve, Ag, mg, rec), inflow_free(sve, 9.9, 10.0))
    s.step(40, 0.5)
    o.step(40, 0.5)
    check(s, o)


@pytest.mark.parametrize("rec", [0, 1])
@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_mpm_channel(sve, rec, storage):
    lx, ly = 4000.0 * 160 / 8192, 1000.0 * 70 / 2048
    h, hu, hv, zb, dx, dy = W.mpm_channel(160, 70, lx=lx, ly=ly)
    s, o = pair2d(sve, (h, hu, hv, zb, lx, ly), mpm(sve, rec), inflow_free(sve, 0.5, 2.0),
                  storage=storage)
    s.step(40, 0.45)
    o.step(40, 0.45)
    check(s, o, TOL64 if storage == "fp64" else TOL32)


@pytest.mark.parametrize("rec", [0, 1])
def test_general_exponent_ag_field_and_friction(sve, rec):
    case = dune(97, 64)
    rng = np.random.default_rng(11)
    Ag = 0.05 * (1.0 + 0.3 * rng.uniform(-1.0, 1.0, case[0].shape))
    p = grass(sve, 0.05, 2.3, rec, momentum_friction=1, friction=sve.FRIC_MANNING,
              fric_coef=0.03)
    s, o = pair2d(sve, case, p, inflow_free(sve, 10.0, 10.0), Ag=Ag)
    s.step(25, 0.5)
    o.step(25, 0.5)
    check(s, o)


def test_fixed_dt_t_end_and_calls_in_a_row(sve):
    case = dune(90, 61)
    p = grass(sve, 0.05)
    s, o = pair2d(sve, case, p, per(sve))
    s.step_fixed_dt(4, 0.02)
    o.step_fixed_dt(4, 0.02)
    check(s, o, close=False)
    for n in (3, 5, 1):                 # CFL steps, then steps clipped at t_end
        s.step(n, 0.5, t_end=0.6)
        o.step(n, 0.5, t_end=0.6)
        check(s, o, close=False)
    assert o.t == pytest.approx(0.6, rel=1e-15) or o.t < 0.6
    s.step(4, 0.5, t_end=0.6)
    o.step(4, 0.5, t_end=0.6)
    f = check(s, o)
    assert o.t == 0.6


def test_split_calls_equal_one_call(sve):
    case = dune(121, 40)
    p = grass(sve, 0.05, rec=1)
    a = sve.Solver(*case[:2], case[3], case[2], lx=1000.0, ly=1000.0, params=p, bcs=per(sve))
    b = sve.Solver(*case[:2], case[3], case[2], lx=1000.0, ly=1000.0, params=p, bcs=per(sve))
    a.step(12, 0.5)
    for n in (5, 7):
        b.step(n, 0.5)
    fa, ta, _, na = a.get_state()
    fb, tb, _, nb = b.get_state()
    a.close()
    b.close()
    assert na == nb == 12 and ta == tb
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("rec", [0, 1])
def test_1d_dune_periodic(sve, rec):
    h, hu, zb, dx = W.dune1d(700)
    p = grass(sve, 0.05, rec=rec)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 2
    s = sve.Solver(h, hu, zb, lx=700.0 * dx, params=p, bcs=bcs)
    o = O.Oracle1D(h, hu, zb, dx, to_oracle_params(p), to_oracle_bcs(bcs))
    s.step(200, 0.5)
    o.step(200, 0.5)
    check(s, o)


@pytest.mark.parametrize("rec", [0, 1])
def test_1d_antidune_inflow_free(sve, rec):
    h, hu, zb, dx = W.antidune1d(600, length=6.0)
    p = grass(sve, 1e-3, rec=rec)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 1.7, 0.0), sve.BC(sve.BC_FREE)]
    s = sve.Solver(h, hu, zb, lx=6.0, params=p, bcs=bcs)
    o = O.Oracle1D(h, hu, zb, dx, to_oracle_params(p), to_oracle_bcs(bcs))
    s.step(300, 0.45)
    o.step(300, 0.45)
    check(s, o)


@pytest.mark.parametrize("shape", [(1, 1), (3, 2), (1, 60), (2, 61), (5, 121), (9, 59),
                                   (4, 180)])
def test_small_and_ragged_grids(sve, shape):
    ny, nx = shape
    rng = np.random.default_rng(nx * 100 + ny)
    zb = 0.2 * rng.uniform(0.0, 1.0, shape)
    h = 2.0 - zb + 0.05 * rng.uniform(-1.0, 1.0, shape)
    hu = 1.0 + 0.2 * rng.uniform(-1.0, 1.0, shape)
    hv = 0.2 * rng.uniform(-1.0, 1.0, shape)
    for bcs in (per(sve), inflow_free(sve, 2.0, 1.0)):
        p = grass(sve, 0.02, 2.5, rec=1)
        s, o = pair2d(sve, (h, hu, hv, zb, 10.0 * nx, 10.0 * ny), p, bcs)
        s.step(8, 0.4)
        o.step(8, 0.4)
        check(s, o)


@pytest.mark.parametrize("rec,law", [(0, "grass3"), (0, "mpm"), (1, "grass2.5")])
def test_lake_at_rest_stays_at_rest(sve, rec, law):
    """Parity over 20 steps (the momentum, round-off on both sides, on the
    scale of the momentum flux max h sqrt(g h)), then preservation to
    round-off over 500 steps on the GPU."""
    nx, ny = 150, 90
    x = W.cell_centres(nx, 1500.0)[None, :]
    y = W.cell_centres(ny, 900.0)[:, None]
    zb = np.ascontiguousarray(0.8 * np.exp(-((x - 700.0) ** 2 + (y - 420.0) ** 2) / 2e4)
                              + 0.2 * np.sin(2 * np.pi * x / 1500.0) * np.cos(2 * np.pi * y / 900.0))
    h = 3.0 - zb
    zero = np.zeros_like(h)
    scale = float(np.max(h * np.sqrt(9.81 * h)))
    p = {"grass3": grass(sve, 0.05, 3.0, rec), "mpm": mpm(sve, rec),
         "grass2.5": grass(sve, 0.05, 2.5, rec)}[law]
    free = [sve.BC(sve.BC_FREE)] * 4
    s, o = pair2d(sve, (h, zero, zero, zb, 1500.0, 900.0), p, free)
    s.step(20, 0.5)
    o.step(20, 0.5)
    f, t, dtl, ns = s.get_state()
    assert ns == 20 and t == pytest.approx(o.t, rel=TOL64)
    assert rel_linf(f[0], o.h) <= TOL64 and rel_linf(f[3], o.z) <= TOL64
    assert np.max(np.abs(f[1] - o.hu)) <= TOL64 * scale
    assert np.max(np.abs(f[2] - o.hv)) <= TOL64 * scale
    s.step(480, 0.5)
    f, t, dtl, ns = s.get_state()
    s.close()
    assert ns == 500
    assert np.max(np.abs(f[1])) <= TOL64 * scale and np.max(np.abs(f[2])) <= TOL64 * scale
    assert np.max(np.abs(f[0] + f[3] - 3.0)) < 1e-12
    assert np.max(np.abs(f[3] - zb)) < 1e-12


def test_full_size_dune(sve):
    """The 2000 x 2000 benchmark grid, 2 CFL steps, every cell compared."""
    h, hu, hv, zb, dx, dy = W.dune2d(2000, 2000)
    p = grass(sve, 1e-3)
    s, o = pair2d(sve, (h, hu, hv, zb, 1000.0, 1000.0), p, per(sve))
    s.step(2, 0.5)
    o.step(2, 0.5)
    check(s, o)


@pytest.mark.parametrize("dim", [1, 2])
def test_dry_first_stage_fails_the_step(sve, dim):
    """Jets leaving a thin layer on both sides: the first stage's interface
    problems or its new depth fail; the oracle raises at step 0 and the
    library fails the first step and keeps the initial state."""
    n = 40
    h = np.full(n, 1.0)
    h[18:23] = 0.05
    hu = np.zeros(n)
    hu[15:20] = -3.0
    hu[21:26] = 3.0
    z = np.zeros(n)
    p = grass(sve, 0.0)
    if dim == 1:
        o = O.Oracle1D(h, hu, z, 1.0, to_oracle_params(p), (O.BC(O.BC_FREE),) * 2)
        s = sve.Solver(h, hu, z, lx=float(n), params=p, bcs=[sve.BC(sve.BC_FREE)] * 2)
    else:
        rep = lambda a: np.ascontiguousarray(np.repeat(a[None, :], 5, axis=0))
        zero = np.zeros((5, n))
        o = O.Oracle2D(rep(h), rep(hu), zero, rep(z), 1.0, 1.0, to_oracle_params(p),
                       (O.BC(O.BC_FREE),) * 4)
        s = sve.Solver(rep(h), rep(hu), rep(z), zero, lx=float(n), ly=5.0, params=p,
                       bcs=[sve.BC(sve.BC_FREE)] * 4)
    with pytest.raises(O.OracleError) as eo, np.errstate(all="ignore"):
        o.step_fixed_dt(1, 0.2)
    assert eo.value.step == 0
    with pytest.raises(sve.SveError) as e:
        s.step_fixed_dt(3, 0.2)
    assert e.value.code in (-3, -4, -5)
    fields, t, dtl, ns = s.get_state()
    s.close()
    assert ns == 0 and t == 0.0
    assert np.array_equal(fields[0].ravel()[:n], h)


def test_unsupported_entry_points_refuse_it(sve):
    from paper_1307_0491_amd.adjoint import AdjointRun
    from paper_1307_0491_amd.ensemble import Ensemble
    h, hu, hv, zb, dx, dy = W.dune2d(64, 64)
    p = grass(sve, 1e-3)
    s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p, bcs=per(sve))
    for path in (sve.PATH_SPLIT, sve.PATH_RESIDUAL):
        with pytest.raises(sve.SveError) as e:
            s.set_path(path)
        assert e.value.code == -1
    s.set_path(sve.PATH_FUSED)
    with pytest.raises(sve.SveError) as e:
        AdjointRun(s).forward(4, 0.01)
    assert e.value.code == -1
    s.step(3, 0.5)                        # the context is still usable
    s.close()
    m = dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0, A_g=1e-3, m_g=3.0)
    with pytest.raises(sve.SveError) as e:
        Ensemble([m], params=p)
    assert e.value.code == -1


def test_1d_fp32_storage(sve):
    h, hu, zb, dx = W.antidune1d(500, length=5.0)
    p = grass(sve, 1e-3, rec=1)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 1.7, 0.0), sve.BC(sve.BC_FREE)]
    s = sve.Solver(h, hu, zb, lx=5.0, params=p, bcs=bcs, storage="fp32")
    o = O.Oracle1D(h, hu, zb, dx, to_oracle_params(p), to_oracle_bcs(bcs), storage="fp32")
    s.step(150, 0.45)
    o.step(150, 0.45)
    check(s, o, TOL32)


def test_order_field_values(sve):
    """order 0 is the first-order scheme (bitwise equal to order 1); orders
    other than 0, 1 and 2 are refused."""
    case = dune(70, 40)
    out = []
    for order in (0, 1):
        p = sve.Params(law=sve.LAW_GRASS, A_g=0.05, m_g=3.0, order=order)
        s = sve.Solver(*case[:2], case[3], case[2], lx=1000.0, ly=1000.0, params=p,
                       bcs=per(sve))
        s.step(10, 0.5)
        out.append(s.get_state())
        s.close()
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
    assert out[0][1] == out[1][1]
    for order in (-1, 3):
        with pytest.raises(sve.SveError) as e:
            sve.Solver(*case[:2], case[3], case[2], lx=1000.0, ly=1000.0,
                       params=sve.Params(order=order), bcs=per(sve))
        assert e.value.code == -1
