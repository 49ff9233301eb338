"""GPU path (HIP kernels through the C ABI) against the FP64 oracle, element
by element on the same seeded inputs.

Tolerances (stated by the build's target): relative L-infinity per field
<= 1e-12 in FP64; <= 1e-5 for float32 state storage against the oracle's
float32-storage emulation.  Grids span several tiles of the fused kernel
(61 columns x 32 rows per wavefront) with ragged tails.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_helpers import (assert_fields_close, dune2d_case, mpm_case, rel_linf,
                         to_oracle_bcs, to_oracle_params)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def grass(sve, Ag=1e-3, mg=3.0, **kw):
    return sve.Params(law=sve.LAW_GRASS, A_g=Ag, m_g=mg, **kw)


def mpm(sve, law=None, friction=None, coef=40.0, **kw):
    return sve.Params(law=sve.LAW_MPM if law is None else law,
                      friction=sve.FRIC_STRICKLER if friction is None else friction,
                      fric_coef=coef, d_s=1e-3, s=2.65, tau_cr=0.05, **kw)


def run_pair(sve, case, params, bcs, nsteps, cfl=0.5, path=None, rows=None,
             storage="fp64", Ag=None, fixed_dt=None, t_end=0.0):
    s = sve.Solver(case["h"], case["hu"], case["zb"], case.get("hv"), lx=case["lx"],
                   ly=case.get("ly", 1.0), params=params, bcs=bcs, Ag=Ag, storage=storage)
    if path is not None:
        s.set_path(path)
    if rows is not None:
        s.set_tile_rows(rows)
    if case.get("hv") is None:
        o = O.Oracle1D(case["h"], case["hu"], case["zb"], case["lx"] / case["h"].shape[0],
                       to_oracle_params(params), to_oracle_bcs(bcs[:2]), Ag=Ag, storage=storage)
    else:
        ny, nx = case["h"].shape
        o = O.Oracle2D(case["h"], case["hu"], case["hv"], case["zb"], case["lx"] / nx,
                       case["ly"] / ny, to_oracle_params(params), to_oracle_bcs(bcs), Ag=Ag,
                       storage=storage)
    if fixed_dt is not None:
        s.step_fixed_dt(nsteps, fixed_dt)
        o.step_fixed_dt(nsteps, fixed_dt)
    else:
        s.step(nsteps, cfl, t_end)
        o.step(nsteps, cfl, t_end if t_end > 0 else None)
    fields, t, dtl, ns = s.get_state()
    s.close()
    return fields, t, dtl, ns, o


PER = None


def per(sve):
    return [sve.BC(sve.BC_PERIODIC)] * 4


PATHS = {"fused": 0, "split": 1, "residual": 3}


@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_dune2d_periodic_fp64(sve, path):
    case = dune2d_case(150, 80)
    p = PATHS[path]
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve), per(sve), 60, path=p)
    assert ns == 60
    assert t == pytest.approx(o.t, rel=TOL64)
    assert dtl == pytest.approx(o.dt_last, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


# rows: one-row tiles, uneven splits (75 rows in tiles of 5 and 8 rows, or
# of 16 with a short last tile), one tile taller than the grid, automatic
@pytest.mark.parametrize("path", ["fused", "residual"])
@pytest.mark.parametrize("rows", [1, 5, 8, 16, 64, 100, 0])
def test_fused_tile_rows_agree(sve, rows, path):
    case = dune2d_case(130, 75)
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=0.05), per(sve), 30, rows=rows,
                                path=PATHS[path])
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("path", ["fused", "residual"])
@pytest.mark.parametrize("rows", [1, 2, 3, 4, 0])
def test_fused_tile_rows_open_boundaries(sve, rows, path):
    """Tiles touching inflow and free boundaries, with uneven splits."""
    case = mpm_case(160, 70)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE)]
    f, t, dtl, ns, o = run_pair(sve, case, mpm(sve), bcs, 40, rows=rows, path=PATHS[path])
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_mpm_strickler_inflow_free_fp64(sve, path):
    case = mpm_case(160, 70)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE)]
    p = PATHS[path]
    f, t, dtl, ns, o = run_pair(sve, case, mpm(sve), bcs, 80, path=p)
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("side", ["E", "S", "N", "WS"])
@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_inflow_on_every_side(sve, side, path):
    """The MPM channel mirrored or transposed so that the inflow boundary is
    the east, south or north side (and west plus south at once): ghost
    columns on the east edge of the last tile, ghost rows below the first
    and above the last tile row."""
    case = mpm_case(160, 70)
    h, hu, hv, zb = case["h"], case["hu"], case["hv"], case["zb"]
    lx, ly = case["lx"], case["ly"]
    free = sve.BC(sve.BC_FREE)
    if side == "E":
        h, hu, hv, zb = h[:, ::-1], -hu[:, ::-1], hv[:, ::-1], zb[:, ::-1]
        bcs = [free, sve.BC(sve.BC_INFLOW, 0.5, -2.0, 0.0), free, free]
    elif side in ("S", "N"):
        h, hu, hv, zb = h.T, hv.T, hu.T, zb.T
        lx, ly = ly, lx
        if side == "N":
            h, hu, hv, zb = h[::-1], hu[::-1], -hv[::-1], zb[::-1]
            bcs = [free, free, free, sve.BC(sve.BC_INFLOW, 0.5, 0.0, -2.0)]
        else:
            bcs = [free, free, sve.BC(sve.BC_INFLOW, 0.5, 0.0, 2.0), free]
    else:
        hv = hu.copy()
        bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 2.0), free, sve.BC(sve.BC_INFLOW, 0.5, 2.0, 2.0),
               free]
    case = dict(h=np.ascontiguousarray(h), hu=np.ascontiguousarray(hu),
                hv=np.ascontiguousarray(hv), zb=np.ascontiguousarray(zb), lx=lx, ly=ly)
    f, t, dtl, ns, o = run_pair(sve, case, mpm(sve), bcs, 40, path=PATHS[path])
    assert ns == 40
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("path", ["fused", "residual"])
def test_mpm_fp32_storage(sve, path):
    case = mpm_case(160, 70)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE)]
    f, t, dtl, ns, o = run_pair(sve, case, mpm(sve), bcs, 80, storage="fp32", path=PATHS[path])
    # every dt comes from the wave speeds of the state as stored (rounded to
    # float32) on both sides, so the times agree to FP64 rounding
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL32)
    for a in f:
        assert np.array_equal(a, a.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("law,fric,coef", [("MPM", "STRICKLER", 40.0),
                                           ("MPM", "MANNING", 0.03),
                                           ("NIELSEN", "STRICKLER", 40.0)])
@pytest.mark.parametrize("path", ["fused", "split"])
def test_threshold_laws_wide_depth_range(sve, law, fric, coef, path):
    """Threshold-law closures, whose shear stress scales with h^(-1/3), on
    depths from 0.01 to 100 m (thirteen binades, every residue of the binary
    exponent mod 3 of the cube-root range reduction), with transport above
    the threshold in every cell.  Free boundaries on all sides."""
    nx, ny = 90, 40
    x = (np.arange(nx) + 0.5) / nx
    h = np.tile(10.0 ** (-2.0 + 4.0 * x), (ny, 1))
    rng = np.random.default_rng(3)
    zb = (1e-3 * np.sin(2 * np.pi * np.arange(ny) / ny)[:, None] * np.ones((1, nx))
          + 1e-4 * rng.standard_normal((ny, nx)))
    hv = 0.2 * h * np.cos(2 * np.pi * np.arange(nx) / nx)[None, :]
    case = dict(h=h, hu=2.0 * h, hv=hv, zb=zb, lx=900.0, ly=400.0)
    p = mpm(sve, law=getattr(sve, "LAW_" + law), friction=getattr(sve, "FRIC_" + fric), coef=coef)
    f, t, dtl, ns, o = run_pair(sve, case, p, [sve.BC(sve.BC_FREE)] * 4, 20, path=PATHS[path])
    assert ns == 20
    assert t == pytest.approx(o.t, rel=TOL64)
    assert np.max(np.abs(o.state[3] - zb)) > 1e-5           # the bed moved
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_dune2d_to_t_end(sve, path):
    """A 2D run stopped at t_end inside a call: the last step is clipped to
    land on t_end and the remaining steps leave the state unchanged."""
    case = dune2d_case(130, 75)
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=0.05), per(sve), 400,
                                path=PATHS[path], t_end=20.0)
    assert t == 20.0 and o.t == 20.0
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("mg", [3.0, 2.5])
@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_fp32_storage_grass_2d(sve, mg, path):
    """Float32 state storage with the Grass closures (m_g = 3 and the
    general exponent) on the periodic dune, against the oracle's
    float32-storage emulation."""
    case = dune2d_case(130, 75)
    case["hv"] = 0.5 * case["zb"]
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=0.05, mg=mg), per(sve), 60,
                                storage="fp32", path=PATHS[path])
    assert ns == 60
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL32)
    for a in f:
        assert np.array_equal(a, a.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("mg", [1.3, 2.5, 3.7])
def test_general_exponent_wide_speed_range(sve, mg):
    """The general-exponent closure (|U|^(m_g-1) by exp and log series on
    the GPU, the library power in the oracle) on speeds from 1e-7 to 4 m/s
    in random directions: |(m_g-3)/2 ln |U|^2| reaches 27."""
    case = dune2d_case(90, 70)
    rng = np.random.default_rng(11)
    speed = 10.0 ** rng.uniform(-7.0, 0.6, case["h"].shape)
    ang = rng.uniform(0.0, 2.0 * np.pi, case["h"].shape)
    case["hu"] = case["h"] * speed * np.cos(ang)
    case["hv"] = case["h"] * speed * np.sin(ang)
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=1e-2, mg=mg), per(sve), 20)
    assert ns == 20
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("mg", [1.0, 1.7, 2.5, 4.0])
@pytest.mark.parametrize("path", ["fused", "residual"])
def test_grass_exponent_and_ag_field(sve, mg, path):
    case = dune2d_case(100, 66)
    rng = np.random.default_rng(5)
    Ag = 1e-2 * (1.0 + 0.3 * rng.uniform(-1, 1, case["h"].shape))
    case["hv"] = 0.5 * case["zb"]
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=1e-2, mg=mg), per(sve), 40, Ag=Ag,
                                path=PATHS[path])
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("law", ["FLVB", "NIELSEN", "RIBBERINK", "CAMENEN"])
@pytest.mark.parametrize("fric", ["MANNING", "DARCY"])
@pytest.mark.parametrize("path", ["fused", "residual"])
def test_other_bedload_laws(sve, law, fric, path):
    case = mpm_case(90, 40)
    case["hv"] = 0.2 * np.sin(np.arange(case["h"].size).reshape(case["h"].shape) * 0.01)
    coef = 0.025 if fric == "MANNING" else 0.05
    p = mpm(sve, law=getattr(sve, "LAW_" + law), friction=getattr(sve, "FRIC_" + fric),
            coef=coef)
    f, t, dtl, ns, o = run_pair(sve, case, p, per(sve), 25, path=PATHS[path])
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("path", ["fused", "residual"])
def test_momentum_friction(sve, path):
    case = mpm_case(120, 40)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_PERIODIC), sve.BC(sve.BC_PERIODIC)]
    f, t, dtl, ns, o = run_pair(sve, case, mpm(sve, momentum_friction=1), bcs, 40,
                                path=PATHS[path])
    assert_fields_close(f, o.state, TOL64)


def test_paths_and_fixed_dt_mixed_in_one_run(sve):
    """Residual, fixed-dt, fused and split steps in one run: the residual
    path rebuilds its residual after any other kind of step."""
    case = dune2d_case(120, 70)
    case["hv"] = 0.3 * case["zb"]
    p = grass(sve, Ag=0.03, mg=2.5)
    s = sve.Solver(case["h"], case["hu"], case["zb"], case["hv"], lx=case["lx"],
                   ly=case["ly"], params=p, bcs=per(sve))
    ny, nx = case["h"].shape
    o = O.Oracle2D(case["h"], case["hu"], case["hv"], case["zb"], case["lx"] / nx,
                   case["ly"] / ny, to_oracle_params(p), to_oracle_bcs(per(sve)))
    plan = [("residual", 7), ("fixed", 4), ("residual", 6), ("fused", 3), ("residual", 1),
            ("split", 2), ("residual", 5)]
    for kind, n in plan:
        if kind == "fixed":
            s.step_fixed_dt(n, 0.004)
            o.step_fixed_dt(n, 0.004)
        else:
            s.set_path(PATHS[kind])
            s.step(n, 0.5)
            o.step(n, 0.5)
    f, t, dtl, ns = s.get_state()
    s.close()
    assert ns == sum(n for _, n in plan)
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


def test_1d_paths_and_fixed_dt_mixed_in_one_run(sve):
    """Resident, one-pass, split and fixed-dt steps in one 1D run, with
    t_end reached in the middle: each path takes over the time and the wave
    speeds the previous one left."""
    h, hu, zb, dx = W.dune1d(1200)
    p = grass(sve, Ag=0.05, mg=2.5)
    bcs = [sve.BC(sve.BC_INFLOW, 9.9, 10.0, 0.0), sve.BC(sve.BC_FREE)]
    s = sve.Solver(h, hu, zb, lx=1000.0, params=p, bcs=bcs)
    o = O.Oracle1D(h, hu, zb, 1000.0 / 1200, to_oracle_params(p), to_oracle_bcs(bcs))
    plan = [("RESIDENT", 9), ("FUSED", 5), ("fixed", 3), ("FUSED", 4), ("SPLIT", 2),
            ("RESIDENT", 3), ("fixed", 2), ("SPLIT", 3), ("FUSED", 6)]
    for kind, n in plan:
        if kind == "fixed":
            s.step_fixed_dt(n, 0.02)
            o.step_fixed_dt(n, 0.02)
        else:
            s.set_path(getattr(sve, "PATH_" + kind))
            s.step(n, 0.5)
            o.step(n, 0.5)
    s.set_path(sve.PATH_FUSED)
    t_end = o.t + 0.07
    s.step(10, 0.5, t_end)
    o.step(10, 0.5, t_end)
    f, t, dtl, ns = s.get_state()
    s.close()
    assert ns == sum(n for _, n in plan) + 10
    assert t == t_end and o.t == t_end
    assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


def test_fixed_dt_2d(sve):
    case = dune2d_case(140, 90)
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=0.02), per(sve), 50, fixed_dt=0.01)
    assert t == pytest.approx(o.t, rel=1e-14)
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (5, 1), (3, 3), (2, 130), (70, 2)])
def test_tiny_and_degenerate_2d_grids(sve, shape):
    ny, nx = shape
    rng = np.random.default_rng(nx * 100 + ny)
    h = 2.0 + 0.3 * rng.uniform(size=shape)
    case = dict(h=h, hu=0.5 + 0.2 * rng.uniform(size=shape), hv=0.1 * rng.uniform(size=shape),
                zb=0.1 * rng.uniform(size=shape), lx=10.0 * nx, ly=10.0 * ny)
    for bcs in (per(sve), [sve.BC(sve.BC_FREE)] * 4):
        for path in (sve.PATH_FUSED, sve.PATH_SPLIT, sve.PATH_RESIDUAL):
            f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=0.01), bcs, 15, path=path)
            assert_fields_close(f, o.state, TOL64)


def test_dune1d_resident_and_split(sve):
    h, hu, zb, dx = W.dune1d(1000)
    case = dict(h=h, hu=hu, zb=zb, lx=1000.0)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 2
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, grass(sve), bcs, 3000, path=path)
        assert ns == 3000
        assert t == pytest.approx(o.t, rel=TOL64)
        assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


def test_dune1d_to_t_end(sve):
    h, hu, zb, dx = W.dune1d(1000)
    case = dict(h=h, hu=hu, zb=zb, lx=1000.0)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 2
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve), bcs, 20000, path=sve.PATH_RESIDENT,
                                t_end=300.0)
    assert t == 300.0 and o.t == 300.0
    assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


def test_antidune1d_inflow_free(sve):
    h, hu, zb, dx = W.antidune1d(1000)
    case = dict(h=h, hu=hu, zb=zb, lx=24.0)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 1.7, 0.0), sve.BC(sve.BC_FREE)]
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, grass(sve), bcs, 2000, path=path)
        assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


def test_antidune1d_mirrored_inflow_east(sve):
    """The antidune channel mirrored: inflow through the east side, free
    outflow through the west (the 1D kernels' ghost cell beyond the last
    cell)."""
    h, hu, zb, dx = W.antidune1d(1000)
    case = dict(h=h[::-1].copy(), hu=-hu[::-1], zb=zb[::-1].copy(), lx=24.0)
    bcs = [sve.BC(sve.BC_FREE), sve.BC(sve.BC_INFLOW, 0.5, -1.7, 0.0)]
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, grass(sve), bcs, 2000, path=path)
        assert ns == 2000
        assert t == pytest.approx(o.t, rel=TOL64)
        assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


@pytest.mark.parametrize("law,fric,friction_src", [("MPM", "STRICKLER", 0), ("NIELSEN", "MANNING", 0),
                                                  ("RIBBERINK", "DARCY", 0), ("CAMENEN", "STRICKLER", 0),
                                                  ("MPM", "STRICKLER", 1)])
def test_1d_threshold_laws_and_friction(sve, law, fric, friction_src):
    """The threshold-law closures and the optional momentum friction in the
    1D kernels (single-workgroup resident kernel and split path): the 1D
    dune with transport above the threshold in every cell."""
    h, hu, zb, dx = W.dune1d(1000)
    case = dict(h=h, hu=hu, zb=zb, lx=1000.0)
    coef = {"STRICKLER": 40.0, "MANNING": 0.025, "DARCY": 0.05}[fric]
    p = mpm(sve, law=getattr(sve, "LAW_" + law), friction=getattr(sve, "FRIC_" + fric), coef=coef,
            momentum_friction=friction_src)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 2
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, p, bcs, 300, path=path)
        assert ns == 300
        assert t == pytest.approx(o.t, rel=TOL64)
        assert np.max(np.abs(o.state[2] - zb)) > 1e-6           # the bed moved
        assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


@pytest.mark.parametrize("closure", ["grass3", "grassm", "nielsen", "mpm"])
def test_1d_resident_largest_grid(sve, closure):
    """The LDS-resident kernel at the largest grid it holds (2922 cells):
    three cells per thread in its 1024-thread form (Grass m_g = 3, MPM), six
    in its 512-thread form (general exponent, the run-time threshold laws)."""
    h, hu, zb, dx = W.dune1d(2922)
    case = dict(h=h, hu=hu, zb=zb, lx=1000.0)
    if closure == "grass3":
        p = grass(sve, Ag=0.05)
    elif closure == "grassm":
        p = grass(sve, Ag=0.05, mg=2.3)
    else:
        p = mpm(sve, law=getattr(sve, "LAW_" + closure.upper()), friction=sve.FRIC_MANNING,
                coef=0.025, momentum_friction=0)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 2
    f, t, dtl, ns, o = run_pair(sve, case, p, bcs, 200, path=sve.PATH_RESIDENT)
    assert ns == 200
    assert t == pytest.approx(o.t, rel=TOL64)
    assert np.max(np.abs(o.state[2] - zb)) > 1e-6           # the bed moved
    assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


@pytest.mark.parametrize("nx", [3000, 6101, 20000])
def test_1d_one_pass_large_grids(sve, nx):
    """The one-pass 1D kernel beyond the resident kernel's size limit (its
    default there): the periodic dune and the inflow / free antidune, on
    grids whose last tile is full (6101 = 100 x 61 + 1 leaves one cell) or
    ragged."""
    h, hu, zb, dx = W.dune1d(nx)
    case = dict(h=h, hu=hu, zb=zb, lx=1000.0)
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=0.05), [sve.BC(sve.BC_PERIODIC)] * 2,
                                200)
    assert ns == 200 and t == pytest.approx(o.t, rel=TOL64)
    assert np.max(np.abs(o.state[2] - zb)) > 1e-6
    assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))
    h, hu, zb, dx = W.antidune1d(nx)
    case = dict(h=h, hu=hu, zb=zb, lx=24.0)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 1.7, 0.0), sve.BC(sve.BC_FREE)]
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve), bcs, 200)
    assert ns == 200 and t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


def test_1d_ag_field(sve):
    """A per-cell A_g field in the 1D kernels (resident and split)."""
    h, hu, zb, dx = W.dune1d(1000)
    case = dict(h=h, hu=hu, zb=zb, lx=1000.0)
    rng = np.random.default_rng(9)
    Ag = 1e-2 * (1.0 + 0.5 * rng.uniform(-1, 1, h.shape))
    bcs = [sve.BC(sve.BC_PERIODIC)] * 2
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=1e-2), bcs, 500, path=path, Ag=Ag)
        assert t == pytest.approx(o.t, rel=TOL64)
        assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


def test_fp32_storage_1d(sve):
    h, hu, zb, dx = W.dune1d(1000)
    case = dict(h=h, hu=hu, zb=zb, lx=1000.0)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 2
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag=0.1), bcs, 500, path=path,
                                    storage="fp32")
        assert_fields_close(f, o.state, TOL32, names=("h", "hu", "z"))


def test_device_tensor_round_trip(sve):
    import torch
    case = dune2d_case(64, 64)
    dev = [torch.tensor(case[k], device="cuda") for k in ("h", "hu", "zb", "hv")]
    s = sve.Solver(dev[0], dev[1], dev[2], dev[3], lx=1000.0, ly=1000.0, params=grass(sve),
                   bcs=per(sve))
    s.step(10, 0.5)
    fields, t, dtl, ns = s.get_state_torch()
    torch.cuda.synchronize()
    host, t2, _, _ = s.get_state()
    for a, b in zip(fields, host):
        assert np.array_equal(a.cpu().numpy(), b)
    assert t == t2
    s.close()
