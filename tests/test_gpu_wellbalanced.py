"""GPU path of the well-balanced variant (hydrostatic reconstruction with the
relaxation interface solver, Params.reconstruction = 1) against the oracle's
variant, element by element on the same seeded inputs: relative L-infinity
per field <= 1e-12 in FP64, <= 1e-5 with float32 storage against the
oracle's float32-storage emulation.

  * the paper's 2D bump (inflow / free boundaries) with the Grass closure,
    and the MPM channel, on every 2D path setting;
  * the periodic 2D dune with a per-cell A_g field and a general exponent;
  * a lake at rest over a bump for Grass exponents below 3 (where the
    paper's scheme lets the bed creep), m_g = 3 and MPM: parity, and
    preservation over 1000 steps on the GPU;
  * 1D: the antidune (inflow / free) and a lake at rest, resident and split
    kernels;
  * float32 storage; tiny grids;
  * the entry points that do not support the variant refuse it.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_helpers import assert_fields_close, rel_linf, to_oracle_bcs, to_oracle_params

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
PATHS = {"fused": 0, "split": 1, "residual": 3}


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def run_pair(sve, case, params, bcs, nsteps, cfl=0.5, path=None, Ag=None, storage="fp64"):
    s = sve.Solver(case["h"], case["hu"], case["zb"], case.get("hv"), lx=case["lx"],
                   ly=case.get("ly", 1.0), params=params, bcs=bcs, Ag=Ag, storage=storage)
    if path is not None:
        s.set_path(path)
    if case.get("hv") is None:
        o = O.Oracle1D(case["h"], case["hu"], case["zb"], case["lx"] / case["h"].shape[0],
                       to_oracle_params(params), to_oracle_bcs(bcs[:2]), Ag=Ag, storage=storage)
    else:
        ny, nx = case["h"].shape
        o = O.Oracle2D(case["h"], case["hu"], case["hv"], case["zb"], case["lx"] / nx,
                       case["ly"] / ny, to_oracle_params(params), to_oracle_bcs(bcs), Ag=Ag,
                       storage=storage)
    s.step(nsteps, cfl)
    o.step(nsteps, cfl)
    fields, t, dtl, ns = s.get_state()
    s.close()
    return fields, t, dtl, ns, o


def grass(sve, Ag=0.05, mg=3.0, **kw):
    return sve.Params(law=sve.LAW_GRASS, A_g=Ag, m_g=mg, reconstruction=1, **kw)


def mpm(sve, **kw):
    return sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3,
                      s=2.65, tau_cr=0.05, reconstruction=1, **kw)


@pytest.mark.parametrize("Ag,mg", [(1.0, 3.0), (0.3, 1.5)])
@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_paper_bump(sve, Ag, mg, path):
    h, hu, hv, zb, dx, dy = W.dune2d(130, 75, base=0.1)
    case = dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0)
    free = sve.BC(sve.BC_FREE)
    bcs = [sve.BC(sve.BC_INFLOW, 9.9, 10.0, 0.0), free, free, free]
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, Ag, mg), bcs, 60, path=PATHS[path])
    assert ns == 60
    assert t == pytest.approx(o.t, rel=TOL64)
    assert dtl == pytest.approx(o.dt_last, rel=TOL64)
    assert np.max(np.abs(o.z - zb)) > 1e-6
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("rows", [1, 2, 3, 0])
def test_fused_tile_heights_and_inflow_sides(sve, rows):
    """The fused kernel's variant at several tile heights, with the bump's
    inflow through the west and (mirrored) the east side."""
    h, hu, hv, zb, dx, dy = W.dune2d(140, 70, base=0.1)
    free = sve.BC(sve.BC_FREE)
    p = grass(sve, 0.5, 2.5)
    for side in ("W", "E"):
        if side == "W":
            case = dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0)
            bcs = [sve.BC(sve.BC_INFLOW, 9.9, 10.0, 0.0), free, free, free]
        else:
            case = dict(h=np.ascontiguousarray(h[:, ::-1]), hu=np.ascontiguousarray(-hu[:, ::-1]),
                        hv=np.ascontiguousarray(hv[:, ::-1]), zb=np.ascontiguousarray(zb[:, ::-1]),
                        lx=1000.0, ly=1000.0)
            bcs = [free, sve.BC(sve.BC_INFLOW, 9.9, -10.0, 0.0), free, free]
        s = sve.Solver(case["h"], case["hu"], case["zb"], case["hv"], lx=1000.0, ly=1000.0,
                       params=p, bcs=bcs)
        s.set_tile_rows(rows)
        s.step(40, 0.5)
        f, t, dtl, ns = s.get_state()
        s.close()
        o = O.Oracle2D(case["h"], case["hu"], case["hv"], case["zb"], 1000.0 / 140, 1000.0 / 70,
                       to_oracle_params(p), to_oracle_bcs(bcs))
        o.step(40, 0.5)
        assert t == pytest.approx(o.t, rel=TOL64), side
        assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("path", ["fused", "split"])
def test_mpm_channel(sve, path):
    lx, ly = 4000.0 * 160 / 8192, 1000.0 * 70 / 2048
    h, hu, hv, zb, dx, dy = W.mpm_channel(160, 70, lx=lx, ly=ly)
    case = dict(h=h, hu=hu, hv=hv, zb=zb, lx=lx, ly=ly)
    free = sve.BC(sve.BC_FREE)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), free, free, free]
    f, t, dtl, ns, o = run_pair(sve, case, mpm(sve), bcs, 60, path=PATHS[path])
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("mg", [1.7, 3.0])
def test_periodic_dune_with_ag_field(sve, mg):
    h, hu, hv, zb, dx, dy = W.dune2d(100, 66)
    case = dict(h=h, hu=hu, hv=0.5 * zb, zb=zb, lx=1000.0, ly=1000.0)
    rng = np.random.default_rng(5)
    Ag = 1e-2 * (1.0 + 0.3 * rng.uniform(-1, 1, h.shape))
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, 1e-2, mg), [sve.BC(sve.BC_PERIODIC)] * 4,
                                40, Ag=Ag)
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


def lake2d(nx, ny, lx=100.0, ly=80.0, level=2.0):
    x = W.cell_centres(nx, lx)[None, :]
    y = W.cell_centres(ny, ly)[:, None]
    z = 0.4 * np.exp(-((x - 40.0) ** 2 + (y - 35.0) ** 2) / 150.0) + 0.1 * np.sin(
        2 * np.pi * y / ly) * np.cos(2 * np.pi * x / lx) + 0.3
    z = np.ascontiguousarray(np.broadcast_to(z, (ny, nx)))
    h = level - z
    return dict(h=h, hu=np.zeros_like(h), hv=np.zeros_like(h), zb=z, lx=lx, ly=ly)


def lake_params(sve, kind):
    if kind == "mpm":
        return mpm(sve)
    return grass(sve, 0.05, float(kind))


@pytest.mark.parametrize("kind", ["1.0", "1.5", "2.5", "3.0", "mpm"])
@pytest.mark.parametrize("bc", ["periodic", "free"])
def test_lake_at_rest_2d(sve, kind, bc):
    case = lake2d(130, 75)
    bcs = [sve.BC(sve.BC_PERIODIC if bc == "periodic" else sve.BC_FREE)] * 4
    p = lake_params(sve, kind)
    scale = float(np.max(case["h"] * np.sqrt(9.81 * case["h"])))
    f, t, dtl, ns, o = run_pair(sve, case, p, bcs, 200)
    # For 1 < m_g < 2 the time step is ill-conditioned at rest: the sediment
    # celerity bound b ~ |U|^((m_g-1)/2) of the round-off velocities a step
    # leaves (|U| ~ 1e-15) moves the outer wave speed by ~ (b/a_f)^2, about
    # 1e-10 for m_g = 1.5 (on the oracle alone a 1e-15 perturbation of the
    # depth changes the time after 50 steps by 5.6e-11).  The state itself
    # stays at rest on both sides.
    t_tol = 1e-9 if kind == "1.5" else TOL64
    assert t == pytest.approx(o.t, rel=t_tol)
    assert rel_linf(f[0], o.h) <= TOL64 and rel_linf(f[3], o.z) <= TOL64
    assert np.max(np.abs(f[1] - o.hu)) <= TOL64 * scale
    assert np.max(np.abs(f[2] - o.hv)) <= TOL64 * scale
    s = sve.Solver(case["h"], case["hu"], case["zb"], case["hv"], lx=case["lx"], ly=case["ly"],
                   params=p, bcs=bcs)
    s.step(1000, 0.5)
    (h, hu, hv, z), t, dtl, ns = s.get_state()
    s.close()
    assert np.max(np.abs(hu)) <= TOL64 * scale and np.max(np.abs(hv)) <= TOL64 * scale
    assert np.max(np.abs(h + z - 2.0)) <= 2.0 * TOL64
    assert np.max(np.abs(z - case["zb"])) <= TOL64 * np.max(case["zb"])


def test_antidune_1d(sve):
    """400 steps: under the variant the supercritical antidune amplifies
    round-off (on the oracle alone a 1e-15 relative perturbation of the
    initial depth grows about tenfold every 400 steps, to 1.4e-9 in z_b after
    2000 steps, where the paper's scheme keeps it below 1e-14), so the
    comparison stops while rounding differences are still below 1e-12."""
    h, hu, zb, dx = W.antidune1d(1000)
    case = dict(h=h, hu=hu, zb=zb, lx=24.0)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 1.7, 0.0), sve.BC(sve.BC_FREE)]
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, grass(sve, 1e-3), bcs, 400, path=path)
        assert ns == 400
        assert t == pytest.approx(o.t, rel=TOL64)
        assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))


@pytest.mark.parametrize("kind", ["1.0", "2.5", "mpm"])
def test_lake_at_rest_1d(sve, kind):
    c2 = lake2d(400, 1)
    case = dict(h=c2["h"][0], hu=c2["hu"][0], zb=c2["zb"][0], lx=c2["lx"])
    p = lake_params(sve, kind)
    scale = float(np.max(case["h"] * np.sqrt(9.81 * case["h"])))
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, p, [sve.BC(sve.BC_FREE)] * 2, 1000, path=path)
        assert t == pytest.approx(o.t, rel=TOL64)
        assert rel_linf(f[0], o.h) <= TOL64 and rel_linf(f[2], o.z) <= TOL64
        assert np.max(np.abs(f[1])) <= TOL64 * scale
        assert np.max(np.abs(f[2] - case["zb"])) <= TOL64 * np.max(case["zb"])


def test_fp32_storage(sve):
    h, hu, hv, zb, dx, dy = W.dune2d(130, 75, base=0.1)
    case = dict(h=h, hu=hu, hv=0.5 * zb, zb=zb, lx=1000.0, ly=1000.0)
    f, t, dtl, ns, o = run_pair(sve, case, grass(sve, 0.3, 2.5), [sve.BC(sve.BC_PERIODIC)] * 4,
                                40, storage="fp32")
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL32)
    for a in f:
        assert np.array_equal(a, a.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (5, 1), (3, 3), (2, 130)])
def test_tiny_grids(sve, shape):
    ny, nx = shape
    rng = np.random.default_rng(nx * 100 + ny)
    case = dict(h=2.0 + 0.3 * rng.uniform(size=shape), hu=0.5 + 0.2 * rng.uniform(size=shape),
                hv=0.1 * rng.uniform(size=shape), zb=0.3 * rng.uniform(size=shape),
                lx=10.0 * nx, ly=10.0 * ny)
    for bcs in ([sve.BC(sve.BC_PERIODIC)] * 4, [sve.BC(sve.BC_FREE)] * 4):
        f, t, dtl, ns, o = run_pair(sve, case, grass(sve, 0.01), bcs, 15)
        assert_fields_close(f, o.state, TOL64)


def test_unsupported_entry_points_refuse_the_variant(sve):
    from paper_1307_0491_amd.adjoint import AdjointRun
    from paper_1307_0491_amd.ensemble import Ensemble
    h, hu, hv, zb, dx, dy = W.dune2d(64, 64)
    s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=grass(sve),
                   bcs=[sve.BC(sve.BC_PERIODIC)] * 4)
    with pytest.raises(sve.SveError) as e:
        AdjointRun(s).forward(4, 0.01)
    assert e.value.code == -1
    s.step(3, 0.5)                        # the context is still usable
    s.close()
    m = dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0, A_g=1e-3, m_g=3.0)
    with pytest.raises(sve.SveError) as e:
        Ensemble([m], params=grass(sve))
    assert e.value.code == -1


@pytest.mark.parametrize("dim", [1, 2])
def test_dry_reconstruction_is_reported(sve, dim):
    """A free surface below the neighbouring bed (h + z_b < z* at an
    interface) reconstructs a zero depth there, which the relaxation solver
    cannot take: the oracle raises and the library reports a step error at
    the first step, keeping the initial state."""
    n = 40
    h = np.full(n, 1.0)
    z = np.zeros(n)
    h[20:24] = 0.2
    z[20:24] = 1.5                     # 1.7 m free surface over a 1 m lake
    hu = np.zeros(n)
    p = grass(sve, 0.01)
    if dim == 1:
        o = O.Oracle1D(h, hu, z, 1.0, to_oracle_params(p), (O.BC(O.BC_FREE),) * 2)
        s = sve.Solver(h, hu, z, lx=float(n), params=p, bcs=[sve.BC(sve.BC_FREE)] * 2)
    else:
        rep = lambda a: np.ascontiguousarray(np.repeat(a[None, :], 6, axis=0))
        o = O.Oracle2D(rep(h), rep(hu), rep(hu), rep(z), 1.0, 1.0, to_oracle_params(p),
                       (O.BC(O.BC_FREE),) * 4)
        s = sve.Solver(rep(h), rep(hu), rep(z), rep(hu), lx=float(n), ly=6.0, params=p,
                       bcs=[sve.BC(sve.BC_FREE)] * 4)
    with pytest.raises(O.OracleError), np.errstate(all="ignore"):
        o.step(1, 0.5)
    with pytest.raises(sve.SveError) as e:
        s.step(3, 0.5)
    assert e.value.code in (-3, -4, -5)
    fields, t, dtl, ns = s.get_state()
    s.close()
    assert ns == 0 and t == 0.0
    assert np.array_equal(fields[0].ravel()[:n], h)
