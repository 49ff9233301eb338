"""GPU path against the FP64 oracle on the configurations the paper's own
runs and edge cases reach:

  * the paper's 2D bump (subsection "2D dune evolution cases"): bed
    0.1 + sin^2 sin^2 bump, h = 10 - z_b, q0 = 10, inflow through the west
    side with the state next to it (9.9, 10, 0), free flow through the other
    sides, Grass closure with m_g = 3 and a general exponent, on every path
    and at several tile heights;
  * a lake at rest over a bump (u = v = 0, flat free surface), which the
    celerity reading keeps at rest to round-off for Grass with m_g >= 3 and
    the threshold laws: periodic and free boundaries, every path, parity
    with the oracle and preservation over 1000 steps.  There the wave-speed
    floor decides b, and the two sides form it in different but equal
    expressions;
  * the optional momentum friction with each friction slope (Strickler,
    Manning, Darcy-Weisbach) in 1D and 2D.

Tolerances: relative L-infinity per field <= 1e-12 (FP64).
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_helpers import assert_fields_close, rel_linf, to_oracle_bcs, to_oracle_params

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
PATHS = {"fused": 0, "split": 1, "residual": 3}


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def run_pair(sve, case, params, bcs, nsteps, cfl=0.5, path=None, rows=None):
    s = sve.Solver(case["h"], case["hu"], case["zb"], case.get("hv"), lx=case["lx"],
                   ly=case.get("ly", 1.0), params=params, bcs=bcs)
    if path is not None:
        s.set_path(path)
    if rows is not None:
        s.set_tile_rows(rows)
    if case.get("hv") is None:
        o = O.Oracle1D(case["h"], case["hu"], case["zb"], case["lx"] / case["h"].shape[0],
                       to_oracle_params(params), to_oracle_bcs(bcs[:2]))
    else:
        ny, nx = case["h"].shape
        o = O.Oracle2D(case["h"], case["hu"], case["hv"], case["zb"], case["lx"] / nx,
                       case["ly"] / ny, to_oracle_params(params), to_oracle_bcs(bcs))
    s.step(nsteps, cfl)
    o.step(nsteps, cfl)
    fields, t, dtl, ns = s.get_state()
    s.close()
    return fields, t, dtl, ns, o


# ----------------------------------------------------------------------------
# the paper's 2D bump with inflow and free boundaries, Grass closure
# ----------------------------------------------------------------------------
def paper_bump(nx, ny):
    h, hu, hv, zb, dx, dy = W.dune2d(nx, ny, base=0.1)
    return dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0)


def paper_bcs(sve):
    free = sve.BC(sve.BC_FREE)
    return [sve.BC(sve.BC_INFLOW, 9.9, 10.0, 0.0), free, free, free]


@pytest.mark.parametrize("Ag,mg", [(1.0, 3.0), (0.1, 3.0), (0.3, 2.5), (0.05, 1.0)])
@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_paper_bump_grass_inflow_free(sve, Ag, mg, path):
    case = paper_bump(130, 75)
    p = sve.Params(law=sve.LAW_GRASS, A_g=Ag, m_g=mg)
    f, t, dtl, ns, o = run_pair(sve, case, p, paper_bcs(sve), 80, path=PATHS[path])
    assert ns == 80
    assert t == pytest.approx(o.t, rel=TOL64)
    assert dtl == pytest.approx(o.dt_last, rel=TOL64)
    assert np.max(np.abs(o.hv)) > 1e-6                 # flow around the bump
    assert np.max(np.abs(o.z - case["zb"])) > 1e-6     # the bed moved
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("mg", [3.0, 2.5])
@pytest.mark.parametrize("path", ["fused", "residual"])
@pytest.mark.parametrize("rows", [1, 2, 3, 4, 0])
def test_paper_bump_tile_heights(sve, rows, path, mg):
    """Tiles touching the inflow column and the free rows and column, with
    uneven splits (70 rows)."""
    case = paper_bump(140, 70)
    p = sve.Params(law=sve.LAW_GRASS, A_g=0.5, m_g=mg)
    f, t, dtl, ns, o = run_pair(sve, case, p, paper_bcs(sve), 40, path=PATHS[path], rows=rows)
    assert t == pytest.approx(o.t, rel=TOL64)
    assert_fields_close(f, o.state, TOL64)


def test_paper_bump_inflow_on_every_side(sve):
    """The bump case transposed and mirrored so that the inflow enters
    through the east, south and north sides (Grass, m_g = 3)."""
    case = paper_bump(120, 90)
    h, hu, hv, zb = case["h"], case["hu"], case["hv"], case["zb"]
    free = sve.BC(sve.BC_FREE)
    p = sve.Params(law=sve.LAW_GRASS, A_g=0.5, m_g=3.0)
    variants = {
        "E": ((h[:, ::-1], -hu[:, ::-1], hv[:, ::-1], zb[:, ::-1]),
              [free, sve.BC(sve.BC_INFLOW, 9.9, -10.0, 0.0), free, free]),
        "S": ((h.T, hv.T, hu.T, zb.T), [free, free, sve.BC(sve.BC_INFLOW, 9.9, 0.0, 10.0), free]),
        "N": ((h.T[::-1], hv.T[::-1], -hu.T[::-1], zb.T[::-1]),
              [free, free, free, sve.BC(sve.BC_INFLOW, 9.9, 0.0, -10.0)]),
    }
    for side, (fields, bcs) in variants.items():
        c = dict(h=np.ascontiguousarray(fields[0]), hu=np.ascontiguousarray(fields[1]),
                 hv=np.ascontiguousarray(fields[2]), zb=np.ascontiguousarray(fields[3]),
                 lx=1000.0, ly=1000.0)
        for path in ("fused", "split", "residual"):
            f, t, dtl, ns, o = run_pair(sve, c, p, bcs, 40, path=PATHS[path])
            assert t == pytest.approx(o.t, rel=TOL64), (side, path)
            assert_fields_close(f, o.state, TOL64)


# ----------------------------------------------------------------------------
# lake at rest
# ----------------------------------------------------------------------------
def lake2d(nx, ny, lx=100.0, ly=80.0, level=2.0):
    x = W.cell_centres(nx, lx)[None, :]
    y = W.cell_centres(ny, ly)[:, None]
    z = 0.4 * np.exp(-((x - 40.0) ** 2 + (y - 35.0) ** 2) / 150.0) + 0.1 * np.sin(
        2 * np.pi * y / ly) * np.cos(2 * np.pi * x / lx) + 0.3
    z = np.ascontiguousarray(np.broadcast_to(z, (ny, nx)))
    h = level - z
    return dict(h=h, hu=np.zeros_like(h), hv=np.zeros_like(h), zb=z, lx=lx, ly=ly)


def lake_params(sve, kind):
    if kind == "grass3":
        return sve.Params(law=sve.LAW_GRASS, A_g=0.05, m_g=3.0)
    if kind == "grass4":
        return sve.Params(law=sve.LAW_GRASS, A_g=0.05, m_g=4.0)
    return sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3,
                      s=2.65, tau_cr=0.05)


def assert_at_rest(fields, case, level=2.0, tol=1e-12):
    h, hu, hv, z = fields
    scale = float(np.max(case["h"] * np.sqrt(9.81 * case["h"])))     # h sqrt(g h)
    assert np.max(np.abs(hu)) <= tol * scale
    assert np.max(np.abs(hv)) <= tol * scale
    assert np.max(np.abs(h + z - level)) <= tol * level
    assert np.max(np.abs(z - case["zb"])) <= tol * np.max(case["zb"])


@pytest.mark.parametrize("kind", ["grass3", "grass4", "mpm"])
@pytest.mark.parametrize("bc", ["periodic", "free"])
@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_lake_at_rest(sve, kind, bc, path):
    case = lake2d(130, 75)
    bcs = [sve.BC(sve.BC_PERIODIC if bc == "periodic" else sve.BC_FREE)] * 4
    p = lake_params(sve, kind)
    # parity with the oracle over 200 steps: depth and bed relative to their
    # maxima, momentum (round-off only) against the scale h sqrt(g h)
    f, t, dtl, ns, o = run_pair(sve, case, p, bcs, 200, path=PATHS[path])
    assert t == pytest.approx(o.t, rel=TOL64)
    assert rel_linf(f[0], o.h) <= TOL64 and rel_linf(f[3], o.z) <= TOL64
    scale = float(np.max(case["h"] * np.sqrt(9.81 * case["h"])))
    assert np.max(np.abs(f[1] - o.hu)) <= TOL64 * scale
    assert np.max(np.abs(f[2] - o.hv)) <= TOL64 * scale
    assert_at_rest(f, case)
    # preservation over 1000 steps on the GPU alone
    s = sve.Solver(case["h"], case["hu"], case["zb"], case["hv"], lx=case["lx"], ly=case["ly"],
                   params=p, bcs=bcs)
    s.set_path(PATHS[path])
    s.step(1000, 0.5)
    fields, t, dtl, ns = s.get_state()
    s.close()
    assert ns == 1000
    assert_at_rest(fields, case)


@pytest.mark.parametrize("kind", ["grass3", "grass4", "mpm"])
@pytest.mark.parametrize("bc", ["periodic", "free"])
def test_lake_at_rest_1d(sve, kind, bc):
    """The 1D kernels (single-workgroup resident kernel and split path)."""
    c2 = lake2d(400, 1)
    case = dict(h=c2["h"][0], hu=c2["hu"][0], zb=c2["zb"][0], lx=c2["lx"])
    bcs = [sve.BC(sve.BC_PERIODIC if bc == "periodic" else sve.BC_FREE)] * 2
    p = lake_params(sve, kind)
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, p, bcs, 1000, path=path)
        assert t == pytest.approx(o.t, rel=TOL64)
        assert rel_linf(f[0], o.h) <= TOL64 and rel_linf(f[2], o.z) <= TOL64
        scale = float(np.max(case["h"] * np.sqrt(9.81 * case["h"])))
        assert np.max(np.abs(f[1] - o.hu)) <= TOL64 * scale
        assert np.max(np.abs(f[1])) <= TOL64 * scale
        assert np.max(np.abs(f[0] + f[2] - 2.0)) <= 2.0 * TOL64


# ----------------------------------------------------------------------------
# momentum friction with each friction slope
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("fric,coef", [("STRICKLER", 40.0), ("MANNING", 0.025),
                                       ("DARCY", 0.05)])
@pytest.mark.parametrize("law", ["MPM", "GRASS"])
@pytest.mark.parametrize("path", ["fused", "split", "residual"])
def test_momentum_friction_laws_2d(sve, fric, coef, law, path):
    lx, ly = 4000.0 * 120 / 8192, 1000.0 * 50 / 2048
    h, hu, hv, zb, dx, dy = W.mpm_channel(120, 50, lx=lx, ly=ly)
    hv = 0.3 * np.sin(np.arange(h.size).reshape(h.shape) * 0.013) * h
    case = dict(h=h, hu=hu, hv=hv, zb=zb, lx=lx, ly=ly)
    common = dict(friction=getattr(sve, "FRIC_" + fric), fric_coef=coef, momentum_friction=1)
    if law == "MPM":
        p = sve.Params(law=sve.LAW_MPM, d_s=1e-3, s=2.65, tau_cr=0.05, **common)
    else:
        p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0, **common)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE), sve.BC(sve.BC_PERIODIC),
           sve.BC(sve.BC_PERIODIC)]
    f, t, dtl, ns, o = run_pair(sve, case, p, bcs, 40, path=PATHS[path])
    assert t == pytest.approx(o.t, rel=TOL64)
    # friction slowed the flow: compare with the same run without the source
    q = O.Oracle2D(h, hu, hv, zb, dx, dy,
                   dataclasses.replace(to_oracle_params(p), momentum_friction=0),
                   to_oracle_bcs(bcs))
    q.step(40, 0.5)
    assert np.mean(np.abs(o.hu)) < np.mean(np.abs(q.hu))
    assert_fields_close(f, o.state, TOL64)


@pytest.mark.parametrize("fric,coef", [("STRICKLER", 40.0), ("MANNING", 0.025),
                                       ("DARCY", 0.05)])
def test_momentum_friction_laws_1d(sve, fric, coef):
    h, hu, zb, dx = W.antidune1d(1000)
    case = dict(h=h, hu=hu, zb=zb, lx=24.0)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0, friction=getattr(sve, "FRIC_" + fric),
                   fric_coef=coef, momentum_friction=1)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 1.7, 0.0), sve.BC(sve.BC_FREE)]
    for path in (sve.PATH_RESIDENT, sve.PATH_SPLIT, sve.PATH_FUSED):
        f, t, dtl, ns, o = run_pair(sve, case, p, bcs, 1500, path=path)
        assert ns == 1500
        assert t == pytest.approx(o.t, rel=TOL64)
        assert_fields_close(f, o.state, TOL64, names=("h", "hu", "z"))
