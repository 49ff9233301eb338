"""Every combination of the library's switches against the oracle on one
small 2D grid (70 x 40 cells, 20 CFL steps, default path): storage (FP64,
FP32), closure family (Grass m_g = 3, Grass general exponent with a per-cell
A_g field, Meyer-Peter & Mueller with Strickler, Nielsen with
Darcy-Weisbach), boundaries (periodic; inflow west with free elsewhere),
momentum friction (off, on), interface problem (the paper's, hydrostatic
reconstruction) and order (the paper's first order, the second-order
variant).  Tolerance: 1e-12 relative L-infinity per field in FP64,
1e-5 with float32 storage against the oracle's float32-storage emulation;
the time to 1e-12 in both (each step's dt comes from the state as
stored)."""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_helpers import assert_fields_close, to_oracle_bcs, to_oracle_params

pytestmark = pytest.mark.gpu

NX, NY, STEPS = 70, 40, 20


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def case():
    lx, ly = 350.0, 200.0
    x = W.cell_centres(NX, lx)[None, :]
    y = W.cell_centres(NY, ly)[:, None]
    zb = np.ascontiguousarray(np.broadcast_to(
        0.05 * np.sin(2 * np.pi * x / 70.0) * np.cos(2 * np.pi * y / 100.0)
        + 0.03 * np.exp(-((x - 150.0) ** 2 + (y - 90.0) ** 2) / 800.0), (NY, NX)))
    h = 0.8 - 0.5 * zb
    hu = np.full((NY, NX), 1.2)
    hv = 0.15 * np.sin(2 * np.pi * x / 90.0) * np.ones((NY, 1))
    return dict(h=h, hu=hu, hv=np.ascontiguousarray(hv), zb=zb, lx=lx, ly=ly)


def params(sve, closure, friction_src, rec, order):
    common = dict(momentum_friction=friction_src, reconstruction=rec, order=order)
    if closure == "grass3":
        return sve.Params(law=sve.LAW_GRASS, A_g=0.05, m_g=3.0, friction=sve.FRIC_MANNING,
                          fric_coef=0.03, **common)
    if closure == "grassm":
        return sve.Params(law=sve.LAW_GRASS, A_g=0.05, m_g=2.2, friction=sve.FRIC_DARCY,
                          fric_coef=0.05, **common)
    if closure == "mpm":
        return sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0,
                          d_s=1e-3, s=2.65, tau_cr=0.05, **common)
    return sve.Params(law=sve.LAW_NIELSEN, friction=sve.FRIC_DARCY, fric_coef=0.05, d_s=1e-3,
                      s=2.65, tau_cr=0.05, **common)


COMBOS = list(itertools.product(["fp64", "fp32"], ["grass3", "grassm", "mpm", "nielsen"],
                                ["periodic", "inflow"], [0, 1], [0, 1], [1, 2]))


@pytest.mark.parametrize("storage,closure,bc,friction_src,rec,order", COMBOS)
def test_switch_combination(sve, storage, closure, bc, friction_src, rec, order):
    c = case()
    p = params(sve, closure, friction_src, rec, order)
    if bc == "periodic":
        bcs = [sve.BC(sve.BC_PERIODIC)] * 4
    else:
        free = sve.BC(sve.BC_FREE)
        bcs = [sve.BC(sve.BC_INFLOW, 0.8, 1.2, 0.0), free, free, free]
    Ag = None
    if closure == "grassm":
        rng = np.random.default_rng(7)
        Ag = 0.05 * (1.0 + 0.3 * rng.uniform(-1, 1, (NY, NX)))
    s = sve.Solver(c["h"], c["hu"], c["zb"], c["hv"], lx=c["lx"], ly=c["ly"], params=p,
                   bcs=bcs, Ag=Ag, storage=storage)
    s.step(STEPS, 0.5)
    f, t, dtl, ns = s.get_state()
    s.close()
    o = O.Oracle2D(c["h"], c["hu"], c["hv"], c["zb"], c["lx"] / NX, c["ly"] / NY,
                   to_oracle_params(p), to_oracle_bcs(bcs), Ag=Ag, storage=storage)
    o.step(STEPS, 0.5)
    assert ns == STEPS
    assert t == pytest.approx(o.t, rel=1e-12)
    assert np.max(np.abs(o.z - c["zb"])) > 1e-9            # the bed moved
    assert_fields_close(f, o.state, 1e-12 if storage == "fp64" else 1e-5)
