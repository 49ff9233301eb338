"""Pins of the oracle's well-balanced variant (hydrostatic reconstruction of
Audusse, Bouchut, Bristeau, Klein and Perthame, 2004, with the relaxation
solver as the interface solver; the paper names well balancing as future
work in sections "Parallelization" and "Conclusions and perspectives"):

  * a lake at rest over a varying bed stays at rest to round-off for every
    Grass exponent (1 <= m_g <= 4, where the paper's scheme lets the bed
    creep for m_g < 3) and for the threshold laws, in 1D and 2D, periodic
    and free boundaries;
  * without bedload (A_g = 0) the bed does not move at all over a varying
    bed (the paper's scheme diffuses it at O(dx)): the variant is exactly
    shallow water plus a fixed bed;
  * on a flat bed it is the paper's scheme;
  * water and sediment volumes are conserved on periodic grids;
  * single-interface hand values: the lake over a bed step (the hydrostatic
    pressure of each side), and a reconstruction that lowers the left
    depth, where the fluxes are the textbook Suliciu solver's between the
    reconstructed states plus the hydrostatic correction g/2 (h^2 - h*^2);
  * the variant and the paper's scheme converge to the same solution
    (difference of first order in dx);
  * the paper's dune still moves downstream and its antidune upstream;
  * planted mistakes in the reconstruction each fail one of these pins.
"""
import dataclasses
import json
import os
import sys
import types

import numpy as np
import pytest

import oracle as O
import oracle.scheme as S0
import workloads as W
from oracle.scheme import fluxes_1d
from test_oracle_riemann import suliciu_textbook

G = 9.81
PER2 = (O.BC(),) * 4
PER1 = (O.BC(),) * 2
FREE2 = (O.BC(O.BC_FREE),) * 4
FREE1 = (O.BC(O.BC_FREE),) * 2


def wb(params):
    return dataclasses.replace(params, reconstruction=1)


def grass(Ag=0.05, mg=3.0, **kw):
    return O.Params(law=O.LAW_GRASS, A_g=Ag, m_g=mg, **kw)


def threshold(law=O.LAW_MPM, friction=O.FRIC_STRICKLER, coef=40.0):
    return O.Params(law=law, friction=friction, fric_coef=coef, d_s=1e-3, s=2.65, tau_cr=0.05)


def lake2d(nx=44, ny=36, level=2.0):
    x = W.cell_centres(nx, 100.0)[None, :]
    y = W.cell_centres(ny, 80.0)[:, None]
    z = (0.4 * np.exp(-((x - 40.0) ** 2 + (y - 35.0) ** 2) / 150.0)
         + 0.1 * np.sin(2 * np.pi * y / 80.0) * np.cos(2 * np.pi * x / 100.0) + 0.3)
    z = np.ascontiguousarray(np.broadcast_to(z, (ny, nx)))
    return level - z, z, 100.0 / nx, 80.0 / ny


def lake1d(nx=200, level=2.0):
    x = W.cell_centres(nx, 100.0)
    z = 0.5 * np.exp(-((x - 45.0) / 9.0) ** 2) + 0.1 * np.sin(2 * np.pi * x / 100.0) + 0.3
    return level - z, z, 100.0 / nx


LAKE_PARAMS = [grass(mg=m) for m in (1.0, 1.5, 2.0, 2.5, 3.0, 4.0)] + [
    threshold(), threshold(O.LAW_NIELSEN, O.FRIC_MANNING, 0.025),
    threshold(O.LAW_CAMENEN, O.FRIC_DARCY, 0.05)]


@pytest.mark.parametrize("params", LAKE_PARAMS)
@pytest.mark.parametrize("bcs", ["periodic", "free"])
def test_lake_at_rest_kept_for_every_law_2d(params, bcs):
    h, z, dx, dy = lake2d()
    o = O.Oracle2D(h, 0 * h, 0 * h, z, dx, dy, wb(params), PER2 if bcs == "periodic" else FREE2)
    o.step(500, 0.5)
    scale = float(np.max(h * np.sqrt(G * h)))
    assert np.max(np.abs(o.hu)) < 1e-12 * scale
    assert np.max(np.abs(o.hv)) < 1e-12 * scale
    assert np.max(np.abs(o.h + o.z - 2.0)) < 1e-13
    assert np.max(np.abs(o.z - z)) < 1e-13


@pytest.mark.parametrize("params", LAKE_PARAMS)
def test_lake_at_rest_kept_for_every_law_1d(params):
    h, z, dx = lake1d()
    o = O.Oracle1D(h, 0 * h, z, dx, wb(params), FREE1)
    o.step(2000, 0.5)
    scale = float(np.max(h * np.sqrt(G * h)))
    assert np.max(np.abs(o.hu)) < 1e-12 * scale
    assert np.max(np.abs(o.h + o.z - 2.0)) < 1e-13
    assert np.max(np.abs(o.z - z)) < 1e-13


def test_paper_scheme_is_not_well_balanced_where_the_variant_is():
    # the contrast the paper describes: with m_g = 1 the bed creeps under a
    # lake at rest in the paper's scheme, not in the variant
    h, z, dx = lake1d()
    base = O.Oracle1D(h, 0 * h, z, dx, grass(mg=1.0), PER1)
    var = O.Oracle1D(h, 0 * h, z, dx, wb(grass(mg=1.0)), PER1)
    base.step(500, 0.5)
    var.step(500, 0.5)
    assert np.max(np.abs(base.z - z)) > 1e-4
    assert np.max(np.abs(var.z - z)) < 1e-13


@pytest.mark.parametrize("dim", [1, 2])
def test_no_bedload_leaves_a_varying_bed_unchanged(dim):
    p = grass(Ag=0.0)
    if dim == 1:
        h, hu, z, dx = W.dune1d(300, base=0.1)
        a = O.Oracle1D(h, hu, z, dx, wb(p), PER1)
        b = O.Oracle1D(h, hu, z, dx, p, PER1)
    else:
        h, hu, hv, z, dx, dy = W.dune2d(60, 50, base=0.1)
        hv = 0.3 * z
        a = O.Oracle2D(h, hu, hv, z, dx, dy, wb(p), PER2)
        b = O.Oracle2D(h, hu, hv, z, dx, dy, p, PER2)
    a.step(200, 0.5)
    b.step(200, 0.5)
    assert np.array_equal(a.z, z)
    assert np.max(np.abs(b.z - z)) > 1e-6          # the paper's scheme diffuses it


def test_flat_bed_is_the_paper_scheme():
    h, hu, hv, zb, dx, dy = W.dune2d(50, 40)
    zf = np.full_like(zb, 0.3)
    hv = 0.2 * zb
    for p, n in ((grass(Ag=0.0, mg=2.5), 60), (grass(Ag=0.05, mg=2.5), 1), (threshold(), 1)):
        a = O.Oracle2D(h, hu, hv, zf, dx, dy, p, PER2)
        b = O.Oracle2D(h, hu, hv, zf, dx, dy, wb(p), PER2)
        a.step(n, 0.5)
        b.step(n, 0.5)
        assert a.t == pytest.approx(b.t, rel=1e-14)
        for x, y in zip(a.state, b.state):
            assert np.max(np.abs(x - y)) <= 1e-13 * max(np.max(np.abs(y)), 1e-300)


@pytest.mark.parametrize("params", [grass(Ag=0.3), grass(Ag=0.3, mg=1.5), threshold()])
def test_conservation_periodic(params):
    h, hu, hv, zb, dx, dy = W.dune2d(48, 40, base=0.1)
    if params.law != O.LAW_GRASS:
        h = 0.5 + 0.1 * zb
        hu = 2.0 + 0.3 * zb
    hv = 0.2 * zb
    o = O.Oracle2D(h, hu, hv, zb, dx, dy, wb(params), PER2)
    m0, s0 = h.sum(), zb.sum()
    o.step(200, 0.5)
    assert abs(o.h.sum() - m0) / m0 < 1e-14
    assert abs(o.z.sum() - s0) / s0 < 1e-13
    assert np.max(np.abs(o.z - zb)) > 1e-6


def two_cell_fluxes(params, left, right):
    """Interface results between two cells (free boundaries around them);
    returns the values at the middle interface."""
    h = np.array([left[0], right[0]])
    hu = np.array([left[0] * left[1], right[0] * right[1]])
    z = np.array([left[2], right[2]])
    r = fluxes_1d(h, hu, z, params, FREE1)
    return r, 1


def test_lake_over_a_bed_step_hand_values():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "lake_at_rest_step_flux.json")
    for c in json.load(open(path))["cases"]:
        L, R = c["left"], c["right"]
        r, k = two_cell_fluxes(wb(grass(Ag=0.0)), (L["h"], 0.0, L["z"]), (R["h"], 0.0, R["z"]))
        assert abs(r.FhuL[k] - c["expected"]["FhuL"]) < 1e-12
        assert abs(r.FhuR[k] - c["expected"]["FhuR"]) < 1e-12
        assert abs(r.Fh[k]) < 1e-14 and r.Fz[k] == 0.0


def test_reconstruction_lowering_the_left_depth_hand_value():
    # left (h 2, u 0.3, z 0), right (h 1, u 0.5, z 0.5): z* = 0.5, the left
    # depth is reconstructed to 1.5, the right one stays 1.  Without bedload
    # the interface problem is the Suliciu problem between (1.5, 0.3) and
    # (1, 0.5) on a flat bed; the left cell also sees g/2 (2^2 - 1.5^2).
    r, k = two_cell_fluxes(wb(grass(Ag=0.0)), (2.0, 0.3, 0.0), (1.0, 0.5, 0.5))
    mk = lambda h, u: O.CellState(h=np.array([h]), tau=np.array([1 / h]), un=np.array([u]),
                                  ut=np.zeros(1), Pi=np.array([0.5 * G * h * h]),
                                  z=np.zeros(1), q=np.zeros(1), b2=np.array([(h * u) ** 2]),
                                  aK=np.array([h * np.sqrt(G * h)]))
    Fh, Fm = suliciu_textbook(mk(1.5, 0.3), mk(1.0, 0.5), r.a[k], G)
    assert r.Fh[k] == pytest.approx(Fh[0], rel=1e-13)
    assert r.FhuL[k] == pytest.approx(Fm[0] + 0.5 * G * (4.0 - 2.25), rel=1e-13)
    assert r.FhuR[k] == pytest.approx(Fm[0], rel=1e-13)
    assert r.Fz[k] == 0.0


def test_variant_and_paper_scheme_converge_to_the_same_solution():
    # smooth periodic bed, both schemes to the same time: their difference
    # shrinks about linearly with dx (both are first order)
    T = 20.0
    diffs = []
    for n in (100, 200, 400):
        h, hu, z, dx = W.smooth_periodic1d(n, amp=0.2)
        p = grass(Ag=5e-3)
        a = O.Oracle1D(h, hu, z, dx, p, PER1)
        b = O.Oracle1D(h, hu, z, dx, wb(p), PER1)
        a.step(100000, 0.5, T)
        b.step(100000, 0.5, T)
        diffs.append(max(np.max(np.abs(a.h - b.h)), np.max(np.abs(a.z - b.z))))
    assert diffs[0] / diffs[1] > 1.6 and diffs[1] / diffs[2] > 1.6, diffs


def test_paper_dune_downstream_and_antidune_upstream():
    h, hu, zb, dx = W.dune1d(1000)
    o = O.Oracle1D(h, hu, zb, dx, wb(grass(Ag=1.0)), PER1)
    x = W.cell_centres(1000, 1000.0)
    o.step(100000, 0.5, 100.0)
    assert x[np.argmax(o.z)] > x[np.argmax(zb)] + 5.0
    h, hu, zb, dx = W.antidune1d(1200)
    o = O.Oracle1D(h, hu, zb, dx, wb(grass(Ag=1e-3)),
                   (O.BC(O.BC_INFLOW, 0.5, 1.7, 0.0), O.BC(O.BC_FREE)))
    x = W.cell_centres(1200, 24.0)
    o.step(100000, 0.5, 10.0)
    assert x[np.argmax(o.z)] < x[np.argmax(zb)] - 0.5


# ----------------------------------------------------------------------------
# planted mistakes in the reconstruction
# ----------------------------------------------------------------------------
SRC = open(os.path.join(os.path.dirname(S0.__file__), "scheme.py")).read()
MUTATIONS = [
    ("zs = _max(zL, zR)", "zs = -_max(-zL, -zR)"),
    ("res.FhuL = res.FhuL + 0.5 * p.g * (hL * hL - hLs * hLs)",
     "res.FhuL = res.FhuL + 0.5 * p.g * (hR * hR - hRs * hRs)"),
    ("res.FhuR = res.FhuR + 0.5 * p.g * (hR * hR - hRs * hRs)",
     "res.FhuR = res.FhuR - 0.5 * p.g * (hR * hR - hRs * hRs)"),
    ("fields = dict(h=hs, hu=hs * u, hv=hs * v, z=zs)",
     "fields = dict(h=hs, hu=Pd[\"hu\"][sl], hv=Pd[\"hv\"][sl], z=zs)"),
    ("fields = dict(h=hs, hu=hs * u, hv=hs * v, z=zs)",
     "fields = dict(h=hs, hu=hs * u, hv=hs * v, z=Pd[\"z\"][sl])"),
    ("hLs = _max(hL + zL - zs, 0.0 * hL)", "hLs = _max(hL - zs, 0.0 * hL)"),
]


def load_variant(old, new):
    assert SRC.count(old) == 1, old
    name = "oracle.scheme_wb_mutant"
    mod = types.ModuleType(name)
    mod.__package__ = "oracle"
    sys.modules[name] = mod
    try:
        exec(compile(SRC.replace(old, new), "scheme_wb_mutant.py", "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def pins_hold(S):
    with np.errstate(all="ignore"):
        try:
            # lake at rest, 1D, m_g = 1
            h, z, dx = lake1d(80)
            o = S.Oracle1D(h, 0 * h, z, dx, wb(grass(mg=1.0)), FREE1)
            o.step(100, 0.5)
            if not (np.max(np.abs(o.hu)) < 1e-11 and np.max(np.abs(o.z - z)) < 1e-13):
                return False
            # flat bed equals the paper's scheme
            hh, hu, hv, zb, dx, dy = W.dune2d(30, 24)
            zf = np.full_like(zb, 0.3)
            a = S.Oracle2D(hh, hu, 0.2 * zb, zf, dx, dy, grass(Ag=0.0, mg=2.5), PER2)
            b = S.Oracle2D(hh, hu, 0.2 * zb, zf, dx, dy, wb(grass(Ag=0.0, mg=2.5)), PER2)
            a.step(10, 0.5)
            b.step(10, 0.5)
            if not all(np.max(np.abs(x - y)) <= 1e-13 * max(np.max(np.abs(y)), 1e-300)
                       for x, y in zip(a.state, b.state)):
                return False
            # hand value of the lowered left depth
            hs = np.array([2.0, 1.0])
            r = S.fluxes_1d(hs, hs * np.array([0.3, 0.5]), np.array([0.0, 0.5]),
                            wb(grass(Ag=0.0)), FREE1)
            mk = lambda h, u: O.CellState(h=np.array([h]), tau=np.array([1 / h]),
                                          un=np.array([u]), ut=np.zeros(1),
                                          Pi=np.array([0.5 * G * h * h]), z=np.zeros(1),
                                          q=np.zeros(1), b2=np.array([(h * u) ** 2]),
                                          aK=np.array([h * np.sqrt(G * h)]))
            Fh, Fm = suliciu_textbook(mk(1.5, 0.3), mk(1.0, 0.5), r.a[1], G)
            if not (abs(r.FhuL[1] - Fm[0] - 0.5 * G * 1.75) < 1e-12 * abs(Fm[0])
                    and abs(r.FhuR[1] - Fm[0]) < 1e-12 * abs(Fm[0])
                    and abs(r.Fh[1] - Fh[0]) < 1e-12 * abs(Fh[0])):
                return False
        except (S.OracleError, FloatingPointError, ValueError):
            return False
    return True


def test_unmutated_variant_passes_the_pins():
    assert pins_hold(S0)


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_mutant_fails_a_pin(old, new):
    assert not pins_hold(load_variant(old, new))
