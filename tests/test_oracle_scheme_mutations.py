"""The pins of the oracle's time step are strong enough: each plausible slip
in ``oracle/scheme.py`` (the time-step rule pairing a direction's speed with
the other direction's spacing, a spacing swapped in the update, the
non-conservative momentum fluctuations of one direction swapped, a ghost
taken from the wrong side, the friction speed losing a component, the
Darcy coefficient off by g), planted in a copy of the module on the CPU,
makes at least one pin fail.

Pins run on each mutant, all independent of the scheme's own code:
  * the CFL time step of uniform flow on an anisotropic grid, from the
    celerities of eq. "ab" (hand value);
  * a y-uniform 2D run equals the 1D run (dx != dy);
  * transpose symmetry on a grid with dx != dy;
  * a lake at rest over a 2D bump stays at rest (free boundaries);
  * mirror symmetry with flow through free boundaries;
  * friction hand values (Darcy and Manning, 2D uniform flow).
"""
import os
import sys
import types

import numpy as np
import pytest

import oracle as O
import oracle.scheme as S0
import workloads as W

SRC = open(os.path.join(os.path.dirname(S0.__file__), "scheme.py")).read()

MUTATIONS = [
    ("return cfl / (Sx / dx + Sy / dy)", "return cfl / (Sx / dy + Sy / dx)"),
    ("    lx = dt / dx\n    ly = dt / dy\n    hn = h - lx",
     "    lx = dt / dy\n    ly = dt / dx\n    hn = h - lx"),
    ("- ly * (Y.FhuL[1:, :] - Y.FhuR[:-1, :])", "- ly * (Y.FhuR[1:, :] - Y.FhuL[:-1, :])"),
    ("    elif lo.kind == BC_FREE or field in (\"z\", \"Ag\"):\n        glo = first",
     "    elif lo.kind == BC_FREE or field in (\"z\", \"Ag\"):\n        glo = last"),
    ("speed = np.sqrt(un * un + vn * vn)", "speed = np.sqrt(un * un)"),
]

CLOSURE_SRC = open(os.path.join(os.path.dirname(S0.__file__), "closures.py")).read()
CLOSURE_MUTATIONS = [
    ("return p.fric_coef * speed / (8.0 * h)", "return p.fric_coef * speed / (8.0 * p.g * h)"),
    ("return p.g * n2 * speed / (h * _cbrt(h))", "return p.g * n2 * speed / (h * h)"),
]


def load_variant(src, old, new, modname):
    assert src.count(old) == 1, old
    name = "oracle." + modname + "_mutant"
    mod = types.ModuleType(name)
    mod.__package__ = "oracle"           # relative imports resolve in the oracle package
    sys.modules[name] = mod              # dataclasses look the module up
    try:
        exec(compile(src.replace(old, new), modname + "_mutant.py", "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def scheme_with_closures(cmod):
    """The unmodified scheme module bound to closure module `cmod`."""
    name = "oracle.scheme_cl_mutant"
    mod = types.ModuleType(name)
    mod.__package__ = "oracle"
    sys.modules[name] = mod
    saved = sys.modules["oracle.closures"]
    sys.modules["oracle.closures"] = cmod
    try:
        exec(compile(SRC, "scheme_cl_mutant.py", "exec"), mod.__dict__)
    finally:
        sys.modules["oracle.closures"] = saved
        del sys.modules[name]
    return mod, cmod


PER2 = (O.BC(),) * 4
PER1 = (O.BC(),) * 2


def pins_hold(S, C=None):
    C = C or O
    g = 9.81
    # CFL time step, uniform flow, flat bed, no bedload, dx != dy
    h0, u0, dx, dy = 4.0, 2.0, 1.0, 3.0
    h = np.full((9, 11), h0)
    o = S.Oracle2D(h, u0 * h, 0 * h, 0 * h, dx, dy, C.Params(law=C.LAW_GRASS, A_g=0.0), PER2)
    expected = 0.5 / ((u0 + np.sqrt(g * h0 + u0 * u0)) / dx + np.sqrt(g * h0) / dy)
    if abs(o.cfl_dt(0.5) - expected) > 1e-13 * expected:
        return False
    # y-uniform 2D equals 1D
    h1, hu1, z1, dx1 = W.dune1d(60, length=500.0)
    rep = lambda a: np.repeat(a[None, :], 4, axis=0)
    p = C.Params(law=C.LAW_GRASS, A_g=0.3, m_g=3.0)
    o2 = S.Oracle2D(rep(h1), rep(hu1), np.zeros((4, 60)), rep(z1), dx1, 3.0, p, PER2)
    o1 = S.Oracle1D(h1, hu1, z1, dx1, p, PER1)
    dt = 0.5 * o1.cfl_dt(1.0)
    o1.step_fixed_dt(10, dt)
    o2.step_fixed_dt(10, dt)
    for j in range(4):
        if not (np.allclose(o2.h[j], o1.h, rtol=1e-14, atol=0)
                and np.allclose(o2.hu[j], o1.hu, rtol=1e-14, atol=1e-14)):
            return False
    # transpose symmetry, dx != dy
    hh, hu, hv, zb, _, _ = W.dune2d(24, 20, lx=1000.0, ly=1000.0)
    hu = hu + 0.5 * zb
    hv = 1.5 * zb
    p = C.Params(law=C.LAW_GRASS, A_g=0.2, m_g=2.5)
    a = S.Oracle2D(hh, hu, hv, zb, 40.0, 55.0, p, PER2)
    b = S.Oracle2D(hh.T, hv.T, hu.T, zb.T, 55.0, 40.0, p, PER2)
    a.step(8, 0.5)
    b.step(8, 0.5)
    if not (abs(a.t - b.t) <= 1e-14 * a.t and np.allclose(a.h, b.h.T, rtol=1e-13, atol=0)
            and np.allclose(a.hu, b.hv.T, rtol=0, atol=1e-12)
            and np.allclose(a.hv, b.hu.T, rtol=0, atol=1e-12)):
        return False
    # lake at rest over an off-centre bump, free boundaries
    x = W.cell_centres(30, 100.0)
    y = W.cell_centres(24, 100.0)
    z = 0.4 * np.exp(-((x[None, :] - 30.0) ** 2 + (y[:, None] - 60.0) ** 2) / 150.0) \
        + 0.002 * x[None, :]
    hl = 2.0 - z
    o = S.Oracle2D(hl, 0 * hl, 0 * hl, z, 100.0 / 30, 100.0 / 24,
                   C.Params(law=C.LAW_GRASS, A_g=1e-3, m_g=3.0), (O.BC(O.BC_FREE),) * 4)
    o.step(50, 0.5)
    if not (np.max(np.abs(o.hu)) < 1e-12 and np.max(np.abs(o.hv)) < 1e-12
            and np.max(np.abs(o.h + o.z - 2.0)) < 1e-12):
        return False
    # mirror symmetry x -> -x with flow through free boundaries
    fb = (O.BC(O.BC_FREE),) * 4
    p = C.Params(law=C.LAW_GRASS, A_g=0.05, m_g=3.0)
    a = S.Oracle2D(hh, hu, hv, zb, 40.0, 55.0, p, fb)
    b = S.Oracle2D(hh[:, ::-1], -hu[:, ::-1], hv[:, ::-1], zb[:, ::-1], 40.0, 55.0, p, fb)
    a.step(8, 0.5)
    b.step(8, 0.5)
    if not (np.allclose(a.h, b.h[:, ::-1], rtol=1e-13, atol=0)
            and np.allclose(a.hu, -b.hu[:, ::-1], rtol=0, atol=1e-12)):
        return False
    # friction hand values (2D uniform flow, |U| = 0.5, h = 8)
    for fric, coef, phi in ((C.FRIC_DARCY, 0.1, 0.1 * 0.5 / 64.0),
                            (C.FRIC_MANNING, 0.5, g * 0.25 * 0.5 / 16.0)):
        pf = C.Params(law=C.LAW_GRASS, A_g=0.0, friction=fric, fric_coef=coef,
                      momentum_friction=1)
        hf = np.full((5, 6), 8.0)
        of = S.Oracle2D(hf, 0.3 * hf, 0.4 * hf, 0 * hf, 1.0, 2.0, pf, PER2)
        of.step_fixed_dt(1, 0.1)
        if not np.allclose(of.hu, 2.4 / (1.0 + 0.1 * phi), rtol=1e-15):
            return False
    return True


def test_unmutated_scheme_passes_the_pins():
    assert pins_hold(S0)


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_scheme_mutant_fails_a_pin(old, new):
    assert not pins_hold(load_variant(SRC, old, new, "scheme"))


@pytest.mark.parametrize("old,new", CLOSURE_MUTATIONS)
def test_friction_mutant_fails_a_pin(old, new):
    S, C = scheme_with_closures(load_variant(CLOSURE_SRC, old, new, "closures"))
    assert not pins_hold(S, C)
