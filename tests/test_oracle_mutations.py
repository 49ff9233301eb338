"""The pins are strong enough: each plausible slip in the oracle's interface
solver (a dropped term, a flipped sign, a wrong index or side) planted in a
copy of the oracle on the CPU makes at least one pin fail.

Checks run on each mutant (all independent of the closed form itself):
raw jump conditions of the five waves, the sub-characteristic bounds of
eq. "ab", the hand-derived lake-at-rest fluxes and the mirror symmetry.
"""
import os
import sys
import types

import numpy as np
import pytest

import oracle.riemann as R0

G = 9.81
SRC = open(os.path.join(os.path.dirname(R0.__file__), "riemann.py")).read()

MUTATIONS = [
    ("T0 = (AR - AL - a * D - c * kappa * dZ)", "T0 = (AR - AL - a * D + c * kappa * dZ)"),
    ("kappa = Hbar * (tmin * tmin * tmin)", "kappa = Hbar * (tmin * tmin)"),
    ("s4 = AR - c * (T0 + D + kappa * dZ)", "s4 = AR - c * (T0 + D - kappa * dZ)"),
    ("C = dO - 0.5 * (s4p + s2p) * dZ", "C = dO + 0.5 * (s4p + s2p) * dZ"),
    ("zeta = -2.0 * C / _where_pos(den_ok, den) + 0.5 * dZ",
     "zeta = -2.0 * C / _where_pos(den_ok, den) - 0.5 * dZ"),
    ("tau1 = T0 - (b * kappa / a) * zeta", "tau1 = T0 + (b * kappa / a) * zeta"),
    ("Os = L.q + sig2 * zeta", "Os = L.q + us * zeta"),
    ("FhuL = P0 + g * Hbar * (Z0 - L.z)", "FhuL = P0 + g * Hbar * (Z0 - R.z)"),
    ("FhuR = P0 + g * Hbar * (Z0 - R.z)", "FhuR = P0 + g * Hbar * (Z0 - L.z)"),
    ("D = (PR - PL) / a2", "D = (PL - PR) / a2"),
    ("c = af2 / (a + b)", "c = af2 / (a + b + b)"),
    ("b2 = _max(_max(L.b2, R.b2)", "b2 = _max(_min(L.b2, R.b2)"),
    ("u_est = 0.5 * (L.un + R.un) - (R.Pi - L.Pi + g * Hbar * dZ)",
     "u_est = 0.5 * (L.un + R.un) - (R.Pi - L.Pi - g * Hbar * dZ)"),
    ("af2 = g * (hmax * hmax * hmax)", "af2 = g * (hmax * hmax)"),
    ("vt0 = np.where(k <= 2, L.ut, R.ut)", "vt0 = np.where(k <= 1, L.ut, R.ut)"),
    ("u4 = AR - a * tau4", "u4 = AR + a * tau4"),
    ("Pi4 = PR - a2 * tau4", "Pi4 = PL - a2 * tau4"),
    ("P0 = u0 * Fh + Pi0", "P0 = u0 * Fh"),
    ("s2p = s2 - 0.5 * eps * dZ", "s2p = s2 + 0.5 * eps * dZ"),
    ("disc = B * B - 8.0 * eps * C", "disc = B * B - 4.0 * eps * C"),
]


def load_variant(old, new):
    assert SRC.count(old) == 1, old
    name = "oracle_riemann_mutant"
    mod = types.ModuleType(name)
    sys.modules[name] = mod          # dataclasses look the module up
    try:
        exec(compile(SRC.replace(old, new), "riemann_mutant.py", "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def sides(R, rng, n):
    def side():
        h = rng.uniform(0.2, 10.0, n)
        u = rng.uniform(-4.0, 4.0, n)
        hu = h * u
        beta = rng.uniform(0.0, 0.05, n)
        return R.CellState(h=h, tau=1.0 / h, un=u, ut=rng.uniform(-1, 1, n),
                           Pi=0.5 * G * h * h, z=rng.uniform(-0.5, 0.5, n),
                           q=rng.uniform(-0.2, 0.2, n),
                           b2=hu * hu + G * h * h * beta, aK=h * np.sqrt(G * h))
    return side(), side()


def pins_hold(R):
    """True when every pin holds for the interface solver module R."""
    rng = np.random.default_rng(7)
    L, Rt = sides(R, rng, 400)
    with np.errstate(all="ignore"):
        r = R.interface_solve(L, Rt, G)
        if np.any(r.err):
            return False
        # raw jump conditions
        W = [(L.tau, L.un, L.Pi, L.z, L.q)] + list(r.states) + [(Rt.tau, Rt.un, Rt.Pi, Rt.z, Rt.q)]
        Hbar = 0.5 * (L.h + Rt.h)
        jv = [r.a, r.b, 0.0, -r.b, -r.a]
        for m in range(5):
            tm, um, pm, zm, om = W[m]
            tp, up, pp, zp, op = W[m + 1]
            s = r.sigma[m]
            Hm, Hp = 1 / tm, 1 / tp
            sc = r.a * r.a * (tm + tp) + 1.0
            eqs = [Hm * (um - s) - jv[m], Hm * (um - s) - Hp * (up - s),
                   (-s * (Hp * up - Hm * um) + (Hp * up * up + pp)
                    - (Hm * um * um + pm) + G * Hbar * (zp - zm)) / sc,
                   -s * (zp - zm) + (op - om)]
            if m in (1, 3):
                eqs.append((-s * (Hp * pp - Hm * pm) + Hp * pp * up + r.a ** 2 * up
                            - Hm * pm * um - r.a ** 2 * um) / (sc * r.a))
            else:
                eqs.append(zp - zm)
            for e in eqs:
                if not np.all(np.abs(e) < 1e-10 * (r.a + 1.0)):
                    return False
        # eq. "ab"
        for S in (L, Rt):
            if not (np.all(r.a >= S.h * np.sqrt(G * S.h) * (1 - 1e-15))
                    and np.all(r.b * r.b >= S.b2 * (1 - 1e-15))):
                return False
        # lake at rest over a step: F_hu^L = g h_L^2/2, F_hu^R = g h_R^2/2
        hl, hr = np.array([3.0]), np.array([3.25])
        mk = lambda h, z: R.CellState(h=h, tau=1 / h, un=0 * h, ut=0 * h,
                                      Pi=0.5 * G * h * h, z=np.array([z]),
                                      q=0 * h, b2=0 * h, aK=h * np.sqrt(G * h))
        rl = R.interface_solve(mk(hl, 0.5), mk(hr, 0.25), G)
        if not (abs(rl.FhuL[0] - 44.145) < 1e-11 and abs(rl.FhuR[0] - 51.8090625) < 1e-11
                and abs(rl.Fz[0]) < 1e-12 and abs(rl.Fh[0]) < 1e-12):
            return False
        # mirror symmetry
        mir = lambda S: R.CellState(h=S.h, tau=S.tau, un=-S.un, ut=S.ut, Pi=S.Pi,
                                    z=S.z, q=-S.q, b2=S.b2, aK=S.aK)
        m = R.interface_solve(mir(Rt), mir(L), G)
        sc = np.max(np.abs(r.FhuL))
        for x, y in ((m.Fh, -r.Fh), (m.FhuL, r.FhuR), (m.FhuR, r.FhuL),
                     (m.Fz, -r.Fz), (m.Fht, -r.Fht)):
            if not np.allclose(x, y, rtol=1e-11, atol=1e-11 * sc):
                return False
    return True


def test_unmutated_oracle_passes_the_pins():
    assert pins_hold(R0)


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_mutant_fails_a_pin(old, new):
    assert not pins_hold(load_variant(old, new))
