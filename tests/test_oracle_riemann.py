"""Pins of the oracle's interface solver against what the relaxation system
fixes independently of the closed form:
  * the raw jump conditions of the five waves (eqs. "relaxh" ... "relaxqs"
    with the straight-path non-conservative product), solved from scratch
    by a 50-digit Newton iteration;
  * the textbook Suliciu solver of the shallow-water system, which the
    fluid part reduces to on a flat bed without bedload (first remark after
    eq. "relaxqs");
  * hand-derived fluxes for uniform flow and for a lake at rest over a bed
    step (fixtures under tests/golden/).
"""
import json
import os

import mpmath as mp
import numpy as np
import pytest

import oracle as O
from oracle.riemann import CellState, interface_solve

G = 9.81
HERE = os.path.dirname(os.path.abspath(__file__))


def random_sides(rng, n, flat=False, no_sed=False):
    def side():
        h = rng.uniform(0.2, 10.0, n)
        u = rng.uniform(-4.0, 4.0, n)
        v = rng.uniform(-1.0, 1.0, n)
        z = np.zeros(n) if flat else rng.uniform(-0.5, 0.5, n)
        q = np.zeros(n) if no_sed else rng.uniform(-0.2, 0.2, n)
        beta = np.zeros(n) if no_sed else rng.uniform(0.0, 0.05, n)
        hu = h * u
        return CellState(h=h, tau=1.0 / h, un=u, ut=v, Pi=0.5 * G * h * h, z=z,
                         q=q, b2=hu * hu + G * h * h * beta,
                         aK=h * np.sqrt(G * h))
    return side(), side()


def jump_residuals(x, L, R, a, b, g, Hbar):
    """The 25 raw conditions for unknowns x = [W1, W2, W3, W4 (each tau, u,
    Pi, Z, Omega), sigma1..sigma5], in mpmath."""
    W = [(L["tau"], L["u"], L["Pi"], L["z"], L["q"])]
    for m in range(4):
        W.append(tuple(x[5 * m:5 * m + 5]))
    W.append((R["tau"], R["u"], R["Pi"], R["z"], R["q"]))
    sig = x[20:25]
    jval = [a, b, 0, -b, -a]
    res = []
    for m in range(5):
        tm, um, pm, zm, om = W[m]
        tp, up, pp, zp, op = W[m + 1]
        s = sig[m]
        Hm, Hp = 1 / tm, 1 / tp
        res.append(Hm * (um - s) - jval[m])                       # mass flux
        res.append(Hm * (um - s) - Hp * (up - s))                 # mass RH
        res.append(-s * (Hp * up - Hm * um)
                   + (Hp * up * up + pp) - (Hm * um * um + pm)
                   + g * Hbar * (zp - zm))                        # momentum RH
        res.append(-s * (zp - zm) + (op - om))                    # Exner RH
        if m in (1, 3):
            res.append(-s * (Hp * pp - Hm * pm)
                       + (Hp * pp * up + a * a * up) - (Hm * pm * um + a * a * um))
        else:
            res.append(zp - zm)                                   # no bed jump
    return res


def newton_mp(f, x0, tol=mp.mpf("1e-40"), maxit=30):
    x = mp.matrix(x0)
    n = len(x0)
    for _ in range(maxit):
        F = mp.matrix(f(x))
        if mp.norm(F) < tol:
            break
        J = mp.matrix(n, n)
        hstep = mp.mpf("1e-25")
        for j in range(n):
            xp = x.copy()
            xp[j] += hstep
            xm = x.copy()
            xm[j] -= hstep
            Fp = f(xp)
            Fm = f(xm)
            for i in range(n):
                J[i, j] = (Fp[i] - Fm[i]) / (2 * hstep)
        x = x - mp.lu_solve(J, F)
    return x


def _pick(side, i):
    return {k: float(getattr(side, k)[i]) for k in ("h", "tau", "un", "Pi", "z", "q")}


def test_closed_form_satisfies_raw_jump_conditions_float64():
    rng = np.random.default_rng(11)
    L, R = random_sides(rng, 4000)
    r = interface_solve(L, R, G)
    assert not np.any(r.err)
    Hbar = 0.5 * (L.h + R.h)
    x = []
    for W in r.states:
        x.extend(W)
    x.extend(r.sigma)
    Ld = dict(tau=L.tau, u=L.un, Pi=L.Pi, z=L.z, q=L.q)
    Rd = dict(tau=R.tau, u=R.un, Pi=R.Pi, z=R.z, q=R.q)
    res = jump_residuals(x, Ld, Rd, r.a, r.b, G, Hbar)
    # scale of each equation: momentum-like terms ~ a^2 tau, mass ~ a
    scale_m = r.a * r.a * np.maximum(L.tau, R.tau) + 1.0
    for i, e in enumerate(res):
        sc = scale_m if (i % 5) in (2, 4) else (r.a + 1.0)
        assert np.max(np.abs(e) / sc) < 5e-13, i


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_closed_form_matches_50_digit_newton_solve(seed):
    mp.mp.dps = 50
    rng = np.random.default_rng(100 + seed)
    L, R = random_sides(rng, 6)
    r = interface_solve(L, R, G)
    for i in range(6):
        Ld = {k: mp.mpf(v) for k, v in _pick(L, i).items()}
        Rd = {k: mp.mpf(v) for k, v in _pick(R, i).items()}
        Ld["u"], Rd["u"] = Ld.pop("un"), Rd.pop("un")
        a = mp.mpf(float(r.a[i]))
        b = mp.mpf(float(r.b[i]))
        Hbar = (1 / Ld["tau"] + 1 / Rd["tau"]) / 2
        x_cf = []
        for W in r.states:
            x_cf.extend(float(c[i]) if np.ndim(c) else float(c) for c in W)
        x_cf.extend(float(s[i]) for s in r.sigma)
        # start 0.1 % away from the closed form and converge independently
        x0 = [mp.mpf(v) * (1 + mp.mpf(float(rng.uniform(-1e-3, 1e-3))))
              + mp.mpf(float(rng.uniform(-1e-4, 1e-4))) for v in x_cf]
        sol = newton_mp(lambda x: jump_residuals(list(x), Ld, Rd, a, b, G, Hbar), x0)
        assert mp.norm(mp.matrix(jump_residuals(list(sol), Ld, Rd, a, b, G, Hbar))) < 1e-30
        for k, v in enumerate(x_cf):
            ref = float(sol[k])
            assert abs(v - ref) <= 1e-12 * max(1.0, abs(ref)), (i, k, v, ref)


def suliciu_textbook(L, R, a, g):
    """Three-wave Suliciu relaxation solver for shallow water (flat bed),
    written from its textbook form: u* and Pi* from the two outer Riemann
    invariants u -/+ a tau ... Pi +/- a u, tau* from u* on each side."""
    us = 0.5 * (L.un + R.un) - (R.Pi - L.Pi) / (2 * a)
    Ps = 0.5 * (L.Pi + R.Pi) - 0.5 * a * (R.un - L.un)
    tLs = L.tau + (us - L.un) / a
    tRs = R.tau - (us - R.un) / a
    s1 = L.un - a * L.tau
    s3 = R.un + a * R.tau
    tau0 = np.where(s1 >= 0, L.tau, np.where(us >= 0, tLs, np.where(s3 > 0, tRs, R.tau)))
    u0 = np.where(s1 >= 0, L.un, np.where(s3 > 0, us, R.un))
    P0 = np.where(s1 >= 0, L.Pi, np.where(s3 > 0, Ps, R.Pi))
    Fh = u0 / tau0
    return Fh, Fh * u0 + P0


def test_flat_bed_no_bedload_reduces_to_suliciu():
    rng = np.random.default_rng(5)
    L, R = random_sides(rng, 3000, flat=True, no_sed=True)
    r = interface_solve(L, R, G)
    Fh, Fm = suliciu_textbook(L, R, r.a, G)
    assert np.allclose(r.Fh, Fh, rtol=1e-13, atol=1e-12)
    assert np.allclose(r.FhuL, Fm, rtol=1e-13, atol=1e-11)
    assert np.allclose(r.FhuR, Fm, rtol=1e-13, atol=1e-11)
    assert np.max(np.abs(r.Fz)) == 0.0


def test_left_and_right_chains_agree():
    rng = np.random.default_rng(9)
    L, R = random_sides(rng, 3000)
    r = interface_solve(L, R, G)
    (t1, u1, P1, Z1, O1), (t2, us, Ps, Zs, Os), (t3, _, _, _, _), (t4, u4, P4, _, _) = r.states
    s1, s2, s3, s4, s5 = r.sigma
    # u* from the right chain: sigma4 - b tau3
    assert np.allclose(us, s4 - r.b * t3, rtol=0, atol=1e-12 * np.max(np.abs(us)) + 1e-12)
    # Exner relation across the right sediment wave
    dz = R.z - Zs
    assert np.allclose(R.q - Os, s4 * dz, rtol=0, atol=1e-13)
    assert np.all(s1 < s2) and np.all(s2 < s3) and np.all(s3 < s4) and np.all(s4 < s5)


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def _side_from(d, beta=0.0, q=0.0):
    h = np.array([d["h"]])
    u = np.array([d["hu"] / d["h"]])
    return CellState(h=h, tau=1.0 / h, un=u, ut=np.zeros(1), Pi=0.5 * G * h * h,
                     z=np.array([d["z"]]), q=np.array([q]),
                     b2=(h * u) ** 2 + G * h * h * beta, aK=h * np.sqrt(G * h))


def test_golden_uniform_flow_flux():
    gdat = _golden("uniform_flow_flux.json")
    for case in gdat["cases"]:
        L = _side_from(case["state"], beta=case["beta"], q=case["q"])
        R = _side_from(case["state"], beta=case["beta"], q=case["q"])
        r = interface_solve(L, R, G)
        exp = case["expected"]
        assert r.Fh[0] == pytest.approx(exp["Fh"], rel=1e-14)
        assert r.FhuL[0] == pytest.approx(exp["Fhu"], rel=1e-14)
        assert r.FhuR[0] == pytest.approx(exp["Fhu"], rel=1e-14)
        assert r.Fz[0] == pytest.approx(exp["Fz"], rel=1e-14, abs=1e-300)


def test_golden_lake_at_rest_bed_step_flux():
    gdat = _golden("lake_at_rest_step_flux.json")
    for case in gdat["cases"]:
        L = _side_from(case["left"])
        R = _side_from(case["right"])
        r = interface_solve(L, R, G)
        exp = case["expected"]
        assert abs(r.Fh[0]) < 1e-12
        assert r.FhuL[0] == pytest.approx(exp["FhuL"], rel=1e-13)
        assert r.FhuR[0] == pytest.approx(exp["FhuR"], rel=1e-13)
        assert abs(r.Fz[0]) < 1e-12


def test_celerities_satisfy_subcharacteristic_bounds():
    # eq. "ab": a >= H sqrt(g H) and b >= sqrt((Hu)^2 + g H^2 d_u Q_s) on
    # both sides of the interface; a > b keeps the five waves ordered
    rng = np.random.default_rng(21)
    L, R = random_sides(rng, 5000)
    r = interface_solve(L, R, G)
    for S in (L, R):
        assert np.all(r.a >= S.h * np.sqrt(G * S.h) * (1 - 1e-15))
        assert np.all(r.b * r.b >= S.b2 * (1 - 1e-15))
    assert np.all(r.a > r.b)


def mirror(S):
    return CellState(h=S.h, tau=S.tau, un=-S.un, ut=S.ut, Pi=S.Pi, z=S.z,
                     q=-S.q, b2=S.b2, aK=S.aK)


def test_mirror_symmetry_of_interface_fluxes():
    rng = np.random.default_rng(22)
    L, R = random_sides(rng, 3000)
    r = interface_solve(L, R, G)
    m = interface_solve(mirror(R), mirror(L), G)
    sc = np.max(np.abs(r.FhuL))
    assert np.allclose(m.Fh, -r.Fh, rtol=1e-12, atol=1e-12 * sc)
    assert np.allclose(m.FhuL, r.FhuR, rtol=1e-12, atol=1e-12 * sc)
    assert np.allclose(m.FhuR, r.FhuL, rtol=1e-12, atol=1e-12 * sc)
    assert np.allclose(m.Fz, -r.Fz, rtol=1e-11, atol=1e-13)
    assert np.allclose(m.Fht, -r.Fht, rtol=1e-12, atol=1e-12 * sc)
