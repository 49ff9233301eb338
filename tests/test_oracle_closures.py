"""Pins of the oracle's bedload closures against what the paper fixes:
  * A_g = 0 gives no transport (remark after eq. "bedload Grass");
  * hand values of the Grass law and of the threshold laws (eqs. "MPM" ...
    "Camenen") at inputs chosen so that the values are exact;
  * the printed Jacobian identities alpha = -u beta (Darcy-Weisbach) and
    alpha = -(7/6) u beta (Manning), alpha = dq_b/dh, beta = dq_b/d(hu)
    (section "Bedload modelling", quasi-linear form), evaluated by complex
    step on q_b(h, hu);
  * beta = dq/du against central differences of q (eq. "ab" uses it);
  * no transport below the threshold, continuity at the threshold.
"""
import numpy as np
import pytest

import oracle as O
from oracle.closures import closure, Params


def test_grass_zero_interaction_means_no_transport():
    p = Params(law=O.LAW_GRASS, A_g=0.0, m_g=3.0)
    u = np.linspace(-3, 3, 11)
    qx, qy, bx, by = closure(np.ones_like(u), u, 0.5 * u, p)
    assert np.all(qx == 0) and np.all(qy == 0) and np.all(bx == 0) and np.all(by == 0)


def test_grass_hand_values():
    # q = A_g |U|^(m-1) (u, v); 1D: A_g u |u|^(m-1); beta = A_g m |u|^(m-1)
    p = Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0)
    qx, qy, bx, by = closure(np.array([1.0]), np.array([2.0]), np.array([0.0]), p)
    assert qx[0] == pytest.approx(8e-3, rel=1e-15)
    assert bx[0] == pytest.approx(12e-3, rel=1e-15)
    qx, qy, bx, by = closure(np.array([1.0]), np.array([1.0]), np.array([2.0]), p)
    assert (qx[0], qy[0]) == (pytest.approx(5e-3), pytest.approx(1e-2))
    assert (bx[0], by[0]) == (pytest.approx(7e-3), pytest.approx(13e-3))
    p2 = Params(law=O.LAW_GRASS, A_g=2.0, m_g=2.0)
    qx, _, bx, _ = closure(np.array([1.0]), np.array([-3.0]), np.array([0.0]), p2)
    assert qx[0] == pytest.approx(-18.0, rel=1e-15)       # 2 * (-3) * 3
    assert bx[0] == pytest.approx(12.0, rel=1e-15)        # 2 * 2 * 3
    p1 = Params(law=O.LAW_GRASS, A_g=0.5, m_g=1.0)
    qx, _, bx, _ = closure(np.array([1.0]), np.array([0.0]), np.array([0.0]), p1)
    assert qx[0] == 0.0 and bx[0] == 0.5


def _unit_threshold_params(law):
    # g = 1, s = 2, d = 1  =>  sqrt((s-1) g d^3) = 1; Darcy: tau* = f u^2 / 8
    return Params(law=law, g=1.0, s=2.0, d_s=1.0, tau_cr=0.05,
                  friction=O.FRIC_DARCY, fric_coef=2.4)


@pytest.mark.parametrize("law,expected", [
    (O.LAW_MPM, 8.0 * 0.125),           # 8 (0.3 - 0.05)^(3/2)
    (O.LAW_FLVB, 5.7 * 0.125),          # 5.7 (0.25)^(3/2)
    (O.LAW_NIELSEN, 12.0 * np.sqrt(0.3) * 0.25),
    (O.LAW_RIBBERINK, 11.0 * 0.25 ** 1.65),
    (O.LAW_CAMENEN, 12.0 * 0.3 ** 1.5 * np.exp(-4.5 * 0.05 / 0.3)),
])
def test_threshold_laws_hand_values(law, expected):
    # f = 2.4, u = 1  =>  tau* = 2.4 / 8 = 0.3
    p = _unit_threshold_params(law)
    qx, qy, _, _ = closure(np.array([1.7]), np.array([1.0]), np.array([0.0]), p)
    assert qx[0] == pytest.approx(expected, rel=1e-14)
    assert qy[0] == 0.0
    # direction follows U
    qx, qy, _, _ = closure(np.array([1.7]), np.array([0.6]), np.array([-0.8]), p)
    assert qx[0] == pytest.approx(0.6 * expected, rel=1e-14)
    assert qy[0] == pytest.approx(-0.8 * expected, rel=1e-14)


def test_strickler_shields_number_hand_value():
    # Strickler: tau* = |U|^2 / ((s-1) d K_s^2 h^(1/3)); pick h = 8, K_s = 1,
    # (s-1) d = 1 => tau* = u^2 / 2; u = 1 => tau* = 0.5, MPM q* = 8 * 0.45^1.5
    p = Params(law=O.LAW_MPM, g=1.0, s=2.0, d_s=1.0, tau_cr=0.05,
               friction=O.FRIC_STRICKLER, fric_coef=1.0)
    qx, _, _, _ = closure(np.array([8.0]), np.array([1.0]), np.array([0.0]), p)
    assert qx[0] == pytest.approx(8.0 * 0.45 ** 1.5, rel=1e-14)
    pm = Params(law=O.LAW_MPM, g=1.0, s=2.0, d_s=1.0, tau_cr=0.05,
                friction=O.FRIC_MANNING, fric_coef=1.0)
    qm, _, _, _ = closure(np.array([8.0]), np.array([1.0]), np.array([0.0]), pm)
    assert qm[0] == pytest.approx(qx[0], rel=1e-14)   # n = 1/K_s


@pytest.mark.parametrize("law", [O.LAW_MPM, O.LAW_FLVB, O.LAW_NIELSEN,
                                 O.LAW_RIBBERINK, O.LAW_CAMENEN])
def test_no_transport_below_threshold_and_continuity(law):
    p = _unit_threshold_params(law)
    # tau* = 2.4 u^2 / 8 = 0.3 u^2 ; threshold 0.05 at u0 = sqrt(1/6)
    u0 = np.sqrt(0.05 / 0.3)
    if law != O.LAW_CAMENEN:
        q, _, b, _ = closure(np.ones(3), np.array([0.0, 0.5 * u0, 0.999 * u0]),
                             np.zeros(3), p)
        assert np.all(q == 0.0) and np.all(b == 0.0)
    q, _, _, _ = closure(np.ones(2), np.array([u0 * (1 + 1e-9), u0 * (1 - 1e-9)]),
                         np.zeros(2), p)
    assert abs(q[0] - q[1]) < 1e-6


def _complex_step(f, x, h=1e-30):
    return np.imag(f(x + 1j * h)) / h


@pytest.mark.parametrize("friction,ratio", [(O.FRIC_DARCY, -1.0),
                                            (O.FRIC_MANNING, -7.0 / 6.0),
                                            (O.FRIC_STRICKLER, -7.0 / 6.0)])
@pytest.mark.parametrize("law", [O.LAW_MPM, O.LAW_FLVB, O.LAW_NIELSEN,
                                 O.LAW_RIBBERINK, O.LAW_CAMENEN])
def test_alpha_beta_identities(law, friction, ratio):
    coef = {O.FRIC_DARCY: 0.05, O.FRIC_MANNING: 0.03, O.FRIC_STRICKLER: 40.0}[friction]
    p = Params(law=law, friction=friction, fric_coef=coef, d_s=1e-3, s=2.65)
    h = np.array([0.4, 1.0, 2.5])
    hu = np.array([1.5, 3.0, -6.0])

    def q_of(hh, qq):
        return closure(hh, qq / hh, np.zeros_like(hh), p)[0]

    alpha = _complex_step(lambda x: q_of(x, hu.astype(complex)), h.astype(complex))
    beta = _complex_step(lambda x: q_of(h.astype(complex), x), hu.astype(complex))
    u = hu / h
    assert np.all(np.abs(beta) > 0)
    assert np.allclose(alpha / (u * beta), ratio, rtol=1e-12)


def test_grass_alpha_beta_identity():
    # q_b depends on u only, as for Darcy-Weisbach: alpha = -u beta
    p = Params(law=O.LAW_GRASS, A_g=0.7, m_g=2.5)
    h = np.array([0.4, 1.0, 2.5])
    hu = np.array([1.5, 3.0, -6.0])

    def q_of(hh, qq):
        return closure(hh, qq / hh, np.zeros_like(hh), p)[0]

    alpha = _complex_step(lambda x: q_of(x, hu.astype(complex)), h.astype(complex))
    beta = _complex_step(lambda x: q_of(h.astype(complex), x), hu.astype(complex))
    assert np.allclose(alpha / ((hu / h) * beta), -1.0, rtol=1e-12)


# the exponent m_g only enters the Grass law
@pytest.mark.parametrize("law,mg", [(O.LAW_GRASS, mg) for mg in (1.0, 1.7, 3.0, 4.0)]
                         + [(law, 3.0) for law in (O.LAW_MPM, O.LAW_FLVB, O.LAW_NIELSEN,
                                                   O.LAW_RIBBERINK, O.LAW_CAMENEN)])
def test_beta_is_normal_derivative(law, mg):
    p = Params(law=law, A_g=2e-3, m_g=mg, friction=O.FRIC_STRICKLER,
               fric_coef=40.0)
    rng = np.random.default_rng(3)
    h = rng.uniform(0.3, 3.0, 50)
    u = rng.uniform(-4, 4, 50)
    v = rng.uniform(-4, 4, 50)
    eps = 1e-6
    qxp = closure(h, u + eps, v, p)[0]
    qxm = closure(h, u - eps, v, p)[0]
    qyp = closure(h, u, v + eps, p)[1]
    qym = closure(h, u, v - eps, p)[1]
    _, _, bx, by = closure(h, u, v, p)
    assert np.allclose(bx, (qxp - qxm) / (2 * eps), rtol=1e-6, atol=1e-12)
    assert np.allclose(by, (qyp - qym) / (2 * eps), rtol=1e-6, atol=1e-12)
    assert np.all(bx >= 0) and np.all(by >= 0)
