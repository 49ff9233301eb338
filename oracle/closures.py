"""Bedload closures of the oracle (section "Bedload modelling").

Test infrastructure only (see the package docstring).

For a cell with depth h and velocity U = (u, v) a closure returns the
bedload flux vector q = (q_x, q_y) and the partial derivatives
beta_x = d q_x / d u (v held fixed) and beta_y = d q_y / d v (u held
fixed).  beta enters the sediment celerity bound of eq. "ab",
b >= sqrt((Hu)^2 + g H^2 d_u Q_s), applied along each interface normal.

Grass (eq. "bedload Grass"): q_b = A_g u |u|^(m_g - 1), 1 <= m_g <= 4, with
no threshold.  In 2D the isotropic form q = A_g |U|^(m_g-1) (u, v) is used
(the paper names a "2D Grass formula" without printing it); it reduces to
the 1D law for v = 0.

Threshold laws (eqs. "MPM", "FLVB", "Nielsen", "Ribberink", "Camenen"):
q_b = q* sqrt((s-1) g d^3) with q* a function of the Shields number
tau* = tau_b / ((rho_s - rho) g d), tau_b = rho g h S_f, and S_f from
  Darcy-Weisbach  S_f = f u|u| / (8 g h),
  Manning         S_f = n^2 u|u| / h^(4/3)   (Strickler: n = 1/K_s).
So tau* = c(h) |U|^2 with
  Strickler  c = 1 / ((s-1) d K_s^2 h^(1/3)),
  Manning    c = n^2 / ((s-1) d h^(1/3)),
  Darcy      c = f / (8 g (s-1) d).
The flux points along U: q = K F(tau*) U / |U|, K = sqrt((s-1) g d^3), hence
beta_x = K [F'(tau*) 2 c u^2 / |U| + F(tau*) v^2 / |U|^3].
The default threshold tau*_cr = 0.05 is the only value the paper prints
(caption of the figure of bedload functions).
"""
from __future__ import annotations

import dataclasses

import numpy as np

LAW_GRASS = 0
LAW_MPM = 1
LAW_FLVB = 2
LAW_NIELSEN = 3
LAW_RIBBERINK = 4
LAW_CAMENEN = 5

FRIC_STRICKLER = 0
FRIC_MANNING = 1
FRIC_DARCY = 2


@dataclasses.dataclass
class Params:
    """Physical parameters of the model (section "Bedload modelling")."""
    law: int = LAW_GRASS
    g: float = 9.81
    A_g: float = 1e-3        # Grass interaction constant (scalar default)
    m_g: float = 3.0         # Grass exponent
    friction: int = FRIC_STRICKLER
    fric_coef: float = 40.0  # K_s (Strickler), n (Manning) or f (Darcy)
    d_s: float = 1e-3        # mean grain diameter [m]
    s: float = 2.65          # rho_s / rho
    tau_cr: float = 0.05     # critical Shields number
    momentum_friction: int = 0  # 1: semi-implicit -g h S_f in momentum
    reconstruction: int = 0  # 1: hydrostatic reconstruction at interfaces
    order: int = 1           # 2: MUSCL reconstruction and Heun's method


def _re(x):
    return np.real(x)


def _where(cond, a, b):
    return np.where(cond, a, b)


def _cbrt(x):
    if np.iscomplexobj(x):
        return x ** (1.0 / 3.0)
    return np.cbrt(x)


def grass(u, v, Ag, mg):
    """Grass law in the isotropic 2D form; returns (qx, qy, bx, by)."""
    w = u * u + v * v
    if mg == 3.0:
        p = w                      # |U|^(m_g - 1) with m_g = 3, exactly
    else:
        p = w ** ((mg - 1.0) / 2.0) if mg != 1.0 else np.ones_like(w)
    qx = Ag * p * u
    qy = Ag * p * v
    if mg == 3.0:
        bx = Ag * (3.0 * u * u + v * v)
        by = Ag * (u * u + 3.0 * v * v)
    else:
        pos = _re(w) > 0.0
        wsafe = _where(pos, w, 1.0)
        bx = _where(pos, Ag * p * (mg * u * u + v * v) / wsafe,
                    Ag if mg == 1.0 else 0.0)
        by = _where(pos, Ag * p * (u * u + mg * v * v) / wsafe,
                    Ag if mg == 1.0 else 0.0)
        bx = bx * np.ones_like(w)
        by = by * np.ones_like(w)
    return qx, qy, bx, by


def shields_coefficient(h, p: Params):
    """c(h) such that tau* = c |U|^2 (friction slope inside tau_b)."""
    sm1 = p.s - 1.0
    if p.friction == FRIC_STRICKLER:
        ks = p.fric_coef
        return 1.0 / (sm1 * p.d_s * ks * ks * _cbrt(h))
    if p.friction == FRIC_MANNING:
        n = p.fric_coef
        return n * n / (sm1 * p.d_s * _cbrt(h))
    if p.friction == FRIC_DARCY:
        return p.fric_coef / (8.0 * p.g * sm1 * p.d_s) * np.ones_like(h)
    raise ValueError("unknown friction law")


def threshold_law(theta, p: Params):
    """q*(tau*) and dq*/dtau* for the threshold laws; zero where the law
    gives no transport."""
    tc = p.tau_cr
    e = theta - tc
    pos = _re(e) > 0.0
    es = _where(pos, e, 1.0)
    if p.law == LAW_MPM:
        F = _where(pos, 8.0 * es ** 1.5, 0.0)
        dF = _where(pos, 12.0 * es ** 0.5, 0.0)
    elif p.law == LAW_FLVB:
        F = _where(pos, 5.7 * es ** 1.5, 0.0)
        dF = _where(pos, 8.55 * es ** 0.5, 0.0)
    elif p.law == LAW_NIELSEN:
        th = _where(pos, theta, 1.0)
        sq = th ** 0.5
        F = _where(pos, 12.0 * sq * es, 0.0)
        dF = _where(pos, 12.0 * (es / (2.0 * sq) + sq), 0.0)
    elif p.law == LAW_RIBBERINK:
        F = _where(pos, 11.0 * es ** 1.65, 0.0)
        dF = _where(pos, 18.15 * es ** 0.65, 0.0)
    elif p.law == LAW_CAMENEN:
        tpos = _re(theta) > 0.0
        th = _where(tpos, theta, 1.0)
        ex = np.exp(-4.5 * tc / th)
        sq = th ** 0.5
        F = _where(tpos, 12.0 * th * sq * ex, 0.0)
        dF = _where(tpos, 12.0 * ex * (1.5 * sq + 4.5 * tc / sq), 0.0)
    else:
        raise ValueError("unknown bedload law")
    return F, dF


def threshold_closure(h, u, v, p: Params):
    """Flux along U for the threshold laws; returns (qx, qy, bx, by)."""
    c = shields_coefficient(h, p)
    w = u * u + v * v
    theta = c * w
    F, dF = threshold_law(theta, p)
    K = np.sqrt((p.s - 1.0) * p.g * p.d_s ** 3)
    pos = _re(w) > 0.0
    wsafe = _where(pos, w, 1.0)
    mag = np.sqrt(wsafe)
    Q = K * F
    qx = _where(pos, Q * u / mag, 0.0)
    qy = _where(pos, Q * v / mag, 0.0)
    bx = _where(pos, K * (dF * 2.0 * c * u * u / mag + F * v * v / (mag * wsafe)), 0.0)
    by = _where(pos, K * (dF * 2.0 * c * v * v / mag + F * u * u / (mag * wsafe)), 0.0)
    return qx, qy, bx, by


def closure(h, u, v, p: Params, Ag=None):
    """q = (qx, qy) and beta = (bx, by) for the configured law.  `Ag` is a
    per-cell Grass constant (array) or None for the scalar p.A_g."""
    if p.law == LAW_GRASS:
        return grass(u, v, p.A_g if Ag is None else Ag, p.m_g)
    return threshold_closure(h, u, v, p)


def friction_factor(h, speed, p: Params):
    """Coefficient phi with -g h S_f = -phi * (hu, hv), used by the optional
    semi-implicit momentum friction (not part of eq. "bedload system")."""
    if p.friction == FRIC_DARCY:
        return p.fric_coef * speed / (8.0 * h)
    n2 = (1.0 / (p.fric_coef * p.fric_coef) if p.friction == FRIC_STRICKLER
          else p.fric_coef * p.fric_coef)
    return p.g * n2 * speed / (h * _cbrt(h))
