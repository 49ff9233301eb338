"""Interface solver of the oracle: exact Riemann solution of the relaxation
system (eqs. "relaxh" ... "relaxqs") with lambda = 0 projection.

Test infrastructure only (see the package docstring).

Derivation (from the relaxation system alone; the paper defers the explicit
solver to its companion analysis).  In the variables (H, u, Pi, Z, Omega)
the relaxation system is block triangular: the (Z, Omega) rows only involve
Z and Omega.  Its five characteristic speeds are u - a/H, u - b/H, u,
u + b/H, u + a/H; in Lagrangian mass coordinates (tau = 1/H) they are the
constants -a, -b, 0, b, a and every field is linearly degenerate, as the
paper's list of properties requires.  Across each wave:
  * waves 1 and 5 (speeds u -/+ a tau): Z, Omega, u -/+ a tau and
    Pi + a^2 tau are continuous;
  * contact (speed u): u, Pi, Z, Omega continuous, tau free;
  * sediment waves 2 and 4 (speeds u -/+ b tau): u -/+ b tau and
    Pi + a^2 tau continuous, the Exner relation [Omega] = sigma [Z], and
    the mass/momentum jump conditions with the non-conservative product
    g H dZ/dx taken along a straight path with H frozen at the interface
    mean H_bar = (h_L + h_R)/2 give [tau] = kappa [Z],
    kappa = g H_bar / (a^2 - b^2).
Eliminating the intermediate states leaves one quadratic equation for the
bed jump zeta = Z* - Z_L across the left sediment wave; the root that is
continuous with the kappa -> 0 limit is taken in the cancellation-free form
-2C / (B + sqrt(B^2 - 8 eps C)).

Celerities (readings of eq. "ab" and of the "stronger bounds" remark):
  a_f^2 = g max(h_L, h_R)^3,  a_f = max(h_L sqrt(g h_L), h_R sqrt(g h_R)),
  b^2 = max(b_L^2, b_R^2, (H_bar u_est)^2, (B_FLOOR a_f)^2) with the cell
  bounds b_K^2 = (h u_n)^2 + g h^2 beta_n and the star-velocity estimate
  u_est = (u_L + u_R)/2 - (Pi_R - Pi_L + g H_bar dZ) / (2 a_f),
  a^2 = a_f^2 + b^2, so a > b, a^2 - b^2 = a_f^2 and kappa = H_bar / h_max^3.
Interface value: the state in the fan at x/t = 0 (waves with sigma < 0
strictly count as left-going).  Fluxes, in fluctuation form for the
non-conservative momentum equation:
  F_h = H(0) u(0),  P0 = H(0) u(0)^2 + Pi(0),
  F_hu^L = P0 + g H_bar (Z(0) - Z_L)   (seen by the left cell),
  F_hu^R = P0 + g H_bar (Z(0) - Z_R)   (seen by the right cell),
  F_ht = F_h v(0) (transverse momentum, v carried by the contact),
  F_z = Omega(0).
"""
from __future__ import annotations

import dataclasses

import numpy as np

B_FLOOR = 1e-14          # floor of b relative to a_f (keeps sigma2 < u < sigma4)
ERR_POSITIVITY = 1       # some intermediate tau_k <= 0
ERR_ORDER = 2            # quadratic discriminant < 0 or B + sqrt(disc) <= 0
ERR_NONFINITE = 4        # non-finite value


def _re(x):
    return np.real(x)


def _max(a, b):
    return np.where(_re(a) >= _re(b), a, b)


def _min(a, b):
    return np.where(_re(a) <= _re(b), a, b)


def _abs(x):
    return np.where(_re(x) < 0.0, -x, x)


@dataclasses.dataclass
class CellState:
    """Projected (lambda = 0) values of one side of an interface.  `un` is
    the velocity normal to the interface, `ut` the transverse one, `q` the
    normal bedload flux Omega = Q_s and `b2` the cell's sediment celerity
    bound (h u_n)^2 + g h^2 d(q_n)/d(u_n)."""
    h: np.ndarray
    tau: np.ndarray
    un: np.ndarray
    ut: np.ndarray
    Pi: np.ndarray
    z: np.ndarray
    q: np.ndarray
    b2: np.ndarray
    aK: np.ndarray


@dataclasses.dataclass
class InterfaceResult:
    Fh: np.ndarray
    FhuL: np.ndarray
    FhuR: np.ndarray
    Fht: np.ndarray
    Fz: np.ndarray
    speed: np.ndarray
    sigma: tuple        # (sigma1, ..., sigma5)
    states: tuple       # W1..W4 as (tau, u, Pi, Z, Omega)
    a: np.ndarray
    b: np.ndarray
    err: np.ndarray     # bit mask of ERR_*


def project(h, hu, hv, z, qx, qy, bx, by, g):
    """Lambda = 0 projection of a cell (relaxation variables at equilibrium:
    Pi = g h^2 / 2, Omega = Q_s).  Returns the per-cell quantities used by
    both interface directions."""
    tau = 1.0 / h
    u = hu * tau
    v = hv * tau
    Pi = 0.5 * g * h * h
    aK = h * np.sqrt(g * h)
    bx2 = hu * hu + g * h * h * bx
    by2 = hv * hv + g * h * h * by
    return dict(h=h, tau=tau, u=u, v=v, Pi=Pi, z=z, qx=qx, qy=qy, bx2=bx2,
                by2=by2, aK=aK)


def interface_solve(L: CellState, R: CellState, g: float) -> InterfaceResult:
    """Riemann solution of the relaxation system between L and R and the
    resulting interface fluxes."""
    # --- celerities -------------------------------------------------------
    hmax = _max(L.h, R.h)
    af2 = g * (hmax * hmax * hmax)
    a_f = _max(L.aK, R.aK)
    Hbar = 0.5 * (L.h + R.h)
    dZ = R.z - L.z
    dO = R.q - L.q
    u_est = 0.5 * (L.un + R.un) - (R.Pi - L.Pi + g * Hbar * dZ) / (2.0 * a_f)
    hb_u = Hbar * u_est
    fl = B_FLOOR * a_f
    b2 = _max(_max(L.b2, R.b2), _max(hb_u * hb_u, fl * fl))
    b = np.sqrt(b2)
    a = np.sqrt(af2 + b2)
    c = af2 / (a + b)                               # a - b without cancellation
    tmin = _min(L.tau, R.tau)
    kappa = Hbar * (tmin * tmin * tmin)             # g H_bar / a_f^2
    # --- closed-form intermediate states ---------------------------------
    a2 = a * a
    PL = L.Pi + a2 * L.tau
    PR = R.Pi + a2 * R.tau
    D = (PR - PL) / a2
    AL = L.un - a * L.tau                           # sigma1
    AR = R.un + a * R.tau                           # sigma5
    T0 = (AR - AL - a * D - c * kappa * dZ) / (2.0 * a)
    eps = c * b * kappa / a
    s2 = AL + c * T0
    s4 = AR - c * (T0 + D + kappa * dZ)
    s2p = s2 - 0.5 * eps * dZ
    s4p = s4 + 0.5 * eps * dZ
    B = s4p - s2p
    C = dO - 0.5 * (s4p + s2p) * dZ
    disc = B * B - 8.0 * eps * C
    disc_ok = _re(disc) >= 0.0
    sq = np.sqrt(_where_pos(disc_ok, disc))
    den = B + sq
    den_ok = _re(den) > 0.0
    zeta = -2.0 * C / _where_pos(den_ok, den) + 0.5 * dZ
    Zs = L.z + zeta
    tau1 = T0 - (b * kappa / a) * zeta
    tau2 = tau1 + kappa * zeta
    tau3 = tau2 + D
    tau4 = tau1 + D + kappa * dZ
    sig1 = AL
    sig2 = AL + c * tau1
    us = sig2 + b * tau2                            # sigma3 = u*
    sig4 = AR - c * tau4
    sig5 = AR
    u1 = AL + a * tau1
    u4 = AR - a * tau4
    Pi1 = PL - a2 * tau1
    Pis = PL - a2 * tau2
    Pi4 = PR - a2 * tau4
    Os = L.q + sig2 * zeta
    # --- state at x/t = 0 ----------------------------------------------
    k = ((_re(sig1) < 0).astype(np.int64) + (_re(sig2) < 0) + (_re(us) < 0)
         + (_re(sig4) < 0) + (_re(sig5) < 0))
    tau0 = _select(k, [L.tau, tau1, tau2, tau3, tau4, R.tau])
    u0 = _select(k, [L.un, u1, us, us, u4, R.un])
    Pi0 = _select(k, [L.Pi, Pi1, Pis, Pis, Pi4, R.Pi])
    Z0 = _select(k, [L.z, L.z, Zs, Zs, R.z, R.z])
    O0 = _select(k, [L.q, L.q, Os, Os, R.q, R.q])
    vt0 = np.where(k <= 2, L.ut, R.ut)
    # --- fluxes -----------------------------------------------------------
    Fh = u0 / tau0
    P0 = u0 * Fh + Pi0
    FhuL = P0 + g * Hbar * (Z0 - L.z)
    FhuR = P0 + g * Hbar * (Z0 - R.z)
    Fht = Fh * vt0
    Fz = O0
    speed = _max(_abs(sig1), _abs(sig5))
    err = np.zeros(np.shape(_re(Fh)), dtype=np.int64)
    err |= np.where(~disc_ok | ~den_ok, ERR_ORDER, 0)
    pos_ok = ((_re(tau1) > 0) & (_re(tau2) > 0) & (_re(tau3) > 0)
              & (_re(tau4) > 0))
    err |= np.where(pos_ok, 0, ERR_POSITIVITY)
    return InterfaceResult(Fh, FhuL, FhuR, Fht, Fz, speed,
                           (sig1, sig2, us, sig4, sig5),
                           ((tau1, u1, Pi1, L.z, L.q), (tau2, us, Pis, Zs, Os),
                            (tau3, us, Pis, Zs, Os), (tau4, u4, Pi4, R.z, R.q)),
                           a, b, err)


def _where_pos(ok, x):
    return np.where(ok, x, 1.0)


def _select(k, choices):
    out = choices[0] * np.ones_like(choices[1])
    for i in range(1, 6):
        out = np.where(k == i, choices[i], out)
    return out


def interface_speed(L: CellState, R: CellState, g: float):
    """max(|sigma1|, |sigma5|) of the interface (same celerities as above)."""
    return interface_solve(L, R, g).speed
