// sve_adjoint.hpp -- reverse mode of one fixed-dt step (Grass closure).
//
// For U^{n+1} = U^n - dt/dx (F^L_{i+1/2} - F^R_{i-1/2}) - dt/dy (...), the
// adjoint of the fluxes of an interface follows from the adjoint state
// lambda^{n+1} of its two cells, and the chain rule is taken backwards
// through the interface solver (sve_device.hpp, iface_flux) and the
// lambda = 0 projection to the conserved variables and the Grass constant.
// Branches of the solver (max/min selections, the fan state at x/t = 0)
// are frozen at their forward values; their derivatives are those of the
// selected expressions.
#pragma once

#include "sve_device.hpp"

namespace sve {

// Adjoints of the projected quantities of one side of an interface (normal
// frame, as in Side).
struct SideAdj {
    double h, tau, un, ut, Pi, z, q, b2;
};

// Adjoints of the projected quantities of a cell (x/y frame, as in Cell).
struct CellAdj {
    double h, tau, u, v, Pi, z, qx, qy, bx2, by2;
};

// a += x where c holds.  Written as a select so that conditional
// accumulations into one of several adjoints compile to selects, not to a
// dynamically indexed temporary array in scratch memory.
__device__ __forceinline__ void add_if(double& a, bool c, double x) { a += c ? x : 0.0; }

__device__ __forceinline__ void add_x(CellAdj& c, const SideAdj& s) {
    c.h += s.h; c.tau += s.tau; c.u += s.un; c.v += s.ut; c.Pi += s.Pi; c.z += s.z;
    c.qx += s.q; c.bx2 += s.b2;
}
__device__ __forceinline__ void add_y(CellAdj& c, const SideAdj& s) {
    c.h += s.h; c.tau += s.tau; c.v += s.un; c.u += s.ut; c.Pi += s.Pi; c.z += s.z;
    c.qy += s.q; c.by2 += s.b2;
}

// Reverse of iface_flux: given the adjoints of (F_h, F_hu^L, F_hu^R, F_ht,
// F_z), accumulate the adjoints of both sides' projected quantities.  The
// forward part repeats iface_flux operation for operation (the same
// reciprocal and square-root helpers), so every branch is taken exactly as
// in the forward step; the reverse part needs five more reciprocals.
__device__ __forceinline__ void iface_vjp(const Side& L, const Side& R, double g,
                                          const Flux& Fb, SideAdj& Lb, SideAdj& Rb) {
    // ---- forward, keeping intermediates -------------------------------
    const bool hmaxL = L.h >= R.h;
    const double hmax = dmax(L.h, R.h);
    const double af2 = g * (hmax * hmax * hmax);
    // 1 / a_f, a_f = max(h sqrt(g h)): the cell with the larger h (hmaxL)
    const double inv_af = dmin(L.inv_aK, R.inv_aK);
    const double Hbar = 0.5 * (L.h + R.h);
    const double gH = g * Hbar;
    const double dZ = R.z - L.z;
    const double w = R.Pi - L.Pi + gH * dZ;
    const double u_est = 0.5 * (L.un + R.un) - w * (0.5 * inv_af);
    const double hbu = Hbar * u_est;
    const double fl2 = B_FLOOR2 * af2;                   // (B_FLOOR a_f)^2
    // b^2 = max(bL^2, bR^2, hbu^2, fl2); ib names the maximum
    const double m01 = dmax(L.b2, R.b2), m23 = fmax(hbu * hbu, fl2);
    const double b2 = dmax(m01, m23);
    const int ib = m01 >= m23 ? (L.b2 >= R.b2 ? 0 : 1) : (hbu * hbu >= fl2 ? 2 : 3);
    const double b = fsqrt(b2);
    const double A2 = af2 + b2;
    const double inv_a = frsq(A2);
    const double a = A2 * inv_a;
    const double a2 = a * a;
    const double apb = a + b;
    const double c = fdiv(af2, apb);
    const bool tminL = L.tau <= R.tau;
    const double tmin = dmin(L.tau, R.tau);
    const double t3 = tmin * tmin * tmin;
    const double kappa = Hbar * t3;
    const double PL = L.Pi + a2 * L.tau;
    const double PR = R.Pi + a2 * R.tau;
    const double ia2 = inv_a * inv_a;
    const double dP = PR - PL;
    const double D = dP * ia2;
    const double AL = L.un - a * L.tau;
    const double AR = R.un + a * R.tau;
    const double kdz = kappa * dZ;
    const double num = AR - AL - a * D - c * kdz;
    const double T0 = num * (0.5 * inv_a);
    const double bk_a = b * kappa * inv_a;
    const double eps = c * bk_a;
    const double s2 = AL + c * T0;
    const double s4 = AR - c * (T0 + D + kdz);
    const double B = (s4 - s2) + eps * dZ;
    const double Cq = (R.q - L.q) - 0.5 * (s4 + s2) * dZ;
    const double disc = B * B - 8.0 * eps * Cq;
    const double sq = fsqrt(fmax(disc, 1e-300));
    const double den = B + sq;
    const double zq = fdiv(-2.0 * Cq, den);
    const double zeta = zq + 0.5 * dZ;
    const double tau1 = T0 - bk_a * zeta;
    const double tau2 = tau1 + kappa * zeta;
    const double tau3 = tau2 + D;
    const double tau4 = tau1 + D + kdz;
    const double sig2 = AL + c * tau1;
    const double us = sig2 + b * tau2;
    const double sig4 = AR - c * tau4;
    const bool c1 = AL < 0.0, l2 = sig2 < 0.0, l3 = us < 0.0, l4 = sig4 < 0.0, l5 = AR < 0.0;
    const bool outer = !l2 || l4;
    const bool right = l3;
    // outer-state tau source: 0 = tau_L, 1 = tau1, 4 = tau4, 5 = tau_R
    const int srcO = right ? (l5 ? 5 : 4) : (c1 ? 1 : 0);
    const double tauO = right ? (l5 ? R.tau : tau4) : (c1 ? tau1 : L.tau);
    const double uO = __builtin_fma(right ? -a : a, tauO, right ? AR : AL);
    const double PiO = __builtin_fma(-a2, tauO, right ? PR : PL);
    const double tauM = l3 ? tau3 : tau2;
    const double PiM = __builtin_fma(-a2, tau2, PL);
    const double tau0 = outer ? tauO : tauM;
    const double u0 = outer ? uO : us;
    const double Pi0 = outer ? PiO : PiM;
    const double Z0 = outer ? (right ? R.z : L.z) : L.z + zeta;
    const double vt0 = right ? R.ut : L.ut;
    const double Fh = fdiv(u0, tau0);

    // ---- reverse ------------------------------------------------------
    Lb = SideAdj{0, 0, 0, 0, 0, 0, 0, 0};
    Rb = SideAdj{0, 0, 0, 0, 0, 0, 0, 0};
    // F_hu^{L,R} = P0 + gH (Z0 - z_{L,R}), F_ht = F_h vt0, F_z = O0
    const double P0b = Fb.FhuL + Fb.FhuR;
    double gHb = Fb.FhuL * (Z0 - L.z) + Fb.FhuR * (Z0 - R.z);
    const double Z0b = gH * (Fb.FhuL + Fb.FhuR);
    Lb.z -= gH * Fb.FhuL;
    Rb.z -= gH * Fb.FhuR;
    const double O0b = Fb.Fz;
    double Fhb = Fb.Fh + Fb.Fht * vt0;
    const double vt0b = Fb.Fht * Fh;
    add_if(Rb.ut, right, vt0b);
    add_if(Lb.ut, !right, vt0b);
    // P0 = u0 F_h + Pi0
    double u0b = P0b * Fh;
    Fhb += P0b * u0;
    const double Pi0b = P0b;
    // F_h = u0 / tau0
    const double inv_tau0 = frcp(tau0);
    u0b += Fhb * inv_tau0;
    const double tau0b = -Fhb * Fh * inv_tau0;
    // fan-state selection
    double tau1b = 0, tau2b = 0, tau3b = 0, tau4b = 0, zetab = 0, sig2b = 0, usb = 0;
    double ALb = 0, ARb = 0, PLb = 0, PRb = 0, ab = 0, a2b = 0;
    if (outer) {
        double tauOb = tau0b;
        // uO = Aside + sa tauO
        add_if(ARb, right, u0b);
        add_if(ALb, !right, u0b);
        ab += (right ? -u0b : u0b) * tauO;
        tauOb += u0b * (right ? -a : a);
        // PiO = Pside - a2 tauO
        add_if(PRb, right, Pi0b);
        add_if(PLb, !right, Pi0b);
        a2b -= Pi0b * tauO;
        tauOb -= Pi0b * a2;
        add_if(Rb.tau, srcO == 5, tauOb);
        add_if(tau4b, srcO == 4, tauOb);
        add_if(tau1b, srcO == 1, tauOb);
        add_if(Lb.tau, srcO == 0, tauOb);
        add_if(Rb.z, right, Z0b);
        add_if(Rb.q, right, O0b);
        add_if(Lb.z, !right, Z0b);
        add_if(Lb.q, !right, O0b);
    } else {
        add_if(tau3b, l3, tau0b);
        add_if(tau2b, !l3, tau0b);
        usb += u0b;
        PLb += Pi0b;
        a2b -= Pi0b * tau2;
        tau2b -= Pi0b * a2;
        // Z0 = zL + zeta ; O0 = qL + sig2 zeta
        Lb.z += Z0b;
        zetab += Z0b;
        Lb.q += O0b;
        sig2b += O0b * zeta;
        zetab += O0b * sig2;
    }
    // us = sig2 + b tau2
    sig2b += usb;
    double bb = usb * tau2;
    tau2b += usb * b;
    // sig2 = AL + c tau1
    ALb += sig2b;
    double cb = sig2b * tau1;
    tau1b += sig2b * c;
    // tau4 = tau1 + D + kdz ; tau3 = tau2 + D ; tau2 = tau1 + kappa zeta
    tau1b += tau4b;
    double Db = tau4b;
    double kdzb = tau4b;
    tau2b += tau3b;
    Db += tau3b;
    tau1b += tau2b;
    double kappab = tau2b * zeta;
    zetab += tau2b * kappa;
    // tau1 = T0 - bk_a zeta
    double T0b = tau1b;
    double bk_ab = -tau1b * zeta;
    zetab -= tau1b * bk_a;
    // zeta = zq + dZ/2, zq = -2 Cq / den
    const double inv_den = frcp(den);
    double Cqb = -2.0 * zetab * inv_den;
    double denb = -zetab * zq * inv_den;
    double dZb = 0.5 * zetab;
    // den = B + sq ; sq = sqrt(disc)
    double Bb = denb;
    const double discb = disc > 0.0 ? 0.5 * denb * frcp(sq) : 0.0;
    // disc = B^2 - 8 eps Cq
    Bb += 2.0 * B * discb;
    double epsb = -8.0 * Cq * discb;
    Cqb -= 8.0 * eps * discb;
    // Cq = (qR - qL) - (s4 + s2) dZ / 2
    Rb.q += Cqb;
    Lb.q -= Cqb;
    double s4b = -0.5 * dZ * Cqb;
    double s2b = s4b;
    dZb -= 0.5 * (s4 + s2) * Cqb;
    // B = s4 - s2 + eps dZ
    s4b += Bb;
    s2b -= Bb;
    epsb += Bb * dZ;
    dZb += Bb * eps;
    // s4 = AR - c (T0 + D + kdz)
    ARb += s4b;
    cb -= s4b * (T0 + D + kdz);
    T0b -= s4b * c;
    Db -= s4b * c;
    kdzb -= s4b * c;
    // s2 = AL + c T0
    ALb += s2b;
    cb += s2b * T0;
    T0b += s2b * c;
    // eps = c bk_a
    cb += epsb * bk_a;
    bk_ab += epsb * c;
    // bk_a = b kappa inv_a
    bb += bk_ab * kappa * inv_a;
    kappab += bk_ab * b * inv_a;
    double inv_ab = bk_ab * b * kappa;
    // T0 = num inv_a / 2, num = AR - AL - a D - c kdz
    const double numb = 0.5 * T0b * inv_a;
    inv_ab += 0.5 * T0b * num;
    ARb += numb;
    ALb -= numb;
    ab -= numb * D;
    Db -= numb * a;
    cb -= numb * kdz;
    kdzb -= numb * c;
    // kdz = kappa dZ
    kappab += kdzb * dZ;
    dZb += kdzb * kappa;
    // AR = uR + a tauR ; AL = uL - a tauL
    Rb.un += ARb;
    ab += ARb * R.tau;
    Rb.tau += ARb * a;
    Lb.un += ALb;
    ab -= ALb * L.tau;
    Lb.tau -= ALb * a;
    // D = (PR - PL) inv_a^2
    PRb += Db * ia2;
    PLb -= Db * ia2;
    inv_ab += 2.0 * Db * dP * inv_a;
    // PR = PiR + a2 tauR ; PL = PiL + a2 tauL
    Rb.Pi += PRb;
    a2b += PRb * R.tau;
    Rb.tau += PRb * a2;
    Lb.Pi += PLb;
    a2b += PLb * L.tau;
    Lb.tau += PLb * a2;
    // kappa = Hbar tmin^3
    double Hbarb = kappab * t3;
    const double tminb = kappab * 3.0 * Hbar * tmin * tmin;
    add_if(Lb.tau, tminL, tminb);
    add_if(Rb.tau, !tminL, tminb);
    // c = af2 / (a + b)
    const double inv_apb = frcp(apb);
    double af2b = cb * inv_apb;
    const double capb = cb * c * inv_apb;
    ab -= capb;
    bb -= capb;
    // a2 = a a ; inv_a = 1 / a
    ab += 2.0 * a * a2b;
    ab -= inv_ab * ia2;
    // a = sqrt(A2) ; A2 = af2 + b2 ; b = sqrt(b2)
    const double A2b = 0.5 * ab * inv_a;
    af2b += A2b;
    double b2b = A2b + 0.5 * bb * frcp(b);
    // b2 = max(bL2, bR2, hbu^2, B_FLOOR^2 af2)
    add_if(Lb.b2, ib == 0, b2b);
    add_if(Rb.b2, ib == 1, b2b);
    const double hbub = ib == 2 ? 2.0 * hbu * b2b : 0.0;
    add_if(af2b, ib == 3, B_FLOOR2 * b2b);
    // hbu = Hbar u_est
    Hbarb += hbub * u_est;
    const double u_estb = hbub * Hbar;
    // u_est = (uL + uR)/2 - w inv_af / 2
    Lb.un += 0.5 * u_estb;
    Rb.un += 0.5 * u_estb;
    const double wb = -0.5 * u_estb * inv_af;
    const double inv_afb = -0.5 * u_estb * w;
    // w = PiR - PiL + gH dZ
    Rb.Pi += wb;
    Lb.Pi -= wb;
    gHb += wb * dZ;
    dZb += wb * gH;
    // inv_af = 1 / a_f
    const double a_fb = -inv_afb * inv_af * inv_af;
    // dZ = zR - zL
    Rb.z += dZb;
    Lb.z -= dZb;
    // gH = g Hbar ; Hbar = (hL + hR)/2
    Hbarb += g * gHb;
    Lb.h += 0.5 * Hbarb;
    Rb.h += 0.5 * Hbarb;
    // af2 = g hmax^3 ; a_f = hmax sqrt(g hmax), whose derivative
    // 1.5 sqrt(g hmax) is 1.5 g hmax^2 / a_f
    const double hmaxb = (af2b * 3.0 + a_fb * 1.5 * inv_af) * g * hmax * hmax;
    add_if(Lb.h, hmaxL, hmaxb);
    add_if(Rb.h, !hmaxL, hmaxb);
}

// Reverse of the projection of a cell with the Grass closure: maps the
// adjoints of the projected quantities to (h, hu, hv, z_b, A_g).  CL is the
// closure family of the forward kernel (CL_GRASS3, CL_GRASS1 or CL_GRASSM).
template <int CL>
__device__ __forceinline__ void project_vjp_grass(const Model& M, double h, double hu, double hv,
                                                  double Ag, const CellAdj& cb, double& hb,
                                                  double& hub, double& hvb, double& zb,
                                                  double& Agb) {
    const double g = M.g;
    const double tau = frcp(h);
    const double u = hu * tau, v = hv * tau;
    const double uu = u * u, vv = v * v, w = uu + vv;
    const double m = CL == CL_GRASS3 ? 3.0 : CL == CL_GRASS1 ? 1.0 : M.mg;
    // closure values and partial derivatives (q = Ag p (u, v), beta = Ag r N)
    double p, dp_dw, r, dr_dw;
    if (CL == CL_GRASS3) {
        p = w; dp_dw = 1.0; r = 1.0; dr_dw = 0.0;
    } else if (CL == CL_GRASS1) {
        p = 1.0; dp_dw = 0.0;
        const double iw = w > 0.0 ? frcp(w) : 0.0;
        r = iw; dr_dw = -iw * iw;
    } else if (w > 1e-300) {
        // the forward closure's evaluation: r = w^((m-3)/2), p = r w
        const double e = 0.5 * (m - 1.0);
        r = gpow(w, 0.5 * (m - 3.0));
        p = r * w;
        dp_dw = e * r;
        dr_dw = (e - 1.0) * r * frcp(w);
    } else {
        p = 0.0; dp_dw = 0.0; r = 0.0; dr_dw = 0.0;
    }
    const double Nx = m * uu + vv, Ny = uu + m * vv;
    double bx, by;
    if (CL == CL_GRASS3) { bx = Ag * (3.0 * uu + vv); by = Ag * (uu + 3.0 * vv); }
    else if (CL == CL_GRASS1) { bx = Ag; by = Ag; }
    else { bx = Ag * r * Nx; by = Ag * r * Ny; }
    const double dqx_du = Ag * (p + 2.0 * uu * dp_dw), dqx_dv = Ag * 2.0 * u * v * dp_dw;
    const double dqy_du = dqx_dv, dqy_dv = Ag * (p + 2.0 * vv * dp_dw);
    double dbx_du, dbx_dv, dby_du, dby_dv, dbx_dA, dby_dA;
    if (CL == CL_GRASS1) {
        dbx_du = dbx_dv = dby_du = dby_dv = 0.0;
        dbx_dA = dby_dA = 1.0;
    } else {
        dbx_du = Ag * (dr_dw * 2.0 * u * Nx + r * 2.0 * m * u);
        dbx_dv = Ag * (dr_dw * 2.0 * v * Nx + r * 2.0 * v);
        dby_du = Ag * (dr_dw * 2.0 * u * Ny + r * 2.0 * u);
        dby_dv = Ag * (dr_dw * 2.0 * v * Ny + r * 2.0 * m * v);
        dbx_dA = CL == CL_GRASS3 ? 3.0 * uu + vv : r * Nx;
        dby_dA = CL == CL_GRASS3 ? uu + 3.0 * vv : r * Ny;
    }
    // b2 = hu^2 + g h^2 beta
    const double gh2 = g * h * h;
    const double bxb = cb.bx2 * gh2, byb = cb.by2 * gh2;
    hub = 2.0 * hu * cb.bx2;
    hvb = 2.0 * hv * cb.by2;
    hb = cb.h + 2.0 * g * h * (bx * cb.bx2 + by * cb.by2);
    // closure
    double ub = cb.u + cb.qx * dqx_du + cb.qy * dqy_du + bxb * dbx_du + byb * dby_du;
    double vb = cb.v + cb.qx * dqx_dv + cb.qy * dqy_dv + bxb * dbx_dv + byb * dby_dv;
    Agb = cb.qx * p * u + cb.qy * p * v + bxb * dbx_dA + byb * dby_dA;
    // u = hu tau, v = hv tau
    hub += ub * tau;
    hvb += vb * tau;
    double taub = cb.tau + ub * hu + vb * hv;
    // Pi = g h^2 / 2 ; tau = 1 / h
    hb += cb.Pi * g * h;
    hb -= taub * tau * tau;
    zb = cb.z;
}

}  // namespace sve
