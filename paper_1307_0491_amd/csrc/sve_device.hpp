// sve_device.hpp -- device-side physics of the relaxation scheme (gfx950).
//
// Per-cell lambda = 0 projection (relaxation variables at equilibrium,
// section "Numerical method"), bedload closures (section "Bedload
// modelling") and the exact Riemann solution of the relaxation system
// (eqs. "relaxh" ... "relaxqs") at one interface.
//
// Riemann solution (derived from the relaxation system's jump conditions;
// the paper defers the explicit solver to its companion analysis):
//   five waves u - a/H < u - b/H < u < u + b/H < u + a/H, Lagrangian speeds
//   -a, -b, 0, b, a.  Outer waves keep Z, Omega, u -/+ a tau and
//   Pi + a^2 tau; the contact keeps u, Pi, Z, Omega; the sediment waves keep
//   u -/+ b tau and Pi + a^2 tau, carry the Exner jump [Omega] = sigma [Z]
//   and, with the non-conservative product g H dZ/dx taken on a straight
//   path with H frozen at H_bar = (h_L + h_R)/2, the depth jump
//   [tau] = kappa [Z], kappa = g H_bar / (a^2 - b^2).  Eliminating the
//   intermediate states leaves a quadratic for the bed jump across the left
//   sediment wave; its root continuous with kappa -> 0 is taken in the form
//   -2C / (B + sqrt(B^2 - 8 eps C)).
// Celerities (eq. "ab" and the remark on stronger bounds):
//   a_f = max(h sqrt(g h)), a_f^2 = g max(h)^3,
//   b^2 = max(b_L^2, b_R^2, (H_bar u_est)^2, (1e-14 a_f)^2), with the cell
//   bound b_K^2 = (h u_n)^2 + g h^2 dq_n/du_n and the star-velocity estimate
//   u_est = (u_L + u_R)/2 - (Pi_R - Pi_L + g H_bar dZ) / (2 a_f),
//   a^2 = a_f^2 + b^2 (so a > b and kappa = H_bar / max(h)^3).
// Interface value: the fan state at x/t = 0, waves with sigma < 0 counted
// as left-going.  Fluxes in fluctuation form for the momentum equation:
//   F_h = u(0)/tau(0), F_hu^{L,R} = F_h u(0) + Pi(0) + g H_bar (Z(0) - Z_{L,R}),
//   F_ht = F_h v(0) (transverse velocity carried by the contact), F_z = Omega(0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sve {

enum { LAW_GRASS = 0, LAW_MPM, LAW_FLVB, LAW_NIELSEN, LAW_RIBBERINK, LAW_CAMENEN };
enum { FRIC_STRICKLER = 0, FRIC_MANNING = 1, FRIC_DARCY = 2 };
enum { BC_PERIODIC = 0, BC_FREE = 1, BC_INFLOW = 2 };
enum { BCW = 0, BCE = 1, BCS = 2, BCN = 3 };
enum : unsigned { ERR_POS = 1u, ERR_ORD = 2u, ERR_NONFIN = 4u };

constexpr double B_FLOOR = 1e-14;
// The floor enters as (B_FLOOR a_f)^2 with a_f = max(h sqrt(g h)) over the two
// cells, i.e. B_FLOOR^2 g max(h)^3: the interface's a_f^2, already formed.
constexpr double B_FLOOR2 = B_FLOOR * B_FLOOR;

// ---------------------------------------------------------------------------
// Reciprocal, division and square root for positive normal operands.
// v_rcp_f64 / v_rsq_f64 are accurate to about 2^-24 (measured on gfx950);
// Newton steps (Newton-Raphson on 1/x and 1/sqrt(x)) and a final residual
// correction bring the results to about one ulp, with fewer and cheaper
// instructions than the IEEE-exact sequences.  Non-positive or non-finite
// operands give non-finite results, which the error checks report.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// a / x: one Newton step on the reciprocal, then a residual correction.
__device__ __forceinline__ double fdiv(double a, double x) {
    double r = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    const double q = a * r;
    const double t = __builtin_fma(-x, q, a);
    return __builtin_fma(t, r, q);
}

// 1 / sqrt(x): two Newton steps.
__device__ __forceinline__ double frsq(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    double t = hx * y;
    double e = __builtin_fma(-t, y, 0.5);
    y = __builtin_fma(y, e, y);
    t = hx * y;
    e = __builtin_fma(-t, y, 0.5);
    return __builtin_fma(y, e, y);
}

// sqrt(x): one Newton step on 1/sqrt(x), then a residual correction.
__device__ __forceinline__ double fsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double t = (0.5 * x) * y;
    const double e = __builtin_fma(-t, y, 0.5);
    y = __builtin_fma(y, e, y);
    const double s = x * y;
    const double d = __builtin_fma(-s, s, x);
    return __builtin_fma(d, 0.5 * y, s);
}

// a b + c as one v_fma_f64.  In a Horner step fma(t, z, C) the compiler
// picks the accumulating form v_fmac_f64 (the sum overwrites its addend)
// and, since the coefficient C is a loop-invariant register it must keep,
// copies C first: one extra instruction per step.  The three-operand form
// needs no copy.
__device__ __forceinline__ double vfma(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// h^(-1/3) for finite h > 0.  With h = 2^(3q) hs, hs in [1/4, 2) (q from
// the binary exponent), a single-precision estimate y = 2^(-log2(hs)/3)
// from the hardware log2/exp2 (relative error about 2^-22) is refined by
// one third-order step of the iteration for hs^(-1/3): with
// e = 1 - hs y^3, hs^(-1/3) = y (1 - e)^(-1/3) = y (1 + e/3 + 2e^2/9 + ...),
// and the dropped terms are below 2^-60.  Within 2 ulp; about 20
// instructions against some 30 for the library function, whose handling of
// zero, infinite and negative arguments this closure does not need.
__device__ __forceinline__ double frcbrt(double h) {
    const int k = __builtin_amdgcn_frexp_exp(h);
    const int q = (int)__builtin_rintf((float)k * (1.0f / 3.0f));   // k - 3q in {-1, 0, 1}
    const double hs = __builtin_amdgcn_ldexp(h, -3 * q);
    const double y = (double)__builtin_amdgcn_exp2f(-(1.0f / 3.0f) *
                                                    __builtin_amdgcn_logf((float)hs));
    const double e = __builtin_fma(-hs, y * y * y, 1.0);
    const double t = e * __builtin_fma(2.0 / 9.0, e, 1.0 / 3.0);
    return __builtin_amdgcn_ldexp(__builtin_fma(y, t, y), -q);
}

// w^p for finite w > 0 and |p| <= 2 (the Grass law's |U|^(m_g - 1)):
// exp(p ln w) with
//   ln w = e ln2 + 2 atanh(s), w = 2^e m, m in [sqrt(1/2), sqrt(2)),
//          s = (m - 1)/(m + 1), |s| <= 0.1716, atanh by its odd Taylor
//          series to s^21 (truncation below 2^-55 relative);
//   exp(y) = 2^k exp(r), k = rint(y / ln2), |r| <= ln2 / 2, exp(r) by its
//          Taylor series to r^13 (truncation below 2^-57);
// ln2 is split into a 42-bit head and a tail so that k ln2 and e ln2 are
// formed without rounding error.  The result is within a few ulp when
// |p ln w| <= 10 (velocities between 1e-3 and 1e2 m/s); beyond that the
// rounding of y adds about |p ln w| ulp.  One reciprocal (v_rcp_f64) and
// about 50 other instructions, against some 200 for the library pow, whose
// extra precision this closure does not need.
__device__ __forceinline__ double gpow(double w, double p) {
    constexpr double LN2_HI = 0x1.62e42fefa3800p-1;   // 42 significant bits
    constexpr double LN2_LO = 0x1.ef35793c76730p-45;  // ln2 - LN2_HI
    constexpr double INV_LN2 = 1.4426950408889634;
    double m = __builtin_amdgcn_frexp_mant(w);        // [1/2, 1)
    int e = __builtin_amdgcn_frexp_exp(w);
    const bool low = m < 0.7071067811865476;
    m = low ? 2.0 * m : m;
    e = low ? e - 1 : e;
    const double s = fdiv(m - 1.0, m + 1.0);
    const double z = s * s;
    double t = 1.0 / 21.0;
    t = vfma(t, z, 1.0 / 19.0);
    t = vfma(t, z, 1.0 / 17.0);
    t = vfma(t, z, 1.0 / 15.0);
    t = vfma(t, z, 1.0 / 13.0);
    t = vfma(t, z, 1.0 / 11.0);
    t = vfma(t, z, 1.0 / 9.0);
    t = vfma(t, z, 1.0 / 7.0);
    t = vfma(t, z, 1.0 / 5.0);
    t = vfma(t, z, 1.0 / 3.0);
    t *= z;                                           // z/3 + z^2/5 + ... + z^10/21
    const double s2 = 2.0 * s;
    const double lnm = __builtin_fma(s2, t, s2);      // 2 atanh(s) = ln m
    const double de = (double)e;
    const double lnw = de * LN2_HI + __builtin_fma(de, LN2_LO, lnm);
    const double y = p * lnw;
    const double kf = __builtin_rint(y * INV_LN2);
    const double r = __builtin_fma(-kf, LN2_LO, __builtin_fma(-kf, LN2_HI, y));
    double q = 1.0 / 6227020800.0;                    // 1/13!
    q = vfma(q, r, 1.0 / 479001600.0);                // 1/12!
    q = vfma(q, r, 1.0 / 39916800.0);
    q = vfma(q, r, 1.0 / 3628800.0);
    q = vfma(q, r, 1.0 / 362880.0);
    q = vfma(q, r, 1.0 / 40320.0);
    q = vfma(q, r, 1.0 / 5040.0);
    q = vfma(q, r, 1.0 / 720.0);
    q = vfma(q, r, 1.0 / 120.0);
    q = vfma(q, r, 1.0 / 24.0);
    q = vfma(q, r, 1.0 / 6.0);
    q = __builtin_fma(q, r, 0.5);
    q = __builtin_fma(q, r, 1.0);
    q = __builtin_fma(q, r, 1.0);
    return __builtin_amdgcn_ldexp(q, (int)kf);
}

// Maximum / minimum of two doubles as a single v_max_f64 / v_min_f64.
// fmax and fmin compile to IEEE maxNum / minNum, which first quiet a
// signalling NaN in every operand not provably canonical (values moved by
// DPP, loaded, or carried around a loop): one more v_max_f64 per such
// operand.  For non-signalling inputs the results are those of fmax / fmin
// (a quiet NaN operand yields the other operand).
__device__ __forceinline__ double dmax(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double dmin(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Everything a kernel needs about the model and the grid, passed by value.
struct Model {
    int law, friction, momentum_friction;
    int wb;               // well-balanced variant (hydrostatic reconstruction)
    int order;            // 1: the paper's first-order scheme; 2: MUSCL and Heun
    int mg_is3, mg_is1;
    int nx, ny;           // ny == 1 with dim == 1 for 1D
    int dim;
    double g, Ag, mg;
    double K;             // sqrt((s-1) g d^3)
    double c_const;       // Shields coefficient constant (see closure)
    double phi_const;     // momentum-friction constant (see friction_phi)
    double tau_cr;
    double dx, dy;
    int bc_kind[4];
    double bc_h[4], bc_hu[4], bc_hv[4];
};

// Control block in device memory.  Wave-speed maxima and times are
// triple-buffered by step index: step n reads slot n%3, accumulates the
// maxima of step n+1 into slot (n+1)%3 and clears slot (n+2)%3.  Each
// slot holds SPEED_PARTS partial maxima on separate 128-byte lines: the
// wavefronts of a launch post to part (workgroup id mod SPEED_PARTS, which
// is also the XCD that round-robin dispatch gives the workgroup), so the
// atomics of some 2000 wavefronts finishing together do not all queue on
// one address; readers take the maximum over the parts.  (Eight parts
// measured faster than 16 or 32, and faster than reading a part before
// posting to skip atomics that cannot raise it.)
constexpr int SPEED_PARTS = 8;
struct Ctrl {
    unsigned long long smax[3][SPEED_PARTS][16];  // bit patterns of max speeds (x, y) in [0], [1]
    double t[3];
    double dt_last;
    unsigned err;
    int fail_step;
    int pad[2];
};

// Projected cell: the lambda = 0 state and the closure.
struct Cell {
    double h, hu, hv, z;     // conserved state (as stored)
    double tau, u, v, Pi;    // 1/h, velocities, pressure g h^2/2
    double qx, qy;           // bedload flux vector
    double bx2, by2;         // (h u)^2 + g h^2 dqx/du, (h v)^2 + g h^2 dqy/dv
    double inv_aK;           // 1 / (h sqrt(g h))
};

// One side of an interface seen along its normal.
struct Side {
    double h, tau, un, ut, Pi, z, q, b2, inv_aK;
};

struct Flux {
    double Fh, FhuL, FhuR, Fht, Fz;
};

__device__ __forceinline__ Side side_x(const Cell& c) {
    return Side{c.h, c.tau, c.u, c.v, c.Pi, c.z, c.qx, c.bx2, c.inv_aK};
}
__device__ __forceinline__ Side side_y(const Cell& c) {
    return Side{c.h, c.tau, c.v, c.u, c.Pi, c.z, c.qy, c.by2, c.inv_aK};
}

// ---------------------------------------------------------------------------
// Closures (section "Bedload modelling")
// ---------------------------------------------------------------------------
// q*(tau*) and dq*/dtau* of the threshold laws (eqs. "MPM" ... "Camenen").
__device__ __forceinline__ void threshold_law(int law, double theta, double tc,
                                              double& F, double& dF) {
    const double e = theta - tc;
    F = 0.0;
    dF = 0.0;
    if (law == LAW_CAMENEN) {
        if (theta > 0.0) {
            const double ex = exp(-4.5 * tc / theta);
            const double sq = sqrt(theta);
            F = 12.0 * theta * sq * ex;
            dF = 12.0 * ex * (1.5 * sq + 4.5 * tc / sq);
        }
        return;
    }
    if (!(e > 0.0)) return;
    if (law == LAW_MPM) {
        const double r = fsqrt(e);
        F = 8.0 * e * r;
        dF = 12.0 * r;
    } else if (law == LAW_FLVB) {
        const double r = fsqrt(e);
        F = 5.7 * e * r;
        dF = 8.55 * r;
    } else if (law == LAW_NIELSEN) {
        const double sq = sqrt(theta);
        F = 12.0 * sq * e;
        dF = 12.0 * (e / (2.0 * sq) + sq);
    } else {  // LAW_RIBBERINK
        const double p = gpow(e, 0.65);
        F = 11.0 * e * p;
        dF = 18.15 * p;
    }
}

// Closure families compiled as separate kernel instantiations, so that the
// common Grass m_g = 3 path carries no pow/exp/cbrt code and the
// Meyer-Peter & Mueller kernels none of the other threshold laws (register
// pressure); CL_THRESH covers the other four threshold laws.
enum { CL_GRASS3 = 0, CL_GRASS1 = 1, CL_GRASSM = 2, CL_THRESH = 3, CL_MPM = 4 };

inline int closure_class(const Model& M) {
    if (M.law == LAW_MPM) return CL_MPM;
    if (M.law != LAW_GRASS) return CL_THRESH;
    if (M.mg_is3) return CL_GRASS3;
    if (M.mg_is1) return CL_GRASS1;
    return CL_GRASSM;
}

// Bedload flux q = (qx, qy) and beta = (dqx/du|v, dqy/dv|u).
//   Grass (isotropic 2D form): q = A_g |U|^(m-1) (u, v),
//     beta_x = A_g |U|^(m-1) (m u^2 + v^2) / |U|^2.
//   Threshold laws: tau* = c |U|^2 with c from the friction slope
//     (Strickler 1/((s-1) d K_s^2 h^(1/3)), Manning n^2/((s-1) d h^(1/3)),
//     Darcy f/(8 g (s-1) d)); q = K q*(tau*) U/|U|, K = sqrt((s-1) g d^3),
//     beta_x = K [q*'(tau*) 2 c u^2/|U| + q*(tau*) v^2/|U|^3].
template <int CL>
__device__ __forceinline__ void closure(const Model& M, double h, double u,
                                        double v, double Ag, double& qx,
                                        double& qy, double& bx, double& by) {
    const double uu = u * u, vv = v * v;
    const double w = uu + vv;
    if (CL != CL_THRESH && CL != CL_MPM) {
        if (CL == CL_GRASS3) {
            qx = Ag * w * u;
            qy = Ag * w * v;
            bx = Ag * (3.0 * uu + vv);
            by = Ag * (uu + 3.0 * vv);
        } else if (CL == CL_GRASS1) {
            qx = Ag * u;
            qy = Ag * v;
            bx = Ag;
            by = Ag;
        } else {
            // r = |U|^(m-3) = w^((m-3)/2), so |U|^(m-1) = r w and
            // beta_x = A_g r (m u^2 + v^2).  At U = 0: q = 0, and beta = A_g
            // for m = 1 (q = A_g U), else 0.  Speeds below 1e-150 count as
            // rest (q and the m > 1 beta are then below A_g 1e-150, and r
            // stays finite).
            const bool moving = w > 1e-300;
            const double r = moving ? gpow(w, 0.5 * (M.mg - 3.0)) : 0.0;
            const double Ap = Ag * (r * w);
            qx = Ap * u;
            qy = Ap * v;
            const double b0 = M.mg_is1 ? Ag : 0.0;
            bx = moving ? Ag * r * (M.mg * uu + vv) : b0;
            by = moving ? Ag * r * (uu + M.mg * vv) : b0;
        }
        return;
    }
    const double c = (M.friction == FRIC_DARCY) ? M.c_const : M.c_const * frcbrt(h);
    double F, dF;
    threshold_law(CL == CL_MPM ? LAW_MPM : M.law, c * w, M.tau_cr, F, dF);
    if (w > 0.0) {
        const double im = frsq(w);                          // 1 / |U|
        const double Q = M.K * F;
        qx = Q * u * im;
        qy = Q * v * im;
        const double t1 = dF * 2.0 * c * im;
        const double t2 = F * (im * im * im);
        bx = M.K * (t1 * uu + t2 * vv);
        by = M.K * (t1 * vv + t2 * uu);
    } else {
        qx = qy = bx = by = 0.0;
    }
}

// lambda = 0 projection of one cell.
template <int CL>
__device__ __forceinline__ Cell project(const Model& M, double h, double hu,
                                        double hv, double z, double Ag) {
    Cell c;
    c.h = h;
    c.hu = hu;
    c.hv = hv;
    c.z = z;
    // one reciprocal square root gives 1/sqrt(g h), hence 1/h = g r^2
    // and 1/(h sqrt(g h)) = r / h
    const double gh = M.g * h;
    const double r = frsq(gh);
    c.tau = M.g * (r * r);
    c.u = hu * c.tau;
    c.v = hv * c.tau;
    c.Pi = 0.5 * gh * h;
    c.inv_aK = c.tau * r;
    double bx, by;
    closure<CL>(M, h, c.u, c.v, Ag, c.qx, c.qy, bx, by);
    const double gh2 = gh * h;
    c.bx2 = hu * hu + gh2 * bx;
    c.by2 = hv * hv + gh2 * by;
    return c;
}

// ---------------------------------------------------------------------------
// Interface celerities
// ---------------------------------------------------------------------------
struct Celer {
    double af2, Hbar, gHbar, dZ, a, b, a2, inv_a, c, kappa;
};

__device__ __forceinline__ Celer celerities(const Side& L, const Side& R, double g) {
    Celer C;
    const double hmax = dmax(L.h, R.h);
    C.af2 = g * (hmax * hmax * hmax);
    const double inv_af = dmin(L.inv_aK, R.inv_aK);       // 1 / max(h sqrt(g h))
    C.Hbar = 0.5 * (L.h + R.h);
    C.gHbar = g * C.Hbar;
    C.dZ = R.z - L.z;
    const double u_est = 0.5 * (L.un + R.un) - (R.Pi - L.Pi + C.gHbar * C.dZ) * (0.5 * inv_af);
    const double hbu = C.Hbar * u_est;
    const double b2 = dmax(dmax(L.b2, R.b2), fmax(hbu * hbu, B_FLOOR2 * C.af2));
    C.b = fsqrt(b2);
    const double A2 = C.af2 + b2;
    C.inv_a = frsq(A2);
    C.a = A2 * C.inv_a;
    C.a2 = C.a * C.a;
    C.c = fdiv(C.af2, C.a + C.b);                          // a - b, no cancellation
    const double tmin = dmin(L.tau, R.tau);
    C.kappa = C.Hbar * (tmin * tmin * tmin);               // g H_bar / a_f^2
    return C;
}

// Largest outer wave speed max(|u_L - a tau_L|, |u_R + a tau_R|).
__device__ __forceinline__ double iface_speed(const Side& L, const Side& R, double g) {
    const double hmax = dmax(L.h, R.h);
    const double af2 = g * (hmax * hmax * hmax);
    const double inv_af = dmin(L.inv_aK, R.inv_aK);
    const double Hbar = 0.5 * (L.h + R.h);
    const double dZ = R.z - L.z;
    const double u_est = 0.5 * (L.un + R.un) - (R.Pi - L.Pi + (g * Hbar) * dZ) * (0.5 * inv_af);
    const double hbu = Hbar * u_est;
    const double b2 = dmax(dmax(L.b2, R.b2), fmax(hbu * hbu, B_FLOOR2 * af2));
    const double a = fsqrt(af2 + b2);
    return fmax(fabs(L.un - a * L.tau), fabs(R.un + a * R.tau));
}

// Fluxes of the exact relaxation Riemann solution; returns ERR_* bits.
// `speed` receives the largest outer wave speed max(|sigma1|, |sigma5|).
__device__ __forceinline__ unsigned iface_flux(const Side& L, const Side& R, double g,
                                               Flux& F, double& speed) {
    const Celer C = celerities(L, R, g);
    const double a = C.a, b = C.b, c = C.c, a2 = C.a2, kappa = C.kappa, dZ = C.dZ;
    const double PL = L.Pi + a2 * L.tau;
    const double PR = R.Pi + a2 * R.tau;
    const double D = (PR - PL) * (C.inv_a * C.inv_a);
    const double AL = L.un - a * L.tau;                    // sigma1
    const double AR = R.un + a * R.tau;                    // sigma5
    const double kdz = kappa * dZ;
    const double T0 = (AR - AL - a * D - c * kdz) * (0.5 * C.inv_a);
    const double bk_a = b * kappa * C.inv_a;
    const double eps = c * bk_a;
    const double s2 = AL + c * T0;
    const double s4 = AR - c * (T0 + D + kdz);
    const double B = (s4 - s2) + eps * dZ;
    const double Cq = (R.q - L.q) - 0.5 * (s4 + s2) * dZ;
    const double disc = B * B - 8.0 * eps * Cq;
    unsigned err = 0;
    const double sq = fsqrt(fmax(disc, 1e-300));
    const double den = B + sq;
    if (!(disc >= 0.0) || !(den > 0.0)) err |= ERR_ORD;
    const double zeta = fdiv(-2.0 * Cq, den) + 0.5 * dZ;
    const double tau1 = T0 - bk_a * zeta;
    const double tau2 = tau1 + kappa * zeta;
    const double tau3 = tau2 + D;
    const double tau4 = tau1 + D + kdz;
    if (!(dmin(dmin(tau1, tau2), dmin(tau3, tau4)) > 0.0)) err |= ERR_POS;
    const double sig2 = AL + c * tau1;
    const double us = sig2 + b * tau2;                     // sigma3 = u*
    const double sig4 = AR - c * tau4;
    // fan state at x/t = 0 (k = number of waves with sigma < 0), selected
    // without branches.  Outer states (k <= 1 or k >= 4) follow from tau by
    // the outer-wave invariants, u = A -/+ a tau and Pi = P - a^2 tau (k = 0
    // and k = 5 are the cell states themselves, tau = tau_L or tau_R);
    // the two states between the sediment waves share u*, Pi*, Z*, Omega*.
    const bool c1 = AL < 0.0, l2 = sig2 < 0.0, l3 = us < 0.0, l4 = sig4 < 0.0, l5 = AR < 0.0;
    const bool outer = !l2 || l4;
    const bool right = l3;                               // state right of the contact
    const double tauO = right ? (l5 ? R.tau : tau4) : (c1 ? tau1 : L.tau);
    const double uO = __builtin_fma(right ? -a : a, tauO, right ? AR : AL);
    const double PiO = __builtin_fma(-a2, tauO, right ? PR : PL);
    const double tauM = l3 ? tau3 : tau2;
    const double PiM = __builtin_fma(-a2, tau2, PL);
    const double tau0 = outer ? tauO : tauM;
    const double u0 = outer ? uO : us;
    const double Pi0 = outer ? PiO : PiM;
    const double Z0 = outer ? (right ? R.z : L.z) : L.z + zeta;
    const double O0 = outer ? (right ? R.q : L.q) : __builtin_fma(sig2, zeta, L.q);
    const double vt0 = right ? R.ut : L.ut;
    F.Fh = fdiv(u0, tau0);
    const double P0 = u0 * F.Fh + Pi0;
    F.FhuL = P0 + C.gHbar * (Z0 - L.z);
    F.FhuR = P0 + C.gHbar * (Z0 - R.z);
    F.Fht = F.Fh * vt0;
    F.Fz = O0;
    speed = fmax(fabs(AL), fabs(AR));
    return err;
}

__device__ __forceinline__ unsigned iface_flux(const Side& L, const Side& R, double g,
                                               Flux& F) {
    double speed;
    return iface_flux(L, R, g, F, speed);
}

// ---------------------------------------------------------------------------
// Well-balanced variant: hydrostatic reconstruction (Audusse, Bouchut,
// Bristeau, Klein and Perthame, 2004) with the relaxation solver above as
// the interface solver.  Between cells A (left or below) and B: z* =
// max(z_A, z_B), h* = max(0, h + z - z*) on each side with the velocities
// kept; the relaxation problem between the projected reconstructed states
// on the bed z*; and the hydrostatic corrections g/2 (h^2 - h*^2) added to
// the momentum flux each cell sees.  A and B are the cells' own projections
// (only h, u, v and z are read); agA, agB their Grass constants.  NX: the
// interface normal is x (else y).
// ---------------------------------------------------------------------------
struct Recon {
    Cell A, B;             // projected reconstructed states
    double corrA, corrB;   // g/2 (h^2 - h*^2) of each side
};

template <int CL>
__device__ __forceinline__ Recon reconstruct(const Model& M, const Cell& A, double agA,
                                             const Cell& B, double agB) {
    Recon r;
    const double zs = dmax(A.z, B.z);
    const double hAs = dmax((A.h + A.z) - zs, 0.0);
    const double hBs = dmax((B.h + B.z) - zs, 0.0);
    r.A = project<CL>(M, hAs, hAs * A.u, hAs * A.v, zs, agA);
    r.B = project<CL>(M, hBs, hBs * B.u, hBs * B.v, zs, agB);
    r.corrA = 0.5 * M.g * (A.h * A.h - hAs * hAs);
    r.corrB = 0.5 * M.g * (B.h * B.h - hBs * hBs);
    return r;
}

template <int CL, bool NX>
__device__ __forceinline__ unsigned wb_iface_flux(const Model& M, const Cell& A, double agA,
                                                  const Cell& B, double agB, Flux& F,
                                                  double& speed) {
    const Recon r = reconstruct<CL>(M, A, agA, B, agB);
    const unsigned e = NX ? iface_flux(side_x(r.A), side_x(r.B), M.g, F, speed)
                          : iface_flux(side_y(r.A), side_y(r.B), M.g, F, speed);
    F.FhuL = F.FhuL + r.corrA;
    F.FhuR = F.FhuR + r.corrB;
    return e;
}

template <int CL, bool NX>
__device__ __forceinline__ double wb_iface_speed(const Model& M, const Cell& A, double agA,
                                                 const Cell& B, double agB) {
    const Recon r = reconstruct<CL>(M, A, agA, B, agB);
    return NX ? iface_speed(side_x(r.A), side_x(r.B), M.g)
              : iface_speed(side_y(r.A), side_y(r.B), M.g);
}

// Coefficient phi of the optional semi-implicit momentum friction,
// -g h S_f = -phi (hu, hv): Darcy f|U|/(8h), Manning/Strickler g n^2 |U| / h^(4/3).
__device__ __forceinline__ double friction_phi(const Model& M, double h, double speed) {
    if (M.friction == FRIC_DARCY) return M.phi_const * speed / h;
    return M.phi_const * speed / (h * cbrt(h));
}

// ---------------------------------------------------------------------------
// Grid access with ghost cells
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

template <typename T>
struct StateView {
    T* h;
    T* hu;
    T* hv;   // unused in 1D
    T* z;
};

// Load cell (i, j), applying the boundary conditions for indices outside
// the grid (one ghost layer; corner ghosts are never used by the stencil).
template <typename T>
__device__ __forceinline__ void fetch(const Model& M, const StateView<T>& S,
                                      const double* __restrict__ Agf, int i, int j,
                                      double& h, double& hu, double& hv, double& z,
                                      double& Ag) {
    int ii = i, jj = j, gx = -1, gy = -1;
    if (i < 0) {
        if (M.bc_kind[BCW] == BC_PERIODIC) ii = wrap(i, M.nx); else { ii = 0; gx = BCW; }
    } else if (i >= M.nx) {
        if (M.bc_kind[BCE] == BC_PERIODIC) ii = wrap(i, M.nx); else { ii = M.nx - 1; gx = BCE; }
    }
    if (M.dim == 2) {
        if (j < 0) {
            if (M.bc_kind[BCS] == BC_PERIODIC) jj = wrap(j, M.ny); else { jj = 0; gy = BCS; }
        } else if (j >= M.ny) {
            if (M.bc_kind[BCN] == BC_PERIODIC) jj = wrap(j, M.ny); else { jj = M.ny - 1; gy = BCN; }
        }
    } else {
        jj = 0;
    }
    const long long k = (long long)jj * M.nx + ii;
    h = (double)S.h[k];
    hu = (double)S.hu[k];
    hv = (M.dim == 2) ? (double)S.hv[k] : 0.0;
    z = (double)S.z[k];
    Ag = Agf ? Agf[k] : M.Ag;
    if (gx >= 0 && M.bc_kind[gx] == BC_INFLOW) { h = M.bc_h[gx]; hu = M.bc_hu[gx]; hv = M.bc_hv[gx]; }
    if (gy >= 0 && M.bc_kind[gy] == BC_INFLOW) { h = M.bc_h[gy]; hu = M.bc_hu[gy]; hv = M.bc_hv[gy]; }
}

// Ghost cell built from an already known interior state (used for the
// wave speeds of the new state at non-periodic boundaries).
__device__ __forceinline__ void ghost_from(const Model& M, int side, double& h,
                                           double& hu, double& hv) {
    if (M.bc_kind[side] == BC_INFLOW) { h = M.bc_h[side]; hu = M.bc_hu[side]; hv = M.bc_hv[side]; }
}

__device__ __forceinline__ double u64_as_double(unsigned long long b) {
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ unsigned long long double_as_u64(double d) {
    return (unsigned long long)__double_as_longlong(d);
}

// Wavefront maximum of non-negative doubles (64 lanes).
// Post non-negative maxima (x, y) of a wavefront or workgroup to part
// `part` of slot `slot` (64-bit atomic max of the bit patterns, which order
// like the values).
__device__ __forceinline__ void post_speeds(Ctrl* ctrl, int slot, int part, double sx,
                                            double sy) {
    unsigned long long* p = ctrl->smax[slot][part % SPEED_PARTS];
    if (sx > 0.0) atomicMax(&p[0], double_as_u64(sx));
    if (sy > 0.0) atomicMax(&p[1], double_as_u64(sy));
}

// Maximum over the parts of slot `slot`, direction `dir` (0: x, 1: y).
__device__ __forceinline__ double speed_max(const Ctrl* ctrl, int slot, int dir) {
    unsigned long long m = 0ull;
    for (int k = 0; k < SPEED_PARTS; ++k) {
        const unsigned long long v = ctrl->smax[slot][k][dir];
        m = v > m ? v : m;
    }
    return u64_as_double(m);
}

// Clear every part of slot `slot` (one thread).
__device__ __forceinline__ void clear_speeds(Ctrl* ctrl, int slot) {
    for (int k = 0; k < SPEED_PARTS; ++k) {
        ctrl->smax[slot][k][0] = 0ull;
        ctrl->smax[slot][k][1] = 0ull;
    }
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Step time and time-step of step n from the control block.
struct StepTime {
    double dt, t, tnew;
};

__device__ __forceinline__ StepTime step_time(const Model& M, const Ctrl* ctrl, int n,
                                              double cfl, double t_end, double fixed_dt) {
    StepTime st;
    st.t = ctrl->t[n % 3];
    if (fixed_dt > 0.0) {
        st.dt = fixed_dt;
        st.tnew = st.t + fixed_dt;
        return st;
    }
    const double Sx = speed_max(ctrl, n % 3, 0);
    double dt;
    if (M.dim == 1) {
        dt = cfl * M.dx / Sx;
    } else {
        const double Sy = speed_max(ctrl, n % 3, 1);
        dt = cfl / (Sx / M.dx + Sy / M.dy);
    }
    double tnew = st.t + dt;
    if (t_end > 0.0) {
        if (st.t >= t_end) {
            dt = 0.0;
            tnew = st.t;
        } else if (dt >= t_end - st.t) {
            dt = t_end - st.t;
            tnew = t_end;
        }
    }
    st.dt = dt;
    st.tnew = tnew;
    return st;
}

}  // namespace sve
