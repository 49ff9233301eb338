// sve_order2.hip -- second-order variant of the step (sve_params.order = 2).
//
// The paper finds its first-order scheme very diffusive and names a higher
// order as future work (sections "Parallelization" and "Conclusions and
// perspectives").  This is the classical second-order extension:
//   * per cell and direction, slopes of h, u, v and eta = h + z_b, each the
//     minmod of the two one-sided differences; face values q -/+ s/2 and
//     the face state (h_f, h_f u_f, h_f v_f, eta_f - h_f);
//   * at each interface the first-order problem (the relaxation Riemann
//     problem, or its hydrostatic reconstruction) between the two facing
//     face states;
//   * inside each cell the bed term g (h_lo + h_hi)/2 (z_hi - z_lo) added to
//     the normal momentum's flux difference (straight path, depth frozen
//     at the mean of the cell's face depths);
//   * rate D = (flux difference [+ cell term]) / dx + ( ... ) / dy;
//   * Heun's method with the Euler stage S(U) = U - dt D(U) (then the
//     optional momentum friction): U^{n+1} = (U^n + S(S(U^n))) / 2, dt from
//     the outer wave speeds of U^n's interface problems.
//
// Two kernels per step:
//   k_o2<.., STAGE2 = false>  D0 = D(U^n) of every owned cell into an FP64
//                             buffer, and the wave speeds of U^n's interface
//                             problems into slot n%3 of the control block;
//   k_o2<.., STAGE2 = true>   dt^n from that slot; U1 = S(U^n) formed from
//                             U^n and D0 for every cell the tile reads (halo
//                             included: D0 is there for every cell), D(U1),
//                             U2 = S(U1) and U^{n+1} = (U^n + U2)/2 of the
//                             owned cells; it also clears slot (n+1)%3 for
//                             the next step's first kernel.
// Tile (one wavefront): lanes 0..63 hold columns i0-2 .. i0+61, i0 = 60 tx;
// lanes 2..61 own their column.  A lane's x-faces need lanes -/+1 (DPP
// shifts), the x-interface (l | l+1) the high face of lane l and the low
// face of lane l+1: owned lanes see every value they need.  Rows
// j0-2 .. jend+1 are loaded once each (one row ahead of the computation in
// the first kernel, two in most forms of the second); row c's y-faces need
// rows c-1 and c+1, so row c-1 is completed in the iteration of row c.
#include <hip/hip_runtime.h>

#include "sve_context.hpp"
#include "sve_kernels.hpp"
#include "sve_fused.hpp"

namespace sve {

namespace {

constexpr int O2_OWN = 60;
// Wavefronts per SIMD each kernel is built for: the first kernel of the
// paper's interface problem with the Grass closure of exponent 1 or 3 or
// the Meyer-Peter & Mueller closure fits in 168 VGPRs (three per SIMD);
// the others need up to 256 (two).
template <int CL, bool WB, bool STAGE2>
constexpr int o2_waves() {
    return (!STAGE2 && !WB && (CL == CL_GRASS3 || CL == CL_GRASS1 || CL == CL_MPM)) ? 3 : 2;
}

__device__ __forceinline__ double minmod(double a, double b) {
    return a * b > 0.0 ? (fabs(a) < fabs(b) ? a : b) : 0.0;
}

// Values the reconstruction reads: depth, velocities, free surface, A_g.
struct Prim {
    double h, u, v, e, ag;
};

struct Face {
    double h, u, v, z;
};

// One row of a lane: the state the stage reconstructs (U^n, or U1 in the
// second kernel) and, in the second kernel, U^n for Heun's average.
struct Row {
    double h, hu, hv, z, ag;
    double nh, nhu, nhv, nz;
};

__device__ __forceinline__ Prim prim_of(const Row& w) {
    Prim p;
    const double r = frcp(w.h);
    p.h = w.h;
    p.u = w.hu * r;
    p.v = w.hv * r;
    p.e = w.h + w.z;
    p.ag = w.ag;
    return p;
}

// Low and high face values of the middle of three cells m | c | p.
__device__ __forceinline__ void faces(const Prim& m, const Prim& c, const Prim& p, Face& lo,
                                      Face& hi) {
    double s = minmod(p.h - c.h, c.h - m.h);
    lo.h = c.h - 0.5 * s;
    hi.h = c.h + 0.5 * s;
    s = minmod(p.u - c.u, c.u - m.u);
    lo.u = c.u - 0.5 * s;
    hi.u = c.u + 0.5 * s;
    s = minmod(p.v - c.v, c.v - m.v);
    lo.v = c.v - 0.5 * s;
    hi.v = c.v + 0.5 * s;
    s = minmod(p.e - c.e, c.e - m.e);
    lo.z = (c.e - 0.5 * s) - lo.h;
    hi.z = (c.e + 0.5 * s) - hi.h;
}

// g (h_lo + h_hi)/2 (z_hi - z_lo): the bed term inside a cell.
__device__ __forceinline__ double cell_term(const Model& M, const Face& lo, const Face& hi) {
    return M.g * (0.5 * (lo.h + hi.h)) * (hi.z - lo.z);
}

template <int CTRL>
__device__ __forceinline__ Prim dpp_prim(const Prim& c) {
    Prim p;
    p.h = dpp<CTRL>(c.h);
    p.u = dpp<CTRL>(c.u);
    p.v = dpp<CTRL>(c.v);
    p.e = dpp<CTRL>(c.e);
    p.ag = 0.0;
    return p;
}

// Interface problem between face A (left of or below the interface) and
// face B; NX: the interface normal is x.
template <int CL, bool WB, bool NX>
__device__ __forceinline__ unsigned face_flux(const Model& M, const Face& A, double agA,
                                              const Face& B, double agB, Flux& F,
                                              double& speed) {
    if constexpr (WB) {
        Cell a{}, b{};
        a.h = A.h; a.u = A.u; a.v = A.v; a.z = A.z;
        b.h = B.h; b.u = B.u; b.v = B.v; b.z = B.z;
        return wb_iface_flux<CL, NX>(M, a, agA, b, agB, F, speed);
    } else {
        const Cell a = project<CL>(M, A.h, A.h * A.u, A.h * A.v, A.z, agA);
        const Cell b = project<CL>(M, B.h, B.h * B.u, B.h * B.v, B.z, agB);
        return NX ? iface_flux(side_x(a), side_x(b), M.g, F, speed)
                  : iface_flux(side_y(a), side_y(b), M.g, F, speed);
    }
}

// Raw loads of row r of the lane's column (wrapped or clamped; D2: 2D).
template <typename T, bool STAGE2, bool D2>
__device__ __forceinline__ Row fetch_row(const Model& M, const StateView<T>& S,
                                         const StateView<double>& R,
                                         const double* __restrict__ Agf, const Ghosts& G,
                                         int ci, int r, int& gyin) {
    int jj = 0;
    gyin = -1;
    if (D2) row_index(M, r, jj, gyin);
    const long long k = (long long)jj * M.nx + ci;
    Row w;
    w.nh = (double)S.h[k];
    w.nhu = (double)S.hu[k];
    w.nhv = D2 ? (double)S.hv[k] : 0.0;
    w.nz = (double)S.z[k];
    w.ag = Agf ? Agf[k] : G.ag;
    if (STAGE2) {           // the rate D0, held in (h, hu, hv, z) until finish_row
        w.h = R.h[k];
        w.hu = R.hu[k];
        w.hv = D2 ? R.hv[k] : 0.0;
        w.z = R.z[k];
    }
    return w;
}

// The state the stage reconstructs: U^n, or U1 = U^n - dt D0 followed by
// the optional friction; then the INFLOW ghost values.
template <bool STAGE2>
__device__ __forceinline__ void finish_row(const Model& M, const Ghosts& G, int gxin, int gyin,
                                           double dt, Row& w) {
    if (STAGE2) {
        w.h = w.nh - dt * w.h;
        w.hu = w.nhu - dt * w.hu;
        w.hv = w.nhv - dt * w.hv;
        w.z = w.nz - dt * w.z;
        if (M.momentum_friction) apply_friction(M, dt, w.h, w.hu, w.hv);
    } else {
        w.h = w.nh;
        w.hu = w.nhu;
        w.hv = w.nhv;
        w.z = w.nz;
    }
    apply_inflow(G, gxin, gyin, w.h, w.hu, w.hv);
}

// x-interface (lane | lane+1) of a row: flux differences of the lane's
// cell (the bed term included in the hu one), error bits of its two
// x-interfaces, and the interface's outer wave speed.
template <int CL, bool WB>
__device__ __forceinline__ void x_row(const Model& M, const Prim& pc, bool agf, double& dXh,
                                      double& dXm, double& dXt, double& dXz, unsigned& eX,
                                      double& speed) {
    Face lo, hi;
    faces(dpp_prim<DPP_PREV>(pc), pc, dpp_prim<DPP_NEXT>(pc), lo, hi);
    Face nb;
    nb.h = dpp<DPP_NEXT>(lo.h);
    nb.u = dpp<DPP_NEXT>(lo.u);
    nb.v = dpp<DPP_NEXT>(lo.v);
    nb.z = dpp<DPP_NEXT>(lo.z);
    const double agn = agf ? dpp<DPP_NEXT>(pc.ag) : pc.ag;
    Flux X;
    const unsigned e = face_flux<CL, WB, true>(M, hi, pc.ag, nb, agn, X, speed);
    dXh = X.Fh - dpp<DPP_PREV>(X.Fh);
    dXm = (X.FhuL - dpp<DPP_PREV>(X.FhuR)) + cell_term(M, lo, hi);
    dXt = X.Fht - dpp<DPP_PREV>(X.Fht);
    dXz = X.Fz - dpp<DPP_PREV>(X.Fz);
    eX = e | dpp_u<DPP_PREV>(e);
}

__device__ __forceinline__ void store_rate(const StateView<double>& R, long long k, double h,
                                           double hu, double hv, double z, bool d2) {
    R.h[k] = h;
    R.hu[k] = hu;
    if (d2) R.hv[k] = hv;
    R.z[k] = z;
}

// Completion of an owned cell from its rate D: the first kernel stores D;
// the second forms U2 = S(U1) and U^{n+1} = (U^n + U2)/2.  Returns error
// bits of the states it checks.
template <typename T, bool STAGE2>
__device__ __forceinline__ unsigned complete(const Model& M, const StateView<double>& R,
                                             const StateView<T>& D, long long k, const Row& w,
                                             double dt, double Dh, double Dhu, double Dhv,
                                             double Dz) {
    if (!STAGE2) {
        store_rate(R, k, Dh, Dhu, Dhv, Dz, M.dim == 2);
        return 0u;
    }
    double h2 = w.h - dt * Dh, hu2 = w.hu - dt * Dhu, hv2 = w.hv - dt * Dhv, z2 = w.z - dt * Dz;
    if (M.momentum_friction) apply_friction(M, dt, h2, hu2, hv2);
    const double h = 0.5 * (w.nh + h2), hu = 0.5 * (w.nhu + hu2);
    const double hv = 0.5 * (w.nhv + hv2), z = 0.5 * (w.nz + z2);
    store_cell(M, D, k, h, hu, hv, z);
    return check_state(w.h, w.hu, w.hv, w.z) | check_state(h, hu, hv, z);
}

// One tile: owned columns [60 tx, 60 tx + 60) (clipped), owned rows
// [j0, jend) (2D) or the single row (1D).  All arguments wave-uniform.
template <typename T, int CL, bool WB, bool STAGE2, bool D2>
__device__ __forceinline__ void o2_tile(const Model& M, const StateView<T>& S,
                                        const StateView<double>& R, const StateView<T>& D,
                                        const double* __restrict__ Agf, Ctrl* ctrl, int n,
                                        double cfl, double t_end, double fixed_dt,
                                        bool bookkeep, int tx, int j0, int jend, double rdx,
                                        double rdy) {
    const int lane = threadIdx.x & 63;
    const int i0 = tx * O2_OWN;
    const int col = i0 - 2 + lane;
    const int l_last = min(O2_OWN, M.nx - i0);          // owned lanes 2 .. l_last + 1
    const bool owned_lane = lane >= 2 && lane <= l_last + 1;
    const bool xghost_w = (i0 == 0) && M.bc_kind[BCW] != BC_PERIODIC;
    const bool yghost_s = D2 && (j0 == 0) && M.bc_kind[BCS] != BC_PERIODIC;
    const bool x_speed_lane = owned_lane || (lane == 1 && xghost_w);
    const bool agf = Agf != nullptr;
    int ci, gxin;
    column_index(M, col, ci, gxin);
    const Ghosts G = make_ghosts(M, gxin);
    if (ctrl->err) return;                              // a previous step failed
    double dt = 0.0;
    if (STAGE2) {
        const StepTime st = step_time(M, ctrl, n, cfl, t_end, fixed_dt);
        if (bookkeep && lane == 0) {
            ctrl->t[(n + 1) % 3] = st.tnew;
            ctrl->dt_last = st.dt;
            clear_speeds(ctrl, (n + 1) % 3);
        }
        dt = st.dt;
    }
    double sx = 0.0, sy = 0.0;
    int gy;
    if constexpr (!D2) {
        Row w = fetch_row<T, STAGE2, false>(M, S, R, Agf, G, ci, 0, gy);
        finish_row<STAGE2>(M, G, gxin, -1, dt, w);
        const Prim pc = prim_of(w);
        double dXh, dXm, dXt, dXz, speed;
        unsigned eX;
        x_row<CL, WB>(M, pc, agf, dXh, dXm, dXt, dXz, eX, speed);
        if (x_speed_lane) sx = speed;
        if (owned_lane) {
            const unsigned e =
                eX | complete<T, STAGE2>(M, R, D, col, w, dt, dXh * rdx, dXm * rdx, 0.0, dXz * rdx);
            if (e) record_error(ctrl, e, n);
        }
    } else {
        auto load = [&](int r) {
            Row w = fetch_row<T, STAGE2, true>(M, S, R, Agf, G, ci, r, gy);
            finish_row<STAGE2>(M, G, gxin, gy, dt, w);
            return w;
        };
        Row wm = load(j0 - 2), wc = load(j0 - 1), wp = load(j0);
        // rows requested ahead: one in the first kernel, two in the second,
        // which reads twice the bytes per row (U^n and the rate), except
        // with the general Grass exponent and the run-time threshold laws,
        // whose closures leave no room for the second row's registers (it
        // spilled 7 to 21 VGPRs; one row ahead: general exponent 323 ->
        // 313 us per 2000^2 step, 350 -> 314 us with the hydrostatic
        // reconstruction)
        int gnx, gnx2 = -1;
        constexpr bool AHEAD2 = STAGE2 && CL != CL_GRASSM && CL != CL_THRESH;
        Row nxt = fetch_row<T, STAGE2, true>(M, S, R, Agf, G, ci, j0 + 1, gnx);
        Row nxt2;
        if (AHEAD2) nxt2 = fetch_row<T, STAGE2, true>(M, S, R, Agf, G, ci, j0 + 2, gnx2);
        Prim pm = prim_of(wm), pc = prim_of(wc), pp = prim_of(wp);
        // carried from the iteration of row c-1
        Face Nf{};                   // high y-face of row c-1
        double Nag = 0.0;
        double dXh = 0, dXm = 0, dXt = 0, dXz = 0, cy = 0;   // row c-1
        unsigned eX = 0;
        double Yh = 0, Yt = 0, YR = 0, Yz = 0;                // y-interface (c-2 | c-1)
        unsigned eY = 0;
        for (int c = j0 - 1; c <= jend; ++c) {
            Face ylo, yhi;
            faces(pm, pc, pp, ylo, yhi);
            double nXh = 0, nXm = 0, nXt = 0, nXz = 0;
            unsigned neX = 0;
            if (c >= j0 && c < jend) {
                double speed;
                x_row<CL, WB>(M, pc, agf, nXh, nXm, nXt, nXz, neX, speed);
                if (!STAGE2 && x_speed_lane) sx = dmax(sx, speed);
            }
            if (c >= j0) {
                Flux Y;
                double speed;
                const unsigned e = face_flux<CL, WB, false>(M, Nf, Nag, ylo, pc.ag, Y, speed);
                if (!STAGE2 && owned_lane && (c > j0 || yghost_s)) sy = dmax(sy, speed);
                if (c > j0 && owned_lane) {
                    const double Dh = dXh * rdx + (Y.Fh - Yh) * rdy;
                    const double Dhu = dXm * rdx + (Y.Fht - Yt) * rdy;
                    const double Dhv = dXt * rdx + ((Y.FhuL - YR) + cy) * rdy;
                    const double Dz = dXz * rdx + (Y.Fz - Yz) * rdy;
                    const long long k = (long long)(c - 1) * M.nx + col;
                    const unsigned ee =
                        eX | eY | e | complete<T, STAGE2>(M, R, D, k, wm, dt, Dh, Dhu, Dhv, Dz);
                    if (ee) record_error(ctrl, ee, n);
                }
                Yh = Y.Fh;
                Yt = Y.Fht;
                YR = Y.FhuR;
                Yz = Y.Fz;
                eY = e;
            }
            if (c == jend) break;
            Nf = yhi;
            Nag = pc.ag;
            cy = cell_term(M, ylo, yhi);
            dXh = nXh; dXm = nXm; dXt = nXt; dXz = nXz;
            eX = neX;
            // rotate the rows: c+2 becomes the newest, c+3 is requested
            wm = wc;
            wc = wp;
            finish_row<STAGE2>(M, G, gxin, gnx, dt, nxt);
            wp = nxt;
            pm = pc;
            pc = pp;
            pp = prim_of(wp);
            if (AHEAD2) {
                nxt = nxt2;
                gnx = gnx2;
                if (c + 4 <= jend + 1)
                    nxt2 = fetch_row<T, STAGE2, true>(M, S, R, Agf, G, ci, c + 4, gnx2);
            } else if (c + 3 <= jend + 1) {
                nxt = fetch_row<T, STAGE2, true>(M, S, R, Agf, G, ci, c + 3, gnx);
            }
        }
    }
    if (!STAGE2) {
        sx = wave_max(sx);
        sy = wave_max(sy);
        if (lane == 0) post_speeds(ctrl, n % 3, blockIdx.x, sx, sy);
    }
}

template <typename T, int CL, bool WB, bool STAGE2, bool D2>
__global__ void __launch_bounds__(64, (o2_waves<CL, WB, STAGE2>()))
k_o2(Model M, StateView<T> S, StateView<double> R, StateView<T> D,
     const double* __restrict__ Agf, Ctrl* ctrl, int n, double cfl, double t_end,
     double fixed_dt, int tiles_y, double rdx, double rdy) {
    const int tiles_x = (M.nx + O2_OWN - 1) / O2_OWN;
    const int t = xcd_tile(blockIdx.x, tiles_x * tiles_y);
    int j0 = 0, jend = 1;
    if (D2) tile_rows(M.ny, tiles_y, t / tiles_x, j0, jend);
    o2_tile<T, CL, WB, STAGE2, D2>(M, S, R, D, Agf, ctrl, n, cfl, t_end, fixed_dt,
                                   blockIdx.x == 0, t % tiles_x, j0, jend, rdx, rdy);
}

// Row tiles of a kernel: tiles of `rows` rows, or (rows = 0) as many as
// keep every wavefront of the launch resident at once (cus x 4 SIMDs x
// waves), with tiles of at least FUSED_MIN_ROWS rows.
int tiles_for(int nx, int ny, int dim, int rows, int cus, int waves) {
    if (dim == 1) return 1;
    if (rows > 0) return (ny + rows - 1) / rows;
    const int tiles_x = (nx + O2_OWN - 1) / O2_OWN;
    int T = cus * 4 * waves / tiles_x;
    T = T < ny / FUSED_MIN_ROWS ? T : ny / FUSED_MIN_ROWS;
    return T < 1 ? 1 : T;
}

template <typename T, int CL, bool WB, bool STAGE2, bool D2>
void launch_k(const Model& M, StateView<T> S, StateView<double> R, StateView<T> D,
              const double* Ag, Ctrl* ctrl, int n, double cfl, double t_end, double fixed_dt,
              int rows, int cus, hipStream_t stream) {
    const int tiles_x = (M.nx + O2_OWN - 1) / O2_OWN;
    const int tiles_y = tiles_for(M.nx, M.ny, M.dim, rows, cus, o2_waves<CL, WB, STAGE2>());
    hipLaunchKernelGGL((k_o2<T, CL, WB, STAGE2, D2>), dim3(tiles_x * tiles_y), dim3(64), 0,
                       stream, M, S, R, D, Ag, ctrl, n, cfl, t_end, fixed_dt, tiles_y,
                       1.0 / M.dx, 1.0 / M.dy);
}

template <typename T, bool WB, bool STAGE2, bool D2>
void launch_cl(const Model& M, StateView<T> S, StateView<double> R, StateView<T> D,
               const double* Ag, Ctrl* ctrl, int n, double cfl, double t_end, double fixed_dt,
               int rows, int cus, hipStream_t stream) {
    const int cl = closure_class(M);
    if (cl == CL_GRASS3)
        launch_k<T, CL_GRASS3, WB, STAGE2, D2>(M, S, R, D, Ag, ctrl, n, cfl, t_end, fixed_dt,
                                               rows, cus, stream);
    else if (cl == CL_GRASS1)
        launch_k<T, CL_GRASS1, WB, STAGE2, D2>(M, S, R, D, Ag, ctrl, n, cfl, t_end, fixed_dt,
                                               rows, cus, stream);
    else if (cl == CL_GRASSM)
        launch_k<T, CL_GRASSM, WB, STAGE2, D2>(M, S, R, D, Ag, ctrl, n, cfl, t_end, fixed_dt,
                                               rows, cus, stream);
    else if (cl == CL_MPM)
        launch_k<T, CL_MPM, WB, STAGE2, D2>(M, S, R, D, Ag, ctrl, n, cfl, t_end, fixed_dt, rows,
                                            cus, stream);
    else
        launch_k<T, CL_THRESH, WB, STAGE2, D2>(M, S, R, D, Ag, ctrl, n, cfl, t_end, fixed_dt,
                                               rows, cus, stream);
}

}  // namespace

template <typename T>
void launch_order2(const Model& M, StateView<T> S, StateView<double> R, StateView<T> D,
                   const double* Ag, Ctrl* ctrl, int n, double cfl, double t_end,
                   double fixed_dt, int rows, int cus, bool stage2, hipStream_t stream) {
    const bool d2 = M.dim == 2;
#define SVE_O2(WB_, S2_, D2_) \
    launch_cl<T, WB_, S2_, D2_>(M, S, R, D, Ag, ctrl, n, cfl, t_end, fixed_dt, rows, cus, stream)
    if (M.wb) {
        if (stage2) { if (d2) SVE_O2(true, true, true); else SVE_O2(true, true, false); }
        else        { if (d2) SVE_O2(true, false, true); else SVE_O2(true, false, false); }
    } else {
        if (stage2) { if (d2) SVE_O2(false, true, true); else SVE_O2(false, true, false); }
        else        { if (d2) SVE_O2(false, false, true); else SVE_O2(false, false, false); }
    }
#undef SVE_O2
}

template void launch_order2<double>(const Model&, StateView<double>, StateView<double>,
                                    StateView<double>, const double*, Ctrl*, int, double, double,
                                    double, int, int, bool, hipStream_t);
template void launch_order2<float>(const Model&, StateView<float>, StateView<double>,
                                   StateView<float>, const double*, Ctrl*, int, double, double,
                                   double, int, int, bool, hipStream_t);

}  // namespace sve
