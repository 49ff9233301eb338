// sve_residual.hpp -- residual form of the 2D CFL step: one pass per step
// that applies the step and solves the interfaces of the new state once.
//
// The update of step n is U^{n+1} = U^n - dt^n R^n with the residual
//   R = (F^L_{i+1/2} - F^R_{i-1/2}) / dx + (G^L_{j+1/2} - G^R_{j-1/2}) / dy
// of the interface fluxes of U^n, and dt^n follows from the outer wave
// speeds of U^n (the same interface solves).  Kernel n reads U^n and R^n,
// forms U^{n+1} (stored in the storage type, then rounded back before it is
// used, as a stored state would be), and solves every interface of U^{n+1}
// once: that gives R^{n+1} (stored in FP64) and the wave-speed maxima of
// U^{n+1}, from which kernel n+1 takes dt^{n+1}.  The initial kernel does
// the same for the current state without an update.
//
// Tile layout as in the fused kernel (sve_fused.hpp): one wavefront per
// tile, lanes 0..63 on columns i0-1 .. i0+62 (61 owned), marching up rows
// j0-1 .. jend; the new state of the halo column and rows is formed from
// U^n and R^n of those cells (ghost cells: from the clamped interior cell,
// then the boundary condition), so each tile needs no data from another
// tile of the same launch.
//
// Errors: a non-finite or non-positive new state belongs to step n; an
// interface error of U^{n+1} belongs to step n+1 (its fluxes are those of
// step n+1); the initial kernel's state and interfaces belong to step n.
#pragma once

#include "sve_fused.hpp"

namespace sve {

template <typename T, int CL, bool INIT>
__device__ __forceinline__ void resid_tile(const Model& M, const StateView<T>& S,
                                           const StateView<double>& RS, const StateView<T>& D,
                                           const StateView<double>& RD,
                                           const double* __restrict__ Agf, Ctrl* ctrl, int n,
                                           double dt, int slot, int tx, int j0, int jend) {
    const int lane = threadIdx.x & 63;
    const int i0 = tx * FUSED_OWN;
    const int col = i0 - 1 + lane;
    const int l_last = min(FUSED_OWN, M.nx - i0);    // owned lanes 1..l_last
    const bool owned_lane = lane >= 1 && lane <= l_last;
    const bool xghost_w = (i0 == 0) && M.bc_kind[BCW] != BC_PERIODIC;
    const bool yghost_s = (j0 == 0) && M.bc_kind[BCS] != BC_PERIODIC;
    const double rdx = 1.0 / M.dx, rdy = 1.0 / M.dy;
    const int flux_step = INIT ? n : n + 1;          // step whose fluxes are solved here

    int ci, gxin;
    column_index(M, col, ci, gxin);
    const Ghosts G = make_ghosts(M, gxin);

    // Row r on this lane's column: U^n, R^n and A_g as loaded (load), then
    // the new state (ghosts included), stored when the cell is owned, and
    // its projection (finish).  Loads run one row ahead of the arithmetic.
    struct Loaded {
        double h, hu, hv, z, ag, rh, rhu, rhv, rz;
        int gyin;
    };
    auto load = [&](int r) -> Loaded {
        int jj, gyin;
        row_index(M, r, jj, gyin);
        const long long k = (long long)jj * M.nx + ci;
        Loaded q;
        q.h = (double)S.h[k];
        q.hu = (double)S.hu[k];
        q.hv = (double)S.hv[k];
        q.z = (double)S.z[k];
        q.ag = Agf ? Agf[k] : G.ag;
        if (!INIT) {
            q.rh = RS.h[k];
            q.rhu = RS.hu[k];
            q.rhv = RS.hv[k];
            q.rz = RS.z[k];
        } else {
            q.rh = q.rhu = q.rhv = q.rz = 0.0;
        }
        q.gyin = gyin;
        return q;
    };
    auto finish = [&](const Loaded& q, int r, bool store) -> Cell {
        double h = q.h, hu = q.hu, hv = q.hv, z = q.z;
        if (INIT && store && owned_lane) {
            const unsigned e = check_state(h, hu, hv, z);
            if (e) record_error(ctrl, e, n);
        }
        if (!INIT) {
            h = __builtin_fma(-dt, q.rh, h);
            hu = __builtin_fma(-dt, q.rhu, hu);
            hv = __builtin_fma(-dt, q.rhv, hv);
            z = __builtin_fma(-dt, q.rz, z);
            if (M.momentum_friction) apply_friction(M, dt, h, hu, hv);
            if (store && owned_lane) {
                const unsigned e = check_state(h, hu, hv, z);
                if (e) record_error(ctrl, e, n);
                store_cell(M, D, (long long)r * M.nx + col, h, hu, hv, z);
            }
            // the state as stored (FP32 storage rounds it)
            h = (double)(T)h;
            hu = (double)(T)hu;
            hv = (double)(T)hv;
            z = (double)(T)z;
        }
        apply_inflow(G, gxin, q.gyin, h, hu, hv);
        return project<CL>(M, h, hu, hv, z, q.ag);
    };

    double sx = 0.0, sy = 0.0;
    // carried from row r-1: its y view, x-flux differences and error bits,
    // and the y-fluxes of the interface below it
    Side Sp;
    double dXh = 0, dXm = 0, dXt = 0, dXz = 0;
    unsigned eX = 0, eYp = 0;
    double Yh = 0, Yt = 0, YR = 0, Yz = 0;
    bool pend = false;                               // residual waiting to be stored
    long long pk = 0;
    double ph = 0, phu = 0, phv = 0, pz = 0;

    // Row r with its loaded data q: x-interfaces (OWN: row r is owned), the
    // y-interface (r-1 | r), and the residual of row r-1.
    auto row = [&](const Loaded& q, int r, auto own) {
        const Cell P = finish(q, r, own.value);
        double nXh = 0, nXm = 0, nXt = 0, nXz = 0;
        unsigned neX = 0;
        if (own.value) {                             // x-interfaces of row r
            Flux X;
            double s;
            const unsigned e = iface_flux(side_x(P), next_side_x(P), M.g, X, s);
            nXh = X.Fh - dpp<DPP_PREV>(X.Fh);
            nXm = X.FhuL - dpp<DPP_PREV>(X.FhuR);
            nXt = X.Fht - dpp<DPP_PREV>(X.Fht);
            nXz = X.Fz - dpp<DPP_PREV>(X.Fz);
            neX = e | dpp_u<DPP_PREV>(e);
            if (owned_lane || (lane == 0 && xghost_w)) sx = fmax(sx, s);
        }
        Flux Y;                                      // y-interface (r-1 | r)
        double s;
        const unsigned eY = iface_flux(Sp, side_y(P), M.g, Y, s);
        if ((r > j0 || yghost_s) && owned_lane) sy = fmax(sy, s);
        if (r > j0 && owned_lane) {                  // row r-1 is complete
            const unsigned e = eX | eYp | eY;
            if (e) record_error(ctrl, e, flux_step);
        }
        // residual of row r-1, stored at the start of the next row: a store
        // issued just before the loop's wait for the next row's loads would
        // hold the wavefront until the write completes
        pend = r > j0;
        pk = (long long)(r - 1) * M.nx + col;
        ph = dXh * rdx + (Y.Fh - Yh) * rdy;
        phu = dXm * rdx + (Y.Fht - Yt) * rdy;
        phv = dXt * rdx + (Y.FhuL - YR) * rdy;
        pz = dXz * rdx + (Y.Fz - Yz) * rdy;
        Sp = side_y(P);
        dXh = nXh; dXm = nXm; dXt = nXt; dXz = nXz;
        eX = neX;
        eYp = eY;
        Yh = Y.Fh; Yt = Y.Fht; YR = Y.FhuR; Yz = Y.Fz;
    };

    auto flush = [&]() {
        if (pend && owned_lane) {
            RD.h[pk] = ph;
            RD.hu[pk] = phu;
            RD.hv[pk] = phv;
            RD.z[pk] = pz;
        }
    };

    // rows j0-1 .. jend, each loaded one row ahead of its arithmetic
    Loaded q1 = load(j0);
    Sp = side_y(finish(load(j0 - 1), j0 - 1, false));
    for (int r = j0; r < jend; ++r) {                // owned rows
        flush();
        const Loaded q = q1;
        q1 = load(r + 1);                            // r + 1 <= jend
        row(q, r, std::true_type{});
    }
    flush();
    row(q1, jend, std::false_type{});               // row above: y-interface only
    flush();
    sx = wave_max(sx);
    sy = wave_max(sy);
    if (lane == 0) {
        post_speeds(ctrl, slot, blockIdx.x, sx, sy);
    }
}

// One wavefront per workgroup; workgroup id runs tile xcd_tile(id) of the
// tiles_x x tiles_y split (row-major; rows by tile_rows).  INIT: residual and wave speeds of the state in S
// (step n's slot); otherwise step n, whose wave speeds are in slot n%3.
template <typename T, int CL, bool INIT>
__global__ void __launch_bounds__(64, FUSED_WAVES_PER_SIMD)
k_resid(Model M, StateView<T> S, StateView<double> RS, StateView<T> D, StateView<double> RD,
        const double* __restrict__ Agf, Ctrl* ctrl, int n, double cfl, double t_end,
        int tiles_y) {
    if (ctrl->err) return;
    double dt = 0.0;
    int slot = n % 3;
    if (!INIT) {
        const StepTime st = step_time(M, ctrl, n, cfl, t_end, 0.0);
        if (blockIdx.x == 0 && threadIdx.x == 0) step_bookkeeping(ctrl, n, st);
        dt = st.dt;
        slot = (n + 1) % 3;
    } else if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the first step kernel accumulates into slot (n+1)%3
        clear_speeds(ctrl, (n + 1) % 3);
    }
    const int tiles_x = (M.nx + FUSED_OWN - 1) / FUSED_OWN;
    const int t = xcd_tile(blockIdx.x, tiles_x * tiles_y);
    int j0, jend;
    tile_rows(M.ny, tiles_y, t / tiles_x, j0, jend);
    resid_tile<T, CL, INIT>(M, S, RS, D, RD, Agf, ctrl, n, dt, slot, t % tiles_x, j0, jend);
}

template <typename T, bool INIT>
void launch_resid(const Model& M, StateView<T> S, StateView<double> RS, StateView<T> D,
                  StateView<double> RD, const double* Ag, Ctrl* ctrl, int n, double cfl,
                  double t_end, int tiles_y, hipStream_t stream) {
    const int tiles_x = (M.nx + FUSED_OWN - 1) / FUSED_OWN;
    const int cl = closure_class(M);
    auto kern = cl == CL_GRASS3 ? k_resid<T, CL_GRASS3, INIT>
              : cl == CL_GRASS1 ? k_resid<T, CL_GRASS1, INIT>
              : cl == CL_GRASSM ? k_resid<T, CL_GRASSM, INIT>
              : cl == CL_MPM    ? k_resid<T, CL_MPM, INIT>
                                : k_resid<T, CL_THRESH, INIT>;
    hipLaunchKernelGGL(kern, dim3(tiles_x * tiles_y), dim3(64), 0, stream, M, S, RS, D, RD, Ag,
                       ctrl, n, cfl, t_end, tiles_y);
}

}  // namespace sve
