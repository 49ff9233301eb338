// sve_fused.hpp -- one-pass 2D step: update of step n and the wave speeds
// of step n+1, one wavefront per tile, marching upward through the rows.
//
// Tile: lanes 0..63 hold columns i0-1 .. i0+62 (i0 = 61 * tile index); lanes
// 1..61 own their column, lane 62 is the ring column and lane 63 its right
// neighbour.  Rows j0-1 .. j_ring+1 are loaded once each, projected once,
// and kept in registers for one iteration; x-interfaces use the right
// neighbour lane's projection (cross-lane shuffle), y-interfaces the
// previous row of the same lane.  The new state is also computed on the ring
// (one extra column and row, not stored), so the outer wave speeds of the
// new state can be evaluated on every interface the tile owns (the right
// and upper interface of each owned cell, plus the boundary interfaces of
// non-periodic edges) and reduced into the control block for the next step.
// Every global access goes through `fetch` (indices wrapped or clamped) or
// a store guarded by the owned-cell test.
#pragma once

#include "sve_context.hpp"
#include "sve_kernels.hpp"

namespace sve {

constexpr int FUSED_OWN = 61;
constexpr int FUSED_WAVES = 4;

__device__ __forceinline__ double shdn(double v) { return __shfl_down(v, 1, 64); }
__device__ __forceinline__ double shup(double v) { return __shfl_up(v, 1, 64); }

// Neighbouring lane's view of a projected cell along x (fields used by the
// interface solver); `down` takes lane+1, otherwise lane-1.
__device__ __forceinline__ Side shfl_side_x_next(const Cell& c) {
    Side s;
    s.h = shdn(c.h);
    s.tau = shdn(c.tau);
    s.un = shdn(c.u);
    s.ut = shdn(c.v);
    s.Pi = shdn(c.Pi);
    s.z = shdn(c.z);
    s.q = shdn(c.qx);
    s.b2 = shdn(c.bx2);
    s.aK = shdn(c.aK);
    s.inv_aK = shdn(c.inv_aK);
    return s;
}

// Lane+1's x view of a projected cell, restricted to what iface_speed reads.
__device__ __forceinline__ Side shfl_speed_x_next(const Cell& c) {
    Side s;
    s.h = shdn(c.h);
    s.tau = shdn(c.tau);
    s.un = shdn(c.u);
    s.ut = 0.0;
    s.Pi = shdn(c.Pi);
    s.z = shdn(c.z);
    s.q = 0.0;
    s.b2 = shdn(c.bx2);
    s.aK = shdn(c.aK);
    s.inv_aK = shdn(c.inv_aK);
    return s;
}

template <typename T, int TY>
__global__ void __launch_bounds__(64 * FUSED_WAVES)
k_fused(Model M, StateView<T> S, StateView<T> D, const double* __restrict__ Agf, Ctrl* ctrl,
        int n, double cfl, double t_end, double fixed_dt, int tiles_y) {
    if (ctrl->err) return;
    const StepTime st = step_time(M, ctrl, n, cfl, t_end, fixed_dt);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) step_bookkeeping(ctrl, n, st);
    const bool speeds = !(fixed_dt > 0.0);
    const int lane = threadIdx.x & 63;
    const int ty = blockIdx.y * FUSED_WAVES + (threadIdx.x >> 6);
    if (ty >= tiles_y) return;                       // whole wavefront
    const int i0 = blockIdx.x * FUSED_OWN;
    const int j0 = ty * TY;
    const int col = i0 - 1 + lane;
    const int jend = min(j0 + TY, M.ny);             // owned rows [j0, jend)
    const int j_ring = jend;
    const int l_last = min(FUSED_OWN, M.nx - i0);    // owned lanes 1..l_last
    const bool owned_lane = lane >= 1 && lane <= l_last;
    const int l_ring = l_last + 1;
    const bool xghost_e = (i0 + l_last == M.nx) && M.bc_kind[BCE] != BC_PERIODIC;
    const bool xghost_w = (i0 == 0) && M.bc_kind[BCW] != BC_PERIODIC;
    const bool yghost_n = (jend == M.ny) && M.bc_kind[BCN] != BC_PERIODIC;
    const bool yghost_s = (j0 == 0) && M.bc_kind[BCS] != BC_PERIODIC;
    const double lx = st.dt / M.dx, ly = st.dt / M.dy;

    Cell Pp;                      // projected row r-1
    Flux Xp{0, 0, 0, 0, 0};       // x-flux (lane, lane+1) of row r-1
    Flux Yp{0, 0, 0, 0, 0};       // y-flux below row r-1
    unsigned eXp = 0, eYp = 0;
    Side Np{};                    // y view of the projected new state of row r-2
    double nh = 0, nhu = 0, nhv = 0, nz = 0;   // new state of row r-2 (north ghost)
    double agp = 0.0;             // A_g of row r-1
    double sx = 0.0, sy = 0.0;

    for (int r = j0 - 1; r <= j_ring + 1; ++r) {
        double h, hu, hv, z, ag;
        fetch(M, S, Agf, col, r, h, hu, hv, z, ag);
        const Cell P = project(M, h, hu, hv, z, ag);
        Flux X{0, 0, 0, 0, 0};
        unsigned eX = 0;
        if (r >= j0 && r <= j_ring) eX = iface_flux(side_x(P), shfl_side_x_next(P), M.g, X);
        Flux Y{0, 0, 0, 0, 0};
        unsigned eY = 0;
        if (r >= j0) eY = iface_flux(side_y(Pp), side_y(P), M.g, Y);
        const int ru = r - 1;                        // row updated in this iteration
        if (ru >= j0) {
            const double fl_h = shup(Xp.Fh), fl_m = shup(Xp.FhuR);
            const double fl_t = shup(Xp.Fht), fl_z = shup(Xp.Fz);
            const unsigned eXl = (unsigned)__shfl_up((int)eXp, 1, 64);
            double hn = Pp.h - lx * (Xp.Fh - fl_h) - ly * (Y.Fh - Yp.Fh);
            double hun = Pp.hu - lx * (Xp.FhuL - fl_m) - ly * (Y.Fht - Yp.Fht);
            double hvn = Pp.hv - lx * (Xp.Fht - fl_t) - ly * (Y.FhuL - Yp.FhuR);
            double zn = Pp.z - lx * (Xp.Fz - fl_z) - ly * (Y.Fz - Yp.Fz);
            if (M.momentum_friction) apply_friction(M, st.dt, hn, hun, hvn);
            const bool owned_row = ru < jend;
            if (owned_row && owned_lane) {
                const unsigned e = check_state(hn, hun, hvn, zn) | eXp | eXl | eYp | eY;
                if (e) record_error(ctrl, e, n);
                store_cell(M, D, (long long)ru * M.nx + col, hn, hun, hvn, zn);
            }
            if (speeds) {
                // new states of ghost cells at non-periodic edges
                if (!owned_row && yghost_n) {
                    hn = nh; hun = nhu; hvn = nhv; zn = nz;
                    ghost_from(M, BCN, hn, hun, hvn);
                }
                if (xghost_e) {
                    const double a = shup(hn), b = shup(hun), c = shup(hvn), d = shup(zn);
                    if (lane == l_ring) {
                        hn = a; hun = b; hvn = c; zn = d;
                        ghost_from(M, BCE, hn, hun, hvn);
                    }
                }
                if (xghost_w) {
                    const double a = shdn(hn), b = shdn(hun), c = shdn(hvn), d = shdn(zn);
                    if (lane == 0) {
                        hn = a; hun = b; hvn = c; zn = d;
                        ghost_from(M, BCW, hn, hun, hvn);
                    }
                }
                // A_g of (col, ru) as fetched with the row: ghosts copy the
                // adjacent interior cell's value, as the boundary rule says
                const Cell PN = project(M, hn, hun, hvn, zn, agp);
                const Side nxt = shfl_speed_x_next(PN);
                if (owned_row && (owned_lane || (lane == 0 && xghost_w)))
                    sx = fmax(sx, iface_speed(side_x(PN), nxt, M.g));
                if (ru - 1 >= j0 && ru - 1 < jend && owned_lane)
                    sy = fmax(sy, iface_speed(Np, side_y(PN), M.g));
                if (ru == j0 && yghost_s && owned_lane) {
                    double gh = hn, ghu = hun, ghv = hvn;
                    ghost_from(M, BCS, gh, ghu, ghv);
                    const Cell G = project(M, gh, ghu, ghv, zn, agp);
                    sy = fmax(sy, iface_speed(side_y(G), side_y(PN), M.g));
                }
                Np = side_y(PN);
                nh = hn; nhu = hun; nhv = hvn; nz = zn;
            }
        }
        Pp = P;
        agp = ag;
        Xp = X;
        Yp = Y;
        eXp = eX;
        eYp = eY;
    }
    if (speeds) {
        sx = wave_max(sx);
        sy = wave_max(sy);
        if (lane == 0) {
            if (sx > 0.0) atomicMax(&ctrl->smax[(n + 1) % 3][0], double_as_u64(sx));
            if (sy > 0.0) atomicMax(&ctrl->smax[(n + 1) % 3][1], double_as_u64(sy));
        }
    }
}

template <typename T, int TY>
void launch_fused_ty(const Model& M, StateView<T> S, StateView<T> D, const double* Ag, Ctrl* ctrl,
                     int n, double cfl, double t_end, double fixed_dt, hipStream_t stream) {
    const int tiles_x = (M.nx + FUSED_OWN - 1) / FUSED_OWN;
    const int tiles_y = (M.ny + TY - 1) / TY;
    const dim3 grid(tiles_x, (tiles_y + FUSED_WAVES - 1) / FUSED_WAVES);
    hipLaunchKernelGGL((k_fused<T, TY>), grid, dim3(64 * FUSED_WAVES), 0, stream, M, S, D, Ag,
                       ctrl, n, cfl, t_end, fixed_dt, tiles_y);
}

}  // namespace sve
