// sve_fused.hpp -- one-pass 2D step: update of step n and the wave speeds
// of step n+1, one wavefront per tile, marching upward through the rows.
//
// Tile: lanes 0..63 hold columns i0-1 .. i0+62 (i0 = 61 * tile index);
// lanes 1..61 own their column, lane 62 is the ring column and lane 63 its
// right neighbour.  Rows j0-1 .. j_ring+1 are read once each (the next row
// is prefetched while the current one is processed), projected once, and
// kept in registers for one iteration.  x-interfaces take the right lane's
// projection through a DPP wavefront shift (wave_shl:1), the left
// interface's flux through wave_shr:1; y-interfaces pair a row with the
// previous row of the same lane.  The new state is also computed on the ring
// (one extra column and row, not stored), so the outer wave speeds of the
// new state can be evaluated on every interface the tile owns (the right and
// upper interface of each owned cell, plus the boundary interfaces of
// non-periodic edges) and reduced into the control block for the next step.
// Every global access uses wrapped or clamped indices, or is a store guarded
// by the owned-cell test.
#pragma once

#include "sve_context.hpp"
#include "sve_kernels.hpp"

#include <type_traits>

namespace sve {

constexpr int FUSED_OWN = 61;
constexpr int FUSED_WAVES_PER_SIMD = 2;   // occupancy the step kernel is built for
constexpr int FUSED_MIN_ROWS = 8;         // shortest tile of the automatic split

// Rows [j0, jend) of tile ty when ny rows are split into T tiles whose
// heights differ by at most one.
__host__ __device__ __forceinline__ void tile_rows(int ny, int T, int ty, int& j0, int& jend) {
    j0 = (int)((long long)ty * ny / T);
    jend = (int)((long long)(ty + 1) * ny / T);
}

// Number of row tiles: ceil(ny / rows) for an explicit tile height, else
// (rows == 0) as many as keep every wavefront of the launch resident at
// once (tiles_x * T <= wave slots of the device), with tiles of at least
// FUSED_MIN_ROWS rows.
inline int fused_tiles_y(int nx, int ny, int rows, int wave_slots) {
    if (rows > 0) return (ny + rows - 1) / rows;
    const int tiles_x = (nx + FUSED_OWN - 1) / FUSED_OWN;
    int T = wave_slots / tiles_x;
    T = T < ny / FUSED_MIN_ROWS ? T : ny / FUSED_MIN_ROWS;
    return T < 1 ? 1 : T;
}
// Tile of workgroup `id` among `nt` tiles numbered row-major (x fastest).
// Workgroups are dispatched to the 8 XCDs in turn (id mod 8); this mapping
// gives XCD k a contiguous band of about nt/8 tiles, so tiles that share
// halo rows and the cache lines at their column edges run under one L2.
// It is a bijection of [0, nt) for any nt.
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_tile(int id, int nt) {
    const int xcd = id % NUM_XCD, slot = id / NUM_XCD;
    const int q = nt / NUM_XCD, r = nt % NUM_XCD;
    return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

constexpr int DPP_NEXT = 0x130;   // wave_shl:1 -- lane i reads lane i+1
constexpr int DPP_PREV = 0x138;   // wave_shr:1 -- lane i reads lane i-1

// Lanes without a source lane (lane 63 for DPP_NEXT, lane 0 for DPP_PREV)
// read 0; their results are never used by an owned cell.
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ unsigned dpp_u(unsigned v) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
}

// The next lane's x view of a projected cell.
__device__ __forceinline__ Side next_side_x(const Cell& c) {
    Side s;
    s.h = dpp<DPP_NEXT>(c.h);
    s.tau = dpp<DPP_NEXT>(c.tau);
    s.un = dpp<DPP_NEXT>(c.u);
    s.ut = dpp<DPP_NEXT>(c.v);
    s.Pi = dpp<DPP_NEXT>(c.Pi);
    s.z = dpp<DPP_NEXT>(c.z);
    s.q = dpp<DPP_NEXT>(c.qx);
    s.b2 = dpp<DPP_NEXT>(c.bx2);
    s.inv_aK = dpp<DPP_NEXT>(c.inv_aK);
    return s;
}

// The next lane's x view restricted to what iface_speed reads.
__device__ __forceinline__ Side next_speed_side(const Side& c) {
    Side s;
    s.h = dpp<DPP_NEXT>(c.h);
    s.tau = dpp<DPP_NEXT>(c.tau);
    s.un = dpp<DPP_NEXT>(c.un);
    s.ut = 0.0;
    s.Pi = dpp<DPP_NEXT>(c.Pi);
    s.z = dpp<DPP_NEXT>(c.z);
    s.q = 0.0;
    s.b2 = dpp<DPP_NEXT>(c.b2);
    s.inv_aK = dpp<DPP_NEXT>(c.inv_aK);
    return s;
}

struct Raw {
    double h, hu, hv, z, ag;
};

// Row r of the tile: wrapped or clamped row index and the INFLOW side that
// replaces (h, hu, hv) of a ghost row (-1 when none).  (The side index is
// wave-uniform, so the model's array is read by a scalar load.)
__device__ __forceinline__ void row_index(const Model& M, int r, int& jj, int& gin) {
    jj = r;
    int g = -1;
    if (r < 0) {
        if (M.bc_kind[BCS] == BC_PERIODIC) jj = wrap(r, M.ny); else { jj = 0; g = BCS; }
    } else if (r >= M.ny) {
        if (M.bc_kind[BCN] == BC_PERIODIC) jj = wrap(r, M.ny); else { jj = M.ny - 1; g = BCN; }
    }
    gin = (g >= 0 && M.bc_kind[g] == BC_INFLOW) ? g : -1;
}

// Column `col` of a lane: wrapped or clamped index and the INFLOW side that
// replaces (h, hu, hv) of a ghost column (-1 when none).  The model's
// array is read with constant indices: a lane-dependent index makes the
// compiler fetch the kernel argument through memory, a round trip before
// the tile's first loads.
__device__ __forceinline__ void column_index(const Model& M, int col, int& ci, int& gin) {
    const int kW = M.bc_kind[BCW], kE = M.bc_kind[BCE];
    ci = col;
    gin = -1;
    if (col < 0) {
        if (kW == BC_PERIODIC) ci = wrap(col, M.nx);
        else { ci = 0; if (kW == BC_INFLOW) gin = BCW; }
    } else if (col >= M.nx) {
        if (kE == BC_PERIODIC) ci = wrap(col, M.nx);
        else { ci = M.nx - 1; if (kE == BC_INFLOW) gin = BCE; }
    }
}

// Inflow values of the ghost cells a tile can touch and the uniform A_g,
// read once per tile with constant indices.  (Indexing the model's arrays
// with a lane- or row-dependent side inside the row loop reads them from
// memory on every row, and those reads stall the loop's other loads.)
struct Ghosts {
    double xh, xhu, xhv;     // this lane's column ghost (used when gxin >= 0)
    double sh, shu, shv;     // south ghost row
    double nh, nhu, nhv;     // north ghost row
    double ag;               // A_g when there is no per-cell field
};

__device__ __forceinline__ Ghosts make_ghosts(const Model& M, int gxin) {
    Ghosts g;
    const bool w = gxin == BCW;
    g.xh = w ? M.bc_h[BCW] : M.bc_h[BCE];
    g.xhu = w ? M.bc_hu[BCW] : M.bc_hu[BCE];
    g.xhv = w ? M.bc_hv[BCW] : M.bc_hv[BCE];
    g.sh = M.bc_h[BCS];
    g.shu = M.bc_hu[BCS];
    g.shv = M.bc_hv[BCS];
    g.nh = M.bc_h[BCN];
    g.nhu = M.bc_hu[BCN];
    g.nhv = M.bc_hv[BCN];
    g.ag = M.Ag;
    return g;
}

// (h, hu, hv) of an INFLOW ghost: x ghost of this lane (gxin >= 0), then
// the ghost row (gyin = BCS or BCN).
__device__ __forceinline__ void apply_inflow(const Ghosts& G, int gxin, int gyin, double& h,
                                             double& hu, double& hv) {
    if (gxin >= 0) { h = G.xh; hu = G.xhu; hv = G.xhv; }
    if (gyin >= 0) {
        const bool s = gyin == BCS;
        h = s ? G.sh : G.nh;
        hu = s ? G.shu : G.nhu;
        hv = s ? G.shv : G.nhv;
    }
}

template <typename T>
__device__ __forceinline__ Raw load_row(const Model& M, const StateView<T>& S,
                                        const double* __restrict__ Agf, const Ghosts& G, int ci,
                                        int gxin, int r) {
    int jj, gyin;
    row_index(M, r, jj, gyin);
    const long long k = (long long)jj * M.nx + ci;
    Raw w;
    w.h = (double)S.h[k];
    w.hu = (double)S.hu[k];
    w.hv = (double)S.hv[k];
    w.z = (double)S.z[k];
    w.ag = Agf ? Agf[k] : G.ag;
    apply_inflow(G, gxin, gyin, w.h, w.hu, w.hv);
    return w;
}

// Row r, 0 <= r < ny, of the tile: no ghost row to apply, and the column's
// INFLOW values are not applied yet (inflow_column does that).
template <typename T>
__device__ __forceinline__ Raw load_row_inner(const Model& M, const StateView<T>& S,
                                              const double* __restrict__ Agf, const Ghosts& G,
                                              int ci, int r) {
    const long long k = (long long)r * M.nx + ci;
    Raw w;
    w.h = (double)S.h[k];
    w.hu = (double)S.hu[k];
    w.hv = (double)S.hv[k];
    w.z = (double)S.z[k];
    w.ag = Agf ? Agf[k] : G.ag;
    return w;
}

// The column's INFLOW values for a row from load_row_inner, applied only in
// tiles that have such a column (xin, wave-uniform).  The empty asm
// statement keeps the test a branch, so the other tiles skip the selects
// instead of executing them on every row.  Called once the row's loads are
// needed anyway: selecting right after the loads would wait for them.
__device__ __forceinline__ void inflow_column(const Ghosts& G, int gxin, bool xin, Raw& w) {
    if (xin) {
        __asm__ volatile("");
        apply_inflow(G, gxin, -1, w.h, w.hu, w.hv);
    }
}

// Side of a ghost cell next to a cell with side `c` (FREE: the same cell;
// INFLOW: the Dirichlet (h, hu, hv) with the cell's bed and A_g).
template <int CL>
__device__ __forceinline__ Side ghost_side_y(const Model& M, int side, const Side& c, double ag) {
    if (M.bc_kind[side] != BC_INFLOW) return c;
    return side_y(project<CL>(M, M.bc_h[side], M.bc_hu[side], M.bc_hv[side], c.z, ag));
}

// Projected ghost cell next to a cell `c` for the well-balanced variant
// (FREE: the cell itself; INFLOW: the Dirichlet (h, hu, hv) with the cell's
// bed and A_g).
template <int CL>
__device__ __forceinline__ Cell ghost_cell(const Model& M, int side, const Cell& c, double ag) {
    if (M.bc_kind[side] != BC_INFLOW) return c;
    return project<CL>(M, M.bc_h[side], M.bc_hu[side], M.bc_hv[side], c.z, ag);
}

// The next lane's h, u, v, z (what the well-balanced interface reads).
__device__ __forceinline__ Cell next_cell(const Cell& c) {
    Cell n;
    n.h = dpp<DPP_NEXT>(c.h);
    n.u = dpp<DPP_NEXT>(c.u);
    n.v = dpp<DPP_NEXT>(c.v);
    n.z = dpp<DPP_NEXT>(c.z);
    return n;
}

// Per-lane state carried from one row to the next.
struct RowCarry {
    double h, tau, u, v, Pi, z, qy, by2, inv, hu, hv, ag;       // projected row r-1
    double dXh, dXm, dXt, dXz;                                 // x-flux differences, row r-1
    unsigned eX, eY;
    double Yh, Yt, YR, Yz;                                     // y-flux below row r-1
    Side N;                                                    // y view, new state of row r-2
    Cell NC;                                                   // the same cell (well-balanced)
    double Nag;                                                // its A_g (well-balanced)
    // new state of the row updated last, stored at the start of the next
    // row: a store issued just before the loop's wait for the next row's
    // loads would hold the wavefront until the write completes
    double ph, phu, phv, pz;
    long long pk;
    bool pend;
};

// One tile of one step, run by one wavefront: tile tx owns columns
// [61 tx, 61 tx + 61) (clipped to the grid) and rows [j0, jend), jend > j0.
// The step's dt follows from the control block (cfl, t_end, fixed_dt as for
// step_time); exactly one tile of the grid passes bookkeep = true and
// records the step.  All arguments must be wave-uniform.
template <typename T, int CL, bool SPEEDS, bool WB = false>
__device__ __forceinline__ void fused_tile(const Model& M, const StateView<T>& S,
                                           const StateView<T>& D, const double* __restrict__ Agf,
                                           Ctrl* ctrl, int n, double cfl, double t_end,
                                           double fixed_dt, bool bookkeep, int tx, int j0,
                                           int jend) {
    const int lane = threadIdx.x & 63;
    const int i0 = tx * FUSED_OWN;
    const int col = i0 - 1 + lane;
    const int j_ring = jend;
    const int l_last = min(FUSED_OWN, M.nx - i0);    // owned lanes 1..l_last
    const bool owned_lane = lane >= 1 && lane <= l_last;
    const int l_ring = l_last + 1;
    const bool xghost_e = (i0 + l_last == M.nx) && M.bc_kind[BCE] != BC_PERIODIC;
    const bool xghost_w = (i0 == 0) && M.bc_kind[BCW] != BC_PERIODIC;
    const bool yghost_n = (jend == M.ny) && M.bc_kind[BCN] != BC_PERIODIC;
    const bool yghost_s = (j0 == 0) && M.bc_kind[BCS] != BC_PERIODIC;

    // column of this lane: wrapped or clamped, and its INFLOW ghost side
    int ci, gxin;
    column_index(M, col, ci, gxin);
    const Ghosts G = make_ghosts(M, gxin);
    // some lane of the tile is an INFLOW ghost column (lane 63 holds the
    // tile's last column, i0 + 62)
    const bool xin = (i0 == 0 && M.bc_kind[BCW] == BC_INFLOW) ||
                     (i0 + 62 >= M.nx && M.bc_kind[BCE] == BC_INFLOW);
    double sx = 0.0, sy = 0.0;
    double dt = 0.0, lx = 0.0, ly = 0.0;            // set once the step's time is known

    // Row r with the row loaded for it in `cur`.  DO_X: x-interfaces of row
    // r; DO_UPD: update of row r-1 (RING: that row is the ring row, not
    // stored); FIRST_UPD: row r-1 is the first owned row (no y-speed below
    // it yet, south boundary speed instead).
    auto flush = [&](RowCarry& c) {
        if (c.pend) store_cell(M, D, c.pk, c.ph, c.phu, c.phv, c.pz);
        c.pend = false;
    };
    auto row = [&](RowCarry& c, const Raw& cur, int r, auto do_x, auto do_upd, auto ring,
                   auto first_upd) {
        flush(c);
        const Cell P = project<CL>(M, cur.h, cur.hu, cur.hv, cur.z, cur.ag);
        double dXh = 0, dXm = 0, dXt = 0, dXz = 0;
        unsigned eXn = 0;
        if (do_x.value) {
            Flux X;
            unsigned e;
            if constexpr (WB) {
                double sp;
                e = wb_iface_flux<CL, true>(M, P, cur.ag, next_cell(P), dpp<DPP_NEXT>(cur.ag), X,
                                            sp);
            } else {
                e = iface_flux(side_x(P), next_side_x(P), M.g, X);
            }
            dXh = X.Fh - dpp<DPP_PREV>(X.Fh);
            dXm = X.FhuL - dpp<DPP_PREV>(X.FhuR);
            dXt = X.Fht - dpp<DPP_PREV>(X.Fht);
            dXz = X.Fz - dpp<DPP_PREV>(X.Fz);
            eXn = e | dpp_u<DPP_PREV>(e);
        }
        Flux Y;
        unsigned eY;
        if constexpr (WB) {
            Cell Lc;
            Lc.h = c.h;
            Lc.u = c.u;
            Lc.v = c.v;
            Lc.z = c.z;
            double sp;
            eY = wb_iface_flux<CL, false>(M, Lc, c.ag, P, cur.ag, Y, sp);
        } else {
            const Side Ls{c.h, c.tau, c.v, c.u, c.Pi, c.z, c.qy, c.by2, c.inv};
            eY = iface_flux(Ls, side_y(P), M.g, Y);
        }
        if (do_upd.value) {
            const int ru = r - 1;
            double hn = c.h - lx * c.dXh - ly * (Y.Fh - c.Yh);
            double hun = c.hu - lx * c.dXm - ly * (Y.Fht - c.Yt);
            double hvn = c.hv - lx * c.dXt - ly * (Y.FhuL - c.YR);
            double zn = c.z - lx * c.dXz - ly * (Y.Fz - c.Yz);
            if (M.momentum_friction) apply_friction(M, dt, hn, hun, hvn);
            if (!ring.value && owned_lane) {
                const unsigned e = check_state(hn, hun, hvn, zn) | c.eX | c.eY | eY;
                if (e) record_error(ctrl, e, n);
                c.pend = true;
                c.pk = (long long)ru * M.nx + col;
                c.ph = hn;
                c.phu = hun;
                c.phv = hvn;
                c.pz = zn;
            }
            if (SPEEDS) {
                // wave speeds of the new state as stored (FP32 storage rounds it)
                hn = (double)(T)hn;
                hun = (double)(T)hun;
                hvn = (double)(T)hvn;
                zn = (double)(T)zn;
                if (xghost_e) {                      // ring lane is the east ghost
                    const double a = dpp<DPP_PREV>(hn), b = dpp<DPP_PREV>(hun);
                    const double cc = dpp<DPP_PREV>(hvn), d = dpp<DPP_PREV>(zn);
                    if (lane == l_ring) {
                        hn = a; hun = b; hvn = cc; zn = d;
                        ghost_from(M, BCE, hn, hun, hvn);
                    }
                }
                if (xghost_w) {                      // lane 0 is the west ghost
                    const double a = dpp<DPP_NEXT>(hn), b = dpp<DPP_NEXT>(hun);
                    const double cc = dpp<DPP_NEXT>(hvn), d = dpp<DPP_NEXT>(zn);
                    if (lane == 0) {
                        hn = a; hun = b; hvn = cc; zn = d;
                        ghost_from(M, BCW, hn, hun, hvn);
                    }
                }
                if constexpr (WB) {
                    Cell NY;
                    if (ring.value && yghost_n) {    // north ghost row of the new state
                        NY = ghost_cell<CL>(M, BCN, c.NC, c.ag);
                    } else {
                        NY = project<CL>(M, hn, hun, hvn, zn, c.ag);
                        if (!ring.value) {
                            const double s = wb_iface_speed<CL, true>(M, NY, c.ag, next_cell(NY),
                                                                      dpp<DPP_NEXT>(c.ag));
                            if (owned_lane || (lane == 0 && xghost_w)) sx = dmax(sx, s);
                        }
                    }
                    if (!first_upd.value) {
                        const double s = wb_iface_speed<CL, false>(M, c.NC, c.Nag, NY, c.ag);
                        if (owned_lane) sy = dmax(sy, s);
                    } else if (yghost_s) {
                        const double s = wb_iface_speed<CL, false>(
                            M, ghost_cell<CL>(M, BCS, NY, c.ag), c.ag, NY, c.ag);
                        if (owned_lane) sy = dmax(sy, s);
                    }
                    c.NC = NY;
                    c.Nag = c.ag;
                } else {
                Side Ny;
                if (ring.value && yghost_n) {        // north ghost row of the new state
                    Ny = ghost_side_y<CL>(M, BCN, c.N, c.ag);
                } else {
                    const Cell PN = project<CL>(M, hn, hun, hvn, zn, c.ag);
                    Ny = side_y(PN);
                    if (!ring.value) {
                        const Side Nx = side_x(PN);
                        const Side nb = next_speed_side(Nx);
                        const double s = iface_speed(Nx, nb, M.g);
                        if (owned_lane || (lane == 0 && xghost_w)) sx = dmax(sx, s);
                    }
                }
                if (!first_upd.value) {
                    const double s = iface_speed(c.N, Ny, M.g);
                    if (owned_lane) sy = dmax(sy, s);
                } else if (yghost_s) {
                    const double s = iface_speed(ghost_side_y<CL>(M, BCS, Ny, c.ag), Ny, M.g);
                    if (owned_lane) sy = dmax(sy, s);
                }
                c.N = Ny;
                }
            }
        }
        c.h = P.h; c.tau = P.tau; c.u = P.u; c.v = P.v; c.Pi = P.Pi; c.z = P.z; c.qy = P.qy;
        c.by2 = P.by2; c.inv = P.inv_aK; c.hu = P.hu; c.hv = P.hv; c.ag = cur.ag;
        c.dXh = dXh; c.dXm = dXm; c.dXt = dXt; c.dXz = dXz; c.eX = eXn; c.eY = eY;
        c.Yh = Y.Fh; c.Yt = Y.Fht; c.YR = Y.FhuR; c.Yz = Y.Fz;
    };
    using Y_ = std::true_type;
    using N_ = std::false_type;

    // The first three rows are requested before the control block is read,
    // so their loads overlap the scalar loads of the error flag and the
    // step's time (the loads are in bounds whatever the flag says).
    const Raw w = load_row(M, S, Agf, G, ci, gxin, j0 - 1);
    Raw cur = load_row(M, S, Agf, G, ci, gxin, j0);
    Raw nxt = load_row(M, S, Agf, G, ci, gxin, j0 + 1);
    if (ctrl->err) return;                           // a previous step failed
    const StepTime st = step_time(M, ctrl, n, cfl, t_end, fixed_dt);
    if (bookkeep && lane == 0) step_bookkeeping(ctrl, n, st);
    dt = st.dt;
    lx = dt / M.dx;
    ly = dt / M.dy;

    // row j0-1: projection only
    RowCarry c{};
    {
        const Cell P = project<CL>(M, w.h, w.hu, w.hv, w.z, w.ag);
        c.h = P.h; c.tau = P.tau; c.u = P.u; c.v = P.v; c.Pi = P.Pi; c.z = P.z; c.qy = P.qy;
        c.by2 = P.by2; c.inv = P.inv_aK; c.hu = P.hu; c.hv = P.hv; c.ag = w.ag;
    }
    row(c, cur, j0, Y_{}, N_{}, N_{}, N_{});                       // row j0: fluxes only
    cur = nxt;
    if (j0 + 1 < j_ring) {
        nxt = load_row(M, S, Agf, G, ci, gxin, j0 + 2);
        row(c, cur, j0 + 1, Y_{}, Y_{}, N_{}, Y_{});               // update of row j0
        cur = nxt;
        for (int r = j0 + 2; r < j_ring - 1; ++r) {               // owned rows j0+1 .. jend-3
            nxt = load_row_inner(M, S, Agf, G, ci, r + 1);           // r + 1 < jend <= ny
            row(c, cur, r, Y_{}, Y_{}, N_{}, N_{});
            cur = nxt;
            inflow_column(G, gxin, xin, cur);
        }
        if (j0 + 2 < j_ring) {                                     // row jend may be a ghost row
            nxt = load_row(M, S, Agf, G, ci, gxin, j_ring);
            row(c, cur, j_ring - 1, Y_{}, Y_{}, N_{}, N_{});       // update of row jend-2
            cur = nxt;
        }
        nxt = load_row(M, S, Agf, G, ci, gxin, j_ring + 1);
        row(c, cur, j_ring, Y_{}, Y_{}, N_{}, N_{});               // update of row jend-1
    } else {                                                       // one owned row
        nxt = load_row(M, S, Agf, G, ci, gxin, j_ring + 1);
        row(c, cur, j_ring, Y_{}, Y_{}, N_{}, Y_{});
    }
    row(c, nxt, j_ring + 1, N_{}, Y_{}, Y_{}, N_{});               // ring row (speeds only)
    flush(c);
    if (SPEEDS) {
        sx = wave_max(sx);
        sy = wave_max(sy);
        if (lane == 0) {
            post_speeds(ctrl, (n + 1) % 3, blockIdx.x, sx, sy);
        }
    }
}

// One wavefront per workgroup: workgroup id runs tile xcd_tile(id) of the
// tiles_x x tiles_y split (row-major; rows by tile_rows).
template <typename T, int CL, bool SPEEDS, bool WB>
__global__ void __launch_bounds__(64, FUSED_WAVES_PER_SIMD)
k_fused(Model M, StateView<T> S, StateView<T> D, const double* __restrict__ Agf, Ctrl* ctrl,
        int n, double cfl, double t_end, double fixed_dt, int tiles_y) {
    const int tiles_x = (M.nx + FUSED_OWN - 1) / FUSED_OWN;
    const int t = xcd_tile(blockIdx.x, tiles_x * tiles_y);
    int j0, jend;
    tile_rows(M.ny, tiles_y, t / tiles_x, j0, jend);
    fused_tile<T, CL, SPEEDS, WB>(M, S, D, Agf, ctrl, n, cfl, t_end, fixed_dt, blockIdx.x == 0,
                                  t % tiles_x, j0, jend);
}

// tiles_y: number of row tiles (fused_tiles_y), 1 <= tiles_y <= ny.  WB:
// the well-balanced variant's kernels (M.wb set).
template <typename T, bool WB = false>
void launch_fused_rows(const Model& M, StateView<T> S, StateView<T> D, const double* Ag,
                       Ctrl* ctrl, int n, double cfl, double t_end, double fixed_dt, int tiles_y,
                       hipStream_t stream) {
    const int tiles_x = (M.nx + FUSED_OWN - 1) / FUSED_OWN;
    const dim3 grid(tiles_x * tiles_y);
    const int cl = closure_class(M);
    const bool sp = !(fixed_dt > 0.0);
    constexpr bool W = WB;
    auto kern = cl == CL_GRASS3 ? (sp ? k_fused<T, CL_GRASS3, true, W> : k_fused<T, CL_GRASS3, false, W>)
              : cl == CL_GRASS1 ? (sp ? k_fused<T, CL_GRASS1, true, W> : k_fused<T, CL_GRASS1, false, W>)
              : cl == CL_GRASSM ? (sp ? k_fused<T, CL_GRASSM, true, W> : k_fused<T, CL_GRASSM, false, W>)
              : cl == CL_MPM    ? (sp ? k_fused<T, CL_MPM, true, W> : k_fused<T, CL_MPM, false, W>)
                                : (sp ? k_fused<T, CL_THRESH, true, W> : k_fused<T, CL_THRESH, false, W>);
    hipLaunchKernelGGL(kern, grid, dim3(64), 0, stream, M, S, D, Ag, ctrl, n, cfl, t_end,
                       fixed_dt, tiles_y);
}

}  // namespace sve
