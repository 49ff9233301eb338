// sve_fused1d.hip -- one-pass 1D step for grids beyond the LDS-resident
// kernel's reach: update of step n and the wave speeds of step n+1 in one
// launch (the first-order scheme of the paper's 1D runs, J up to 20 000).
//
// One wavefront per tile of 61 cells, as one row of the 2D fused kernel:
// lanes 0..63 hold cells i0-1 .. i0+62, lanes 1..61 own theirs, lane 62 is
// the ring cell and lane 63 its right neighbour.  Each lane projects its
// cell, solves the interface on its right with the next lane's projection
// (DPP wave_shl:1) and takes the left interface's flux from the previous
// lane (wave_shr:1); the owned lanes store the new state.  The new state is
// also formed on the ring cell, so every owned lane can evaluate the outer
// wave speed of the new state on its right interface (and lane 0 on the
// west boundary interface of a non-periodic grid); the wavefront's maximum
// goes into one part of slot (n+1)%3 of the control block.  A 1D step is
// then one launch instead of the split path's two (update, then speeds),
// whose tiny grids are each bound by latency.
#include <hip/hip_runtime.h>

#include "sve_context.hpp"
#include "sve_fused.hpp"
#include "sve_kernels.hpp"

namespace sve {

namespace {

template <typename T, int CL, bool SPEEDS, bool WB>
__global__ void __launch_bounds__(64, 2)
k_fused_1d(Model M, StateView<T> S, StateView<T> D, const double* __restrict__ Agf, Ctrl* ctrl,
           int n, double cfl, double t_end, double fixed_dt) {
    const int lane = threadIdx.x & 63;
    const int i0 = blockIdx.x * FUSED_OWN;
    const int col = i0 - 1 + lane;
    const int l_last = min(FUSED_OWN, M.nx - i0);      // owned lanes 1..l_last
    const bool owned_lane = lane >= 1 && lane <= l_last;
    const int l_ring = l_last + 1;
    const bool xghost_e = (i0 + l_last == M.nx) && M.bc_kind[BCE] != BC_PERIODIC;
    const bool xghost_w = (i0 == 0) && M.bc_kind[BCW] != BC_PERIODIC;
    int ci, gxin;
    column_index(M, col, ci, gxin);
    const Ghosts G = make_ghosts(M, gxin);
    // the cell's state (the INFLOW ghost's values replace h and hu)
    double h = (double)S.h[ci];
    double hu = (double)S.hu[ci];
    const double z = (double)S.z[ci];
    const double ag = Agf ? Agf[ci] : G.ag;
    if (gxin >= 0) {
        h = G.xh;
        hu = G.xhu;
    }
    if (ctrl->err) return;                              // a previous step failed
    const StepTime st = step_time(M, ctrl, n, cfl, t_end, fixed_dt);
    if (blockIdx.x == 0 && lane == 0) step_bookkeeping(ctrl, n, st);
    const double dt = st.dt, lx = dt / M.dx;

    const Cell P = project<CL>(M, h, hu, 0.0, z, ag);
    Flux X;
    unsigned e;
    if constexpr (WB) {
        double sp;
        e = wb_iface_flux<CL, true>(M, P, ag, next_cell(P), dpp<DPP_NEXT>(ag), X, sp);
    } else {
        e = iface_flux(side_x(P), next_side_x(P), M.g, X);
    }
    const double dXh = X.Fh - dpp<DPP_PREV>(X.Fh);
    const double dXm = X.FhuL - dpp<DPP_PREV>(X.FhuR);
    const double dXz = X.Fz - dpp<DPP_PREV>(X.Fz);
    const unsigned eX = e | dpp_u<DPP_PREV>(e);
    double hn = h - lx * dXh;
    double hun = hu - lx * dXm;
    double hvn = 0.0;
    double zn = z - lx * dXz;
    if (M.momentum_friction) apply_friction(M, dt, hn, hun, hvn);
    if (owned_lane) {
        const unsigned ee = check_state(hn, hun, 0.0, zn) | eX;
        if (ee) record_error(ctrl, ee, n);
        store_cell(M, D, (long long)col, hn, hun, 0.0, zn);
    }
    if (SPEEDS) {
        // wave speeds of the new state as stored (FP32 storage rounds it)
        hn = (double)(T)hn;
        hun = (double)(T)hun;
        zn = (double)(T)zn;
        if (xghost_e) {                                 // ring lane is the east ghost
            const double a = dpp<DPP_PREV>(hn), b = dpp<DPP_PREV>(hun), d = dpp<DPP_PREV>(zn);
            if (lane == l_ring) {
                hn = a; hun = b; zn = d;
                ghost_from(M, BCE, hn, hun, hvn);
            }
        }
        if (xghost_w) {                                 // lane 0 is the west ghost
            const double a = dpp<DPP_NEXT>(hn), b = dpp<DPP_NEXT>(hun), d = dpp<DPP_NEXT>(zn);
            if (lane == 0) {
                hn = a; hun = b; zn = d;
                ghost_from(M, BCW, hn, hun, hvn);
            }
        }
        hvn = 0.0;
        const Cell PN = project<CL>(M, hn, hun, 0.0, zn, ag);
        double s;
        if constexpr (WB) {
            s = wb_iface_speed<CL, true>(M, PN, ag, next_cell(PN), dpp<DPP_NEXT>(ag));
        } else {
            const Side Nx = side_x(PN);
            s = iface_speed(Nx, next_speed_side(Nx), M.g);
        }
        double sx = (owned_lane || (lane == 0 && xghost_w)) ? s : 0.0;
        sx = wave_max(sx);
        if (lane == 0) post_speeds(ctrl, (n + 1) % 3, blockIdx.x, sx, 0.0);
    }
}

template <typename T, bool SPEEDS, bool WB>
void launch_cl(const Model& M, StateView<T> S, StateView<T> D, const double* Ag, Ctrl* ctrl,
               int n, double cfl, double t_end, double fixed_dt, hipStream_t stream) {
    const int cl = closure_class(M);
    auto kern = cl == CL_GRASS3 ? k_fused_1d<T, CL_GRASS3, SPEEDS, WB>
              : cl == CL_GRASS1 ? k_fused_1d<T, CL_GRASS1, SPEEDS, WB>
              : cl == CL_GRASSM ? k_fused_1d<T, CL_GRASSM, SPEEDS, WB>
              : cl == CL_MPM    ? k_fused_1d<T, CL_MPM, SPEEDS, WB>
                                : k_fused_1d<T, CL_THRESH, SPEEDS, WB>;
    const unsigned tiles = (unsigned)((M.nx + FUSED_OWN - 1) / FUSED_OWN);
    hipLaunchKernelGGL(kern, dim3(tiles), dim3(64), 0, stream, M, S, D, Ag, ctrl, n, cfl, t_end,
                       fixed_dt);
}

}  // namespace

template <typename T>
void launch_fused_1d(const Model& M, StateView<T> S, StateView<T> D, const double* Ag,
                     Ctrl* ctrl, int n, double cfl, double t_end, double fixed_dt,
                     hipStream_t stream) {
    const bool speeds = !(fixed_dt > 0.0);
    if (M.wb) {
        if (speeds) launch_cl<T, true, true>(M, S, D, Ag, ctrl, n, cfl, t_end, fixed_dt, stream);
        else launch_cl<T, false, true>(M, S, D, Ag, ctrl, n, cfl, t_end, fixed_dt, stream);
    } else {
        if (speeds) launch_cl<T, true, false>(M, S, D, Ag, ctrl, n, cfl, t_end, fixed_dt, stream);
        else launch_cl<T, false, false>(M, S, D, Ag, ctrl, n, cfl, t_end, fixed_dt, stream);
    }
}

template void launch_fused_1d<double>(const Model&, StateView<double>, StateView<double>,
                                      const double*, Ctrl*, int, double, double, double,
                                      hipStream_t);
template void launch_fused_1d<float>(const Model&, StateView<float>, StateView<float>,
                                     const double*, Ctrl*, int, double, double, double,
                                     hipStream_t);

}  // namespace sve
