// sve_kernels.hpp -- step kernels of the relaxation scheme (gfx950).
//
//   k_speeds   one thread per interface: outer wave speed, wavefront and
//              workgroup max, one 64-bit atomicMax per workgroup and
//              direction (non-negative doubles order like their bit
//              patterns).
//   k_update   one thread per cell: five-point stencil, four interface
//              solves, conservative update (split path and reference).
// plus the per-cell helpers the row kernels share (error bits, stores,
// friction, step bookkeeping).  The one-pass 2D kernels are in
// sve_fused.hpp (k_fused) and sve_residual.hpp (k_resid), the 1D
// LDS-resident kernel in sve_resident.hpp.
#pragma once

#include "sve_device.hpp"

namespace sve {

constexpr int SPEED_BLOCK = 256;
constexpr int UPDATE_BLOCK = 256;

__device__ __forceinline__ void record_error(Ctrl* ctrl, unsigned bits, int n) {
    atomicOr(&ctrl->err, bits);
    atomicMin(&ctrl->fail_step, n);
}

// Workgroup max of non-negative values; thread 0 returns the result.
template <int BLOCK>
__device__ __forceinline__ double block_max(double v, double* sh) {
    v = wave_max(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < BLOCK / 64; ++w) r = fmax(r, sh[w]);
    }
    return r;
}

template <typename T, int CL, bool WB>
__global__ void __launch_bounds__(SPEED_BLOCK)
k_speeds(Model M, StateView<T> S, const double* __restrict__ Agf, Ctrl* ctrl, int slot) {
    __shared__ double sh[2][SPEED_BLOCK / 64];
    if (ctrl->err) return;
    const long long nxi = (long long)(M.nx + 1) * M.ny;              // x-interfaces
    const long long nyi = (M.dim == 2) ? (long long)M.nx * (M.ny + 1) : 0;
    const long long t = (long long)blockIdx.x * SPEED_BLOCK + threadIdx.x;
    double sx = 0.0, sy = 0.0;
    if (t < nxi) {
        const int j = (int)(t / (M.nx + 1)), m = (int)(t % (M.nx + 1));
        double h, hu, hv, z, agL, agR;
        fetch(M, S, Agf, m - 1, j, h, hu, hv, z, agL);
        const Cell L = project<CL>(M, h, hu, hv, z, agL);
        fetch(M, S, Agf, m, j, h, hu, hv, z, agR);
        const Cell R = project<CL>(M, h, hu, hv, z, agR);
        sx = WB ? wb_iface_speed<CL, true>(M, L, agL, R, agR)
                : iface_speed(side_x(L), side_x(R), M.g);
    } else if (t < nxi + nyi) {
        const long long u = t - nxi;
        const int i = (int)(u % M.nx), m = (int)(u / M.nx);
        double h, hu, hv, z, agL, agR;
        fetch(M, S, Agf, i, m - 1, h, hu, hv, z, agL);
        const Cell L = project<CL>(M, h, hu, hv, z, agL);
        fetch(M, S, Agf, i, m, h, hu, hv, z, agR);
        const Cell R = project<CL>(M, h, hu, hv, z, agR);
        sy = WB ? wb_iface_speed<CL, false>(M, L, agL, R, agR)
                : iface_speed(side_y(L), side_y(R), M.g);
    }
    const double bx = block_max<SPEED_BLOCK>(sx, sh[0]);
    const double by = block_max<SPEED_BLOCK>(sy, sh[1]);
    if (threadIdx.x == 0) {
        post_speeds(ctrl, slot, blockIdx.x, bx, by);
    }
}

// Outer wave speeds of the state S into slot `slot` of the control block
// (one thread per interface).
template <typename T>
void launch_speeds_model(const Model& M, StateView<T> S, const double* Ag, Ctrl* ctrl, int slot,
                         hipStream_t stream) {
    const long long nint = (long long)(M.nx + 1) * M.ny +
                           (M.dim == 2 ? (long long)M.nx * (M.ny + 1) : 0);
    const unsigned blocks = (unsigned)((nint + SPEED_BLOCK - 1) / SPEED_BLOCK);
    const int cl = closure_class(M);
    auto kern = M.wb ? (cl == CL_GRASS3 ? k_speeds<T, CL_GRASS3, true>
                      : cl == CL_GRASS1 ? k_speeds<T, CL_GRASS1, true>
                      : cl == CL_GRASSM ? k_speeds<T, CL_GRASSM, true>
                      : cl == CL_MPM    ? k_speeds<T, CL_MPM, true>
                                        : k_speeds<T, CL_THRESH, true>)
                     : (cl == CL_GRASS3 ? k_speeds<T, CL_GRASS3, false>
                      : cl == CL_GRASS1 ? k_speeds<T, CL_GRASS1, false>
                      : cl == CL_GRASSM ? k_speeds<T, CL_GRASSM, false>
                      : cl == CL_MPM    ? k_speeds<T, CL_MPM, false>
                                        : k_speeds<T, CL_THRESH, false>);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(SPEED_BLOCK), 0, stream, M, S, Ag, ctrl, slot);
}

// Per-step bookkeeping done by one thread of step n: time of step n+1,
// last dt, and clearing of the maxima slot used by step n+2.
__device__ __forceinline__ void step_bookkeeping(Ctrl* ctrl, int n, const StepTime& st) {
    ctrl->t[(n + 1) % 3] = st.tnew;
    ctrl->dt_last = st.dt;
    clear_speeds(ctrl, (n + 2) % 3);
}

template <typename T>
__device__ __forceinline__ void store_cell(const Model& M, const StateView<T>& D, long long k,
                                           double h, double hu, double hv, double z) {
    D.h[k] = (T)h;
    D.hu[k] = (T)hu;
    if (M.dim == 2) D.hv[k] = (T)hv;
    D.z[k] = (T)z;
}

__device__ __forceinline__ unsigned check_state(double h, double hu, double hv, double z) {
    unsigned e = 0;
    if (!(fabs(h) < INFINITY && fabs(hu) < INFINITY && fabs(hv) < INFINITY && fabs(z) < INFINITY))
        e |= ERR_NONFIN;
    else if (!(h > 0.0))
        e |= ERR_POS;
    return e;
}

__device__ __forceinline__ void apply_friction(const Model& M, double dt, double h, double& hu,
                                               double& hv) {
    const double u = hu / h, v = hv / h;
    const double phi = friction_phi(M, h, sqrt(u * u + v * v));
    const double den = 1.0 + dt * phi;
    hu = hu / den;
    hv = hv / den;
}

// Interface flux between projected cells A and B (A left of or below B):
// the relaxation solve, or that of the hydrostatic reconstruction (WB).
template <int CL, bool WB, bool NX>
__device__ __forceinline__ unsigned cell_flux(const Model& M, const Cell& A, double agA,
                                              const Cell& B, double agB, Flux& F) {
    double sp;
    if (WB) return wb_iface_flux<CL, NX>(M, A, agA, B, agB, F, sp);
    return NX ? iface_flux(side_x(A), side_x(B), M.g, F, sp)
              : iface_flux(side_y(A), side_y(B), M.g, F, sp);
}

template <typename T, int CL, bool WB>
__global__ void __launch_bounds__(UPDATE_BLOCK)
k_update(Model M, StateView<T> S, StateView<T> D, const double* __restrict__ Agf, Ctrl* ctrl,
         int n, double cfl, double t_end, double fixed_dt) {
    if (ctrl->err) return;
    const StepTime st = step_time(M, ctrl, n, cfl, t_end, fixed_dt);
    if (blockIdx.x == 0 && threadIdx.x == 0) step_bookkeeping(ctrl, n, st);
    const long long N = (long long)M.nx * M.ny;
    const long long k = (long long)blockIdx.x * UPDATE_BLOCK + threadIdx.x;
    if (k >= N) return;
    const int i = (int)(k % M.nx), j = (int)(k / M.nx);
    double h, hu, hv, z, agC, agW, agE;
    fetch(M, S, Agf, i, j, h, hu, hv, z, agC);
    const Cell C = project<CL>(M, h, hu, hv, z, agC);
    fetch(M, S, Agf, i - 1, j, h, hu, hv, z, agW);
    const Cell W = project<CL>(M, h, hu, hv, z, agW);
    fetch(M, S, Agf, i + 1, j, h, hu, hv, z, agE);
    const Cell E = project<CL>(M, h, hu, hv, z, agE);
    Flux fl, fr;
    unsigned err = cell_flux<CL, WB, true>(M, W, agW, C, agC, fl);
    err |= cell_flux<CL, WB, true>(M, C, agC, E, agE, fr);
    const double lx = st.dt / M.dx;
    double hn, hun, hvn, zn;
    if (M.dim == 2) {
        double agS, agN;
        fetch(M, S, Agf, i, j - 1, h, hu, hv, z, agS);
        const Cell So = project<CL>(M, h, hu, hv, z, agS);
        fetch(M, S, Agf, i, j + 1, h, hu, hv, z, agN);
        const Cell No = project<CL>(M, h, hu, hv, z, agN);
        Flux gb, gt;
        err |= cell_flux<CL, WB, false>(M, So, agS, C, agC, gb);
        err |= cell_flux<CL, WB, false>(M, C, agC, No, agN, gt);
        const double ly = st.dt / M.dy;
        hn = C.h - lx * (fr.Fh - fl.Fh) - ly * (gt.Fh - gb.Fh);
        hun = C.hu - lx * (fr.FhuL - fl.FhuR) - ly * (gt.Fht - gb.Fht);
        hvn = C.hv - lx * (fr.Fht - fl.Fht) - ly * (gt.FhuL - gb.FhuR);
        zn = C.z - lx * (fr.Fz - fl.Fz) - ly * (gt.Fz - gb.Fz);
    } else {
        hn = C.h - lx * (fr.Fh - fl.Fh);
        hun = C.hu - lx * (fr.FhuL - fl.FhuR);
        hvn = 0.0;
        zn = C.z - lx * (fr.Fz - fl.Fz);
    }
    if (M.momentum_friction) apply_friction(M, st.dt, hn, hun, hvn);
    err |= check_state(hn, hun, hvn, zn);
    if (err) record_error(ctrl, err, n);
    store_cell(M, D, k, hn, hun, hvn, zn);
}

// State initialisation: convert caller doubles to storage type and check.
template <typename T>
__global__ void k_load_state(Model M, const double* __restrict__ h, const double* __restrict__ hu,
                             const double* __restrict__ hv, const double* __restrict__ z,
                             StateView<T> D, Ctrl* ctrl) {
    const long long N = (long long)M.nx * M.ny;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double vh = h[k], vhu = hu[k], vhv = hv ? hv[k] : 0.0, vz = z[k];
    unsigned e = check_state(vh, vhu, vhv, vz);
    if (e) atomicOr(&ctrl->err, e);
    store_cell(M, D, k, vh, vhu, vhv, vz);
}

template <typename T>
__global__ void k_store_state(Model M, StateView<T> S, double* h, double* hu, double* hv,
                              double* z) {
    const long long N = (long long)M.nx * M.ny;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    if (h) h[k] = (double)S.h[k];
    if (hu) hu[k] = (double)S.hu[k];
    if (hv) hv[k] = (M.dim == 2) ? (double)S.hv[k] : 0.0;
    if (z) z[k] = (double)S.z[k];
}

static __global__ void k_reset_ctrl(Ctrl* ctrl, double t0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int s = 0; s < 3; ++s) {
            clear_speeds(ctrl, s);
            ctrl->t[s] = t0;
        }
        ctrl->dt_last = 0.0;
        ctrl->err = 0u;
        ctrl->fail_step = 0x7fffffff;
    }
}

static __global__ void k_clear_slot(Ctrl* ctrl, int slot) {
    if (threadIdx.x == 0 && blockIdx.x == 0) clear_speeds(ctrl, slot);
}

template <typename T>
__global__ void k_poke(StateView<T> S, int field, long long k, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        T* p = field == 0 ? S.h : field == 1 ? S.hu : field == 2 ? S.hv : S.z;
        p[k] = (T)v;
    }
}

}  // namespace sve
