// sve_resident.hpp -- 1D grids that fit in LDS: one workgroup holds the
// whole state and runs all requested steps in one launch (the 1D dune of
// the paper has 1000 cells: a grid-wide pass per step would be launch-bound).
//
// Per step: one pass over the interfaces gives the fluxes (into LDS) and
// the outer wave speeds of the current state (reduced in LDS into the time
// step), barrier, cell update in place (the old cells kept in registers),
// barrier; on an error every thread writes its old cells back.  The loop ends after n steps, or early when t
// reaches t_end (the remaining steps would leave the state unchanged) or on
// an error (the state before the failing step is kept).
#pragma once

#include "sve_context.hpp"
#include "sve_kernels.hpp"

namespace sve {

constexpr int RES_BLOCK = 1024;
// cells per thread: the LDS of one workgroup (160 KiB, 56 B per cell) holds
// at most 2922 cells, so three per thread cover every grid that fits
constexpr int RES_PER_THREAD = 3;
constexpr int RES_NMAX = RES_BLOCK * RES_PER_THREAD;
// Largest grid the resident kernel is chosen for by default.  Its step time
// grows with the cells per thread (2.5, 3.7, 4.7, 6.0 and 8.4 us at 500,
// 1000, 1500, 2000 and 2922 cells), while the one-pass 1D kernel takes
// about 4.8 us at any size up to 20 000 cells (latency of one launch); the
// two meet near 1500 cells.
constexpr int RES_DEFAULT_NMAX = 1536;

// Threads of the workgroup for a closure.  1024 threads leave 128 VGPRs a
// thread; the general Grass exponent and the run-time threshold laws need
// more (at 1024 they spilled 17 to 48 VGPRs), so they run 512 threads with
// six cells each.
template <int CL>
constexpr int res_block() {
    return (CL == CL_GRASSM || CL == CL_THRESH) ? RES_BLOCK / 2 : RES_BLOCK;
}

// LDS layout, carved from dynamic shared memory sized for nx.
struct ResLds {
    double *h, *hu, *z;                // nx each
    double *Fh, *FL, *FR, *Fz;         // nx + 1 each
    double* red;                       // RES_BLOCK / 64
    unsigned* err;
};

__host__ __device__ inline size_t res_lds_bytes(int nx) {
    return sizeof(double) * (3 * (size_t)nx + 4 * ((size_t)nx + 1) + RES_BLOCK / 64) + 16;
}

__device__ __forceinline__ ResLds res_carve(double* base, int nx) {
    ResLds L;
    L.h = base;
    L.hu = L.h + nx;
    L.z = L.hu + nx;
    L.Fh = L.z + nx;
    L.FL = L.Fh + nx + 1;
    L.FR = L.FL + nx + 1;
    L.Fz = L.FR + nx + 1;
    L.red = L.Fz + nx + 1;
    L.err = reinterpret_cast<unsigned*>(L.red + RES_BLOCK / 64);
    return L;
}

__device__ __forceinline__ void res_cell(const Model& M, const ResLds& L,
                                         const double* __restrict__ Agf, int i, double& h,
                                         double& hu, double& z, double& ag) {
    int ii = i, g = -1;
    if (i < 0) {
        if (M.bc_kind[BCW] == BC_PERIODIC) ii = M.nx - 1; else { ii = 0; g = BCW; }
    } else if (i >= M.nx) {
        if (M.bc_kind[BCE] == BC_PERIODIC) ii = 0; else { ii = M.nx - 1; g = BCE; }
    }
    h = L.h[ii];
    hu = L.hu[ii];
    z = L.z[ii];
    ag = Agf ? Agf[ii] : M.Ag;
    if (g >= 0 && M.bc_kind[g] == BC_INFLOW) { h = M.bc_h[g]; hu = M.bc_hu[g]; }
}

template <int CL, bool WB, int BLOCK>
__device__ __forceinline__ double res_max_speed(const Model& M, const ResLds& L,
                                                const double* __restrict__ Agf) {
    double s = 0.0;
    for (int m = threadIdx.x; m <= M.nx; m += BLOCK) {
        double h, hu, z, agA, agB;
        res_cell(M, L, Agf, m - 1, h, hu, z, agA);
        const Cell A = project<CL>(M, h, hu, 0.0, z, agA);
        res_cell(M, L, Agf, m, h, hu, z, agB);
        const Cell B = project<CL>(M, h, hu, 0.0, z, agB);
        s = fmax(s, WB ? wb_iface_speed<CL, true>(M, A, agA, B, agB)
                       : iface_speed(side_x(A), side_x(B), M.g));
    }
    s = wave_max(s);
    if ((threadIdx.x & 63) == 0) L.red[threadIdx.x >> 6] = s;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) r = fmax(r, L.red[w]);
    __syncthreads();
    return r;
}

template <typename T, int CL, bool WB, int BLOCK = res_block<CL>()>
__global__ void __launch_bounds__(BLOCK)
k_resident_1d(Model M, StateView<T> S, StateView<T> D, const double* __restrict__ Agf,
              Ctrl* ctrl, int n0, int nsteps, double cfl, double t_end, double fixed_dt) {
    extern __shared__ double lds_raw[];
    ResLds L = res_carve(lds_raw, M.nx);
    if (ctrl->err) return;
    constexpr int PER_THREAD = RES_NMAX / BLOCK;
    const int nx = M.nx;
    for (int i = threadIdx.x; i < nx; i += BLOCK) {
        L.h[i] = (double)S.h[i];
        L.hu[i] = (double)S.hu[i];
        L.z[i] = (double)S.z[i];
    }
    if (threadIdx.x == 0) *L.err = 0u;
    __syncthreads();
    const bool cfl_mode = !(fixed_dt > 0.0);
    double t = ctrl->t[n0 % 3];
    double S_cur = 0.0;                              // outer wave speed of the state in LDS
    bool S_known = false;
    double dt_last = ctrl->dt_last;
    int done = 0;
    unsigned err = 0u;
    for (; done < nsteps; ++done) {
        if (cfl_mode && t_end > 0.0 && t >= t_end) {   // remaining steps are no-ops
            done = nsteps;
            dt_last = 0.0;
            break;
        }
        // fluxes and outer wave speeds of the current state
        unsigned e = 0u;
        double s = 0.0;
        for (int m = threadIdx.x; m <= nx; m += BLOCK) {
            double h, hu, z, agA, agB;
            res_cell(M, L, Agf, m - 1, h, hu, z, agA);
            const Cell A = project<CL>(M, h, hu, 0.0, z, agA);
            res_cell(M, L, Agf, m, h, hu, z, agB);
            const Cell B = project<CL>(M, h, hu, 0.0, z, agB);
            Flux F;
            double sp;
            e |= WB ? wb_iface_flux<CL, true>(M, A, agA, B, agB, F, sp)
                    : iface_flux(side_x(A), side_x(B), M.g, F, sp);
            s = dmax(s, sp);
            L.Fh[m] = F.Fh;
            L.FL[m] = F.FhuL;
            L.FR[m] = F.FhuR;
            L.Fz[m] = F.Fz;
        }
        if (cfl_mode) {
            s = wave_max(s);
            if ((threadIdx.x & 63) == 0) L.red[threadIdx.x >> 6] = s;
        }
        __syncthreads();
        double dt, tnew;
        if (cfl_mode) {
            S_cur = 0.0;
            for (int w = 0; w < BLOCK / 64; ++w) S_cur = fmax(S_cur, L.red[w]);
            S_known = true;
            dt = cfl * M.dx / S_cur;
            tnew = t + dt;
            if (t_end > 0.0 && dt >= t_end - t) {
                dt = t_end - t;
                tnew = t_end;
            }
        } else {
            dt = fixed_dt;
            tnew = t + dt;
        }
        const double lx = dt / M.dx;
        // new state written in place (each thread reads and writes only its
        // own cells here); the old state stays in registers (constant
        // indices after unrolling) until the step is known to be free of
        // errors, and is written back if it is not
        double oh[PER_THREAD], ohu[PER_THREAD], oz[PER_THREAD];
#pragma unroll
        for (int c = 0; c < PER_THREAD; ++c) {
            const int i = threadIdx.x + c * BLOCK;
            if (i >= nx) continue;
            oh[c] = L.h[i];
            ohu[c] = L.hu[i];
            oz[c] = L.z[i];
            double hn = oh[c] - lx * (L.Fh[i + 1] - L.Fh[i]);
            double hun = ohu[c] - lx * (L.FL[i + 1] - L.FR[i]);
            double zn = oz[c] - lx * (L.Fz[i + 1] - L.Fz[i]);
            if (M.momentum_friction) {
                double hvn = 0.0;
                apply_friction(M, dt, hn, hun, hvn);
            }
            e |= check_state(hn, hun, 0.0, zn);
            L.h[i] = (double)(T)hn;
            L.hu[i] = (double)(T)hun;
            L.z[i] = (double)(T)zn;
        }
        if (e) atomicOr(L.err, e);
        __syncthreads();
        err = *L.err;
        if (err) {                                   // keep the state before this step
#pragma unroll
            for (int c = 0; c < PER_THREAD; ++c) {
                const int i = threadIdx.x + c * BLOCK;
                if (i >= nx) continue;
                L.h[i] = oh[c];
                L.hu[i] = ohu[c];
                L.z[i] = oz[c];
            }
            __syncthreads();
            break;
        }
        t = tnew;
        dt_last = dt;
        S_known = false;
    }
    // outer wave speed of the state left in LDS, for the next call's first step
    if (cfl_mode && !S_known) S_cur = res_max_speed<CL, WB, BLOCK>(M, L, Agf);
    // write back the last good state into the buffer the host expects
    const StateView<T>& out = (done & 1) ? D : S;
    for (int i = threadIdx.x; i < nx; i += BLOCK) {
        out.h[i] = (T)L.h[i];
        out.hu[i] = (T)L.hu[i];
        out.z[i] = (T)L.z[i];
    }
    if (threadIdx.x == 0) {
        const int nend = n0 + done;
        if (err) {
            atomicOr(&ctrl->err, err);
            atomicMin(&ctrl->fail_step, nend);
        }
        ctrl->t[nend % 3] = t;
        ctrl->dt_last = dt_last;
        for (int k = 0; k < 3; ++k) clear_speeds(ctrl, k);
        ctrl->smax[nend % 3][0][0] = cfl_mode ? double_as_u64(S_cur) : 0ull;
    }
}

}  // namespace sve

inline bool resident_supported(const sve_ctx* c) {
    if (c->M.dim != 1 || c->M.nx > sve::RES_NMAX || c->M.order == 2) return false;
    int dev = 0, max_lds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
        hipSuccess)
        return false;
    return sve::res_lds_bytes(c->M.nx) <= (size_t)max_lds;
}

template <typename T>
void launch_resident(sve_ctx* c, int n, double cfl, double t_end, double fixed_dt) {
    using namespace sve;
    const int src = c->cur, dst = src ^ 1;
    StateView<T> S, D;
    T* b0 = static_cast<T*>(c->buf[src]);
    T* b1 = static_cast<T*>(c->buf[dst]);
    S = StateView<T>{b0, b0 + c->pitch, b0 + 2 * c->pitch, b0 + 3 * c->pitch};
    D = StateView<T>{b1, b1 + c->pitch, b1 + 2 * c->pitch, b1 + 3 * c->pitch};
    const size_t lds = res_lds_bytes(c->M.nx);
    const int cl = closure_class(c->M);
    const bool wb = c->M.wb;
    auto kern = wb ? (cl == CL_GRASS3 ? k_resident_1d<T, CL_GRASS3, true>
                    : cl == CL_GRASS1 ? k_resident_1d<T, CL_GRASS1, true>
                    : cl == CL_GRASSM ? k_resident_1d<T, CL_GRASSM, true>
                    : cl == CL_MPM    ? k_resident_1d<T, CL_MPM, true>
                                      : k_resident_1d<T, CL_THRESH, true>)
                   : (cl == CL_GRASS3 ? k_resident_1d<T, CL_GRASS3, false>
                    : cl == CL_GRASS1 ? k_resident_1d<T, CL_GRASS1, false>
                    : cl == CL_GRASSM ? k_resident_1d<T, CL_GRASSM, false>
                    : cl == CL_MPM    ? k_resident_1d<T, CL_MPM, false>
                                      : k_resident_1d<T, CL_THRESH, false>);
    const int block = (cl == CL_GRASSM || cl == CL_THRESH) ? res_block<CL_GRASSM>() : RES_BLOCK;
    static_assert(res_block<CL_GRASSM>() == res_block<CL_THRESH>() &&
                      res_block<CL_GRASS3>() == RES_BLOCK && res_block<CL_GRASS1>() == RES_BLOCK &&
                      res_block<CL_MPM>() == RES_BLOCK,
                  "launch block sizes follow res_block");
    hipLaunchKernelGGL(kern, dim3(1), dim3(block), lds, c->stream,
                       c->M, S, D, (const double*)c->Ag, c->ctrl, (int)c->nsteps, n, cfl, t_end,
                       fixed_dt);
}
