// sve_context.hpp -- host-side context of one solver instance.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/sve.h"
#include "sve_device.hpp"

struct sve_adjoint_state;

struct sve_ctx {
    sve::Model M;
    int storage = SVE_FP64;
    long long N = 0;        // nx * ny
    long long pitch = 0;    // elements between fields (multiple of 64)
    void* buf[2] = {nullptr, nullptr};   // double-buffered state, 4 fields each
    double* Ag = nullptr;   // per-cell Grass constant, or null
    sve::Ctrl* ctrl = nullptr;
    sve::Ctrl* h_ctrl = nullptr;         // pinned host mirror of ctrl
    double* staging = nullptr;           // 4*N doubles for host transfers
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int cur = 0;                // buffer holding the current state
    long long nsteps = 0;
    double t = 0.0, dt_last = 0.0;
    int path = SVE_PATH_FUSED;
    int fused_ty = 0;           // tile rows of the fused kernel (0: automatic)
    int adj_ty = 0;             // tile rows of the reverse-step kernel (0: automatic)
    int wave_slots = 2048;      // resident wavefronts of the step kernels on the device
    int sticky = SVE_OK;
    bool speeds_valid = false;  // slot nsteps%3 holds the speeds of the state
    double* rbuf[2] = {nullptr, nullptr};  // residuals of the residual path, rate D0 of the
                                           // second-order variant (FP64, 4 fields)
    bool resid_valid = false;   // rbuf[cur] and slot nsteps%3 belong to the state
    bool last_resid = false;    // the last run_steps used the residual path
    int pending = SVE_OK;       // error of the step after the last call (residual path)
    double last_ms = 0.0;
    sve_adjoint_state* adj = nullptr;
};

namespace sve {
Model make_model(int nx, int ny, double Lx, double Ly, int dim, const sve_params* p,
                 const sve_bc* bc);
// SVE_OK when the model parameters and boundary conditions are valid for a
// grid of dimension `dim`, else SVE_ERR_ARG.
int validate_params(const sve_params* p, int dim, const sve_bc* bc);

// Second-order variant (sve_order2.hip): launch of the step's first
// (stage2 = false: rate D0 of U^n into R, wave speeds into slot n%3) or
// second kernel (U^{n+1} into D).  rows: tile height (0: automatic, from
// the device's `cus` compute units and the kernel's occupancy).
template <typename T>
void launch_order2(const Model& M, StateView<T> S, StateView<double> R, StateView<T> D,
                   const double* Ag, Ctrl* ctrl, int n, double cfl, double t_end,
                   double fixed_dt, int rows, int cus, bool stage2, hipStream_t stream);

// One-pass 1D step (sve_fused1d.hip): update of step n from S into D and,
// in CFL mode (fixed_dt <= 0), the wave speeds of the new state into slot
// (n+1)%3.
template <typename T>
void launch_fused_1d(const Model& M, StateView<T> S, StateView<T> D, const double* Ag,
                     Ctrl* ctrl, int n, double cfl, double t_end, double fixed_dt,
                     hipStream_t stream);
}

// Frees the adjoint buffers of a context (defined with the adjoint).
void sve_adjoint_release(sve_ctx* ctx);
