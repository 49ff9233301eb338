// sve_api.hip -- C ABI of the solver (declarations and contracts in sve.h).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "../../include/sve.h"
#include "sve_context.hpp"
#include "sve_kernels.hpp"
#include "sve_fused.hpp"
#include "sve_resident.hpp"
#include "sve_residual.hpp"

using namespace sve;

namespace {

inline long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

template <typename T>
StateView<T> view_of(sve_ctx* c, int b) {
    T* base = static_cast<T*>(c->buf[b]);
    StateView<T> v;
    v.h = base;
    v.hu = base + c->pitch;
    v.hv = base + 2 * c->pitch;
    v.z = base + 3 * c->pitch;
    return v;
}

// HIP failures are reported as SVE_ERR_HIP; with SVE_VERBOSE set in the
// environment the failing call and the runtime's message go to stderr.
int hip_fail(hipError_t e, const char* what, int line) {
    static const bool verbose = std::getenv("SVE_VERBOSE") != nullptr;
    if (verbose)
        std::fprintf(stderr, "sve: %s failed at line %d: %s\n", what, line, hipGetErrorString(e));
    return SVE_ERR_HIP;
}
#define HIP_OK(call) ((call) == hipSuccess)
#define HIP_TRY(call)                                               \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return hip_fail(e_, #call, __LINE__); \
    } while (0)

int check_hip(hipError_t e) { return e == hipSuccess ? SVE_OK : hip_fail(e, "HIP call", 0); }

int code_from_bits(unsigned bits) {
    if (bits & ERR_NONFIN) return SVE_ERR_NONFINITE;
    if (bits & ERR_POS) return SVE_ERR_POSITIVITY;
    if (bits & ERR_ORD) return SVE_ERR_ORDER;
    return SVE_OK;
}

}  // namespace

int sve::validate_params(const sve_params* p, int dim, const sve_bc* bc) {
    if (!p || !bc) return SVE_ERR_ARG;
    if (!(p->g > 0.0) || !std::isfinite(p->g)) return SVE_ERR_ARG;
    if (p->law < SVE_LAW_GRASS || p->law > SVE_LAW_CAMENEN) return SVE_ERR_ARG;
    if (p->reconstruction != 0 && p->reconstruction != 1) return SVE_ERR_ARG;
    if (p->order < 0 || p->order > 2) return SVE_ERR_ARG;
    if (p->law == SVE_LAW_GRASS) {
        if (!(p->m_g >= 1.0 && p->m_g <= 4.0)) return SVE_ERR_ARG;
        if (!std::isfinite(p->A_g)) return SVE_ERR_ARG;
    } else {
        if (!(p->d_s > 0.0) || !(p->s > 1.0) || !(p->tau_cr >= 0.0)) return SVE_ERR_ARG;
    }
    if (p->law != SVE_LAW_GRASS || p->momentum_friction) {
        if (p->friction < SVE_FRIC_STRICKLER || p->friction > SVE_FRIC_DARCY) return SVE_ERR_ARG;
        if (!(p->fric_coef > 0.0)) return SVE_ERR_ARG;
    }
    const int nb = dim == 2 ? 4 : 2;
    for (int s = 0; s < nb; ++s) {
        if (bc[s].kind < SVE_BC_PERIODIC || bc[s].kind > SVE_BC_INFLOW) return SVE_ERR_ARG;
        if (bc[s].kind == SVE_BC_INFLOW && !(bc[s].h > 0.0)) return SVE_ERR_ARG;
    }
    // periodicity must be set on both sides of a direction
    if ((bc[0].kind == SVE_BC_PERIODIC) != (bc[1].kind == SVE_BC_PERIODIC)) return SVE_ERR_ARG;
    if (dim == 2 && (bc[2].kind == SVE_BC_PERIODIC) != (bc[3].kind == SVE_BC_PERIODIC))
        return SVE_ERR_ARG;
    return SVE_OK;
}

Model sve::make_model(int nx, int ny, double Lx, double Ly, int dim, const sve_params* p,
                      const sve_bc* bc) {
    Model M;
    std::memset(&M, 0, sizeof(M));
    M.law = p->law;
    M.friction = p->friction;
    M.momentum_friction = p->momentum_friction ? 1 : 0;
    M.wb = p->reconstruction ? 1 : 0;
    M.order = p->order == 2 ? 2 : 1;
    M.mg_is3 = (p->m_g == 3.0);
    M.mg_is1 = (p->m_g == 1.0);
    M.nx = nx;
    M.ny = ny;
    M.dim = dim;
    M.g = p->g;
    M.Ag = p->A_g;
    M.mg = p->m_g;
    const double sm1 = p->s - 1.0;
    M.K = (p->law == SVE_LAW_GRASS) ? 0.0 : std::sqrt(sm1 * p->g * p->d_s * p->d_s * p->d_s);
    M.tau_cr = p->tau_cr;
    if (p->law != SVE_LAW_GRASS) {
        if (p->friction == SVE_FRIC_STRICKLER)
            M.c_const = 1.0 / (sm1 * p->d_s * p->fric_coef * p->fric_coef);
        else if (p->friction == SVE_FRIC_MANNING)
            M.c_const = p->fric_coef * p->fric_coef / (sm1 * p->d_s);
        else
            M.c_const = p->fric_coef / (8.0 * p->g * sm1 * p->d_s);
    }
    if (p->friction == SVE_FRIC_DARCY)
        M.phi_const = p->fric_coef / 8.0;
    else if (p->friction == SVE_FRIC_STRICKLER)
        M.phi_const = p->g / (p->fric_coef * p->fric_coef);
    else
        M.phi_const = p->g * p->fric_coef * p->fric_coef;
    M.dx = Lx / nx;
    M.dy = (dim == 2) ? Ly / ny : 1.0;
    const int nb = dim == 2 ? 4 : 2;
    for (int s = 0; s < 4; ++s) {
        const sve_bc b = s < nb ? bc[s] : sve_bc{SVE_BC_PERIODIC, 0, 0, 0};
        M.bc_kind[s] = b.kind;
        M.bc_h[s] = b.h;
        M.bc_hu[s] = b.hu;
        M.bc_hv[s] = b.hv;
    }
    return M;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
namespace {

template <typename T>
void launch_speeds(sve_ctx* c, int buf, int slot) {
    launch_speeds_model<T>(c->M, view_of<T>(c, buf), c->Ag, c->ctrl, slot, c->stream);
}

template <typename T>
void launch_update(sve_ctx* c, int src, int dst, int n, double cfl, double t_end,
                   double fixed_dt) {
    const Model& M = c->M;
    const long long N = (long long)M.nx * M.ny;
    const unsigned blocks = (unsigned)((N + UPDATE_BLOCK - 1) / UPDATE_BLOCK);
    const int cl = closure_class(M);
    auto kern = M.wb ? (cl == CL_GRASS3 ? k_update<T, CL_GRASS3, true>
                      : cl == CL_GRASS1 ? k_update<T, CL_GRASS1, true>
                      : cl == CL_GRASSM ? k_update<T, CL_GRASSM, true>
                      : cl == CL_MPM    ? k_update<T, CL_MPM, true>
                                        : k_update<T, CL_THRESH, true>)
                     : (cl == CL_GRASS3 ? k_update<T, CL_GRASS3, false>
                      : cl == CL_GRASS1 ? k_update<T, CL_GRASS1, false>
                      : cl == CL_GRASSM ? k_update<T, CL_GRASSM, false>
                      : cl == CL_MPM    ? k_update<T, CL_MPM, false>
                                        : k_update<T, CL_THRESH, false>);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(UPDATE_BLOCK), 0, c->stream, M,
                       view_of<T>(c, src), view_of<T>(c, dst), (const double*)c->Ag, c->ctrl,
                       n, cfl, t_end, fixed_dt);
}

template <typename T>
void launch_fused(sve_ctx* c, int src, int dst, int n, double cfl, double t_end,
                  double fixed_dt) {
    const int tiles_y = fused_tiles_y(c->M.nx, c->M.ny, c->fused_ty, c->wave_slots);
    if (c->M.wb)
        launch_fused_rows<T, true>(c->M, view_of<T>(c, src), view_of<T>(c, dst), c->Ag, c->ctrl,
                                   n, cfl, t_end, fixed_dt, tiles_y, c->stream);
    else
        launch_fused_rows<T>(c->M, view_of<T>(c, src), view_of<T>(c, dst), c->Ag, c->ctrl, n,
                             cfl, t_end, fixed_dt, tiles_y, c->stream);
}

StateView<double> rview(sve_ctx* c, int b) {
    double* p = c->rbuf[b];
    return StateView<double>{p, p + c->pitch, p + 2 * c->pitch, p + 3 * c->pitch};
}

// Second-order steps: two kernels per step (rate of U^n and wave speeds;
// then Heun's stages), the rate in rbuf[0].
template <typename T>
int run_steps_order2(sve_ctx* c, int n, double cfl, double t_end, double fixed_dt) {
    if (!c->rbuf[0])
        HIP_TRY(hipMalloc((void**)&c->rbuf[0], 4 * (size_t)c->pitch * sizeof(double)));
    const int cus = c->wave_slots / (4 * FUSED_WAVES_PER_SIMD);
    hipLaunchKernelGGL(k_clear_slot, dim3(1), dim3(64), 0, c->stream, c->ctrl,
                       (int)(c->nsteps % 3));
    (void)hipEventRecord(c->ev0, c->stream);
    for (int s = 0; s < n; ++s) {
        const int step = (int)(c->nsteps + s);
        const int src = (c->cur + s) & 1, dst = src ^ 1;
        launch_order2<T>(c->M, view_of<T>(c, src), rview(c, 0), view_of<T>(c, dst), c->Ag,
                         c->ctrl, step, cfl, t_end, fixed_dt, c->fused_ty, cus, false,
                         c->stream);
        launch_order2<T>(c->M, view_of<T>(c, src), rview(c, 0), view_of<T>(c, dst), c->Ag,
                         c->ctrl, step, cfl, t_end, fixed_dt, c->fused_ty, cus, true,
                         c->stream);
    }
    (void)hipEventRecord(c->ev1, c->stream);
    HIP_TRY(hipGetLastError());
    c->speeds_valid = false;
    c->resid_valid = false;
    c->last_resid = false;
    return SVE_OK;
}

template <typename T>
int run_steps(sve_ctx* c, int n, double cfl, double t_end, double fixed_dt) {
    if (c->M.order == 2) return run_steps_order2<T>(c, n, cfl, t_end, fixed_dt);
    const bool cfl_mode = !(fixed_dt > 0.0);
    // the residual path has no well-balanced variant: its steps run fused
    const bool resid = cfl_mode && c->path == SVE_PATH_RESIDUAL && c->M.dim == 2 && !c->M.wb;
    c->last_resid = resid;
    const int tiles_y = fused_tiles_y(c->M.nx, c->M.ny, c->fused_ty, c->wave_slots);
    if (resid) {
        for (int b = 0; b < 2; ++b)
            if (!c->rbuf[b])
                HIP_TRY(hipMalloc((void**)&c->rbuf[b], 4 * (size_t)c->pitch * sizeof(double)));
        if (!c->resid_valid) {
            // residual and wave speeds of the current state
            const int slot = (int)(c->nsteps % 3);
            hipLaunchKernelGGL(k_clear_slot, dim3(1), dim3(64), 0, c->stream, c->ctrl, slot);
            launch_resid<T, true>(c->M, view_of<T>(c, c->cur), rview(c, c->cur),
                                  view_of<T>(c, c->cur), rview(c, c->cur), c->Ag, c->ctrl,
                                  (int)c->nsteps, cfl, t_end, tiles_y, c->stream);
        }
    } else if (cfl_mode && !c->speeds_valid) {
        // wave speeds of the current state into the slot of the next step
        const int slot = (int)(c->nsteps % 3);
        hipLaunchKernelGGL(k_clear_slot, dim3(1), dim3(64), 0, c->stream, c->ctrl, slot);
        launch_speeds<T>(c, c->cur, slot);
    }
    (void)hipEventRecord(c->ev0, c->stream);
    if (c->path == SVE_PATH_RESIDENT) {
        launch_resident<T>(c, n, cfl, t_end, fixed_dt);
    } else {
        for (int s = 0; s < n; ++s) {
            const int step = (int)(c->nsteps + s);
            const int src = (c->cur + s) & 1, dst = src ^ 1;
            if (resid) {
                launch_resid<T, false>(c->M, view_of<T>(c, src), rview(c, src), view_of<T>(c, dst),
                                       rview(c, dst), c->Ag, c->ctrl, step, cfl, t_end, tiles_y,
                                       c->stream);
            } else if ((c->path == SVE_PATH_FUSED || c->path == SVE_PATH_RESIDUAL) &&
                       c->M.dim == 2) {
                launch_fused<T>(c, src, dst, step, cfl, t_end, fixed_dt);
            } else if (c->path == SVE_PATH_FUSED || c->path == SVE_PATH_RESIDUAL) {
                launch_fused_1d<T>(c->M, view_of<T>(c, src), view_of<T>(c, dst), c->Ag, c->ctrl,
                                   step, cfl, t_end, fixed_dt, c->stream);
            } else {
                launch_update<T>(c, src, dst, step, cfl, t_end, fixed_dt);
                if (cfl_mode) launch_speeds<T>(c, dst, (step + 1) % 3);
            }
        }
    }
    (void)hipEventRecord(c->ev1, c->stream);
    HIP_TRY(hipGetLastError());
    c->speeds_valid = cfl_mode;
    c->resid_valid = resid;
    return SVE_OK;
}

int finish_steps(sve_ctx* c, int n) {
    HIP_TRY(hipMemcpyAsync(c->h_ctrl, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) c->last_ms = ms;
    const Ctrl& h = *c->h_ctrl;
    if (h.err && c->last_resid && h.fail_step == c->nsteps + n) {
        // the residual pass found an interface error of the state its last
        // step reached: the n steps completed; the next step fails
        c->cur = (int)((c->cur + n) & 1);
        c->nsteps += n;
        c->t = h.t[c->nsteps % 3];
        c->dt_last = h.dt_last;
        c->pending = code_from_bits(h.err);
        if (c->pending == SVE_OK) c->pending = SVE_ERR_STATE;
        c->speeds_valid = false;
        c->resid_valid = false;
        return SVE_OK;
    }
    if (h.err) {
        long long fail = h.fail_step;
        if (fail < c->nsteps || fail >= c->nsteps + n) fail = c->nsteps;
        const long long done = fail - c->nsteps;
        c->cur = (int)((c->cur + done) & 1);
        c->nsteps = fail;
        c->t = h.t[fail % 3];
        c->sticky = code_from_bits(h.err);
        if (c->sticky == SVE_OK) c->sticky = SVE_ERR_STATE;
        c->speeds_valid = false;
        c->resid_valid = false;
        return c->sticky;
    }
    c->cur = (int)((c->cur + n) & 1);
    c->nsteps += n;
    c->t = h.t[c->nsteps % 3];
    c->dt_last = h.dt_last;
    return SVE_OK;
}

int do_steps(sve_ctx* c, int n, double cfl, double t_end, double fixed_dt) {
    if (!c) return SVE_ERR_ARG;
    if (c->sticky) return c->sticky;
    if (n < 0) return SVE_ERR_ARG;
    if (c->pending && n > 0) {                   // the first of these steps fails
        c->sticky = c->pending;
        c->pending = SVE_OK;
        return c->sticky;
    }
    if (n == 0) return SVE_OK;
    if (c->nsteps + n >= INT_MAX) return SVE_ERR_ARG;
    int rc = c->storage == SVE_FP32 ? run_steps<float>(c, n, cfl, t_end, fixed_dt)
                                    : run_steps<double>(c, n, cfl, t_end, fixed_dt);
    if (rc) return rc;
    return finish_steps(c, n);
}

template <typename T>
int init_common(sve_ctx* c, const double* h, const double* hu, const double* hv,
                const double* z) {
    const Model& M = c->M;
    const long long N = (long long)M.nx * M.ny;
    const unsigned blocks = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_reset_ctrl, dim3(1), dim3(64), 0, c->stream, c->ctrl, 0.0);
    hipLaunchKernelGGL(k_load_state<T>, dim3(blocks), dim3(256), 0, c->stream, M, h, hu, hv, z,
                       view_of<T>(c, 0), c->ctrl);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(c->h_ctrl, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->h_ctrl->err) return SVE_ERR_ARG;
    launch_speeds<T>(c, 0, 0);
    HIP_TRY(hipGetLastError());
    c->speeds_valid = true;
    // small 1D grids run on the LDS-resident kernel, larger ones on the
    // one-pass kernel (the fused path)
    if (resident_supported(c) && c->M.nx <= RES_DEFAULT_NMAX) c->path = SVE_PATH_RESIDENT;
    return SVE_OK;
}

int init_impl(sve_ctx** out, int nx, int ny, double Lx, double Ly, const double* h,
              const double* hu, const double* hv, const double* zb, const double* Ag,
              const sve_params* p, const sve_bc bc[4], int storage, void* stream, bool dev) {
    if (!out) return SVE_ERR_ARG;
    *out = nullptr;
    if (!h || !hu || !zb) return SVE_ERR_ARG;
    if (nx < 1 || ny < 1) return SVE_ERR_ARG;
    const int dim = hv ? 2 : 1;
    if (dim == 1 && ny != 1) return SVE_ERR_ARG;
    if (!(Lx > 0.0) || (dim == 2 && !(Ly > 0.0))) return SVE_ERR_ARG;
    if (storage != SVE_FP64 && storage != SVE_FP32) return SVE_ERR_ARG;
    if ((long long)nx * ny > (1ll << 31) - 1) return SVE_ERR_ARG;
    int rc = validate_params(p, dim, bc);
    if (rc) return rc;
    sve_ctx* c = new (std::nothrow) sve_ctx();
    if (!c) return SVE_ERR_HIP;
    c->M = make_model(nx, ny, Lx, Ly, dim, p, bc);
    c->storage = storage;
    c->stream = (hipStream_t)stream;
    {
        int dev_id = 0, cus = 0;
        if (hipGetDevice(&dev_id) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) ==
                hipSuccess &&
            cus > 0)
            c->wave_slots = cus * 4 * FUSED_WAVES_PER_SIMD;   // 4 SIMDs per compute unit
    }
    c->N = (long long)nx * ny;
    c->pitch = round_up(c->N, 64);
    const size_t esz = storage == SVE_FP32 ? sizeof(float) : sizeof(double);
    const size_t fields = 4;
    rc = SVE_OK;
    auto alloc = [&](hipError_t e, const char* what) {
        if (rc == SVE_OK && e != hipSuccess) rc = hip_fail(e, what, __LINE__);
    };
    for (int b = 0; b < 2; ++b) alloc(hipMalloc(&c->buf[b], fields * c->pitch * esz), "hipMalloc state");
    alloc(hipMalloc((void**)&c->ctrl, sizeof(Ctrl)), "hipMalloc ctrl");
    alloc(hipHostMalloc((void**)&c->h_ctrl, sizeof(Ctrl), hipHostMallocDefault), "hipHostMalloc");
    alloc(hipEventCreate(&c->ev0), "hipEventCreate");
    alloc(hipEventCreate(&c->ev1), "hipEventCreate");
    if (Ag) alloc(hipMalloc((void**)&c->Ag, c->N * sizeof(double)), "hipMalloc Ag");
    if (!dev) alloc(hipMalloc((void**)&c->staging, 4 * c->N * sizeof(double)), "hipMalloc staging");
    if (rc) {
        sve_destroy(c);
        return rc;
    }
    const double *dh = h, *dhu = hu, *dhv = hv, *dz = zb;
    const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (!dev) {
        double* s = c->staging;
        const size_t bytes = c->N * sizeof(double);
        hipError_t e = hipMemcpyAsync(s, h, bytes, kind, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s + c->N, hu, bytes, kind, c->stream);
        if (e == hipSuccess && hv) e = hipMemcpyAsync(s + 2 * c->N, hv, bytes, kind, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s + 3 * c->N, zb, bytes, kind, c->stream);
        if (e != hipSuccess) {
            sve_destroy(c);
            return hip_fail(e, "hipMemcpyAsync initial state", __LINE__);
        }
        dh = s;
        dhu = s + c->N;
        dhv = hv ? s + 2 * c->N : nullptr;
        dz = s + 3 * c->N;
    }
    if (Ag) {
        const hipError_t e = hipMemcpyAsync(c->Ag, Ag, c->N * sizeof(double), kind, c->stream);
        if (e != hipSuccess) {
            sve_destroy(c);
            return hip_fail(e, "hipMemcpyAsync A_g", __LINE__);
        }
    }
    rc = storage == SVE_FP32 ? init_common<float>(c, dh, dhu, dhv, dz)
                             : init_common<double>(c, dh, dhu, dhv, dz);
    if (rc) {
        sve_destroy(c);
        return rc;
    }
    *out = c;
    return SVE_OK;
}

template <typename T>
int get_impl(sve_ctx* c, double* h, double* hu, double* hv, double* zb, bool dev) {
    const long long N = c->N;
    const unsigned blocks = (unsigned)((N + 255) / 256);
    if (dev) {
        hipLaunchKernelGGL(k_store_state<T>, dim3(blocks), dim3(256), 0, c->stream, c->M,
                           view_of<T>(c, c->cur), h, hu, hv, zb);
        return check_hip(hipGetLastError());
    }
    if (!c->staging && hipMalloc((void**)&c->staging, 4 * N * sizeof(double)) != hipSuccess)
        return SVE_ERR_HIP;
    double* s = c->staging;
    hipLaunchKernelGGL(k_store_state<T>, dim3(blocks), dim3(256), 0, c->stream, c->M,
                       view_of<T>(c, c->cur), s, s + N, s + 2 * N, s + 3 * N);
    const size_t bytes = N * sizeof(double);
    double* outs[4] = {h, hu, hv, zb};
    for (int f = 0; f < 4; ++f) {
        if (!outs[f]) continue;
        if (f == 2 && c->M.dim == 1) {
            std::memset(outs[f], 0, bytes);
            continue;
        }
        if (hipMemcpyAsync(outs[f], s + f * N, bytes, hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess)
            return SVE_ERR_HIP;
    }
    return check_hip(hipStreamSynchronize(c->stream));
}

}  // namespace

// ---------------------------------------------------------------------------
// exported C ABI
// ---------------------------------------------------------------------------
extern "C" {

int sve_init_state(sve_ctx** ctx, int nx, int ny, double Lx, double Ly, const double* h,
                   const double* hu, const double* hv, const double* zb, const double* Ag_field,
                   const sve_params* p, const sve_bc bc[4], int storage, void* stream) {
    return init_impl(ctx, nx, ny, Lx, Ly, h, hu, hv, zb, Ag_field, p, bc, storage, stream, false);
}

int sve_init_state_dev(sve_ctx** ctx, int nx, int ny, double Lx, double Ly, const double* h,
                       const double* hu, const double* hv, const double* zb,
                       const double* Ag_field, const sve_params* p, const sve_bc bc[4],
                       int storage, void* stream) {
    return init_impl(ctx, nx, ny, Lx, Ly, h, hu, hv, zb, Ag_field, p, bc, storage, stream, true);
}

int sve_step(sve_ctx* ctx, int n, double cfl, double t_end, double* t_out) {
    if (ctx && !(cfl > 0.0)) return SVE_ERR_ARG;
    const int rc = do_steps(ctx, n, cfl, t_end, 0.0);
    if (t_out && ctx) *t_out = ctx->t;
    return rc;
}

int sve_step_fixed_dt(sve_ctx* ctx, int n, double dt) {
    if (ctx && !(dt > 0.0 && std::isfinite(dt))) return SVE_ERR_ARG;
    return do_steps(ctx, n, 0.0, 0.0, dt);
}

int sve_get_state(sve_ctx* ctx, double* h, double* hu, double* hv, double* zb, double* t,
                  double* dt_last, long long* nsteps) {
    if (!ctx) return SVE_ERR_ARG;
    const int rc = ctx->storage == SVE_FP32 ? get_impl<float>(ctx, h, hu, hv, zb, false)
                                            : get_impl<double>(ctx, h, hu, hv, zb, false);
    if (t) *t = ctx->t;
    if (dt_last) *dt_last = ctx->dt_last;
    if (nsteps) *nsteps = ctx->nsteps;
    return rc;
}

int sve_get_state_dev(sve_ctx* ctx, double* h, double* hu, double* hv, double* zb, double* t,
                      double* dt_last, long long* nsteps) {
    if (!ctx) return SVE_ERR_ARG;
    const int rc = ctx->storage == SVE_FP32 ? get_impl<float>(ctx, h, hu, hv, zb, true)
                                            : get_impl<double>(ctx, h, hu, hv, zb, true);
    if (t) *t = ctx->t;
    if (dt_last) *dt_last = ctx->dt_last;
    if (nsteps) *nsteps = ctx->nsteps;
    return rc;
}

int sve_destroy(sve_ctx* ctx) {
    if (!ctx) return SVE_OK;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream); else (void)hipDeviceSynchronize();
    for (int b = 0; b < 2; ++b)
        if (ctx->buf[b]) (void)hipFree(ctx->buf[b]);
    if (ctx->ctrl) (void)hipFree(ctx->ctrl);
    if (ctx->h_ctrl) (void)hipHostFree(ctx->h_ctrl);
    if (ctx->Ag) (void)hipFree(ctx->Ag);
    if (ctx->staging) (void)hipFree(ctx->staging);
    for (int b = 0; b < 2; ++b)
        if (ctx->rbuf[b]) (void)hipFree(ctx->rbuf[b]);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    sve_adjoint_release(ctx);
    delete ctx;
    return SVE_OK;
}

const char* sve_strerror(int code) {
    switch (code) {
        case SVE_OK: return "success";
        case SVE_ERR_ARG: return "invalid argument";
        case SVE_ERR_HIP: return "HIP runtime failure";
        case SVE_ERR_POSITIVITY: return "non-positive depth in a Riemann fan or after an update";
        case SVE_ERR_ORDER: return "bed-jump quadratic without an admissible root";
        case SVE_ERR_NONFINITE: return "non-finite value in the state";
        case SVE_ERR_STATE: return "call out of order or context in an error state";
        default: return "unknown error code";
    }
}

int sve_set_path(sve_ctx* ctx, int path) {
    if (!ctx) return SVE_ERR_ARG;
    if (path != SVE_PATH_FUSED && path != SVE_PATH_SPLIT && path != SVE_PATH_RESIDENT &&
        path != SVE_PATH_RESIDUAL)
        return SVE_ERR_ARG;
    if (path == SVE_PATH_RESIDENT && !resident_supported(ctx)) return SVE_ERR_ARG;
    if (ctx->M.order == 2 && path != SVE_PATH_FUSED) return SVE_ERR_ARG;
    ctx->path = path;
    return SVE_OK;
}

int sve_set_tile_rows(sve_ctx* ctx, int rows) {
    if (!ctx || rows < 0 || rows > 65536) return SVE_ERR_ARG;
    ctx->fused_ty = rows;
    return SVE_OK;
}

int sve_debug_poke(sve_ctx* ctx, int field, long long k, double value) {
    if (!ctx || field < 0 || field > 3 || k < 0 || k >= ctx->N) return SVE_ERR_ARG;
    if (field == 2 && ctx->M.dim == 1) return SVE_ERR_ARG;
    if (ctx->storage == SVE_FP32)
        hipLaunchKernelGGL(k_poke<float>, dim3(1), dim3(64), 0, ctx->stream,
                           view_of<float>(ctx, ctx->cur), field, k, value);
    else
        hipLaunchKernelGGL(k_poke<double>, dim3(1), dim3(64), 0, ctx->stream,
                           view_of<double>(ctx, ctx->cur), field, k, value);
    ctx->speeds_valid = false;
    ctx->resid_valid = false;
    return check_hip(hipStreamSynchronize(ctx->stream));
}

int sve_last_elapsed_ms(sve_ctx* ctx, double* ms) {
    if (!ctx || !ms) return SVE_ERR_ARG;
    *ms = ctx->last_ms;
    return SVE_OK;
}

}  // extern "C"
