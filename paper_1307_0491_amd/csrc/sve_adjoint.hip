// sve_adjoint.hip -- discrete adjoint of fixed-dt steps with sqrt(N)
// checkpointing (C ABI in include/sve_adjoint.h).
//
// Forward: n fixed-dt steps of the fused kernel, the state saved every k
// steps (k = ceil(sqrt(n)) by default).  Backward: for each segment, last
// first, the segment's states are recomputed from its checkpoint into a
// segment buffer, then the reverse step kernel runs from the segment's last
// step down to its first, mapping lambda^{n+1} to lambda^n and accumulating
// dL/dA_g.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/sve.h"
#include "../../include/sve_adjoint.h"
#include "sve_adjoint.hpp"
#include "sve_context.hpp"
#include "sve_fused.hpp"

using namespace sve;

struct sve_adjoint_state {
    int nsteps = 0, every = 0;
    double dt = 0.0;
    std::vector<double*> ckpt;     // state at steps 0, every, 2 every, ... (4 pitch each)
    double* seg = nullptr;         // `every` states of the current segment
    double* lam[2] = {nullptr, nullptr};
    Ctrl* ctrl = nullptr;          // control block of the recomputation
    bool ready = false;
};

namespace {

constexpr int ADJ_BLOCK = 256;

StateView<double> view(double* base, long long pitch) {
    return StateView<double>{base, base + pitch, base + 2 * pitch, base + 3 * pitch};
}

// lambda^n = (dU^{n+1}/dU^n)^T lambda^{n+1}; gAg += (dU^{n+1}/dA_g)^T lambda^{n+1}.
// One thread per cell: the four interfaces of the cell are solved in reverse
// and the cell's own share of each is accumulated (periodic grid).
template <int CL>
__global__ void __launch_bounds__(ADJ_BLOCK)
k_adjoint_step(Model M, StateView<double> U, const double* __restrict__ Agf,
               StateView<double> Lin, StateView<double> Lout, double* __restrict__ gAg,
               double dt) {
    const long long N = (long long)M.nx * M.ny;
    const long long k = (long long)blockIdx.x * ADJ_BLOCK + threadIdx.x;
    if (k >= N) return;
    const int i = (int)(k % M.nx), j = (int)(k / M.nx);
    const int iw = i == 0 ? M.nx - 1 : i - 1, ie = i == M.nx - 1 ? 0 : i + 1;
    const int js = j == 0 ? M.ny - 1 : j - 1, jn = j == M.ny - 1 ? 0 : j + 1;
    const long long kc = k, kw = (long long)j * M.nx + iw, ke = (long long)j * M.nx + ie;
    const long long ks = (long long)js * M.nx + i, kn = (long long)jn * M.nx + i;
    auto ag = [&](long long q) { return Agf ? Agf[q] : M.Ag; };
    auto cell = [&](long long q) {
        return project<CL>(M, U.h[q], U.hu[q], U.hv[q], U.z[q], ag(q));
    };
    const Cell C = cell(kc), W = cell(kw), E = cell(ke), S = cell(ks), No = cell(kn);
    const double lx = dt / M.dx, ly = dt / M.dy;
    auto lam = [&](long long q, double& a, double& b, double& c, double& d) {
        a = Lin.h[q]; b = Lin.hu[q]; c = Lin.hv[q]; d = Lin.z[q];
    };
    double lc_h, lc_u, lc_v, lc_z;
    lam(kc, lc_h, lc_u, lc_v, lc_z);
    CellAdj acc{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    SideAdj Lb, Rb;
    {   // west interface (W | C): C is the right cell
        double a, b, c, d;
        lam(kw, a, b, c, d);
        const Flux Fb{lx * (lc_h - a), -lx * b, lx * lc_u, lx * (lc_v - c), lx * (lc_z - d)};
        iface_vjp(side_x(W), side_x(C), M.g, Fb, Lb, Rb);
        add_x(acc, Rb);
    }
    {   // east interface (C | E): C is the left cell
        double a, b, c, d;
        lam(ke, a, b, c, d);
        const Flux Fb{lx * (a - lc_h), -lx * lc_u, lx * b, lx * (c - lc_v), lx * (d - lc_z)};
        iface_vjp(side_x(C), side_x(E), M.g, Fb, Lb, Rb);
        add_x(acc, Lb);
    }
    {   // south interface (S | C): normal momentum hv, transverse hu
        double a, b, c, d;
        lam(ks, a, b, c, d);
        const Flux Fb{ly * (lc_h - a), -ly * c, ly * lc_v, ly * (lc_u - b), ly * (lc_z - d)};
        iface_vjp(side_y(S), side_y(C), M.g, Fb, Lb, Rb);
        add_y(acc, Rb);
    }
    {   // north interface (C | N)
        double a, b, c, d;
        lam(kn, a, b, c, d);
        const Flux Fb{ly * (a - lc_h), -ly * lc_v, ly * c, ly * (b - lc_u), ly * (d - lc_z)};
        iface_vjp(side_y(C), side_y(No), M.g, Fb, Lb, Rb);
        add_y(acc, Lb);
    }
    double hb, hub, hvb, zb, Agb;
    project_vjp_grass(M, C.h, C.hu, C.hv, ag(kc), acc, hb, hub, hvb, zb, Agb);
    Lout.h[kc] = lc_h + hb;
    Lout.hu[kc] = lc_u + hub;
    Lout.hv[kc] = lc_v + hvb;
    Lout.z[kc] = lc_z + zb;
    if (gAg) gAg[kc] += Agb;
}

__global__ void k_copy4(StateView<double> dst, const double* __restrict__ src, long long N) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    dst.h[k] = src[k];
    dst.hu[k] = src[N + k];
    dst.hv[k] = src[2 * N + k];
    dst.z[k] = src[3 * N + k];
}

__global__ void k_copy4_out(double* dst, StateView<double> src, long long N) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    dst[k] = src.h[k];
    dst[N + k] = src.hu[k];
    dst[2 * N + k] = src.hv[k];
    dst[3 * N + k] = src.z[k];
}

__global__ void k_zero(double* p, long long n) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0.0;
}

int adjoint_supported(const sve_ctx* c) {
    const Model& M = c->M;
    if (M.dim != 2 || c->storage != SVE_FP64 || M.law != LAW_GRASS || M.momentum_friction)
        return SVE_ERR_ARG;
    for (int s = 0; s < 4; ++s)
        if (M.bc_kind[s] != BC_PERIODIC) return SVE_ERR_ARG;
    return SVE_OK;
}

unsigned blocks_for(long long n, int b) { return (unsigned)((n + b - 1) / b); }

void free_adj(sve_adjoint_state* a) {
    if (!a) return;
    for (double* p : a->ckpt)
        if (p) (void)hipFree(p);
    a->ckpt.clear();
    if (a->seg) (void)hipFree(a->seg);
    a->seg = nullptr;
    for (int i = 0; i < 2; ++i) {
        if (a->lam[i]) (void)hipFree(a->lam[i]);
        a->lam[i] = nullptr;
    }
    if (a->ctrl) (void)hipFree(a->ctrl);
    a->ctrl = nullptr;
    a->ready = false;
}

// One fixed-dt step from `src` to `dst` with the fused kernel.
void fwd_step(sve_ctx* c, Ctrl* ctrl, double* src, double* dst, int n, double dt) {
    launch_fused_rows<double>(c->M, view(src, c->pitch), view(dst, c->pitch), c->Ag, ctrl, n, 0.0,
                              0.0, dt, c->fused_ty, c->stream);
}

int reverse_step(sve_ctx* c, double* U, double* lin, double* lout, double* gAg, double dt) {
    const int cl = closure_class(c->M);
    auto kern = cl == CL_GRASS3 ? k_adjoint_step<CL_GRASS3>
              : cl == CL_GRASS1 ? k_adjoint_step<CL_GRASS1>
                                : k_adjoint_step<CL_GRASSM>;
    hipLaunchKernelGGL(kern, dim3(blocks_for(c->N, ADJ_BLOCK)), dim3(ADJ_BLOCK), 0, c->stream, c->M, view(U, c->pitch), (const double*)c->Ag,
                       view(lin, c->pitch), view(lout, c->pitch), gAg, dt);
    return hipGetLastError() == hipSuccess ? SVE_OK : SVE_ERR_HIP;
}

}  // namespace

void sve_adjoint_release(sve_ctx* ctx) {
    if (!ctx || !ctx->adj) return;
    free_adj(ctx->adj);
    delete ctx->adj;
    ctx->adj = nullptr;
}

extern "C" {

int sve_adj_forward(sve_ctx* ctx, int nsteps, double dt, int every) {
    if (!ctx || nsteps < 1 || !(dt > 0.0) || !std::isfinite(dt)) return SVE_ERR_ARG;
    if (ctx->sticky) return ctx->sticky;
    int rc = adjoint_supported(ctx);
    if (rc) return rc;
    if (every <= 0) every = (int)std::ceil(std::sqrt((double)nsteps));
    if (every > nsteps) every = nsteps;
    if (!ctx->adj) ctx->adj = new (std::nothrow) sve_adjoint_state();
    if (!ctx->adj) return SVE_ERR_HIP;
    sve_adjoint_state* a = ctx->adj;
    free_adj(a);
    const size_t bytes = 4 * (size_t)ctx->pitch * sizeof(double);
    const int nck = (nsteps + every - 1) / every;
    a->ckpt.assign(nck, nullptr);
    bool ok = true;
    for (int s = 0; s < nck && ok; ++s) ok = hipMalloc((void**)&a->ckpt[s], bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->seg, (size_t)every * bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&a->ctrl, sizeof(Ctrl)) == hipSuccess;
    if (!ok) {
        free_adj(a);
        return SVE_ERR_HIP;
    }
    hipLaunchKernelGGL(k_reset_ctrl, dim3(1), dim3(64), 0, ctx->stream, a->ctrl, 0.0);
    // checkpoints are taken from the context's own stepping, one segment
    // per call (one stream synchronisation per segment)
    for (int sgi = 0; sgi < nck; ++sgi) {
        (void)hipMemcpyAsync(a->ckpt[sgi], ctx->buf[ctx->cur], bytes, hipMemcpyDeviceToDevice,
                             ctx->stream);
        const int len = std::min(every, nsteps - sgi * every);
        rc = sve_step_fixed_dt(ctx, len, dt);
        if (rc) {
            free_adj(a);
            return rc;
        }
    }
    a->nsteps = nsteps;
    a->every = every;
    a->dt = dt;
    a->ready = true;
    return SVE_OK;
}

int sve_adj_backward(sve_ctx* ctx, const double* gT, double* g0, double* gAg) {
    if (!ctx || !gT || !g0) return SVE_ERR_ARG;
    sve_adjoint_state* a = ctx->adj;
    if (!a || !a->ready) return SVE_ERR_STATE;
    const long long N = ctx->N, P = ctx->pitch;
    const size_t bytes = 4 * (size_t)P * sizeof(double);
    for (int i = 0; i < 2; ++i)
        if (!a->lam[i] && hipMalloc((void**)&a->lam[i], bytes) != hipSuccess) return SVE_ERR_HIP;
    hipLaunchKernelGGL(k_copy4, dim3(blocks_for(N, 256)), dim3(256), 0, ctx->stream,
                       view(a->lam[0], P), gT, N);
    if (gAg)
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(N, 256)), dim3(256), 0, ctx->stream, gAg, N);
    int cur = 0;
    const int nck = (int)a->ckpt.size();
    int step_id = 0;
    hipLaunchKernelGGL(k_reset_ctrl, dim3(1), dim3(64), 0, ctx->stream, a->ctrl, 0.0);
    for (int sgi = nck - 1; sgi >= 0; --sgi) {
        const int s0 = sgi * a->every;
        const int s1 = std::min(s0 + a->every, a->nsteps);
        // recompute states s0 .. s1-1 into the segment buffer
        (void)hipMemcpyAsync(a->seg, a->ckpt[sgi], bytes, hipMemcpyDeviceToDevice, ctx->stream);
        for (int s = s0 + 1; s < s1; ++s) {
            double* src = a->seg + (size_t)(s - 1 - s0) * 4 * P;
            double* dst = a->seg + (size_t)(s - s0) * 4 * P;
            fwd_step(ctx, a->ctrl, src, dst, step_id++, a->dt);
        }
        for (int s = s1 - 1; s >= s0; --s) {
            double* U = a->seg + (size_t)(s - s0) * 4 * P;
            const int rc = reverse_step(ctx, U, a->lam[cur], a->lam[cur ^ 1], gAg, a->dt);
            if (rc) return rc;
            cur ^= 1;
        }
    }
    hipLaunchKernelGGL(k_copy4_out, dim3(blocks_for(N, 256)), dim3(256), 0, ctx->stream, g0,
                       view(a->lam[cur], P), N);
    Ctrl hc;
    if (hipMemcpyAsync(&hc, a->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return SVE_ERR_HIP;
    if (hc.err) return SVE_ERR_STATE;
    return SVE_OK;
}

int sve_adj_step_vjp(sve_ctx* ctx, double dt, const double* lam_in, double* lam_out,
                     double* gAg) {
    if (!ctx || !lam_in || !lam_out || !(dt > 0.0)) return SVE_ERR_ARG;
    int rc = adjoint_supported(ctx);
    if (rc) return rc;
    if (!ctx->adj) ctx->adj = new (std::nothrow) sve_adjoint_state();
    if (!ctx->adj) return SVE_ERR_HIP;
    sve_adjoint_state* a = ctx->adj;
    const long long N = ctx->N, P = ctx->pitch;
    const size_t bytes = 4 * (size_t)P * sizeof(double);
    for (int i = 0; i < 2; ++i)
        if (!a->lam[i] && hipMalloc((void**)&a->lam[i], bytes) != hipSuccess) return SVE_ERR_HIP;
    hipLaunchKernelGGL(k_copy4, dim3(blocks_for(N, 256)), dim3(256), 0, ctx->stream,
                       view(a->lam[0], P), lam_in, N);
    if (gAg)
        hipLaunchKernelGGL(k_zero, dim3(blocks_for(N, 256)), dim3(256), 0, ctx->stream, gAg, N);
    rc = reverse_step(ctx, (double*)ctx->buf[ctx->cur], a->lam[0], a->lam[1], gAg, dt);
    if (rc) return rc;
    hipLaunchKernelGGL(k_copy4_out, dim3(blocks_for(N, 256)), dim3(256), 0, ctx->stream, lam_out,
                       view(a->lam[1], P), N);
    return hipStreamSynchronize(ctx->stream) == hipSuccess ? SVE_OK : SVE_ERR_HIP;
}

}  // extern "C"
