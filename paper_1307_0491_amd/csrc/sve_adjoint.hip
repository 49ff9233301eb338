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
    double* seg[2] = {nullptr, nullptr};   // `every` states of a segment, two segments
    double* lam[2] = {nullptr, nullptr};
    Ctrl* ctrl = nullptr;          // control block of the recomputation
    hipStream_t side = nullptr;    // stream of the recomputation
    hipEvent_t ev_start = nullptr, ev_recomp[2] = {nullptr, nullptr},
               ev_rev[2] = {nullptr, nullptr};
    bool ready = false;
};

namespace {

StateView<double> view(double* base, long long pitch) {
    return StateView<double>{base, base + pitch, base + 2 * pitch, base + 3 * pitch};
}

struct Lam {
    double h, hu, hv, z;
};

__device__ __forceinline__ SideAdj prev_lane(const SideAdj& s) {
    return SideAdj{dpp<DPP_PREV>(s.h),  dpp<DPP_PREV>(s.tau), dpp<DPP_PREV>(s.un),
                   dpp<DPP_PREV>(s.ut), dpp<DPP_PREV>(s.Pi),  dpp<DPP_PREV>(s.z),
                   dpp<DPP_PREV>(s.q),  dpp<DPP_PREV>(s.b2)};
}

// lambda^n = (dU^{n+1}/dU^n)^T lambda^{n+1}; gAg += (dU^{n+1}/dA_g)^T lambda^{n+1}
// on a periodic grid.
//
// The tile layout is that of the forward step kernel: one wavefront per
// tile, lanes 0..63 holding columns i0-1 .. i0+62 (i0 = 61 * tile index,
// lanes 1..61 owned), marching upward from row j0-1 to row jend.  Every
// interface the tile needs is solved in reverse once.  At row r, each lane
// first solves the y-interface (row r-1 | row r), which completes row r-1
// (then mapped back through the projection and stored) and starts row r;
// then the x-interface (lane | lane+1) of row r, keeping the left cell's
// share and passing the right cell's share one lane up (wave_shr:1).  The
// adjoint seed of an interface's fluxes comes from lambda^{n+1} of its two
// cells: U' = U - dt/dx (F^L_{i+1/2} - F^R_{i-1/2}) - ...
//
// One wavefront per workgroup, two per SIMD (the register budget is 256),
// except with the general Grass exponent, whose form needs more: at two per
// SIMD it spilled 26 VGPRs to scratch memory; at one per SIMD the excess
// goes to AGPRs (forward and reverse sweep of 500 steps at 1024^2: 62.1 ->
// 56.3 ms).  Workgroup id runs tile xcd_tile(id) of the tiles_x x tiles_y
// split (row-major; rows by tile_rows), so each XCD gets a contiguous band.
template <int CL>
__global__ void __launch_bounds__(64, (CL == CL_GRASSM ? 1 : 2))
k_adjoint_march(Model M, StateView<double> U, const double* __restrict__ Agf,
                StateView<double> Lin, StateView<double> Lout, double* __restrict__ gAg,
                double dt, int tiles_y) {
    const int lane = threadIdx.x & 63;
    const int tiles_x = (M.nx + FUSED_OWN - 1) / FUSED_OWN;
    const int t = xcd_tile(blockIdx.x, tiles_x * tiles_y);
    const int i0 = (t % tiles_x) * FUSED_OWN;
    int j0, jend;                                    // owned rows [j0, jend)
    tile_rows(M.ny, tiles_y, t / tiles_x, j0, jend);
    const int l_last = min(FUSED_OWN, M.nx - i0);    // owned lanes 1..l_last
    const bool owned = lane >= 1 && lane <= l_last;
    const int col = i0 - 1 + lane;
    const int ci = wrap(col, M.nx);
    const double lx = dt / M.dx, ly = dt / M.dy;

    auto load = [&](int r, Cell& P, Lam& l, double& ag) {
        const long long k = (long long)wrap(r, M.ny) * M.nx + ci;
        ag = Agf ? Agf[k] : M.Ag;
        P = project<CL>(M, U.h[k], U.hu[k], U.hv[k], U.z[k], ag);
        l = Lam{Lin.h[k], Lin.hu[k], Lin.hv[k], Lin.z[k]};
    };

    // row r-1, carried: its y view, stored state, A_g, lambda and the
    // adjoint of its projected quantities gathered so far
    Side Sp;
    double hp, hup, hvp, agp;
    Lam lp;
    CellAdj acc{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    {
        Cell P;
        load(j0 - 1, P, lp, agp);
        Sp = side_y(P);
        hp = P.h; hup = P.hu; hvp = P.hv;
    }
    for (int r = j0; r <= jend; ++r) {
        Cell P;
        Lam l;
        double ag;
        load(r, P, l, ag);
        CellAdj an{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        {                                            // y-interface (r-1 | r)
            const Flux Fb{ly * (l.h - lp.h), -ly * lp.hv, ly * l.hv, ly * (l.hu - lp.hu),
                          ly * (l.z - lp.z)};
            SideAdj Lb, Rb;
            iface_vjp(Sp, side_y(P), M.g, Fb, Lb, Rb);
            if (r > j0) {                            // row r-1 is complete
                add_y(acc, Lb);
                double hb, hub, hvb, zb, Agb;
                project_vjp_grass<CL>(M, hp, hup, hvp, agp, acc, hb, hub, hvb, zb, Agb);
                if (owned) {
                    const long long k = (long long)(r - 1) * M.nx + col;
                    Lout.h[k] = lp.h + hb;
                    Lout.hu[k] = lp.hu + hub;
                    Lout.hv[k] = lp.hv + hvb;
                    Lout.z[k] = lp.z + zb;
                    if (gAg) gAg[k] += Agb;
                }
            }
            add_y(an, Rb);
        }
        if (r < jend) {                              // x-interfaces of row r
            const double rh = dpp<DPP_NEXT>(l.h), ru = dpp<DPP_NEXT>(l.hu);
            const double rv = dpp<DPP_NEXT>(l.hv), rz = dpp<DPP_NEXT>(l.z);
            const Flux Fb{lx * (rh - l.h), -lx * l.hu, lx * ru, lx * (rv - l.hv), lx * (rz - l.z)};
            SideAdj Lb, Rb;
            iface_vjp(side_x(P), next_side_x(P), M.g, Fb, Lb, Rb);
            add_x(an, Lb);
            add_x(an, prev_lane(Rb));
        }
        Sp = side_y(P);
        hp = P.h; hup = P.hu; hvp = P.hv; agp = ag;
        lp = l;
        acc = an;
    }
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
    if (M.dim != 2 || c->storage != SVE_FP64 || M.law != LAW_GRASS || M.momentum_friction ||
        M.wb || M.order == 2)
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
    for (int i = 0; i < 2; ++i) {
        if (a->seg[i]) (void)hipFree(a->seg[i]);
        a->seg[i] = nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        if (a->lam[i]) (void)hipFree(a->lam[i]);
        a->lam[i] = nullptr;
    }
    if (a->ctrl) (void)hipFree(a->ctrl);
    a->ctrl = nullptr;
    a->ready = false;
}

// One fixed-dt step from `src` to `dst` with the fused kernel.
void fwd_step(sve_ctx* c, Ctrl* ctrl, double* src, double* dst, int n, double dt,
              hipStream_t stream) {
    launch_fused_rows<double>(c->M, view(src, c->pitch), view(dst, c->pitch), c->Ag, ctrl, n, 0.0,
                              0.0, dt, fused_tiles_y(c->M.nx, c->M.ny, c->fused_ty, c->wave_slots),
                              stream);
}

// Stream and events of the pipelined backward sweep, created once.
int ensure_sync(sve_adjoint_state* a) {
    if (a->side) return SVE_OK;
    bool ok = hipStreamCreateWithFlags(&a->side, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&a->ev_start, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < 2 && ok; ++i)
        ok = hipEventCreateWithFlags(&a->ev_recomp[i], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&a->ev_rev[i], hipEventDisableTiming) == hipSuccess;
    return ok ? SVE_OK : SVE_ERR_HIP;
}

void release_sync(sve_adjoint_state* a) {
    if (a->side) {
        (void)hipStreamSynchronize(a->side);
        (void)hipStreamDestroy(a->side);
        a->side = nullptr;
    }
    hipEvent_t* evs[5] = {&a->ev_start, &a->ev_recomp[0], &a->ev_recomp[1], &a->ev_rev[0],
                          &a->ev_rev[1]};
    for (hipEvent_t* e : evs) {
        if (*e) (void)hipEventDestroy(*e);
        *e = nullptr;
    }
}

// Recompute the states of segment `sgi` into segment buffer `b`, on the
// side stream.
void recompute_segment(sve_ctx* ctx, sve_adjoint_state* a, int sgi, int b, int& step_id) {
    const long long P = ctx->pitch;
    const size_t bytes = 4 * (size_t)P * sizeof(double);
    const int s0 = sgi * a->every;
    const int s1 = std::min(s0 + a->every, a->nsteps);
    (void)hipMemcpyAsync(a->seg[b], a->ckpt[sgi], bytes, hipMemcpyDeviceToDevice, a->side);
    for (int s = s0 + 1; s < s1; ++s) {
        double* src = a->seg[b] + (size_t)(s - 1 - s0) * 4 * P;
        double* dst = a->seg[b] + (size_t)(s - s0) * 4 * P;
        fwd_step(ctx, a->ctrl, src, dst, step_id++, a->dt, a->side);
    }
}

int reverse_step(sve_ctx* c, double* U, double* lin, double* lout, double* gAg, double dt) {
    const int cl = closure_class(c->M);
    auto kern = cl == CL_GRASS3 ? k_adjoint_march<CL_GRASS3>
              : cl == CL_GRASS1 ? k_adjoint_march<CL_GRASS1>
                                : k_adjoint_march<CL_GRASSM>;
    const int tiles_x = (c->M.nx + FUSED_OWN - 1) / FUSED_OWN;
    const int tiles_y = fused_tiles_y(c->M.nx, c->M.ny, c->adj_ty, c->wave_slots);
    hipLaunchKernelGGL(kern, dim3(tiles_x * tiles_y), dim3(64), 0, c->stream, c->M,
                       view(U, c->pitch), (const double*)c->Ag, view(lin, c->pitch),
                       view(lout, c->pitch), gAg, dt, tiles_y);
    return hipGetLastError() == hipSuccess ? SVE_OK : SVE_ERR_HIP;
}

}  // namespace

void sve_adjoint_release(sve_ctx* ctx) {
    if (!ctx || !ctx->adj) return;
    release_sync(ctx->adj);
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
    const size_t bytes = 4 * (size_t)ctx->pitch * sizeof(double);
    const int nck = (nsteps + every - 1) / every;
    // buffers of an earlier run with the same segment layout are reused
    const bool reuse =
        (int)a->ckpt.size() == nck && a->every == every && a->seg[0] && a->seg[1] && a->ctrl;
    a->ready = false;
    if (!reuse) {
        free_adj(a);
        a->ckpt.assign(nck, nullptr);
        bool ok = true;
        for (int s = 0; s < nck && ok; ++s)
            ok = hipMalloc((void**)&a->ckpt[s], bytes) == hipSuccess;
        for (int i = 0; i < 2; ++i)
            ok = ok && hipMalloc((void**)&a->seg[i], (size_t)every * bytes) == hipSuccess;
        ok = ok && hipMalloc((void**)&a->ctrl, sizeof(Ctrl)) == hipSuccess;
        if (!ok) {
            free_adj(a);
            return SVE_ERR_HIP;
        }
    }
    a->every = every;
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
    if (ensure_sync(a)) return SVE_ERR_HIP;
    // Segments are swept last to first.  The recomputation of segment k-1
    // (side stream, segment buffer (k-1)&1) does not depend on the reverse
    // steps of segment k (context stream, buffer k&1), so the two overlap;
    // events order each buffer's reuse.
    int cur = 0;
    const int nck = (int)a->ckpt.size();
    int step_id = 0;
    hipLaunchKernelGGL(k_reset_ctrl, dim3(1), dim3(64), 0, ctx->stream, a->ctrl, 0.0);
    if (hipEventRecord(a->ev_start, ctx->stream) != hipSuccess ||
        hipStreamWaitEvent(a->side, a->ev_start, 0) != hipSuccess)
        return SVE_ERR_HIP;
    recompute_segment(ctx, a, nck - 1, (nck - 1) & 1, step_id);
    (void)hipEventRecord(a->ev_recomp[(nck - 1) & 1], a->side);
    for (int sgi = nck - 1; sgi >= 0; --sgi) {
        const int b = sgi & 1;
        if (sgi > 0) {
            // buffer b^1 was last read by the reverse steps of segment sgi+1
            if (sgi + 1 < nck) (void)hipStreamWaitEvent(a->side, a->ev_rev[b ^ 1], 0);
            recompute_segment(ctx, a, sgi - 1, b ^ 1, step_id);
            (void)hipEventRecord(a->ev_recomp[b ^ 1], a->side);
        }
        (void)hipStreamWaitEvent(ctx->stream, a->ev_recomp[b], 0);
        const int s0 = sgi * a->every;
        const int s1 = std::min(s0 + a->every, a->nsteps);
        for (int s = s1 - 1; s >= s0; --s) {
            double* U = a->seg[b] + (size_t)(s - s0) * 4 * P;
            const int rc = reverse_step(ctx, U, a->lam[cur], a->lam[cur ^ 1], gAg, a->dt);
            if (rc) {
                (void)hipStreamSynchronize(a->side);
                return rc;
            }
            cur ^= 1;
        }
        (void)hipEventRecord(a->ev_rev[b], ctx->stream);
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

int sve_adj_set_tile_rows(sve_ctx* ctx, int rows) {
    if (!ctx || rows < 0 || rows > 65536) return SVE_ERR_ARG;
    ctx->adj_ty = rows;
    return SVE_OK;
}

}  // extern "C"
