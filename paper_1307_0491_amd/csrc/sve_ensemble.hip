// sve_ensemble.hip -- many independent 2D runs advanced together (C ABI in
// include/sve_ensemble.h).
//
// All members step in lockstep (global step index n, read from device memory
// so that a captured graph can be replayed); each member keeps its own
// control block (wave-speed maxima, time) and hence its own CFL time step.
// The ensemble kernel runs the single-grid kernel's tile routine on tiles of
// any member: in queue mode a fixed set of resident wavefronts pulls tile
// indices from an atomic counter until the tile list (largest members
// first) is exhausted, in grid mode one wavefront is launched per tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/sve.h"
#include "../../include/sve_ensemble.h"
#include "sve_context.hpp"
#include "sve_fused.hpp"

using namespace sve;

namespace {

struct EnsMember {
    Model M;
    double* buf[2];
    long long pitch;
    Ctrl* ctrl;
    int tiles_x, tiles_y;
};

struct EnsTile {
    int m, tx, ty, pad;
};

constexpr int ENS_WAVES = 4;

__host__ __device__ inline StateView<double> view(double* base, long long pitch) {
    return StateView<double>{base, base + pitch, base + 2 * pitch, base + 3 * pitch};
}

__device__ __forceinline__ void ens_tile(const EnsMember* __restrict__ mem, const EnsTile& t,
                                         int n, double cfl, int TY) {
    const EnsMember& E = mem[t.m];
    Ctrl* ctrl = E.ctrl;
    const StateView<double> S = view(E.buf[n & 1], E.pitch);
    const StateView<double> D = view(E.buf[(n + 1) & 1], E.pitch);
    const int j0 = t.ty * TY;
    // the tile checks the member's error flag and does the member's step
    // bookkeeping (its first tile) after requesting its first rows
    fused_tile<double, CL_GRASSM, true>(E.M, S, D, nullptr, ctrl, n, cfl, 0.0, 0.0,
                                        t.tx == 0 && t.ty == 0, t.tx, j0,
                                        min(j0 + TY, E.M.ny));
}

// Persistent wavefronts: pull tiles until the list is exhausted (every
// wavefront reaches the exit once the counter passes ntiles).
__global__ void __launch_bounds__(64 * ENS_WAVES, 2)
k_ens_queue(const EnsMember* __restrict__ mem, const EnsTile* __restrict__ tiles, int ntiles,
            unsigned* __restrict__ counter, const int* __restrict__ base, int s, double cfl,
            int TY) {
    const int n = *base + s;
    const unsigned inc = (threadIdx.x & 63) == 0 ? 1u : 0u;
    for (;;) {
        // every lane takes part (lane 0 adds 1, the others 0) so the loop
        // stays in uniform control flow; the tile index is lane 0's result
        const int w = __builtin_amdgcn_readfirstlane((int)atomicAdd(counter, inc));
        if (w >= ntiles) break;
        const EnsTile t = tiles[w];
        ens_tile(mem, EnsTile{__builtin_amdgcn_readfirstlane(t.m),
                              __builtin_amdgcn_readfirstlane(t.tx),
                              __builtin_amdgcn_readfirstlane(t.ty), 0},
                 n, cfl, TY);
    }
}

// One wavefront per tile.
__global__ void __launch_bounds__(64 * ENS_WAVES)
k_ens_grid(const EnsMember* __restrict__ mem, const EnsTile* __restrict__ tiles, int ntiles,
           const int* __restrict__ base, int s, double cfl, int TY) {
    const int n = *base + s;
    const int w = blockIdx.x * ENS_WAVES + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (w >= ntiles) return;
    const EnsTile t = tiles[w];
    ens_tile(mem, EnsTile{__builtin_amdgcn_readfirstlane(t.m),
                          __builtin_amdgcn_readfirstlane(t.tx),
                          __builtin_amdgcn_readfirstlane(t.ty), 0},
             n, cfl, TY);
}

__global__ void k_ens_zero(unsigned* p, int count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = 0u;
}

__global__ void k_ens_advance(int* base, int by) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *base += by;
}

}  // namespace

struct sve_ens {
    int n = 0;
    std::vector<EnsMember> mem;          // host copy of the member table
    EnsMember* dmem = nullptr;
    Ctrl* dctrl = nullptr;
    Ctrl* hctrl = nullptr;               // pinned mirror of the control blocks
    double* pool = nullptr;
    size_t pool_bytes = 0;
    double* snapshot = nullptr;
    EnsTile* dtiles = nullptr;
    int ntiles = 0, tiles_rows = 0;
    unsigned* counters = nullptr;
    int ncounters = 0;
    int* dbase = nullptr;                // global step index of the next step
    hipStream_t stream = nullptr;
    int rows = 16, mode = SVE_ENS_QUEUE;
    long long nsteps = 0;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int g_steps = 0, g_rows = 0, g_mode = -1;
    double g_cfl = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_ms = 0.0;
    int queue_blocks = 512;
    int wave_slots = 2048;     // resident wavefronts of the single-grid step kernel
    std::vector<int> fail_step;          // per member, -1 when healthy
    int sticky = SVE_OK;
};

namespace {

void drop_graph(sve_ens* e);

int build_tiles(sve_ens* e, int rows) {
    if (e->dtiles && e->tiles_rows == rows) return SVE_OK;
    std::vector<int> order(e->n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (long long)e->mem[a].M.nx * e->mem[a].M.ny >
               (long long)e->mem[b].M.nx * e->mem[b].M.ny;
    });
    std::vector<EnsTile> t;
    for (int m : order) {
        const int tx = (e->mem[m].M.nx + FUSED_OWN - 1) / FUSED_OWN;
        const int ty = (e->mem[m].M.ny + rows - 1) / rows;
        for (int y = 0; y < ty; ++y)
            for (int x = 0; x < tx; ++x) t.push_back(EnsTile{m, x, y, 0});
    }
    // a captured graph holds the old tile list in its kernel arguments
    drop_graph(e);
    if (e->dtiles) (void)hipFree(e->dtiles);
    e->dtiles = nullptr;
    if (hipMalloc((void**)&e->dtiles, t.size() * sizeof(EnsTile)) != hipSuccess) return SVE_ERR_HIP;
    if (hipMemcpy(e->dtiles, t.data(), t.size() * sizeof(EnsTile), hipMemcpyHostToDevice) !=
        hipSuccess)
        return SVE_ERR_HIP;
    e->ntiles = (int)t.size();
    e->tiles_rows = rows;
    return SVE_OK;
}

int ensure_counters(sve_ens* e, int count) {
    if (e->ncounters >= count) return SVE_OK;
    if (e->counters) (void)hipFree(e->counters);
    e->counters = nullptr;
    e->ncounters = 0;
    if (hipMalloc((void**)&e->counters, (size_t)count * sizeof(unsigned)) != hipSuccess)
        return SVE_ERR_HIP;
    e->ncounters = count;
    return SVE_OK;
}

// Launch the ensemble kernels of `steps` steps on the stream (also used
// under graph capture): counters cleared by a kernel, then one kernel per
// step, then the device step index advanced.
void enqueue_steps(sve_ens* e, int steps, double cfl) {
    hipLaunchKernelGGL(k_ens_zero, dim3((steps + 255) / 256), dim3(256), 0, e->stream,
                       e->counters, steps);
    for (int s = 0; s < steps; ++s) {
        if (e->mode == SVE_ENS_QUEUE) {
            const int blocks = std::min(e->queue_blocks, (e->ntiles + ENS_WAVES - 1) / ENS_WAVES);
            hipLaunchKernelGGL(k_ens_queue, dim3(blocks), dim3(64 * ENS_WAVES), 0, e->stream,
                               e->dmem, e->dtiles, e->ntiles, e->counters + s, e->dbase, s, cfl,
                               e->rows);
        } else {
            hipLaunchKernelGGL(k_ens_grid, dim3((e->ntiles + ENS_WAVES - 1) / ENS_WAVES),
                               dim3(64 * ENS_WAVES), 0, e->stream, e->dmem, e->dtiles, e->ntiles,
                               e->dbase, s, cfl, e->rows);
        }
    }
    hipLaunchKernelGGL(k_ens_advance, dim3(1), dim3(64), 0, e->stream, e->dbase, steps);
}

void drop_graph(sve_ens* e) {
    if (e->gexec) (void)hipGraphExecDestroy(e->gexec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->gexec = nullptr;
    e->graph = nullptr;
    e->g_steps = 0;
}

int collect_errors(sve_ens* e) {
    if (hipMemcpyAsync(e->hctrl, e->dctrl, e->n * sizeof(Ctrl), hipMemcpyDeviceToHost,
                       e->stream) != hipSuccess ||
        hipStreamSynchronize(e->stream) != hipSuccess)
        return SVE_ERR_HIP;
    int first = SVE_OK;
    for (int m = 0; m < e->n; ++m) {
        const Ctrl& c = e->hctrl[m];
        if (c.err && e->fail_step[m] < 0) e->fail_step[m] = c.fail_step;
        if (c.err && first == SVE_OK)
            first = (c.err & ERR_NONFIN) ? SVE_ERR_NONFINITE
                  : (c.err & ERR_POS)    ? SVE_ERR_POSITIVITY
                                         : SVE_ERR_ORDER;
    }
    if (first) e->sticky = first;
    return first;
}

void free_ens(sve_ens* e) {
    if (!e) return;
    if (e->stream) (void)hipStreamSynchronize(e->stream); else (void)hipDeviceSynchronize();
    drop_graph(e);
    if (e->dmem) (void)hipFree(e->dmem);
    if (e->dctrl) (void)hipFree(e->dctrl);
    if (e->hctrl) (void)hipHostFree(e->hctrl);
    if (e->pool) (void)hipFree(e->pool);
    if (e->snapshot) (void)hipFree(e->snapshot);
    if (e->dtiles) (void)hipFree(e->dtiles);
    if (e->counters) (void)hipFree(e->counters);
    if (e->dbase) (void)hipFree(e->dbase);
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    delete e;
}

}  // namespace

extern "C" {

int sve_ens_create(sve_ens** out, int n, const sve_member* members, const sve_params* p,
                   void* stream) {
    if (!out || n < 1 || !members || !p) return SVE_ERR_ARG;
    *out = nullptr;
    if (p->law != SVE_LAW_GRASS || !(p->g > 0.0) || p->reconstruction ||
        p->order == 2)
        return SVE_ERR_ARG;
    sve_bc bc[4] = {{SVE_BC_PERIODIC, 0, 0, 0}, {SVE_BC_PERIODIC, 0, 0, 0},
                    {SVE_BC_PERIODIC, 0, 0, 0}, {SVE_BC_PERIODIC, 0, 0, 0}};
    for (int m = 0; m < n; ++m) {
        const sve_member& s = members[m];
        if (s.nx < 1 || s.ny < 1 || !(s.Lx > 0.0) || !(s.Ly > 0.0)) return SVE_ERR_ARG;
        if (!(s.m_g >= 1.0 && s.m_g <= 4.0) || !std::isfinite(s.A_g)) return SVE_ERR_ARG;
        if (!s.h || !s.hu || !s.hv || !s.zb) return SVE_ERR_ARG;
        const long long N = (long long)s.nx * s.ny;
        for (long long k = 0; k < N; ++k)
            if (!(s.h[k] > 0.0) || !std::isfinite(s.h[k]) || !std::isfinite(s.hu[k]) ||
                !std::isfinite(s.hv[k]) || !std::isfinite(s.zb[k]))
                return SVE_ERR_ARG;
    }
    sve_ens* e = new (std::nothrow) sve_ens();
    if (!e) return SVE_ERR_HIP;
    e->n = n;
    e->stream = (hipStream_t)stream;
    e->mem.resize(n);
    e->fail_step.assign(n, -1);
    size_t total = 0;
    std::vector<size_t> off(n);
    for (int m = 0; m < n; ++m) {
        const long long N = (long long)members[m].nx * members[m].ny;
        const long long pitch = (N + 63) / 64 * 64;
        off[m] = total;
        total += 2 * 4 * (size_t)pitch;
        sve_params q = *p;
        q.A_g = members[m].A_g;
        q.m_g = members[m].m_g;
        e->mem[m].M = make_model(members[m].nx, members[m].ny, members[m].Lx, members[m].Ly, 2,
                                 &q, bc);
        e->mem[m].pitch = pitch;
        e->mem[m].tiles_x = (members[m].nx + FUSED_OWN - 1) / FUSED_OWN;
    }
    e->pool_bytes = total * sizeof(double);
    bool ok = hipMalloc((void**)&e->pool, e->pool_bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&e->dctrl, n * sizeof(Ctrl)) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&e->hctrl, n * sizeof(Ctrl), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc((void**)&e->dmem, n * sizeof(EnsMember)) == hipSuccess;
    ok = ok && hipMalloc((void**)&e->dbase, sizeof(int)) == hipSuccess;
    ok = ok && hipEventCreate(&e->ev0) == hipSuccess && hipEventCreate(&e->ev1) == hipSuccess;
    if (!ok) {
        free_ens(e);
        return SVE_ERR_HIP;
    }
    for (int m = 0; m < n; ++m) {
        EnsMember& E = e->mem[m];
        E.buf[0] = e->pool + off[m];
        E.buf[1] = E.buf[0] + 4 * E.pitch;
        E.ctrl = e->dctrl + m;
        const size_t bytes = (size_t)members[m].nx * members[m].ny * sizeof(double);
        const double* src[4] = {members[m].h, members[m].hu, members[m].hv, members[m].zb};
        for (int f = 0; f < 4; ++f)
            if (hipMemcpyAsync(E.buf[0] + f * E.pitch, src[f], bytes, hipMemcpyHostToDevice,
                               e->stream) != hipSuccess) {
                free_ens(e);
                return SVE_ERR_HIP;
            }
        hipLaunchKernelGGL(k_reset_ctrl, dim3(1), dim3(64), 0, e->stream, E.ctrl, 0.0);
    }
    int zero = 0;
    ok = hipMemcpyAsync(e->dmem, e->mem.data(), n * sizeof(EnsMember), hipMemcpyHostToDevice,
                        e->stream) == hipSuccess &&
         hipMemcpyAsync(e->dbase, &zero, sizeof(int), hipMemcpyHostToDevice, e->stream) ==
             hipSuccess;
    // wave speeds of every member's initial state (slot 0)
    for (int m = 0; m < n && ok; ++m) {
        const EnsMember& E = e->mem[m];
        const long long nint = (long long)(E.M.nx + 1) * E.M.ny + (long long)E.M.nx * (E.M.ny + 1);
        hipLaunchKernelGGL((k_speeds<double, CL_GRASSM, false>), dim3((unsigned)((nint + 255) / 256)),
                           dim3(SPEED_BLOCK), 0, e->stream, E.M, view(E.buf[0], E.pitch),
                           (const double*)nullptr, E.ctrl, 0);
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    e->queue_blocks = 2 * cus;                       // two resident workgroups per CU
    e->wave_slots = cus * 4 * FUSED_WAVES_PER_SIMD;
    ok = ok && hipStreamSynchronize(e->stream) == hipSuccess && hipGetLastError() == hipSuccess;
    if (!ok || build_tiles(e, e->rows) != SVE_OK) {
        free_ens(e);
        return SVE_ERR_HIP;
    }
    *out = e;
    return SVE_OK;
}

int sve_ens_step(sve_ens* e, int nsteps, double cfl) {
    if (!e || nsteps < 0 || !(cfl > 0.0)) return SVE_ERR_ARG;
    if (nsteps == 0) return SVE_OK;
    if (build_tiles(e, e->rows) != SVE_OK || ensure_counters(e, nsteps) != SVE_OK)
        return SVE_ERR_HIP;
    if (!e->gexec || e->g_steps != nsteps || e->g_cfl != cfl || e->g_rows != e->rows ||
        e->g_mode != e->mode) {
        drop_graph(e);
        hipStream_t cap = nullptr;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return SVE_ERR_HIP;
        hipStream_t saved = e->stream;
        e->stream = cap;
        bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) enqueue_steps(e, nsteps, cfl);
        ok = (hipStreamEndCapture(cap, &e->graph) == hipSuccess) && ok;
        e->stream = saved;
        (void)hipStreamDestroy(cap);
        ok = ok && hipGraphInstantiate(&e->gexec, e->graph, nullptr, nullptr, 0) == hipSuccess;
        if (!ok) {
            drop_graph(e);
            return SVE_ERR_HIP;
        }
        e->g_steps = nsteps;
        e->g_cfl = cfl;
        e->g_rows = e->rows;
        e->g_mode = e->mode;
    }
    (void)hipEventRecord(e->ev0, e->stream);
    if (hipGraphLaunch(e->gexec, e->stream) != hipSuccess) return SVE_ERR_HIP;
    (void)hipEventRecord(e->ev1, e->stream);
    const int rc = collect_errors(e);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e->ev0, e->ev1) == hipSuccess) e->last_ms = ms;
    e->nsteps += nsteps;
    return rc;
}

int sve_ens_step_sequential(sve_ens* e, int nsteps, double cfl) {
    if (!e || nsteps < 0 || !(cfl > 0.0)) return SVE_ERR_ARG;
    if (nsteps == 0) return SVE_OK;
    (void)hipEventRecord(e->ev0, e->stream);
    const int n0 = (int)e->nsteps;
    for (int m = 0; m < e->n; ++m) {
        const EnsMember& E = e->mem[m];
        for (int s = 0; s < nsteps; ++s) {
            const int n = n0 + s;
            launch_fused_rows<double>(E.M, view(E.buf[n & 1], E.pitch),
                                      view(E.buf[(n + 1) & 1], E.pitch), nullptr, E.ctrl, n, cfl,
                                      0.0, 0.0, fused_tiles_y(E.M.nx, E.M.ny, 0, e->wave_slots),
                                      e->stream);
        }
    }
    hipLaunchKernelGGL(k_ens_advance, dim3(1), dim3(64), 0, e->stream, e->dbase, nsteps);
    (void)hipEventRecord(e->ev1, e->stream);
    if (hipGetLastError() != hipSuccess) return SVE_ERR_HIP;
    const int rc = collect_errors(e);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e->ev0, e->ev1) == hipSuccess) e->last_ms = ms;
    e->nsteps += nsteps;
    return rc;
}

int sve_ens_get(sve_ens* e, int m, double* h, double* hu, double* hv, double* zb, double* t,
                long long* nsteps) {
    if (!e || m < 0 || m >= e->n) return SVE_ERR_ARG;
    const EnsMember& E = e->mem[m];
    const long long n = e->fail_step[m] >= 0 ? e->fail_step[m] : e->nsteps;
    double* b = E.buf[n & 1];
    const size_t bytes = (size_t)E.M.nx * E.M.ny * sizeof(double);
    double* outs[4] = {h, hu, hv, zb};
    for (int f = 0; f < 4; ++f)
        if (outs[f] && hipMemcpyAsync(outs[f], b + f * E.pitch, bytes, hipMemcpyDeviceToHost,
                                      e->stream) != hipSuccess)
            return SVE_ERR_HIP;
    Ctrl c;
    if (hipMemcpyAsync(&c, E.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, e->stream) != hipSuccess ||
        hipStreamSynchronize(e->stream) != hipSuccess)
        return SVE_ERR_HIP;
    if (t) *t = c.t[n % 3];
    if (nsteps) *nsteps = n;
    return SVE_OK;
}

int sve_ens_set_schedule(sve_ens* e, int rows, int mode) {
    if (!e || (rows != 8 && rows != 16 && rows != 32 && rows != 48 && rows != 64 && rows != 96 &&
               rows != 128))
        return SVE_ERR_ARG;
    if (mode != SVE_ENS_QUEUE && mode != SVE_ENS_GRID) return SVE_ERR_ARG;
    e->rows = rows;
    e->mode = mode;
    return build_tiles(e, rows);
}

int sve_ens_autotune(sve_ens* e, int nprobe, double cfl, int* rows, int* mode) {
    if (!e || nprobe < 1 || !(cfl > 0.0)) return SVE_ERR_ARG;
    if (e->sticky) return e->sticky;
    if (!e->snapshot && hipMalloc((void**)&e->snapshot, e->pool_bytes) != hipSuccess)
        return SVE_ERR_HIP;
    std::vector<Ctrl> ctrl_save(e->n);
    if (hipMemcpyAsync(e->snapshot, e->pool, e->pool_bytes, hipMemcpyDeviceToDevice, e->stream) !=
            hipSuccess ||
        hipMemcpyAsync(ctrl_save.data(), e->dctrl, e->n * sizeof(Ctrl), hipMemcpyDeviceToHost,
                       e->stream) != hipSuccess ||
        hipStreamSynchronize(e->stream) != hipSuccess)
        return SVE_ERR_HIP;
    const long long n_saved = e->nsteps;
    // a member that fails during a probe marks fail_step and sticky; both
    // are rewound with the state
    const std::vector<int> fail_saved = e->fail_step;
    const int sticky_saved = e->sticky;
    int base_saved = 0;
    if (hipMemcpy(&base_saved, e->dbase, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return SVE_ERR_HIP;
    auto restore = [&]() {
        bool ok = hipMemcpyAsync(e->pool, e->snapshot, e->pool_bytes, hipMemcpyDeviceToDevice,
                                 e->stream) == hipSuccess &&
                  hipMemcpyAsync(e->dctrl, ctrl_save.data(), e->n * sizeof(Ctrl),
                                 hipMemcpyHostToDevice, e->stream) == hipSuccess &&
                  hipMemcpyAsync(e->dbase, &base_saved, sizeof(int), hipMemcpyHostToDevice,
                                 e->stream) == hipSuccess &&
                  hipStreamSynchronize(e->stream) == hipSuccess;
        e->nsteps = n_saved;
        e->fail_step = fail_saved;
        e->sticky = sticky_saved;
        return ok;
    };
    const int cand_rows[7] = {8, 16, 32, 48, 64, 96, 128};
    double best = 1e300;
    int best_rows = e->rows, best_mode = e->mode;
    for (int md = 0; md < 2; ++md) {
        for (int r : cand_rows) {
            if (sve_ens_set_schedule(e, r, md) != SVE_OK) return SVE_ERR_HIP;
            int rc = sve_ens_step(e, nprobe, cfl);          // capture + warm-up
            if (!restore()) return SVE_ERR_HIP;
            if (rc) return rc;
            rc = sve_ens_step(e, nprobe, cfl);              // timed replay
            const double ms = e->last_ms;
            if (!restore()) return SVE_ERR_HIP;
            if (rc) return rc;
            if (ms < best) {
                best = ms;
                best_rows = r;
                best_mode = md;
            }
        }
    }
    drop_graph(e);
    if (sve_ens_set_schedule(e, best_rows, best_mode) != SVE_OK) return SVE_ERR_HIP;
    if (rows) *rows = best_rows;
    if (mode) *mode = best_mode;
    return SVE_OK;
}

int sve_ens_last_elapsed_ms(sve_ens* e, double* ms) {
    if (!e || !ms) return SVE_ERR_ARG;
    *ms = e->last_ms;
    return SVE_OK;
}

int sve_ens_destroy(sve_ens* e) {
    free_ens(e);
    return SVE_OK;
}

}  // extern "C"
