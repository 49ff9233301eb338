// sve_noalloc.hip -- CFL steps on caller-owned device state without any
// device allocation (declaration and contract in include/sve.h,
// sve_step_dev_noalloc).
//
// The one buffer the step kernels need besides the two states is the
// control block (wave-speed maxima, times, error word).  Here it lives in a
// file-scope device array, `scratch`, of SCRATCH_BYTES bytes: every GPU the
// library runs on holds one copy of it until the process ends, and every
// call on that GPU shares it.  In host code the array's name is not a device
// address; its address on each device is taken once with
// hipGetSymbolAddress (with that device current) and kept per device, and
// only that address is handed to kernels.  The caller's two state buffers
// serve as the double buffer of the steps.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstddef>
#include <mutex>

#include "../../include/sve.h"
#include "sve_context.hpp"
#include "sve_fused.hpp"
#include "sve_kernels.hpp"

using namespace sve;

namespace {

constexpr size_t SCRATCH_BYTES = 4096;
static_assert(sizeof(Ctrl) <= SCRATCH_BYTES, "control block larger than the scratch array");
static_assert(alignof(Ctrl) <= 256, "control block alignment");

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

struct DeviceScratch {
    Ctrl* ctrl = nullptr;    // address of `scratch` on the device
    int wave_slots = 0;      // resident wavefronts of the step kernel
};

std::mutex g_mutex;
DeviceScratch g_dev[MAX_DEVICES];

// Address of the scratch array on the current device, taken on the first
// call on that device.
int device_scratch(DeviceScratch& out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SVE_ERR_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return SVE_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_mutex);
    DeviceScratch& d = g_dev[dev];
    if (!d.ctrl) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return SVE_ERR_HIP;
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            cus <= 0)
            return SVE_ERR_HIP;
        d.wave_slots = cus * 4 * FUSED_WAVES_PER_SIMD;   // 4 SIMDs per compute unit
        d.ctrl = static_cast<Ctrl*>(ptr);
    }
    out = d;
    return SVE_OK;
}

// Input state checked as sve_init_state checks it: finite, h > 0.
__global__ void k_check_input(Model M, StateView<double> S, Ctrl* ctrl) {
    const long long N = (long long)M.nx * M.ny;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const unsigned e = check_state(S.h[k], S.hu[k], S.hv[k], S.z[k]);
    if (e) atomicOr(&ctrl->err, e);
}

// The fields of the control block the host reads after a call.
struct CtrlTail {
    double t[3];
    double dt_last;
    unsigned err;
    int fail_step;
};

static_assert(offsetof(Ctrl, fail_step) - offsetof(Ctrl, t) == offsetof(CtrlTail, fail_step),
              "CtrlTail mirrors the end of the control block");

int copy_state(const StateView<double>& from, const StateView<double>& to, long long N,
               hipStream_t stream) {
    const size_t bytes = (size_t)N * sizeof(double);
    const double* src[4] = {from.h, from.hu, from.hv, from.z};
    double* dst[4] = {to.h, to.hu, to.hv, to.z};
    for (int f = 0; f < 4; ++f)
        if (hipMemcpyAsync(dst[f], src[f], bytes, hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return SVE_ERR_HIP;
    return SVE_OK;
}

bool overlaps(const double* a, const double* b, long long n) {
    return a < b + n && b < a + n;
}

}  // namespace

extern "C" int sve_step_dev_noalloc(int nx, int ny, double Lx, double Ly, const sve_params* p,
                                    const sve_bc bc[4], double* h, double* hu, double* hv,
                                    double* zb, double* h_out, double* hu_out, double* hv_out,
                                    double* zb_out, int n, double cfl, double t_end, double* t,
                                    double* dt_last, void* stream) {
    if (!h || !hu || !hv || !zb || !h_out || !hu_out || !hv_out || !zb_out || !t)
        return SVE_ERR_ARG;
    if (nx < 1 || ny < 1 || (long long)nx * ny > (long long)INT_MAX) return SVE_ERR_ARG;
    if (!(Lx > 0.0) || !(Ly > 0.0) || n < 0 || !(cfl > 0.0) || !std::isfinite(*t))
        return SVE_ERR_ARG;
    if (validate_params(p, 2, bc) != SVE_OK || p->reconstruction ||
        p->order == 2)
        return SVE_ERR_ARG;
    const long long N = (long long)nx * ny;
    double* ins[4] = {h, hu, hv, zb};
    double* outs[4] = {h_out, hu_out, hv_out, zb_out};
    for (int a = 0; a < 8; ++a)
        for (int b = a + 1; b < 8; ++b) {
            const double* x = a < 4 ? ins[a] : outs[a - 4];
            const double* y = b < 4 ? ins[b] : outs[b - 4];
            if (overlaps(x, y, N)) return SVE_ERR_ARG;
        }
    DeviceScratch ds;
    int rc = device_scratch(ds);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Model M = make_model(nx, ny, Lx, Ly, 2, p, bc);
    const StateView<double> buf[2] = {StateView<double>{h, hu, hv, zb},
                                      StateView<double>{h_out, hu_out, hv_out, zb_out}};
    Ctrl* ctrl = ds.ctrl;
    // the control block keeps the last call's contents: reset it (a kernel,
    // not a memset) and check the input
    hipLaunchKernelGGL(k_reset_ctrl, dim3(1), dim3(64), 0, s, ctrl, *t);
    hipLaunchKernelGGL(k_check_input, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, M,
                       buf[0], ctrl);
    // wave speeds of the input state (step 0 reads slot 0)
    launch_speeds_model<double>(M, buf[0], nullptr, ctrl, 0, s);
    const int tiles_y = fused_tiles_y(nx, ny, 0, ds.wave_slots);
    for (int k = 0; k < n; ++k)
        launch_fused_rows<double>(M, buf[k & 1], buf[(k + 1) & 1], nullptr, ctrl, k, cfl, t_end,
                                  0.0, tiles_y, s);
    if (hipGetLastError() != hipSuccess) return SVE_ERR_HIP;
    CtrlTail tail;
    const char* base = reinterpret_cast<const char*>(ctrl);
    if (hipMemcpyAsync(&tail, base + offsetof(Ctrl, t), sizeof(CtrlTail), hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SVE_ERR_HIP;
    int done = n;
    rc = SVE_OK;
    if (tail.err) {
        if (tail.fail_step < 0 || tail.fail_step >= n) return SVE_ERR_ARG;   // input rejected
        done = tail.fail_step;
        rc = (tail.err & ERR_NONFIN) ? SVE_ERR_NONFINITE
           : (tail.err & ERR_POS)    ? SVE_ERR_POSITIVITY
                                     : SVE_ERR_ORDER;
    }
    // the state after `done` steps is in buf[done & 1]; the result goes to
    // the output arrays
    if ((done & 1) == 0) {
        if (copy_state(buf[0], buf[1], N, s) != SVE_OK || hipStreamSynchronize(s) != hipSuccess)
            return SVE_ERR_HIP;
    }
    *t = tail.t[done % 3];
    if (dt_last && rc == SVE_OK) *dt_last = n > 0 ? tail.dt_last : 0.0;
    return rc;
}
