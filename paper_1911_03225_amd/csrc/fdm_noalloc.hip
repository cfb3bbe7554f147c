// fdm_noalloc.hip -- fdm_transport_step_noalloc: the transport step of one
// float32 instance without any device allocation.
//
// The stage buffer and the max |v0| partials live in a file-scope device
// array, `scratch`, instead of memory from hipMalloc.  In host code the
// array's name only stands for the symbol: the kernels get its device
// address, looked up once per device with hipGetSymbolAddress (each GPU
// holds its own copy at its own address) and kept in g_scratch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/fdm.h"
#include "fdm_host.h"
#include "fdm_internal.h"

using fdm::InstDev;
using namespace fdm::host;

namespace {

constexpr int64_t kMaxNodes = FDM_NOALLOC_MAX_NODES;
constexpr size_t kStageBytes = 2 * (size_t)kMaxNodes * sizeof(float);   // both components
constexpr size_t kScratchBytes = kStageBytes + fdm::kAbsmaxBlocks * sizeof(float);

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch`, per device

// The current device's address of `scratch`, looked up on the first call on
// that device (with the device current).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

fdm_status reject(fdm_status st, const std::string &msg)
{
    set_init_error(msg);
    return st;
}

fdm_status device_error(const char *what, hipError_t e)
{
    return reject(e == hipErrorOutOfMemory ? FDM_ERR_OUT_OF_MEMORY : FDM_ERR_DEVICE,
                  std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" fdm_status fdm_transport_step_noalloc(const fdm_transport_desc *desc, void *alpha11, void *alpha12,
                                                 int32_t n_steps, void *hip_stream)
{
    // host checks first, as in fdm_transport_init
    if (!desc) return reject(FDM_ERR_INVALID_ARG, "desc must not be NULL");
    const fdm_transport_desc &d = *desc;
    const std::string m = check_desc(d);
    if (!m.empty()) return reject(FDM_ERR_INVALID_ARG, m);
    const int64_t n = (int64_t)d.nx * d.ny;
    if (n > kMaxNodes)
        return reject(FDM_ERR_INVALID_ARG, "nx*ny = " + std::to_string(n) + " exceeds the allocation-free maximum of " +
                                               std::to_string(kMaxNodes) + " nodes");
    if (n_steps < 0) return reject(FDM_ERR_INVALID_ARG, "n_steps must be >= 0");
    if (!alpha11 || !alpha12) return reject(FDM_ERR_INVALID_ARG, "alpha11 and alpha12 must not be NULL");
    if (alpha11 == alpha12) return reject(FDM_ERR_INVALID_ARG, "alpha11 and alpha12 alias");
    const bool fd = d.scheme == FDM_SCHEME_FULLY_DISCRETE;
    const int32_t order = d.time_order == 0 ? (fd ? 1 : 2) : d.time_order;
    const bool field = d.velocity == FDM_VELOCITY_LAW && d.v0_field;
    if (!(field && d.dt > 0.0)) {
        const std::string c = check_courant(d, order, std::fabs((double)(float)d.v0));
        if (!c.empty()) return reject(FDM_ERR_CFL, c);
    }
    if (n_steps == 0) return FDM_OK;

    hipStream_t s = (hipStream_t)hip_stream;
    void *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) return device_error("hipGetSymbolAddress(scratch)", e);
    char *const stage = static_cast<char *>(base);
    float *const partials = reinterpret_cast<float *>(stage + kStageBytes);

    double smax;
    if (field) {   // max |v0| of the field, read back as fdm_transport_init does
        float host[fdm::kAbsmaxBlocks];
        if ((e = fdm::launch_absmax(d.v0_field, n, partials, s)) != hipSuccess) return device_error("absmax", e);
        if ((e = hipMemcpyAsync(host, partials, sizeof(host), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return device_error("hipMemcpyAsync", e);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return device_error("hipStreamSynchronize", e);
        float mx = 0.0f;
        for (float v : host) {
            if (std::isnan(v)) return reject(FDM_ERR_INVALID_ARG, "v0_field is not finite");
            mx = std::fmax(mx, v);
        }
        smax = mx;
        if (d.dt > 0.0) {
            const std::string c = check_courant(d, order, smax);
            if (!c.empty()) return reject(FDM_ERR_CFL, c);
        }
    } else {
        smax = smax_uniform(d);
    }

    // one instance, the default schedule of fdm_transport_init (one stage
    // launch per stage, default tile height): the same kernels and bits
    InstDev I;
    fill_inst(I, d, step_dt(d, smax), stage, stage + (size_t)n * sizeof(float));
    I.a11 = alpha11;
    I.a12 = alpha12;
    I.rows = pick_rows(strip_rows_of(d), d.ny, 0);
    I.strips = (d.nx + fdm::kStrip - 1) / fdm::kStrip;
    I.fstrips = (d.nx + fdm::kFusedStrip - 1) / fdm::kFusedStrip;
    I.chunks = fdm::tiles_along_y(d.ny, I.rows);
    for (int32_t step = 0; step < n_steps; ++step) {
        int modes[2];
        const int nm = stage_modes(order, step, modes);
        for (int k = 0; k < nm; ++k)
            if ((e = fdm::launch_stage(I, modes[k], fdm::PREC_FP32, s)) != hipSuccess)
                return device_error("stage launch", e);
    }
    // one Euler stage ping-pongs between the state and the stage buffer
    if (order == 1 && (n_steps & 1)) {
        if ((e = fdm::launch_copy(alpha11, I.w11, n, fdm::PREC_FP32, s)) != hipSuccess)
            return device_error("copy", e);
        if ((e = fdm::launch_copy(alpha12, I.w12, n, fdm::PREC_FP32, s)) != hipSuccess)
            return device_error("copy", e);
    }
    return FDM_OK;
}
