// fdm_static.hip -- static problem of the layer case on the GPU.
//
// Layer-averaged shear stress tau13 at the layer nodes for given densities
// (Morin, Brenner & Suquet, arXiv:1911.03225, sec. 3.1.2 and 3.2.1): a
// periodic cell of homogeneous isotropic elasticity (mu, lambda), n3 voxels
// high, holds a layer of h voxels carrying U^p = phi(x1,x2) e1 (x) e3.  The
// homogeneous Green-operator solution sigma^ = (C:Gamma^ - I):C:U^p^ gives,
// for this ansatz,
//     sigma13^(xi) = -mu phi^ chi^(xi3) G(xi),
//     G = xi2^2/|xi|^2 + 2/(1-nu) xi1^2 xi3^2/|xi|^4,
// so the layer average folds x3 into a 2-D multiplier:
//     tau13^ = -mu K phi^,  K = (n3/h) sum_m3 |chi^[m3]|^2 G(xi1, xi2, xi3(m3)),
// and the mean is sigma_bar_13 = 2 mu eps_bar_13 - mu (h/n3) <phi>.
// phi^ comes from the densities: alpha12 = D1 phi, alpha11 = -D2 phi are
// forward differences on the staggered grid, with Fourier symbols
// d = (e^{i 2 pi m/n} - 1)/d, inverted in least squares:
//     phi^ = (conj(d1) alpha12^ - conj(d2) alpha11^) / (|d1|^2 + |d2|^2).
//
// GPU pipeline per solve: pack the two density arrays (rocFFT may overwrite
// an out-of-place input), one batched real-to-complex FFT (rocFFT), the
// pointwise multiplier kernel below, one complex-to-real FFT into tau13.
// K is built once per plan by a kernel (FP64 sum over m3).
#pragma clang fp contract(off)
#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "fdm_static.h"

namespace fdm {
namespace {

constexpr double kPi = 3.14159265358979323846;

// K[m2 * nxh + m1] over the half spectrum m1 = 0 .. nx/2; FP64 throughout.
template <typename T>
__global__ __launch_bounds__(256) void layer_multiplier_kernel(T *K, int nx, int ny, int nxh, double dx, double dy,
                                                                int n3, const double *c2, const double *xi3sq,
                                                                double two_over_1mnu, double n3_over_h)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nxh * ny) return;
    const int m1 = (int)(idx % nxh), m2 = (int)(idx / nxh);
    const int f1 = m1 <= nx - m1 ? m1 : nx - m1;          // |signed frequency|
    const int f2 = m2 <= ny - m2 ? m2 : ny - m2;
    const double x1 = 2.0 * kPi * f1 / (nx * dx), x2 = 2.0 * kPi * f2 / (ny * dy);
    const double x1s = x1 * x1, x2s = x2 * x2;
    double acc = 0.0;
    if (m1 != 0 || m2 != 0) {
        for (int m3 = 0; m3 < n3; ++m3) {
            const double s = x1s + x2s + xi3sq[m3];
            const double g = x2s / s + two_over_1mnu * x1s * xi3sq[m3] / (s * s);
            acc += c2[m3] * g;
        }
    }
    K[idx] = (T)(acc * n3_over_h);
}

// out[m] = -mu K[m] phi^[m] / N (m != 0), out[0] = sigma_bar; spec holds the
// two transforms alpha11^ then alpha12^ (interleaved complex).
template <typename T>
__global__ __launch_bounds__(256) void green_kernel(const T *spec, T *out, const T *K, const T *d1, const T *d2,
                                                     int nxh, int ny, T neg_mu_over_n, const double *sigma_bar)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nmodes = (int64_t)nxh * ny;
    if (idx >= nmodes) return;
    const int m1 = (int)(idx % nxh), m2 = (int)(idx / nxh);
    const T a11r = spec[2 * idx], a11i = spec[2 * idx + 1];
    const T a12r = spec[2 * (nmodes + idx)], a12i = spec[2 * (nmodes + idx) + 1];
    const T d1r = d1[2 * m1], d1i = d1[2 * m1 + 1];
    const T d2r = d2[2 * m2], d2i = d2[2 * m2 + 1];
    T re, im;
    if (idx == 0) {
        re = (T)*sigma_bar;
        im = T(0);
    } else {
        // conj(d1) a12 - conj(d2) a11
        const T nr = (d1r * a12r + d1i * a12i) - (d2r * a11r + d2i * a11i);
        const T ni = (d1r * a12i - d1i * a12r) - (d2r * a11i - d2i * a11r);
        const T den = (d1r * d1r + d1i * d1i) + (d2r * d2r + d2i * d2i);
        const T f = neg_mu_over_n * K[idx] / den;
        re = f * nr;
        im = f * ni;
    }
    out[2 * idx] = re;
    out[2 * idx + 1] = im;
}

template <typename T>
__global__ __launch_bounds__(256) void pack_kernel(T *dst, const T *a11, const T *a12, int64_t n, SlipArgs slip)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        dst[i] = a11[i];
        dst[n + i] = a12[i];
    }
    // the previous coupled step's slip update, ahead of every reader of the
    // mean stress and slip (the later kernels of this solve)
    if (slip.cd != nullptr && blockIdx.x == 0) {
        __shared__ double2 lds[256];
        coupled_slip_block(slip, lds);
    }
}

// Celerity field (float32), m = mobility * mfield[i]:
//   threshold: v0 = -m S_tau0(tau13), S the soft threshold;
//   wiggly:    v0 = m (tau_y cos(phi / beta) - tau13).
template <typename T, bool WIGGLY>
__global__ __launch_bounds__(256) void velocity_law_kernel(const T *tau, const T *phi, const float *mfield, float *v0,
                                                            int64_t n, T tau0, T mobility, T tau_y, T beta,
                                                            float *partial)
{
    __shared__ float lds[4];
    float amax = 0.0f;   // this thread's max |v0|, NaN once a non-finite value is seen
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const T t = tau[i];
        const T m = mfield ? mobility * T(mfield[i]) : mobility;
        T v;
        if constexpr (WIGGLY) {
            v = m * (tau_y * cos(phi[i] / beta) - t);
        } else {
            const T a = fabs(t) - tau0;
            const T s = a > T(0) ? copysign(a, t) : T(0);
            v = -(m * s);
        }
        const float vf = (float)v;
        v0[i] = vf;
        bad |= !isfinite(vf);
        amax = fmaxf(amax, fabsf(vf));
    }
    // block partial of max |v0| for the step size (NaN marks a non-finite value)
    if (bad) amax = __builtin_nanf("");
    for (int o = 32; o > 0; o >>= 1) {
        const float other = __shfl_xor(amax, o, 64);
        amax = (isnan(amax) || isnan(other)) ? __builtin_nanf("") : fmaxf(amax, other);
    }
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = amax;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = lds[0];
        for (int w = 1; w < 4; ++w) r = (isnan(r) || isnan(lds[w])) ? __builtin_nanf("") : fmaxf(r, lds[w]);
        partial[blockIdx.x] = r;
    }
}

// phi^ / N at every mode (phi_mean at the mean), for a complex-to-real
// transform; spec holds alpha11^ then alpha12^.
template <typename T>
__global__ __launch_bounds__(256) void phi_kernel(const T *spec, T *out, const T *d1, const T *d2, int nxh, int ny,
                                                   T inv_n, const double *phi_mean)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nmodes = (int64_t)nxh * ny;
    if (idx >= nmodes) return;
    const int m1 = (int)(idx % nxh), m2 = (int)(idx / nxh);
    T re, im;
    if (idx == 0) {
        re = (T)*phi_mean;
        im = T(0);
    } else {
        const T a11r = spec[2 * idx], a11i = spec[2 * idx + 1];
        const T a12r = spec[2 * (nmodes + idx)], a12i = spec[2 * (nmodes + idx) + 1];
        const T d1r = d1[2 * m1], d1i = d1[2 * m1 + 1];
        const T d2r = d2[2 * m2], d2i = d2[2 * m2 + 1];
        const T nr = (d1r * a12r + d1i * a12i) - (d2r * a11r + d2i * a11i);
        const T ni = (d1r * a12i - d1i * a12r) - (d2r * a11i - d2i * a11r);
        const T den = (d1r * d1r + d1i * d1i) + (d2r * d2r + d2i * d2i);
        const T f = inv_n / den;
        re = f * nr;
        im = f * ni;
    }
    out[2 * idx] = re;
    out[2 * idx + 1] = im;
}

std::once_flag g_rocfft_once;
rocfft_status g_rocfft_setup = rocfft_status_success;

const char *rocfft_message(rocfft_status s)
{
    switch (s) {
    case rocfft_status_success: return "success";
    case rocfft_status_failure: return "failure";
    case rocfft_status_invalid_arg_value: return "invalid argument value";
    case rocfft_status_invalid_dimensions: return "invalid dimensions";
    case rocfft_status_invalid_array_type: return "invalid array type";
    case rocfft_status_invalid_strides: return "invalid strides";
    case rocfft_status_invalid_distance: return "invalid distance";
    case rocfft_status_invalid_offset: return "invalid offset";
    case rocfft_status_invalid_work_buffer: return "invalid work buffer";
    default: return "unknown rocFFT status";
    }
}

}  // namespace

struct StaticPlan {
    int nx = 0, ny = 0, nxh = 0;
    bool f64 = false;
    double mu = 1.0;
    rocfft_plan fwd = nullptr, inv = nullptr;
    rocfft_execution_info info = nullptr;
    void *work = nullptr;
    void *real2 = nullptr;   // packed densities, 2 * nx * ny reals
    void *spec = nullptr;    // 2 spectra, 2 * ny * nxh complex
    void *K = nullptr;       // ny * nxh reals
    void *d1 = nullptr;      // nxh complex
    void *d2 = nullptr;      // ny complex
    double *scal = nullptr;  // [mean stress, mean slip] of one-off solves
};

#define ST_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                          \
            return e_ == hipErrorOutOfMemory ? StaticStatus::OutOfMemory : StaticStatus::Device; \
        }                                                                                     \
    } while (0)
#define ST_FFT(call)                                                                          \
    do {                                                                                      \
        rocfft_status r_ = (call);                                                            \
        if (r_ != rocfft_status_success) {                                                    \
            err = std::string(#call) + ": " + rocfft_message(r_);                             \
            return StaticStatus::Device;                                                      \
        }                                                                                     \
    } while (0)

void static_plan_destroy(StaticPlan *p)
{
    if (!p) return;
    if (p->fwd) (void)rocfft_plan_destroy(p->fwd);
    if (p->inv) (void)rocfft_plan_destroy(p->inv);
    if (p->info) (void)rocfft_execution_info_destroy(p->info);
    for (void *b : {p->work, p->real2, p->spec, p->K, p->d1, p->d2, (void *)p->scal})
        if (b) (void)hipFree(b);
    delete p;
}

StaticStatus static_plan_create(const StaticParams &q, hipStream_t s, StaticPlan **out, std::string &err)
{
    *out = nullptr;
    std::call_once(g_rocfft_once, [] { g_rocfft_setup = rocfft_setup(); });
    if (g_rocfft_setup != rocfft_status_success) {
        err = std::string("rocfft_setup: ") + rocfft_message(g_rocfft_setup);
        return StaticStatus::Device;
    }
    StaticPlan *p = new StaticPlan;
    StaticStatus st = [&]() -> StaticStatus {
        p->nx = q.nx;
        p->ny = q.ny;
        p->nxh = q.nx / 2 + 1;
        p->f64 = q.f64;
        p->mu = q.mu;
        const size_t es = q.f64 ? sizeof(double) : sizeof(float);
        const int64_t n = (int64_t)q.nx * q.ny, nm = (int64_t)p->nxh * q.ny;
        ST_HIP(hipMalloc(&p->real2, es * 2 * n));
        ST_HIP(hipMalloc(&p->spec, es * 2 * 2 * nm));
        ST_HIP(hipMalloc(&p->K, es * nm));
        ST_HIP(hipMalloc(&p->d1, es * 2 * p->nxh));
        ST_HIP(hipMalloc(&p->d2, es * 2 * q.ny));
        ST_HIP(hipMalloc((void **)&p->scal, 2 * sizeof(double)));

        // symbols of the forward differences, in FP64 on the host
        std::vector<double> d1(2 * p->nxh), d2(2 * q.ny);
        for (int m = 0; m < p->nxh; ++m) {
            const double t = 2.0 * kPi * m / q.nx;
            d1[2 * m] = (std::cos(t) - 1.0) / q.dx;
            d1[2 * m + 1] = std::sin(t) / q.dx;
        }
        for (int m = 0; m < q.ny; ++m) {
            const double t = 2.0 * kPi * m / q.ny;
            d2[2 * m] = (std::cos(t) - 1.0) / q.dy;
            d2[2 * m + 1] = std::sin(t) / q.dy;
        }
        // |chi^[m3]|^2 of h consecutive voxels out of n3, and xi3^2
        std::vector<double> c2(q.n3), x3(q.n3);
        for (int m = 0; m < q.n3; ++m) {
            double re = 0.0, im = 0.0;
            for (int z = 0; z < q.h; ++z) {
                const double t = -2.0 * kPi * (double)m * z / q.n3;
                re += std::cos(t);
                im += std::sin(t);
            }
            c2[m] = (re * re + im * im) / ((double)q.n3 * q.n3);
            const int f = m <= q.n3 - m ? m : q.n3 - m;
            const double xi = 2.0 * kPi * f / (q.n3 * q.dx);
            x3[m] = xi * xi;
        }
        double *dc2 = nullptr, *dx3 = nullptr;
        ST_HIP(hipMalloc((void **)&dc2, sizeof(double) * q.n3));
        hipError_t e = hipMalloc((void **)&dx3, sizeof(double) * q.n3);
        if (e != hipSuccess) {
            (void)hipFree(dc2);
            ST_HIP(e);
        }
        auto upload = [&]() -> StaticStatus {
            ST_HIP(hipMemcpyAsync(dc2, c2.data(), sizeof(double) * q.n3, hipMemcpyHostToDevice, s));
            ST_HIP(hipMemcpyAsync(dx3, x3.data(), sizeof(double) * q.n3, hipMemcpyHostToDevice, s));
            const double nu = q.lambda / (2.0 * (q.lambda + q.mu));
            const unsigned blocks = (unsigned)((nm + 255) / 256);
            if (q.f64) {
                std::vector<double> t1(d1), t2(d2);
                ST_HIP(hipMemcpyAsync(p->d1, t1.data(), sizeof(double) * t1.size(), hipMemcpyHostToDevice, s));
                ST_HIP(hipMemcpyAsync(p->d2, t2.data(), sizeof(double) * t2.size(), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(layer_multiplier_kernel<double>, dim3(blocks), dim3(256), 0, s, (double *)p->K, q.nx,
                                   q.ny, p->nxh, q.dx, q.dy, q.n3, dc2, dx3, 2.0 / (1.0 - nu), (double)q.n3 / q.h);
                ST_HIP(hipGetLastError());
                ST_HIP(hipStreamSynchronize(s));   // host tables go out of scope
            } else {
                std::vector<float> t1(d1.begin(), d1.end()), t2(d2.begin(), d2.end());
                ST_HIP(hipMemcpyAsync(p->d1, t1.data(), sizeof(float) * t1.size(), hipMemcpyHostToDevice, s));
                ST_HIP(hipMemcpyAsync(p->d2, t2.data(), sizeof(float) * t2.size(), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(layer_multiplier_kernel<float>, dim3(blocks), dim3(256), 0, s, (float *)p->K, q.nx,
                                   q.ny, p->nxh, q.dx, q.dy, q.n3, dc2, dx3, 2.0 / (1.0 - nu), (double)q.n3 / q.h);
                ST_HIP(hipGetLastError());
                ST_HIP(hipStreamSynchronize(s));
            }
            return StaticStatus::Ok;
        };
        StaticStatus us = upload();
        (void)hipFree(dc2);
        (void)hipFree(dx3);
        if (us != StaticStatus::Ok) return us;

        const rocfft_precision prec = q.f64 ? rocfft_precision_double : rocfft_precision_single;
        const size_t len[2] = {(size_t)q.nx, (size_t)q.ny};   // fastest first
        ST_FFT(rocfft_plan_create(&p->fwd, rocfft_placement_notinplace, rocfft_transform_type_real_forward, prec, 2,
                                  len, 2, nullptr));
        ST_FFT(rocfft_plan_create(&p->inv, rocfft_placement_notinplace, rocfft_transform_type_real_inverse, prec, 2,
                                  len, 1, nullptr));
        size_t w1 = 0, w2 = 0;
        ST_FFT(rocfft_plan_get_work_buffer_size(p->fwd, &w1));
        ST_FFT(rocfft_plan_get_work_buffer_size(p->inv, &w2));
        ST_FFT(rocfft_execution_info_create(&p->info));
        const size_t w = w1 > w2 ? w1 : w2;
        if (w > 0) {
            ST_HIP(hipMalloc(&p->work, w));
            ST_FFT(rocfft_execution_info_set_work_buffer(p->info, p->work, w));
        }
        return StaticStatus::Ok;
    }();
    if (st != StaticStatus::Ok) {
        static_plan_destroy(p);
        return st;
    }
    *out = p;
    return StaticStatus::Ok;
}

namespace {
StaticStatus run_impl(StaticPlan *p, const void *a11, const void *a12, void *tau13, void *phi,
                      const double *sigma_bar, const double *phi_mean, const SlipArgs *slip, hipStream_t s,
                      std::string &err);
}

double *static_plan_scalars(StaticPlan *p) { return p->scal; }

StaticStatus static_plan_run(StaticPlan *p, const void *a11, const void *a12, void *tau13, const double *sigma_bar,
                             const SlipArgs *slip, hipStream_t s, std::string &err)
{
    return run_impl(p, a11, a12, tau13, nullptr, sigma_bar, nullptr, slip, s, err);
}

StaticStatus static_plan_run_phi(StaticPlan *p, const void *a11, const void *a12, void *tau13, void *phi,
                                 const double *sigma_bar, const double *phi_mean, const SlipArgs *slip,
                                 hipStream_t s, std::string &err)
{
    return run_impl(p, a11, a12, tau13, phi, sigma_bar, phi_mean, slip, s, err);
}

namespace {
StaticStatus run_impl(StaticPlan *p, const void *a11, const void *a12, void *tau13, void *phi,
                      const double *sigma_bar, const double *phi_mean, const SlipArgs *slip, hipStream_t s,
                      std::string &err)
{
    SlipArgs sa{};
    if (slip) sa = *slip;
    const int64_t n = (int64_t)p->nx * p->ny, nm = (int64_t)p->nxh * p->ny;
    ST_FFT(rocfft_execution_info_set_stream(p->info, s));
    const unsigned pb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    const unsigned gb = (unsigned)((nm + 255) / 256);
    if (p->f64) {
        hipLaunchKernelGGL(pack_kernel<double>, dim3(pb), dim3(256), 0, s, (double *)p->real2, (const double *)a11,
                           (const double *)a12, n, sa);
    } else {
        hipLaunchKernelGGL(pack_kernel<float>, dim3(pb), dim3(256), 0, s, (float *)p->real2, (const float *)a11,
                           (const float *)a12, n, sa);
    }
    ST_HIP(hipGetLastError());
    void *in[1] = {p->real2}, *outb[1] = {p->spec};
    ST_FFT(rocfft_execute(p->fwd, in, outb, p->info));
    if (phi) {
        // phi^ into the (consumed) packed-input buffer, then to the nodes
        if (p->f64)
            hipLaunchKernelGGL(phi_kernel<double>, dim3(gb), dim3(256), 0, s, (const double *)p->spec,
                               (double *)p->real2, (const double *)p->d1, (const double *)p->d2, p->nxh, p->ny,
                               1.0 / (double)n, phi_mean);  // device pointer
        else
            hipLaunchKernelGGL(phi_kernel<float>, dim3(gb), dim3(256), 0, s, (const float *)p->spec,
                               (float *)p->real2, (const float *)p->d1, (const float *)p->d2, p->nxh, p->ny,
                               (float)(1.0 / (double)n), phi_mean);
        ST_HIP(hipGetLastError());
        void *pin[1] = {p->real2}, *pout[1] = {phi};
        ST_FFT(rocfft_execute(p->inv, pin, pout, p->info));
    }
    // the product overwrites alpha11^ in place: each thread reads its own
    // mode of both spectra before writing that mode
    void *prod = p->spec;
    if (p->f64) {
        hipLaunchKernelGGL(green_kernel<double>, dim3(gb), dim3(256), 0, s, (const double *)p->spec, (double *)prod,
                           (const double *)p->K, (const double *)p->d1, (const double *)p->d2, p->nxh, p->ny,
                           -p->mu / (double)n, sigma_bar);  // device pointer
    } else {
        hipLaunchKernelGGL(green_kernel<float>, dim3(gb), dim3(256), 0, s, (const float *)p->spec, (float *)prod,
                           (const float *)p->K, (const float *)p->d1, (const float *)p->d2, p->nxh, p->ny,
                           (float)(-p->mu / (double)n), sigma_bar);
    }
    ST_HIP(hipGetLastError());
    void *in2[1] = {prod}, *out2[1] = {tau13};
    ST_FFT(rocfft_execute(p->inv, in2, out2, p->info));
    return StaticStatus::Ok;
}
}  // namespace

static_assert(kLawBlocks <= kMaxPartials, "the stage kernels reduce at most kMaxPartials partials");
int velocity_law_blocks(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, kLawBlocks); }

StaticStatus velocity_law(const void *tau13, const void *phi, bool f64, float *v0, int64_t n, const LawParams &L,
                          float *partial, hipStream_t s, std::string &err)
{
    const unsigned b = (unsigned)velocity_law_blocks(n);
    if (f64) {
        if (L.wiggly)
            hipLaunchKernelGGL((velocity_law_kernel<double, true>), dim3(b), dim3(256), 0, s, (const double *)tau13,
                               (const double *)phi, L.mfield, v0, n, L.tau0, L.mobility, L.tau_y, L.beta, partial);
        else
            hipLaunchKernelGGL((velocity_law_kernel<double, false>), dim3(b), dim3(256), 0, s, (const double *)tau13,
                               (const double *)phi, L.mfield, v0, n, L.tau0, L.mobility, L.tau_y, L.beta, partial);
    } else {
        if (L.wiggly)
            hipLaunchKernelGGL((velocity_law_kernel<float, true>), dim3(b), dim3(256), 0, s, (const float *)tau13,
                               (const float *)phi, L.mfield, v0, n, (float)L.tau0, (float)L.mobility,
                               (float)L.tau_y, (float)L.beta, partial);
        else
            hipLaunchKernelGGL((velocity_law_kernel<float, false>), dim3(b), dim3(256), 0, s, (const float *)tau13,
                               (const float *)phi, L.mfield, v0, n, (float)L.tau0, (float)L.mobility,
                               (float)L.tau_y, (float)L.beta, partial);
    }
    ST_HIP(hipGetLastError());
    return StaticStatus::Ok;
}

}  // namespace fdm
