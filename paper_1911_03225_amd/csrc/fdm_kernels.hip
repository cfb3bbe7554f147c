// fdm_kernels.hip -- reductions and helpers of the transport hot path, and
// the precision dispatch of the stage kernels (fdm_stage_f32.hip,
// fdm_stage_f64.hip).
#include "fdm_internal.h"

namespace fdm {

hipError_t launch_stage_f32(const InstDev &I, int mode, hipStream_t s);
hipError_t launch_stage_batched_f32(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles,
                                    int mode, bool fd, hipStream_t s);
hipError_t launch_stage_f64(const InstDev &I, int mode, bool f64_state, hipStream_t s);
hipError_t launch_stage_batched_f64(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles,
                                    int mode, bool fd, bool f64_state, hipStream_t s);

hipError_t launch_stage(const InstDev &I, int mode, int precision, hipStream_t s)
{
    if (precision == PREC_FP32) return launch_stage_f32(I, mode, s);
    return launch_stage_f64(I, mode, precision == PREC_FP64, s);
}

hipError_t launch_stage_batched(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles,
                                int mode, bool fd, int precision, hipStream_t s)
{
    if (precision == PREC_FP32) return launch_stage_batched_f32(d_inst, d_tile_inst, total_tiles, mode, fd, s);
    return launch_stage_batched_f64(d_inst, d_tile_inst, total_tiles, mode, fd, precision == PREC_FP64, s);
}

namespace {

// ---------------------------------------------------------------- reductions

// Error-free sum of two doubles folded into a compensated pair.
__device__ __forceinline__ void pair_add(double &s, double &c, double s2, double c2)
{
    const double t = s + s2;
    const double bp = t - s;
    const double e = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = c + c2 + e;
}

__device__ __forceinline__ double shfl_xor_d(double v, int m)
{
    return __shfl_xor(v, m, 64);
}

// Fixed-order butterfly over the wave, then over the block's waves.
__device__ void block_reduce(StatsPartial &p, StatsPartial *lds)
{
    for (int m = 1; m < 64; m <<= 1) {
        double s11 = shfl_xor_d(p.s11, m), c11 = shfl_xor_d(p.c11, m);
        double s12 = shfl_xor_d(p.s12, m), c12 = shfl_xor_d(p.c12, m);
        double sab = shfl_xor_d(p.sab, m), cab = shfl_xor_d(p.cab, m);
        double mx = shfl_xor_d(p.maxn, m), nf = shfl_xor_d(p.nonfinite, m);
        // combine in lane order so both partners compute the same value
        const bool lower = (threadIdx.x & m) == 0;
        StatsPartial a = p, b;
        b.s11 = s11; b.c11 = c11; b.s12 = s12; b.c12 = c12; b.sab = sab; b.cab = cab;
        b.maxn = mx; b.nonfinite = nf;
        StatsPartial &x = lower ? a : b;
        StatsPartial &y = lower ? b : a;
        pair_add(x.s11, x.c11, y.s11, y.c11);
        pair_add(x.s12, x.c12, y.s12, y.c12);
        pair_add(x.sab, x.cab, y.sab, y.cab);
        x.maxn = fmax(x.maxn, y.maxn);
        x.nonfinite = x.nonfinite + y.nonfinite;
        p = x;
    }
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[wave] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        StatsPartial r = lds[0];
        for (int w = 1; w < nw; ++w) {
            pair_add(r.s11, r.c11, lds[w].s11, lds[w].c11);
            pair_add(r.s12, r.c12, lds[w].s12, lds[w].c12);
            pair_add(r.sab, r.cab, lds[w].sab, lds[w].cab);
            r.maxn = fmax(r.maxn, lds[w].maxn);
            r.nonfinite += lds[w].nonfinite;
        }
        p = r;
    }
}

__device__ __forceinline__ void neumaier(double &s, double &c, double x)
{
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

template <typename S>
__global__ __launch_bounds__(256) void stats_partial_kernel(const S *__restrict__ a11,
                                                            const S *__restrict__ a12, int64_t n,
                                                            StatsPartial *__restrict__ out)
{
    __shared__ StatsPartial lds[4];
    StatsPartial p = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const S x = a11[i], y = a12[i];
        if (!isfinite(x) || !isfinite(y)) {
            p.nonfinite += 1.0;
            continue;
        }
        const double dx = x, dy = y;
        neumaier(p.s11, p.c11, dx);
        neumaier(p.s12, p.c12, dy);
        neumaier(p.sab, p.cab, fabs(dx) + fabs(dy));
        p.maxn = fmax(p.maxn, sqrt(dx * dx + dy * dy));
    }
    block_reduce(p, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = p;
}

// One block folds the kStatsBlocks partials in fixed order:
// out = {sum11, sum12, sum_abs, max_norm, nonfinite}.
__global__ __launch_bounds__(kStatsBlocks) void stats_final_kernel(const StatsPartial *__restrict__ parts,
                                                                   double *__restrict__ out)
{
    __shared__ StatsPartial lds[kStatsBlocks / 64];
    StatsPartial p = parts[threadIdx.x];
    block_reduce(p, lds);
    if (threadIdx.x == 0) {
        out[0] = p.s11 + p.c11;
        out[1] = p.s12 + p.c12;
        out[2] = p.sab + p.cab;
        out[3] = p.maxn;
        out[4] = p.nonfinite;
    }
}

// Largest |v| per block (NaN if the block saw a non-finite value).  Blocks
// of 1024 threads (16 waves per CU) read four float4 each per trip, so
// enough loads are in flight to stream the field at HBM rate; a misaligned
// pointer or the last n % 4 values take the scalar loop.
constexpr int kAbsmaxThreads = 1024;

__global__ __launch_bounds__(kAbsmaxThreads) void absmax_kernel(const float *__restrict__ v, int64_t n,
                                                                float *__restrict__ partial)
{
    __shared__ float lds[kAbsmaxThreads / 64];
    float m = 0.0f;
    bool bad = false;
    auto take = [&](float x) {
        bad |= !isfinite(x);
        m = fmaxf(m, fabsf(x));
    };
    const int64_t nt = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n4 = (reinterpret_cast<uintptr_t>(v) & 15) == 0 ? n / 4 : 0;
    const float4 *__restrict__ v4 = reinterpret_cast<const float4 *>(v);
    int64_t i = tid;
    for (; i + 3 * nt < n4; i += 4 * nt) {
        float4 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) q[u] = v4[i + u * nt];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            take(q[u].x);
            take(q[u].y);
            take(q[u].z);
            take(q[u].w);
        }
    }
    for (; i < n4; i += nt) {
        const float4 q = v4[i];
        take(q.x);
        take(q.y);
        take(q.z);
        take(q.w);
    }
    for (int64_t j = 4 * n4 + tid; j < n; j += nt) take(v[j]);
    if (bad) m = __builtin_nanf("");
    for (int o = 32; o > 0; o >>= 1) {
        const float other = __shfl_xor(m, o, 64);
        m = (isnan(m) || isnan(other)) ? __builtin_nanf("") : fmaxf(m, other);
    }
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = lds[0];
        for (int w = 1; w < kAbsmaxThreads / 64; ++w)
            r = (isnan(r) || isnan(lds[w])) ? __builtin_nanf("") : fmaxf(r, lds[w]);
        partial[blockIdx.x] = r;
    }
}

template <typename S>
__global__ __launch_bounds__(256) void copy_kernel(S *__restrict__ dst, const S *__restrict__ src, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// One block: the slip update of a coupled step.
__global__ __launch_bounds__(256) void coupled_slip_kernel(SlipArgs a)
{
    __shared__ double2 lds[256];
    coupled_slip_block(a, lds);
}

}  // namespace

hipError_t launch_coupled_slip(const SlipArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(coupled_slip_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_absmax(const float *v, int64_t n, float *d_partial, hipStream_t s)
{
    hipLaunchKernelGGL(absmax_kernel, dim3(kAbsmaxBlocks), dim3(kAbsmaxThreads), 0, s, v, n, d_partial);
    return hipGetLastError();
}

hipError_t launch_stats(const void *a11, const void *a12, int64_t n, int precision, StatsPartial *d_partials,
                        double *d_out, hipStream_t s)
{
    if (precision == PREC_FP64)
        hipLaunchKernelGGL(stats_partial_kernel<double>, dim3(kStatsBlocks), dim3(256), 0, s,
                           static_cast<const double *>(a11), static_cast<const double *>(a12), n, d_partials);
    else
        hipLaunchKernelGGL(stats_partial_kernel<float>, dim3(kStatsBlocks), dim3(256), 0, s,
                           static_cast<const float *>(a11), static_cast<const float *>(a12), n, d_partials);
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(kStatsBlocks), 0, s, d_partials, d_out);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, int64_t n, int precision, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (precision == PREC_FP64)
        hipLaunchKernelGGL(copy_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<double *>(dst), static_cast<const double *>(src), n);
    else
        hipLaunchKernelGGL(copy_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<float *>(dst), static_cast<const float *>(src), n);
    return hipGetLastError();
}

}  // namespace fdm
