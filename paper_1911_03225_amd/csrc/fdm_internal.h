// fdm_internal.h -- shared between the gfx950 kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdm {

// Wave tiling of the stencil kernels.  One wave64 owns a strip of kStrip
// consecutive columns plus kHalo columns on each side (the x stencil reaches
// two edges each way) and walks a chunk of `rows` rows downwards, keeping the
// y stencil in registers.
constexpr int kWave = 64;
constexpr int kHalo = 2;
constexpr int kStrip = kWave - 2 * kHalo;   // 60 output columns per wave
constexpr int kFusedStrip = kWave - 8;      // 56: the fused Heun kernel's (4 halo lanes a side)
constexpr int kWavesPerBlock = 4;

// Row tiles of a grid of ny rows (ny may be as large as 2^31 - 1, so the
// rounding-up sum is taken in 64 bits).
__host__ __device__ inline int tiles_along_y(int ny, int rows)
{
    return (int)(((int64_t)ny + rows - 1) / rows);
}
constexpr int kBlock = kWave * kWavesPerBlock;

// Limiter and Hamiltonian codes (values of the public enums).
enum : int { LIM_NONE = 0, LIM_MINMOD = 1, LIM_MC = 2, LIM_THETA = 3, LIM_SUPERBEE = 4 };
// Hamiltonian kind (bit 0: LAW or PRESCRIBED) and scheme (bit 1: the fully
// discrete scheme of sec. 3.2.3 instead of its dt -> 0 limit).
enum : int { VK_LAW = 0, VK_PRESCRIBED = 1, VK_FD = 2, VK_LAW_FD = 2, VK_PRESCRIBED_FD = 3 };

// What one stage launch reads and writes.
//   MODE_FWD   : w = a + dt L(a)                 (first stage / Euler step)
//   MODE_BWD   : a = w + dt L(w)                 (Euler step, other direction)
//   MODE_HEUN2 : a = a/2 + (w + dt L(w))/2       (second Heun stage, in place)
//   MODE_MID2  : a = a + dt L(w)                 (second midpoint stage, in place)
//   MODE_MID1  : w = a + (dt/2) L(a)             (first midpoint stage: the
//                MODE_FWD kernel with the step coefficients halved, exactly)
enum : int { MODE_FWD = 0, MODE_BWD = 1, MODE_HEUN2 = 2, MODE_MID2 = 3, MODE_MID1 = 4 };

// Precision modes (values of fdm_precision): arithmetic type / state type.
//   PREC_FP32       float  / float
//   PREC_FP64_ARITH double / float
//   PREC_FP64       double / double
enum : int { PREC_FP32 = 0, PREC_FP64_ARITH = 1, PREC_FP64 = 2 };

// Step coefficients computed on the device (coupled runs): the stage kernels
// read them through InstDev::coef instead of the values in InstDev.
struct StepCoef {
    double dtd, cxd, cyd;    // dt, dt/dx, dt/dy
    float cx, cy;            // the same in float
    float dt, vmax;          // the float32 step and max |v0| it came from
    int32_t nonfinite, pad;  // a non-finite celerity was seen
};

// The step of a coupled run from the block partials of max |v0| (a NaN
// partial marks a non-finite celerity): the largest float not above
// min(cfl_h / max|v0|, dt_max) (dt_max when nothing moves) and the stage
// coefficients.  Evaluated by one whole wave, in two parts so that callers
// can put other loads in flight beside the partials': x holds the lane's
// partials lane + 64 j (0 where j indexes past the np <= kMaxPartials
// partials).
constexpr int kMaxPartials = 1024;

__device__ __forceinline__ StepCoef step_coef_from_loaded(const float (&x)[kMaxPartials / 64], double cfl_h,
                                                          double dt_max, double dx, double dy)
{
    float m = 0.0f;
    int bad = 0;
#pragma unroll
    for (int j = 0; j < kMaxPartials / 64; ++j) {
        bad |= __builtin_isnan(x[j]) ? 1 : 0;
        m = fmaxf(m, x[j]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        m = fmaxf(m, __shfl_xor(m, o, 64));
        bad |= __shfl_xor(bad, o, 64);
    }
    const double bound = m > 0.0f ? fmin(cfl_h / (double)m, dt_max) : dt_max;
    float f = (float)bound;
    if ((double)f > bound) f = nextafterf(f, 0.0f);
    StepCoef c;
    c.dtd = (double)f;
    c.cxd = (double)f / dx;
    c.cyd = (double)f / dy;
    c.cx = (float)c.cxd;
    c.cy = (float)c.cyd;
    c.dt = f;
    c.vmax = m;
    c.nonfinite = bad;
    c.pad = 0;
    return c;
}

// Scalars of a coupled run, advanced on the device step by step.
struct CoupledDev {
    StepCoef coef;
    double eps13, phi_mean, t, sigma_bar;
};

// The mean-slip update that ends a coupled step: from the per-tile sums of
// Hhat of the step's stages, the mean slip, mean strain, time and mean
// stress.
struct SlipArgs {
    CoupledDev *cd;
    const double *hsum;   // first stage's tile sums, then the second's
    int64_t tiles;
    int32_t time_order;
    int32_t increments;   // the sums hold node increments phi^{n+1} - phi^n (fully discrete, FP64)
    double rate, mu, frac, n_nodes;   // strain rate, shear modulus, h / L3, nodes
};

// Fixed-order compensated sums of u[0..n) and v[0..n) (v may be null: 0)
// by one block of 256 threads: thread t adds elements t, t + 256, ... in
// index order, then a pairwise tree over the threads.
__device__ __forceinline__ void block_sums256(const double *u, const double *v, int64_t n, double2 *lds,
                                              double &su, double &sv)
{
    double s[2] = {0.0, 0.0}, c[2] = {0.0, 0.0};
    auto add = [&](int k, double x) {
        const double t = s[k] + x;
        c[k] += fabs(s[k]) >= fabs(x) ? (s[k] - t) + x : (x - t) + s[k];
        s[k] = t;
    };
    for (int64_t base = threadIdx.x; base < n; base += 256 * 4) {
        double x[4], y[4];   // the loads first, then the sums in index order
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool in = base + 256 * q < n;
            x[q] = in ? u[base + 256 * q] : 0.0;
            y[q] = in && v ? v[base + 256 * q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (base + 256 * q >= n) break;
            add(0, x[q]);
            add(1, y[q]);
        }
    }
    lds[threadIdx.x] = make_double2(s[0] + c[0], s[1] + c[1]);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            lds[threadIdx.x].x += lds[threadIdx.x + w].x;
            lds[threadIdx.x].y += lds[threadIdx.x + w].y;
        }
        __syncthreads();
    }
    su = lds[0].x;
    sv = lds[0].y;
    __syncthreads();
}

// The slip update by one whole block of 256 threads (no contraction into
// fused multiply-adds, whichever kernel runs it).
__device__ __forceinline__ void coupled_slip_block(const SlipArgs &a, double2 *lds)
{
#pragma clang fp contract(off)
    double s1, s2;
    block_sums256(a.hsum, a.time_order == 1 ? nullptr : a.hsum + a.tiles, a.tiles, lds, s1, s2);
    if (threadIdx.x == 0) {
        // Euler: Hhat of the state; Heun: mean of the two stages; midpoint: the half-step state
        CoupledDev *cd = a.cd;
        const double dt = (double)cd->coef.dt;
        double hmean = s1 / a.n_nodes;
        if (a.increments) hmean = -hmean / dt;   // the mean rate of phi over the step
        if (a.time_order == 2) hmean = 0.5 * (hmean + s2 / a.n_nodes);
        if (a.time_order == 3) hmean = s2 / a.n_nodes;
        const double phi = cd->phi_mean - dt * hmean;
        const double eps = cd->eps13 + a.rate * dt;
        cd->phi_mean = phi;
        cd->eps13 = eps;
        cd->t = cd->t + dt;
        cd->sigma_bar = 2.0 * a.mu * eps - a.mu * a.frac * phi;
    }
}

// Device view of one transport instance.
struct InstDev {
    void *a11, *a12;         // state, caller-owned (float, or double in PREC_FP64)
    void *w11, *w12;         // stage buffer, library-owned, same type
    const float *v0f;        // node celerity field or nullptr
    int32_t nx, ny;
    float v0, V1, V2;        // uniform celerity / prescribed velocity
    float cx, cy;            // dt/dx, dt/dy
    float theta;             // minmod-family parameter
    int32_t limiter, vkind;
    int32_t rows;            // rows per wave tile
    int32_t strips, chunks;  // tiles along x and y
    int32_t fstrips;         // tiles along x of the fused Heun kernel (56 columns)
    int64_t tile_begin;      // first global tile of this instance (batched)
    double cxd, cyd, thetad; // the same coefficients for FP64 arithmetic
    double dtd, dxd, dyd;    // step and spacings (FP64 update in definition form)
    double *hsum;            // per-tile sums of Hhat (coupled runs) or nullptr
    // Coupled runs: the step comes from the velocity law's max |v0|
    // partials, reduced by every wave of the stage kernels (so no launch
    // stands between the law and the first stage); the wave of tile 0 of
    // the first stage stores it in coef_out for the slip update and the host.
    const float *vpart;      // the partials, or nullptr (the step in this struct)
    StepCoef *coef_out;      // or nullptr
    int32_t nvpart, pad2;
    double cfl_h, dt_max;    // cfl min(dx, dy), the largest step
};

// Per-block partial of the diagnostics reduction (compensated sums).
struct StatsPartial {
    double s11, c11, s12, c12, sab, cab, maxn, nonfinite;
};

constexpr int kStatsBlocks = 512;   // fixed => deterministic reduction order

hipError_t launch_stage(const InstDev &I, int mode, int precision, hipStream_t s);
// fd: the instances use the fully discrete scheme (all or none of a batch)
hipError_t launch_stage_batched(const InstDev *d_inst, const int32_t *d_tile_inst,
                                int64_t total_tiles, int mode, bool fd, int precision, hipStream_t s);
hipError_t launch_absmax(const float *v, int64_t n, float *d_partial, hipStream_t s);
// Fused two-stage step of one instance (float state and arithmetic,
// semi-discrete scheme; Heun, or the explicit midpoint when mid): dir 0 from
// the state into the stage buffer, dir 1 back; tiles of I.rows rows and 56
// columns.
hipError_t launch_fused(const InstDev &I, int dir, bool mid, hipStream_t s);
// The same for every instance of a batched context in one launch (the tile
// map and tile_begin of the fused tiling).
hipError_t launch_fused_batched(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles, int dir,
                                bool mid, hipStream_t s);
hipError_t launch_stats(const void *a11, const void *a12, int64_t n, int precision,
                        StatsPartial *d_partials, double *d_out, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, int64_t n, int precision, hipStream_t s);

constexpr int kAbsmaxBlocks = 256;

// Coupled runs: the slip update of the last step before the host reads the
// scalars back (one block; within a chunk the next step's pack kernel runs
// it).
hipError_t launch_coupled_slip(const SlipArgs &a, hipStream_t s);

}  // namespace fdm
