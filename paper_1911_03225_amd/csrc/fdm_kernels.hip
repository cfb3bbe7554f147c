// fdm_kernels.hip -- gfx950 kernels of the layer-case transport hot path.
//
// Scheme (Morin, Brenner & Suquet, arXiv:1911.03225, sec. 3.2.2-3.2.3): the
// central-upwind Godunov-type update of U^p_13, carried out on its edge
// differences, the in-plane Nye components alpha_12 (x-edges) and alpha_11
// (y-edges).  Per node and stage:
//   Step 1   limited slope of each component along its own axis (limited
//            second difference of U^p_13, minmod family eq. 43-44, or
//            superbee);
//   Step 2   one-sided derivatives px-+, py-+ (eq. 46 per axis) and one-sided
//            speeds a-+, b-+ over the four (+-,+-) combinations (eq. 53);
//   Step 3-4 the dt -> 0 limit of the intermediate-point solve and projection
//            (eq. 54-55), with the tensor-product (sign-corrected) weights:
//            Hhat = sum w_s v_t H(px^s, py^t) + a+a-/(a+-a-) (px+ - px-)
//                                             + b+b-/(b+-b-) (py+ - py-);
//   update   alpha_12 -= dt/dx (Hhat_{j+1,k} - Hhat_{jk}),
//            alpha_11 += dt/dy (Hhat_{j,k+1} - Hhat_{jk})  (eq. 57 form).
//
// Data movement (gfx950, wave64).  The stencil reaches two edges along each
// axis.  A wave owns a strip of 60 output columns plus 2 halo lanes on each
// side, one column per lane, and walks `rows` rows downwards:
//   * y neighbours stay in registers (a sliding window of alpha_11 rows and
//     the previous row's Hhat), so every row is read once per strip;
//   * x neighbours come from adjacent lanes through DPP wave shifts;
//   * no LDS, no barriers; every global access is a row of 64 consecutive
//     floats.
// Hhat is pure VALU work (4 rsq, 2 rcp per node); there is no contraction
// for MFMA here.
#include "fdm_internal.h"

namespace fdm {
namespace {

// ---------------------------------------------------------------- lane moves

// lane l receives lane l-1's value (lane 0 receives 0)
__device__ __forceinline__ float from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}

// lane l receives lane l+1's value (lane 63 receives 0)
__device__ __forceinline__ float from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ double from_left(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double from_right(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// ------------------------------------------------------- arithmetic types
//
// float: the default FP32 arithmetic.  double: FP64 register arithmetic on
// the same float32 state (loads widened, results rounded once when stored);
// FP64 VALU issues at the non-packed FP32 rate on gfx950.

__device__ __forceinline__ float vmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ float vmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ float vabs(float a) { return fabsf(a); }
__device__ __forceinline__ float vsign(float m, float s) { return copysignf(m, s); }
__device__ __forceinline__ double vmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ double vmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ double vabs(double a) { return fabs(a); }
__device__ __forceinline__ double vsign(double m, double s) { return copysign(m, s); }

template <typename R> struct Arith;

template <> struct Arith<float> {
    static constexpr float tiny = 1.17549435e-38f;   // FLT_MIN
    static __device__ __forceinline__ float rsq(float r) { return __builtin_amdgcn_rsqf(r); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
};

template <> struct Arith<double> {
    static constexpr double tiny = 2.2250738585072014e-308;   // DBL_MIN
    // hardware estimates refined by one Newton step
    static __device__ __forceinline__ double rsq(double r)
    {
        const double y = __builtin_amdgcn_rsq(r);
        return y * (1.5 - 0.5 * r * y * y);
    }
    static __device__ __forceinline__ double rcp(double x)
    {
        const double y = __builtin_amdgcn_rcp(x);
        return y * (2.0 - x * y);
    }
};

// ---------------------------------------------------------------- Step 1

// Limiter kinds compiled separately: the minmod family shares one body with
// a runtime theta (1 for minmod, 2 for MC), so every launch form runs the
// same instructions for a given limiter.
enum : int { LK_NONE = 0, LK_THETA = 1, LK_SUPERBEE = 2 };

__host__ __device__ constexpr int limiter_kind(int lim)
{
    return lim == LIM_NONE ? LK_NONE : (lim == LIM_SUPERBEE ? LK_SUPERBEE : LK_THETA);
}

// Limited slope at an edge from three consecutive values along its axis.
// theta-minmod: minmod(theta*D+, (w+ - w-)/2, theta*D-), written as
// max(min3, 0) + min(max3, 0): the minimum if all three are positive, the
// maximum if all are negative, else zero.  Odd in w, exactly.
template <int LK, typename R>
__device__ __forceinline__ R limited_slope(R wm, R w0, R wp, R theta)
{
    if constexpr (LK == LK_NONE) {
        return R(0);
    } else if constexpr (LK == LK_SUPERBEE) {
        const R dm = w0 - wm, dp = wp - w0;
        const R adm = vabs(dm), adp = vabs(dp);
        const R mag = vmax(vmin(R(2) * adm, adp), vmin(adm, R(2) * adp));
        return (dm * dp > R(0)) ? vsign(mag, dp) : R(0);
    } else {
        const R dm = w0 - wm, dp = wp - w0;
        const R a = theta * dp, b = R(0.5) * (wp - wm), c = theta * dm;
        const R lo = vmin(vmin(a, b), c), hi = vmax(vmax(a, b), c);
        return vmax(lo, R(0)) + vmin(hi, R(0));
    }
}

// ---------------------------------------------------------- Steps 2 to 4

template <int VK, typename R>
__device__ __forceinline__ R numerical_hamiltonian(R pxm, R pxp, R pym, R pyp, R v0, R V1, R V2)
{
    if constexpr (VK == VK_PRESCRIBED) {
        // H = V.p: the central-upwind weights reduce to pure upwinding.
        const R px = V1 > R(0) ? pxm : pxp;
        const R py = V2 > R(0) ? pym : pyp;
        return V1 * px + V2 * py;
    } else {
        // H = v0 |p| at the four corners (s,t) in {-,+}^2, dH/dp = v0 p/|p|.
        // |p|^2 is clamped below at the smallest normal number before the
        // reciprocal square root (v_rsq reads a subnormal as zero): p = 0
        // still gives H = 0 and speed 0, and gradients below 1e-19 (float)
        // move with speed v0 p / 1e-19 instead of a full-speed direction.
        constexpr R kTiny = Arith<R>::tiny;
        const R xm2 = pxm * pxm, xp2 = pxp * pxp, ym2 = pym * pym, yp2 = pyp * pyp;
        const R r00 = xm2 + ym2, r01 = xm2 + yp2, r10 = xp2 + ym2, r11 = xp2 + yp2;
        const R g00 = v0 * Arith<R>::rsq(vmax(r00, kTiny));
        const R g01 = v0 * Arith<R>::rsq(vmax(r01, kTiny));
        const R g10 = v0 * Arith<R>::rsq(vmax(r10, kTiny));
        const R g11 = v0 * Arith<R>::rsq(vmax(r11, kTiny));
        const R H00 = r00 * g00, H01 = r01 * g01, H10 = r10 * g10, H11 = r11 * g11;
        const R hx00 = pxm * g00, hx01 = pxm * g01, hx10 = pxp * g10, hx11 = pxp * g11;
        const R hy00 = pym * g00, hy01 = pyp * g01, hy10 = pym * g10, hy11 = pyp * g11;
        // Step 2: one-sided local speeds over the four combinations
        const R ap = vmax(vmax(vmax(hx00, hx01), vmax(hx10, hx11)), R(0));
        const R am = vmin(vmin(vmin(hx00, hx01), vmin(hx10, hx11)), R(0));
        const R bp = vmax(vmax(vmax(hy00, hy01), vmax(hy10, hy11)), R(0));
        const R bm = vmin(vmin(vmin(hy00, hy01), vmin(hy10, hy11)), R(0));
        // Steps 3-4 (dt -> 0): projection weights; 1/2 each and no viscosity
        // when nothing moves along that axis.  The sum keeps the order of
        // the definition (weighted corner values, then the two viscosity
        // terms): rewriting it, e.g. with w_+ = 1 - w_-, lets FMA
        // contraction turn exact cancellations between equal corner values
        // into product rounding errors, which the kink of |p| at p = 0
        // then amplifies.
        const R da = ap - am, db = bp - bm;
        const bool mx = da >= kTiny, my = db >= kTiny;
        const R ia = mx ? Arith<R>::rcp(da) : R(0);
        const R ib = my ? Arith<R>::rcp(db) : R(0);
        const R wxm = mx ? ap * ia : R(0.5), wxp = mx ? -am * ia : R(0.5);
        const R wym = my ? bp * ib : R(0.5), wyp = my ? -bm * ib : R(0.5);
        const R visc_x = ap * am * ia, visc_y = bp * bm * ib;
        return wxm * (wym * H00 + wyp * H01) + wxp * (wym * H10 + wyp * H11)
             + visc_x * (pxp - pxm) + visc_y * (pyp - pym);
    }
}

__device__ __forceinline__ int next_row(int k, int ny)
{
    k += 1;
    return k == ny ? 0 : k;
}

// Row `row` of a field, at this lane's byte offset: the row address is
// wave-uniform (scalar registers), the offset a 32-bit lane value.
__device__ __forceinline__ const float *row_ptr(const float *base, int row, int nx)
{
    return base + (size_t)row * (size_t)nx;
}

__device__ __forceinline__ float at(const float *row, uint32_t off)
{
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(row) + off);
}

__device__ __forceinline__ void put(float *row, uint32_t off, float v)
{
    *reinterpret_cast<float *>(reinterpret_cast<char *>(row) + off) = v;
}

// One wave: columns strip*60 .. strip*60+59 (lanes 2..61), rows
// chunk*rows .. +rows-1, of one stage, in arithmetic type R.  Loads run one
// row ahead of the arithmetic so their latency overlaps the previous row.
template <typename R, int LK, int VK, bool FIELD, int MODE>
__device__ __forceinline__ void run_tile(const InstDev &I, int strip, int chunk, int lane)
{
    constexpr bool kF64 = sizeof(R) == 8;
    constexpr bool kBase = MODE == MODE_HEUN2;
    const int nx = I.nx, ny = I.ny;
    const float *s12 = MODE == MODE_FWD ? I.a12 : I.w12;
    const float *s11 = MODE == MODE_FWD ? I.a11 : I.w11;
    float *d12 = MODE == MODE_FWD ? I.w12 : I.a12;
    float *d11 = MODE == MODE_FWD ? I.w11 : I.a11;
    const R theta = kF64 ? R(I.thetad) : R(I.theta);
    const R cx = kF64 ? R(I.cxd) : R(I.cx);
    const R cy = kF64 ? R(I.cyd) : R(I.cy);
    const R V1 = R(I.V1), V2 = R(I.V2);

    const int gcol = strip * kStrip - kHalo + lane;
    int col = gcol % nx;
    if (col < 0) col += nx;
    const uint32_t off = (uint32_t)col * 4u;
    const bool out_col = lane >= kHalo && lane < kHalo + kStrip && gcol < nx;
    const int k0 = chunk * I.rows;
    const int nrows = min(I.rows, ny - k0);

    // alpha_11 = -w_y on y-edges; the window holds rows k-2, k-1, k.
    int k = (k0 - 2) % ny;
    if (k < 0) k += ny;
    const R ym2 = R(at(row_ptr(s11, k, nx), off));
    k = next_row(k, ny);
    R ym1 = R(at(row_ptr(s11, k, nx), off));
    const int kprev0 = k;
    k = next_row(k, ny);
    R y0 = R(at(row_ptr(s11, k, nx), off));
    R sm1 = limited_slope<LK>(ym2, ym1, y0, theta);   // slope at edge k-1/2
    R hprev = R(0);
    int kprev = kprev0;

    // first row's operands
    int kn = next_row(k, ny);
    float f_wx = at(row_ptr(s12, k, nx), off);
    float f_yp1 = at(row_ptr(s11, kn, nx), off);
    float f_v0 = FIELD ? at(row_ptr(I.v0f, k, nx), off) : 0.0f;
    float f_b12 = kBase ? at(row_ptr(d12, k, nx), off) : 0.0f;
    float f_b11 = kBase ? at(row_ptr(d11, kprev, nx), off) : 0.0f;

    for (int it = 0; it <= nrows; ++it) {
        const R wx = R(f_wx), yp1 = R(f_yp1);
        const R v0 = FIELD ? R(f_v0) : R(I.v0);
        const R b12 = R(f_b12), b11 = R(f_b11);
        const int knn = next_row(kn, ny);
        if (it < nrows) {   // operands of the next row (wave-uniform branch)
            f_wx = at(row_ptr(s12, kn, nx), off);
            f_yp1 = at(row_ptr(s11, knn, nx), off);
            if constexpr (FIELD) f_v0 = at(row_ptr(I.v0f, kn, nx), off);
            if constexpr (kBase) {
                f_b12 = at(row_ptr(d12, kn, nx), off);
                f_b11 = at(row_ptr(d11, k, nx), off);
            }
        }

        // Steps 1-2 along y (alpha_11 = -w_y, slopes are odd)
        const R s0 = limited_slope<LK>(ym1, y0, yp1, theta);
        const R pyp = -(y0 - R(0.5) * s0);
        const R pym = -(ym1 + R(0.5) * sm1);
        // Steps 1-2 along x (alpha_12 = w_x), neighbours from adjacent lanes
        const R wl = from_left(wx), wr = from_right(wx);
        const R sx = limited_slope<LK>(wl, wx, wr, theta);
        const R pxp = wx - R(0.5) * sx;
        const R pxm = from_left(wx + R(0.5) * sx);
        // Steps 2-4
        const R h = numerical_hamiltonian<VK>(pxm, pxp, pym, pyp, v0, V1, V2);
        const R hr = from_right(h);

        if (out_col) {
            if (it < nrows) {            // x-edge (j+1/2, k)
                R nv = wx - cx * (hr - h);
                if constexpr (kBase) nv = R(0.5) * b12 + R(0.5) * nv;
                put(const_cast<float *>(row_ptr(d12, k, nx)), off, float(nv));
            }
            if (it > 0) {                // y-edge (j, k-1/2)
                R nv = ym1 + cy * (h - hprev);
                if constexpr (kBase) nv = R(0.5) * b11 + R(0.5) * nv;
                put(const_cast<float *>(row_ptr(d11, kprev, nx)), off, float(nv));
            }
        }
        hprev = h;
        kprev = k;
        k = kn;
        kn = knn;
        ym1 = y0;
        y0 = yp1;
        sm1 = s0;
    }
}

// Hardware places block b on XCD b % 8.  Give each XCD a contiguous run of
// tiles (vertically adjacent chunks of the same strips) so halo rows are
// re-read from that XCD's L2.
__device__ __forceinline__ int64_t xcd_tile(int blocks_per_xcd)
{
    const int b = blockIdx.x;
    const int64_t logical = (int64_t)(b & 7) * blocks_per_xcd + (b >> 3);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    return logical * kWavesPerBlock + wave;
}

template <typename R, int LK, int VK, bool FIELD, int MODE>
__global__ __launch_bounds__(kBlock) void stage_kernel(InstDev I, int64_t total_tiles, int blocks_per_xcd)
{
    const int64_t tile = xcd_tile(blocks_per_xcd);
    if (tile >= total_tiles) return;
    const int t = (int)tile;
    run_tile<R, LK, VK, FIELD, MODE>(I, t / I.chunks, t % I.chunks, threadIdx.x & 63);
}

// Batched: one launch for every tile of every instance; tile_inst maps a
// global tile to its instance.  Limiter, Hamiltonian and field presence are
// per instance and uniform over a wave.
template <typename R, int MODE>
__global__ __launch_bounds__(kBlock) void stage_kernel_batched(const InstDev *__restrict__ insts,
                                                               const int32_t *__restrict__ tile_inst,
                                                               int64_t total_tiles, int blocks_per_xcd)
{
    const int64_t tile = xcd_tile(blocks_per_xcd);
    if (tile >= total_tiles) return;
    const InstDev I = insts[tile_inst[tile]];
    const int local = (int)(tile - I.tile_begin);
    const int strip = local / I.chunks, chunk = local % I.chunks;
    const int lane = threadIdx.x & 63;
    const int lk = limiter_kind(I.limiter);
    if (I.vkind == VK_PRESCRIBED) {
        if (lk == LK_NONE) run_tile<R, LK_NONE, VK_PRESCRIBED, false, MODE>(I, strip, chunk, lane);
        else if (lk == LK_SUPERBEE) run_tile<R, LK_SUPERBEE, VK_PRESCRIBED, false, MODE>(I, strip, chunk, lane);
        else run_tile<R, LK_THETA, VK_PRESCRIBED, false, MODE>(I, strip, chunk, lane);
    } else if (I.v0f != nullptr) {
        if (lk == LK_NONE) run_tile<R, LK_NONE, VK_LAW, true, MODE>(I, strip, chunk, lane);
        else if (lk == LK_SUPERBEE) run_tile<R, LK_SUPERBEE, VK_LAW, true, MODE>(I, strip, chunk, lane);
        else run_tile<R, LK_THETA, VK_LAW, true, MODE>(I, strip, chunk, lane);
    } else {
        if (lk == LK_NONE) run_tile<R, LK_NONE, VK_LAW, false, MODE>(I, strip, chunk, lane);
        else if (lk == LK_SUPERBEE) run_tile<R, LK_SUPERBEE, VK_LAW, false, MODE>(I, strip, chunk, lane);
        else run_tile<R, LK_THETA, VK_LAW, false, MODE>(I, strip, chunk, lane);
    }
}

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

__global__ __launch_bounds__(256) void stats_partial_kernel(const float *__restrict__ a11,
                                                            const float *__restrict__ a12, int64_t n,
                                                            StatsPartial *__restrict__ out)
{
    __shared__ StatsPartial lds[4];
    StatsPartial p = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float x = a11[i], y = a12[i];
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

// Largest |v| per block (NaN if the block saw a non-finite value).
__global__ __launch_bounds__(256) void absmax_kernel(const float *__restrict__ v, int64_t n,
                                                     float *__restrict__ partial)
{
    __shared__ float lds[4];
    float m = 0.0f;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float x = v[i];
        bad |= !isfinite(x);
        m = fmaxf(m, fabsf(x));
    }
    if (bad) m = __builtin_nanf("");
    for (int o = 32; o > 0; o >>= 1) {
        const float other = __shfl_xor(m, o, 64);
        m = (isnan(m) || isnan(other)) ? __builtin_nanf("") : fmaxf(m, other);
    }
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = lds[0];
        for (int w = 1; w < 4; ++w) r = (isnan(r) || isnan(lds[w])) ? __builtin_nanf("") : fmaxf(r, lds[w]);
        partial[blockIdx.x] = r;
    }
}

__global__ __launch_bounds__(256) void copy_kernel(float *__restrict__ dst, const float *__restrict__ src,
                                                   int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

template <typename R, int LK, int VK, bool FIELD>
hipError_t launch_stage_t(const InstDev &I, int mode, hipStream_t s)
{
    const int64_t tiles = (int64_t)I.strips * I.chunks;
    const int64_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_xcd = (int)((blocks + 7) / 8);
    const dim3 grid(8 * per_xcd), block(kBlock);
    if (mode == MODE_FWD)
        hipLaunchKernelGGL((stage_kernel<R, LK, VK, FIELD, MODE_FWD>), grid, block, 0, s, I, tiles, per_xcd);
    else if (mode == MODE_BWD)
        hipLaunchKernelGGL((stage_kernel<R, LK, VK, FIELD, MODE_BWD>), grid, block, 0, s, I, tiles, per_xcd);
    else
        hipLaunchKernelGGL((stage_kernel<R, LK, VK, FIELD, MODE_HEUN2>), grid, block, 0, s, I, tiles, per_xcd);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_stage_r(const InstDev &I, int mode, hipStream_t s)
{
    const int lk = limiter_kind(I.limiter);
    if (I.vkind == VK_PRESCRIBED) {
        if (lk == LK_NONE) return launch_stage_t<R, LK_NONE, VK_PRESCRIBED, false>(I, mode, s);
        if (lk == LK_SUPERBEE) return launch_stage_t<R, LK_SUPERBEE, VK_PRESCRIBED, false>(I, mode, s);
        return launch_stage_t<R, LK_THETA, VK_PRESCRIBED, false>(I, mode, s);
    }
    if (I.v0f != nullptr) {
        if (lk == LK_NONE) return launch_stage_t<R, LK_NONE, VK_LAW, true>(I, mode, s);
        if (lk == LK_SUPERBEE) return launch_stage_t<R, LK_SUPERBEE, VK_LAW, true>(I, mode, s);
        return launch_stage_t<R, LK_THETA, VK_LAW, true>(I, mode, s);
    }
    if (lk == LK_NONE) return launch_stage_t<R, LK_NONE, VK_LAW, false>(I, mode, s);
    if (lk == LK_SUPERBEE) return launch_stage_t<R, LK_SUPERBEE, VK_LAW, false>(I, mode, s);
    return launch_stage_t<R, LK_THETA, VK_LAW, false>(I, mode, s);
}

template <typename R>
hipError_t launch_batched_r(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles, int mode,
                            hipStream_t s)
{
    const int64_t blocks = (total_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_xcd = (int)((blocks + 7) / 8);
    const dim3 grid(8 * per_xcd), block(kBlock);
    if (mode == MODE_FWD)
        hipLaunchKernelGGL((stage_kernel_batched<R, MODE_FWD>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles, per_xcd);
    else if (mode == MODE_BWD)
        hipLaunchKernelGGL((stage_kernel_batched<R, MODE_BWD>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles, per_xcd);
    else
        hipLaunchKernelGGL((stage_kernel_batched<R, MODE_HEUN2>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles, per_xcd);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stage(const InstDev &I, int mode, int precision, hipStream_t s)
{
    return precision == PREC_FP64 ? launch_stage_r<double>(I, mode, s) : launch_stage_r<float>(I, mode, s);
}

hipError_t launch_stage_batched(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles,
                                int mode, int precision, hipStream_t s)
{
    return precision == PREC_FP64 ? launch_batched_r<double>(d_inst, d_tile_inst, total_tiles, mode, s)
                                  : launch_batched_r<float>(d_inst, d_tile_inst, total_tiles, mode, s);
}

hipError_t launch_absmax(const float *v, int64_t n, float *d_partial, hipStream_t s)
{
    hipLaunchKernelGGL(absmax_kernel, dim3(kAbsmaxBlocks), dim3(256), 0, s, v, n, d_partial);
    return hipGetLastError();
}

hipError_t launch_stats(const float *a11, const float *a12, int64_t n, StatsPartial *d_partials,
                        double *d_out, hipStream_t s)
{
    hipLaunchKernelGGL(stats_partial_kernel, dim3(kStatsBlocks), dim3(256), 0, s, a11, a12, n, d_partials);
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(kStatsBlocks), 0, s, d_partials, d_out);
    return hipGetLastError();
}

hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace fdm
