// fdm_stage.h -- gfx950 stage kernels of the layer-case transport hot path.
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

#pragma once
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

// FP64 modes: the numerical Hamiltonian evaluated with the definition's
// operations in the definition's order -- correctly rounded square root and
// division, |p| = sqrt(px^2 + py^2), dH/dpx = (v0 px)/|p| (0 at p = 0), the
// speeds as running max/min from 0, weights a+/(a+ - a-), -a-/(a+ - a-),
// viscosity (a+ a-)/(a+ - a-), and the sum accumulated corner by corner from
// zero, then the two viscosity terms.  With IEEE operations and no
// contraction (the FP64 translation unit) this reproduces a plain float64
// evaluation of the scheme bit for bit, including which tiny gradients are
// exactly zero -- which matters because the speed p/|p| is discontinuous
// there.
template <int VK>
__device__ __forceinline__ double numerical_hamiltonian_ieee(double pxm, double pxp, double pym, double pyp,
                                                             double v0, double V1, double V2)
{
    if constexpr (VK == VK_PRESCRIBED) {
        const double px = V1 > 0.0 ? pxm : pxp;
        const double py = V2 > 0.0 ? pym : pyp;
        return V1 * px + V2 * py;
    } else {
        const double px[2] = {pxm, pxp};
        const double py[2] = {pym, pyp};
        double H[2][2], Hx[2][2], Hy[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const double r = sqrt(px[s] * px[s] + py[t] * py[t]);
                H[s][t] = v0 * r;
                Hx[s][t] = r > 0.0 ? v0 * px[s] / r : 0.0;
                Hy[s][t] = r > 0.0 ? v0 * py[t] / r : 0.0;
            }
        double ap = 0.0, am = 0.0, bp = 0.0, bm = 0.0;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                ap = Hx[s][t] > ap ? Hx[s][t] : ap;
                am = Hx[s][t] < am ? Hx[s][t] : am;
                bp = Hy[s][t] > bp ? Hy[s][t] : bp;
                bm = Hy[s][t] < bm ? Hy[s][t] : bm;
            }
        double wx[2], wy[2], visc_x, visc_y;
        if (ap - am > 0.0) {
            wx[0] = ap / (ap - am);
            wx[1] = -am / (ap - am);
            visc_x = ap * am / (ap - am);
        } else {
            wx[0] = 0.5;
            wx[1] = 0.5;
            visc_x = 0.0;
        }
        if (bp - bm > 0.0) {
            wy[0] = bp / (bp - bm);
            wy[1] = -bm / (bp - bm);
            visc_y = bp * bm / (bp - bm);
        } else {
            wy[0] = 0.5;
            wy[1] = 0.5;
            visc_y = 0.0;
        }
        double hhat = 0.0;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int t = 0; t < 2; ++t) hhat += wx[s] * wy[t] * H[s][t];
        hhat += visc_x * (pxp - pxm) + visc_y * (pyp - pym);
        return hhat;
    }
}

__device__ __forceinline__ int next_row(int k, int ny)
{
    k += 1;
    return k == ny ? 0 : k;
}

// Row `row` of a field, at this lane's byte offset: the row address is
// wave-uniform (scalar registers), the offset a 32-bit lane value.
template <typename T>
__device__ __forceinline__ const T *row_ptr(const void *base, int row, int nx)
{
    return static_cast<const T *>(base) + (size_t)row * (size_t)nx;
}

template <typename T>
__device__ __forceinline__ T at(const T *row, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(row) + off);
}

template <typename T>
__device__ __forceinline__ void put(const T *row, uint32_t off, T v)
{
    *reinterpret_cast<T *>(const_cast<char *>(reinterpret_cast<const char *>(row)) + off) = v;
}

// One wave: columns strip*60 .. strip*60+59 (lanes 2..61), rows
// chunk*rows .. +rows-1, of one stage; arithmetic in R, state stored as S.
// Loads run one row ahead of the arithmetic so their latency overlaps the
// previous row.
template <typename R, typename S, int LK, int VK, bool FIELD, int MODE>
__device__ __forceinline__ void run_tile(const InstDev &I, int strip, int chunk, int lane)
{
    constexpr bool kF64 = sizeof(R) == 8;
    constexpr bool kBase = MODE == MODE_HEUN2;
    const int nx = I.nx, ny = I.ny;
    const void *s12 = MODE == MODE_FWD ? I.a12 : I.w12;
    const void *s11 = MODE == MODE_FWD ? I.a11 : I.w11;
    const void *d12 = MODE == MODE_FWD ? I.w12 : I.a12;
    const void *d11 = MODE == MODE_FWD ? I.w11 : I.a11;
    const R theta = kF64 ? R(I.thetad) : R(I.theta);
    const R cx = kF64 ? R(I.cxd) : R(I.cx);
    const R cy = kF64 ? R(I.cyd) : R(I.cy);
    const R V1 = R(I.V1), V2 = R(I.V2);

    const int gcol = strip * kStrip - kHalo + lane;
    int col = gcol % nx;
    if (col < 0) col += nx;
    const uint32_t off = (uint32_t)col * (uint32_t)sizeof(S);
    const uint32_t off_v = (uint32_t)col * 4u;
    const bool out_col = lane >= kHalo && lane < kHalo + kStrip && gcol < nx;
    const int k0 = chunk * I.rows;
    const int nrows = min(I.rows, ny - k0);

    // alpha_11 = -w_y on y-edges; the window holds rows k-2, k-1, k.
    int k = (k0 - 2) % ny;
    if (k < 0) k += ny;
    const R ym2 = R(at(row_ptr<S>(s11, k, nx), off));
    k = next_row(k, ny);
    R ym1 = R(at(row_ptr<S>(s11, k, nx), off));
    const int kprev0 = k;
    k = next_row(k, ny);
    R y0 = R(at(row_ptr<S>(s11, k, nx), off));
    R sm1 = limited_slope<LK>(ym2, ym1, y0, theta);   // slope at edge k-1/2
    R hprev = R(0);
    int kprev = kprev0;

    // first row's operands
    int kn = next_row(k, ny);
    S f_wx = at(row_ptr<S>(s12, k, nx), off);
    S f_yp1 = at(row_ptr<S>(s11, kn, nx), off);
    float f_v0 = FIELD ? at(row_ptr<float>(I.v0f, k, nx), off_v) : 0.0f;
    S f_b12 = kBase ? at(row_ptr<S>(d12, k, nx), off) : S(0);
    S f_b11 = kBase ? at(row_ptr<S>(d11, kprev, nx), off) : S(0);

    for (int it = 0; it <= nrows; ++it) {
        const R wx = R(f_wx), yp1 = R(f_yp1);
        const R v0 = FIELD ? R(f_v0) : R(I.v0);
        const R b12 = R(f_b12), b11 = R(f_b11);
        const int knn = next_row(kn, ny);
        if (it < nrows) {   // operands of the next row (wave-uniform branch)
            f_wx = at(row_ptr<S>(s12, kn, nx), off);
            f_yp1 = at(row_ptr<S>(s11, knn, nx), off);
            if constexpr (FIELD) f_v0 = at(row_ptr<float>(I.v0f, kn, nx), off_v);
            if constexpr (kBase) {
                f_b12 = at(row_ptr<S>(d12, kn, nx), off);
                f_b11 = at(row_ptr<S>(d11, k, nx), off);
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
        R h;
        if constexpr (kF64)
            h = numerical_hamiltonian_ieee<VK>(pxm, pxp, pym, pyp, v0, V1, V2);
        else
            h = numerical_hamiltonian<VK>(pxm, pxp, pym, pyp, v0, V1, V2);
        const R hr = from_right(h);

        if (out_col) {
            if (it < nrows) {            // x-edge (j+1/2, k): d(alpha_12)/dt = -(Hhat_{j+1} - Hhat_j)/dx
                R nv;
                if constexpr (kF64) nv = wx + I.dtd * (-(hr - h) / I.dxd);
                else nv = wx - cx * (hr - h);
                if constexpr (kBase) nv = R(0.5) * b12 + R(0.5) * nv;
                put(row_ptr<S>(d12, k, nx), off, S(nv));
            }
            if (it > 0) {                // y-edge (j, k-1/2): d(alpha_11)/dt = (Hhat_k - Hhat_{k-1})/dy
                R nv;
                if constexpr (kF64) nv = ym1 + I.dtd * ((h - hprev) / I.dyd);
                else nv = ym1 + cy * (h - hprev);
                if constexpr (kBase) nv = R(0.5) * b11 + R(0.5) * nv;
                put(row_ptr<S>(d11, kprev, nx), off, S(nv));
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

template <typename R, typename S, int LK, int VK, bool FIELD, int MODE>
__global__ __launch_bounds__(kBlock) void stage_kernel(InstDev I, int64_t total_tiles, int blocks_per_xcd)
{
    const int64_t tile = xcd_tile(blocks_per_xcd);
    if (tile >= total_tiles) return;
    const int t = (int)tile;
    run_tile<R, S, LK, VK, FIELD, MODE>(I, t / I.chunks, t % I.chunks, threadIdx.x & 63);
}

// Batched: one launch for every tile of every instance; tile_inst maps a
// global tile to its instance.  Limiter, Hamiltonian and field presence are
// per instance and uniform over a wave.
template <typename R, typename S, int MODE>
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
        if (lk == LK_NONE) run_tile<R, S, LK_NONE, VK_PRESCRIBED, false, MODE>(I, strip, chunk, lane);
        else if (lk == LK_SUPERBEE) run_tile<R, S, LK_SUPERBEE, VK_PRESCRIBED, false, MODE>(I, strip, chunk, lane);
        else run_tile<R, S, LK_THETA, VK_PRESCRIBED, false, MODE>(I, strip, chunk, lane);
    } else if (I.v0f != nullptr) {
        if (lk == LK_NONE) run_tile<R, S, LK_NONE, VK_LAW, true, MODE>(I, strip, chunk, lane);
        else if (lk == LK_SUPERBEE) run_tile<R, S, LK_SUPERBEE, VK_LAW, true, MODE>(I, strip, chunk, lane);
        else run_tile<R, S, LK_THETA, VK_LAW, true, MODE>(I, strip, chunk, lane);
    } else {
        if (lk == LK_NONE) run_tile<R, S, LK_NONE, VK_LAW, false, MODE>(I, strip, chunk, lane);
        else if (lk == LK_SUPERBEE) run_tile<R, S, LK_SUPERBEE, VK_LAW, false, MODE>(I, strip, chunk, lane);
        else run_tile<R, S, LK_THETA, VK_LAW, false, MODE>(I, strip, chunk, lane);
    }
}

template <typename R, typename S, int LK, int VK, bool FIELD>
hipError_t launch_stage_t(const InstDev &I, int mode, hipStream_t s)
{
    const int64_t tiles = (int64_t)I.strips * I.chunks;
    const int64_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_xcd = (int)((blocks + 7) / 8);
    const dim3 grid(8 * per_xcd), block(kBlock);
    if (mode == MODE_FWD)
        hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_FWD>), grid, block, 0, s, I, tiles, per_xcd);
    else if (mode == MODE_BWD)
        hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_BWD>), grid, block, 0, s, I, tiles, per_xcd);
    else
        hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_HEUN2>), grid, block, 0, s, I, tiles, per_xcd);
    return hipGetLastError();
}

template <typename R, typename S>
hipError_t launch_stage_r(const InstDev &I, int mode, hipStream_t s)
{
    const int lk = limiter_kind(I.limiter);
    if (I.vkind == VK_PRESCRIBED) {
        if (lk == LK_NONE) return launch_stage_t<R, S, LK_NONE, VK_PRESCRIBED, false>(I, mode, s);
        if (lk == LK_SUPERBEE) return launch_stage_t<R, S, LK_SUPERBEE, VK_PRESCRIBED, false>(I, mode, s);
        return launch_stage_t<R, S, LK_THETA, VK_PRESCRIBED, false>(I, mode, s);
    }
    if (I.v0f != nullptr) {
        if (lk == LK_NONE) return launch_stage_t<R, S, LK_NONE, VK_LAW, true>(I, mode, s);
        if (lk == LK_SUPERBEE) return launch_stage_t<R, S, LK_SUPERBEE, VK_LAW, true>(I, mode, s);
        return launch_stage_t<R, S, LK_THETA, VK_LAW, true>(I, mode, s);
    }
    if (lk == LK_NONE) return launch_stage_t<R, S, LK_NONE, VK_LAW, false>(I, mode, s);
    if (lk == LK_SUPERBEE) return launch_stage_t<R, S, LK_SUPERBEE, VK_LAW, false>(I, mode, s);
    return launch_stage_t<R, S, LK_THETA, VK_LAW, false>(I, mode, s);
}

template <typename R, typename S>
hipError_t launch_batched_r(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles, int mode,
                            hipStream_t s)
{
    const int64_t blocks = (total_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_xcd = (int)((blocks + 7) / 8);
    const dim3 grid(8 * per_xcd), block(kBlock);
    if (mode == MODE_FWD)
        hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_FWD>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles, per_xcd);
    else if (mode == MODE_BWD)
        hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_BWD>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles, per_xcd);
    else
        hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_HEUN2>), grid, block, 0, s, d_inst, d_tile_inst, total_tiles, per_xcd);
    return hipGetLastError();
}

}  // namespace
}  // namespace fdm
