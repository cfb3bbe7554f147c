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

// lane l receives lane l-1's value (lane 0 receives 0: bound_ctrl writes
// zero where the source lane does not exist, so no old value is needed)
__device__ __forceinline__ float from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}

// lane l receives lane l+1's value (lane 63 receives 0)
__device__ __forceinline__ float from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
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

// Multiply-add.  float: always one fused operation.  Both stage files turn
// implicit contraction off, so every fusion is written out here and each of
// the eight unrolled copies of the row loop rounds identically: otherwise the
// compiler may fuse a different product in different copies, a row's Hhat
// then depends on which copy computes it (the tile height), and the two tiles
// that both compute a boundary row can disagree in the last bit.  double:
// separate multiply and add, as in the definition.
__device__ __forceinline__ float madd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double madd(double a, double b, double c) { return a * b + c; }

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

// Two independent float evaluations in lock step: each operation applies
// the scalar operation to both components, so results are those of two
// scalar evaluations bit for bit, and the compiler sees the two instruction
// streams interleaved (the fused kernel evaluates its two stages' nodes of
// a row this way).
struct F2 {
    float a, b;
    __host__ __device__ constexpr F2() : a(0.0f), b(0.0f) {}
    __host__ __device__ constexpr F2(float v) : a(v), b(v) {}
    __host__ __device__ constexpr F2(float x, float y) : a(x), b(y) {}
};
__device__ __forceinline__ F2 operator+(F2 x, F2 y) { return F2(x.a + y.a, x.b + y.b); }
__device__ __forceinline__ F2 operator-(F2 x, F2 y) { return F2(x.a - y.a, x.b - y.b); }
__device__ __forceinline__ F2 operator*(F2 x, F2 y) { return F2(x.a * y.a, x.b * y.b); }
__device__ __forceinline__ F2 operator-(F2 x) { return F2(-x.a, -x.b); }
__device__ __forceinline__ F2 vmin(F2 x, F2 y) { return F2(fminf(x.a, y.a), fminf(x.b, y.b)); }
__device__ __forceinline__ F2 vmax(F2 x, F2 y) { return F2(fmaxf(x.a, y.a), fmaxf(x.b, y.b)); }
__device__ __forceinline__ F2 madd(F2 x, F2 y, F2 z)
{
    return F2(__builtin_fmaf(x.a, y.a, z.a), __builtin_fmaf(x.b, y.b, z.b));
}
__device__ __forceinline__ F2 from_left(F2 v) { return F2(from_left(v.a), from_left(v.b)); }
__device__ __forceinline__ F2 from_right(F2 v) { return F2(from_right(v.a), from_right(v.b)); }

template <> struct Arith<F2> {
    static constexpr F2 tiny = F2(Arith<float>::tiny);
    static __device__ __forceinline__ F2 rsq(F2 r) { return F2(Arith<float>::rsq(r.a), Arith<float>::rsq(r.b)); }
    static __device__ __forceinline__ F2 rcp(F2 x) { return F2(Arith<float>::rcp(x.a), Arith<float>::rcp(x.b)); }
};

// float arithmetic (one value or a lock-step pair)
template <typename R> struct IsF32 {
    static constexpr bool value = false;
};
template <> struct IsF32<float> {
    static constexpr bool value = true;
};
template <> struct IsF32<F2> {
    static constexpr bool value = true;
};

// The middle of three values; +-infinity with the sign of s; a when v > 0
// else b (v is the same in both components of a pair).
__device__ __forceinline__ float med3(float x, float y, float z) { return __builtin_amdgcn_fmed3f(x, y, z); }
__device__ __forceinline__ F2 med3(F2 x, F2 y, F2 z) { return F2(med3(x.a, y.a, z.a), med3(x.b, y.b, z.b)); }
__device__ __forceinline__ float sign_inf(float s) { return copysignf(__builtin_inff(), s); }
__device__ __forceinline__ F2 sign_inf(F2 s) { return F2(sign_inf(s.a), sign_inf(s.b)); }
__device__ __forceinline__ float pick_pos(float v, float a, float b) { return v > 0.0f ? a : b; }
__device__ __forceinline__ double pick_pos(double v, double a, double b) { return v > 0.0 ? a : b; }
__device__ __forceinline__ F2 pick_pos(F2 v, F2 a, F2 b) { return F2(pick_pos(v.a, a.a, b.a), pick_pos(v.b, a.b, b.b)); }

// ---------------------------------------------------------------- Step 1

// Limiter kinds compiled separately.  The minmod family shares one body with
// a runtime theta (2 for MC, or a given theta), so every launch form runs the
// same instructions for a given limiter.  Minmod itself (theta = 1) has its
// own float body: there the centred argument (D+ + D-)/2 always lies between
// D+ and D-, so the three-argument minmod is the two-argument minmod(D-, D+).
// The float64 arithmetic keeps the definition's three arguments (bit for bit
// with the oracle), so there minmod stays a theta kind.
enum : int { LK_NONE = 0, LK_THETA = 1, LK_SUPERBEE = 2, LK_MINMOD = 3 };

template <int K> struct LimTag {
    static constexpr int value = K;
};

// f(LimTag<kind>{}) for a limiter code (the public enum), one instantiation
// per kind; F32: float arithmetic, where minmod is a kind of its own.
template <bool F32, typename F>
__host__ __device__ __forceinline__ decltype(auto) with_limiter(int lim, F &&f)
{
    if (lim == LIM_NONE) return f(LimTag<LK_NONE>{});
    if (lim == LIM_SUPERBEE) return f(LimTag<LK_SUPERBEE>{});
    if constexpr (F32) {
        if (lim == LIM_MINMOD) return f(LimTag<LK_MINMOD>{});
    }
    return f(LimTag<LK_THETA>{});
}

// Limited slope at an edge from three consecutive values along its axis.
// Every limiter here returns one of its candidate values (or zero), so the
// result does not depend on how the selection is written.
//
// float: with med3(a, b, 0) = minmod(a, b) (the middle of a, b and 0 is the
// smaller magnitude when the signs agree and 0 otherwise), theta-minmod is
// med3(med3(theta*D+, theta*D-, 0), (w+ - w-)/2, 0), and superbee
// picks the larger of minmod(2D-, D+) and minmod(D-, 2D+) -- both carry the
// sign of D+ or are zero -- as med3(s1, s2, copysign(inf, D+)).
//
// double (no FP64 med3 on gfx950): theta-minmod as max(min3, 0) +
// min(max3, 0), superbee as sign * max(min(2|D-|, |D+|), min(|D-|, 2|D+|))
// when D- D+ > 0.
template <int LK, typename R>
__device__ __forceinline__ R limited_slope(R wm, R w0, R wp, R theta)
{
    if constexpr (LK == LK_NONE) {
        return R(0);
    } else if constexpr (LK == LK_MINMOD) {
        static_assert(IsF32<R>::value, "minmod has its own kind in float arithmetic only");
        return med3(w0 - wm, wp - w0, R(0.0f));
    } else if constexpr (IsF32<R>::value && LK == LK_SUPERBEE) {
        const R dm = w0 - wm, dp = wp - w0;
        const R s1 = med3(R(2.0f) * dm, dp, R(0.0f));
        const R s2 = med3(dm, R(2.0f) * dp, R(0.0f));
        return med3(s1, s2, sign_inf(dp));
    } else if constexpr (IsF32<R>::value) {
        const R a = theta * (wp - w0), b = R(0.5f) * (wp - wm), c = theta * (w0 - wm);
        return med3(med3(a, c, R(0.0f)), b, R(0.0f));
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

// float, along the y walk: the backward difference of row k is the forward
// difference of row k-1, bit for bit (same operands, same operation), so it
// is carried from the previous row together with its scaled form (2 D for
// superbee, theta D for the minmod family).  Same results as limited_slope,
// two instructions fewer.  dm, dms: in, the carried difference and its scaled
// form; out, this row's.
template <int LK, typename R>
__device__ __forceinline__ R y_slope_carried(R wm, R w0, R wp, R theta, R &dm, R &dms)
{
    static_assert(IsF32<R>::value, "the carried y slope is a float path");
    if constexpr (LK == LK_NONE) {
        return R(0.0f);
    } else {
        const R dp = wp - w0;
        R s, dps;
        if constexpr (LK == LK_MINMOD) {
            dps = dp;
            s = med3(dm, dp, R(0.0f));
        } else if constexpr (LK == LK_SUPERBEE) {
            dps = R(2.0f) * dp;
            const R s1 = med3(dms, dp, R(0.0f));
            const R s2 = med3(dm, dps, R(0.0f));
            s = med3(s1, s2, sign_inf(dp));
        } else {
            dps = theta * dp;
            const R b = R(0.5f) * (wp - wm);
            s = med3(med3(dps, dms, R(0.0f)), b, R(0.0f));
        }
        dm = dp;
        dms = dps;
        return s;
    }
}

// ---------------------------------------------------------- Steps 2 to 4

template <int VK, typename R>
__device__ __forceinline__ R numerical_hamiltonian(R pxm, R pxp, R pym, R pyp, R v0, R V1, R V2)
{
    if constexpr (VK == VK_PRESCRIBED) {
        // H = V.p: the central-upwind weights reduce to pure upwinding.
        const R px = pick_pos(V1, pxm, pxp);
        const R py = pick_pos(V2, pym, pyp);
        return madd(V2, py, V1 * px);
    } else {
        // H = v0 |p| at the four corners (s,t) in {-,+}^2, dH/dp = v0 p/|p|.
        // |p|^2 is clamped below at the smallest normal number before the
        // reciprocal square root (v_rsq reads a subnormal as zero): p = 0
        // still gives H = 0 and speed 0, and gradients below 1e-19 (float)
        // move with speed v0 p / 1e-19 instead of a full-speed direction.
        // (Folding the bound into the squares as fma(p, p, FLT_MIN) would
        // save the four clamps but make H(0) = v0 2^-63: under a celerity
        // field that seeds 1e-19 densities in empty regions, whose speeds
        // are then O(v0) -- measurably worse parity.)
        constexpr R kTiny = Arith<R>::tiny;
        const R xm2 = pxm * pxm, xp2 = pxp * pxp;
        const R r00 = madd(pym, pym, xm2), r01 = madd(pyp, pyp, xm2);
        const R r10 = madd(pym, pym, xp2), r11 = madd(pyp, pyp, xp2);
        const R g00 = v0 * Arith<R>::rsq(vmax(r00, kTiny));
        const R g01 = v0 * Arith<R>::rsq(vmax(r01, kTiny));
        const R g10 = v0 * Arith<R>::rsq(vmax(r10, kTiny));
        const R g11 = v0 * Arith<R>::rsq(vmax(r11, kTiny));
        const R H00 = r00 * g00, H01 = r01 * g01, H10 = r10 * g10, H11 = r11 * g11;
        const R hx00 = pxm * g00, hx01 = pxm * g01, hx10 = pxp * g10, hx11 = pxp * g11;
        const R hy00 = pym * g00, hy01 = pyp * g01, hy10 = pym * g10, hy11 = pyp * g11;
        // Step 2: one-sided local speeds over the four combinations, bounded
        // by +-FLT_MIN instead of 0 (two three-operand max/min each).  Then
        // a+ - a- >= 2 FLT_MIN always: where nothing moves along an axis the
        // weights come out as exactly 1/2 (2^-126 * rcp(2^-125)) and the
        // viscosity as -FLT_MIN/2, which is the scheme's degenerate case up
        // to a term below the smallest normal number per unit gradient jump,
        // with no compare or select; a one-sided speed of 0 becomes 1.2e-38,
        // which moves nothing representable against normal densities.
        const R ap = vmax(vmax(vmax(vmax(hx00, hx01), hx10), hx11), kTiny);
        const R am = vmin(vmin(vmin(vmin(hx00, hx01), hx10), hx11), -kTiny);
        const R bp = vmax(vmax(vmax(vmax(hy00, hy01), hy10), hy11), kTiny);
        const R bm = vmin(vmin(vmin(vmin(hy00, hy01), hy10), hy11), -kTiny);
        // Steps 3-4 (dt -> 0): projection weights.  The sum keeps the order
        // of the definition (weighted corner values, then the two viscosity
        // terms): rewriting it, e.g. with w_+ = 1 - w_-, lets FMA
        // contraction turn exact cancellations between equal corner values
        // into product rounding errors, which the kink of |p| at p = 0
        // then amplifies.
        const R ia = Arith<R>::rcp(ap - am), ib = Arith<R>::rcp(bp - bm);
        const R wxm = ap * ia, wxp = -am * ia;
        const R wym = bp * ib, wyp = -bm * ib;
        // viscosity a+ a- / (a+ - a-) = -(a+ w+), one product instead of two
        const R nvx = ap * wxp, nvy = bp * wyp;
        const R sum = madd(wxp, madd(wyp, H11, wym * H10), wxm * madd(wyp, H01, wym * H00));
        return madd(-nvy, pyp - pym, madd(-nvx, pxp - pxm, sum));
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

// Fully discrete scheme (sec. 3.2.3), float.  With the separable quadratic
// interpolant the value over phi_jk at the corner (x_j + a^s dt, y_k + b^t dt)
// is X_s + Y_t, X_s = dt a^s (p_x^s + a^s dt sx^s / (2 dx)), and its slope is
// q_x^s = p_x^s + a^s (dt/dx) sx^s (likewise along y).  Projecting
// X_s + Y_t - dt H(q^s, q^t) with the weights and dividing by -dt gives the
// node's rate in the same units as the semi-discrete Hhat:
//   Hhat_fd = sum_st w_s v_t H(q_x^s, q_y^t)
//           + a+a-/(a+ - a-) [(p_x^+ - p_x^-) + (dt/dx)/2 (a+ sx^+ - a- sx^-)]
//           + the same along y,
// because w_+ a+ = -a+a-/(a+ - a-) = -w_- a-.  sx^+- are the limited slopes
// (in density units) of the edges right/left of the node, sy^+- above/below;
// cx = dt/dx, cy = dt/dy.  The speeds and weights are those of the
// semi-discrete scheme (same FLT_MIN bounds); |q| uses the hardware square
// root (|q| = 0 gives H = 0).
template <int VH>
__device__ __forceinline__ float fd_hamiltonian(float pxm, float pxp, float pym, float pyp, float sxm, float sxp,
                                                float sym, float syp, float v0, float V1, float V2, float cx,
                                                float cy)
{
    float ap, am, bp, bm;
    if constexpr (VH == VK_PRESCRIBED) {
        ap = vmax(V1, Arith<float>::tiny);
        am = vmin(V1, -Arith<float>::tiny);
        bp = vmax(V2, Arith<float>::tiny);
        bm = vmin(V2, -Arith<float>::tiny);
    } else {
        constexpr float kTiny = Arith<float>::tiny;
        const float xm2 = pxm * pxm, xp2 = pxp * pxp;
        const float g00 = v0 * Arith<float>::rsq(vmax(madd(pym, pym, xm2), kTiny));
        const float g01 = v0 * Arith<float>::rsq(vmax(madd(pyp, pyp, xm2), kTiny));
        const float g10 = v0 * Arith<float>::rsq(vmax(madd(pym, pym, xp2), kTiny));
        const float g11 = v0 * Arith<float>::rsq(vmax(madd(pyp, pyp, xp2), kTiny));
        const float hx00 = pxm * g00, hx01 = pxm * g01, hx10 = pxp * g10, hx11 = pxp * g11;
        const float hy00 = pym * g00, hy01 = pyp * g01, hy10 = pym * g10, hy11 = pyp * g11;
        ap = vmax(vmax(vmax(vmax(hx00, hx01), hx10), hx11), kTiny);
        am = vmin(vmin(vmin(vmin(hx00, hx01), hx10), hx11), -kTiny);
        bp = vmax(vmax(vmax(vmax(hy00, hy01), hy10), hy11), kTiny);
        bm = vmin(vmin(vmin(vmin(hy00, hy01), hy10), hy11), -kTiny);
    }
    // slopes of the interpolant at the intermediate points
    const float qxm = madd(cx * am, sxm, pxm), qxp = madd(cx * ap, sxp, pxp);
    const float qym = madd(cy * bm, sym, pym), qyp = madd(cy * bp, syp, pyp);
    float H00, H01, H10, H11;
    if constexpr (VH == VK_PRESCRIBED) {
        H00 = madd(V2, qym, V1 * qxm);
        H01 = madd(V2, qyp, V1 * qxm);
        H10 = madd(V2, qym, V1 * qxp);
        H11 = madd(V2, qyp, V1 * qxp);
    } else {
        const float xm2 = qxm * qxm, xp2 = qxp * qxp;
        H00 = v0 * __builtin_amdgcn_sqrtf(madd(qym, qym, xm2));
        H01 = v0 * __builtin_amdgcn_sqrtf(madd(qyp, qyp, xm2));
        H10 = v0 * __builtin_amdgcn_sqrtf(madd(qym, qym, xp2));
        H11 = v0 * __builtin_amdgcn_sqrtf(madd(qyp, qyp, xp2));
    }
    const float ia = Arith<float>::rcp(ap - am), ib = Arith<float>::rcp(bp - bm);
    const float wxm = ap * ia, wxp = -am * ia;
    const float wym = bp * ib, wyp = -bm * ib;
    const float nvx = ap * wxp, nvy = bp * wyp;   // minus the viscosities
    const float corr_x = madd(0.5f * cx, madd(ap, sxp, -(am * sxm)), pxp - pxm);
    const float corr_y = madd(0.5f * cy, madd(bp, syp, -(bm * sym)), pyp - pym);
    const float sum = madd(wxp, madd(wyp, H11, wym * H10), wxm * madd(wyp, H01, wym * H00));
    return madd(-nvy, corr_y, madd(-nvx, corr_x, sum));
}

// Fully discrete scheme, FP64 modes, in the definition's own form: the
// node increment phi^{n+1} - phi^n of Steps 1-4 (sec. 3.2.2-3.2.3), whose
// differences between neighbouring nodes are the density updates.  One
// piece of the quadratic interpolant (eq. 42) as an increment over phi at
// the node and its slope at x_j + h: side +1 is the piece on [x_j, x_j+d]
// (h >= 0), side -1 the piece on [x_j-d, x_j] (h <= 0, whose left end lies
// D below the node); D and Dp are the edge's (Delta phi) and (Delta phi)'.
__device__ __forceinline__ void fd_piece_ieee(int side, double D, double Dp, double d, double h, double &val,
                                              double &slope)
{
    const double c = Dp / (2.0 * d * d);
    if (side > 0) {
        val = D / d * h + c * h * (h - d);
        slope = D / d + c * ((h - d) + h);
    } else {
        val = -D + D / d * (d + h) + c * (d + h) * h;
        slope = D / d + c * (h + (d + h));
    }
}

// The increment at one node from the densities w and limited slopes s (per
// unit length) of its four edges: x to the left (l) and right (r), y below
// (d) and above (u).  IEEE operations in the definition's order: one-sided
// derivatives (the pieces' slopes at the node), the four-corner speeds
// (eq. 53, running max/min from 0), the interpolant and its slope at the
// points x_j + a^-+ dt and y_k + b^-+ dt, the projection weights (1/2 where
// nothing moves along an axis) and the weighted sum of phi at the four
// points after the step, accumulated corner by corner from zero.
template <int VH>
__device__ __forceinline__ double fd_increment_ieee(double wxl, double sxl, double wxr, double sxr, double wyd,
                                                    double syd, double wyu, double syu, double v0, double V1,
                                                    double V2, double dx, double dy, double dt)
{
    double unused, px[2], py[2];
    fd_piece_ieee(-1, dx * wxl, dx * sxl, dx, 0.0, unused, px[0]);
    fd_piece_ieee(+1, dx * wxr, dx * sxr, dx, 0.0, unused, px[1]);
    fd_piece_ieee(-1, dy * wyd, dy * syd, dy, 0.0, unused, py[0]);
    fd_piece_ieee(+1, dy * wyu, dy * syu, dy, 0.0, unused, py[1]);
    double ap = 0.0, am = 0.0, bp = 0.0, bm = 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            double hx, hy;
            if constexpr (VH == VK_PRESCRIBED) {
                hx = V1;
                hy = V2;
            } else {
                const double r = sqrt(px[s] * px[s] + py[t] * py[t]);
                hx = r > 0.0 ? v0 * px[s] / r : 0.0;
                hy = r > 0.0 ? v0 * py[t] / r : 0.0;
            }
            ap = hx > ap ? hx : ap;
            am = hx < am ? hx : am;
            bp = hy > bp ? hy : bp;
            bm = hy < bm ? hy : bm;
        }
    double X[2], Xs[2], Y[2], Ys[2];
    fd_piece_ieee(-1, dx * wxl, dx * sxl, dx, am * dt, X[0], Xs[0]);
    fd_piece_ieee(+1, dx * wxr, dx * sxr, dx, ap * dt, X[1], Xs[1]);
    fd_piece_ieee(-1, dy * wyd, dy * syd, dy, bm * dt, Y[0], Ys[0]);
    fd_piece_ieee(+1, dy * wyu, dy * syu, dy, bp * dt, Y[1], Ys[1]);
    double wx[2], wy[2];
    if (ap - am > 0.0) {
        wx[0] = ap / (ap - am);
        wx[1] = -am / (ap - am);
    } else {
        wx[0] = 0.5;
        wx[1] = 0.5;
    }
    if (bp - bm > 0.0) {
        wy[0] = bp / (bp - bm);
        wy[1] = -bm / (bp - bm);
    } else {
        wy[0] = 0.5;
        wy[1] = 0.5;
    }
    double inc = 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const double H = VH == VK_PRESCRIBED ? V1 * Xs[s] + V2 * Ys[t]
                                                 : v0 * sqrt(Xs[s] * Xs[s] + Ys[t] * Ys[t]);
            inc += wx[s] * wy[t] * ((X[s] + Y[t]) - dt * H);
        }
    return inc;
}

__device__ __forceinline__ int next_row(int k, int ny)
{
    k += 1;
    return k == ny ? 0 : k;
}

// Rows are addressed through buffer resources: a wave-uniform row base
// (scalar registers) plus this lane's 32-bit byte offset, so no access needs
// 64-bit vector address arithmetic.  The hardware range check does the
// masking: an offset at or beyond the row's byte size (kSkip for lanes that
// must not write) loads 0 and drops stores, and a row built with `live`
// false has size 0, which drops every lane.  Stores are therefore issued
// unconditionally, with no branches around them, and the memory counter
// waits stay exact.
constexpr uint32_t kBufWord3 = 0x00020000u;   // gfx9: 32-bit data format, raw access
constexpr uint32_t kSkip = 0x80000000u;       // > any row size (rows are < 2^31 bytes)

template <typename T> struct RowRef {
    __amdgpu_buffer_rsrc_t r;
};

template <typename T>
__device__ __forceinline__ RowRef<T> row_ptr(const void *base, int row, int nx, bool live = true)
{
    T *p = const_cast<T *>(static_cast<const T *>(base)) + (size_t)row * (size_t)nx;
    const int bytes = live ? nx * (int)sizeof(T) : 0;
    return RowRef<T>{__builtin_amdgcn_make_buffer_rsrc(p, 0, bytes, (int)kBufWord3)};
}

__device__ __forceinline__ float at(RowRef<float> row, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(row.r, (int)off, 0, 0));
}

__device__ __forceinline__ double at(RowRef<double> row, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(row.r, (int)off, 0, 0));
}

__device__ __forceinline__ void put(RowRef<float> row, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), row.r, (int)off, 0, 0);
}

__device__ __forceinline__ void put(RowRef<double> row, uint32_t off, double v)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), row.r, (int)off, 0, 0);
}

template <int P> struct Phase {
    static constexpr int value = P;
};

// One wave: columns strip*60 .. strip*60+59 (lanes 2..61), rows
// chunk*rows .. +rows-1, of one stage; arithmetic in R, state stored as S.
// Loads run kAhead rows ahead of the arithmetic, so each load has the
// arithmetic of kAhead rows to arrive.  The row loop is unrolled eight times
// by hand: every value on the sliding window (alpha_11 rows from in flight
// down to the row below the current one; the other loads; slopes and Hhat)
// sits in a ring slot fixed by the row number, so no copies rotate it.
constexpr int kAhead = 2;

// The first midpoint stage runs the MODE_FWD kernel with half the step:
// halving is exact in float and double, so the coefficients are those of
// dt/2.
// Coupled runs: the step is chosen on the device, from the velocity law's
// max |v0| partials (each wave loads them first, beside its first rows, and
// reduces them: a few kilobytes from L2).
// The partials this lane reduces (zeros, with no memory read, when the
// instance has none).
__device__ __forceinline__ void load_partials(const InstDev &I, float (&x)[kMaxPartials / 64])
{
    const int lane = threadIdx.x & 63;
    const auto row = row_ptr<float>(I.vpart, 0, I.nvpart, I.vpart != nullptr);
#pragma unroll
    for (int j = 0; j < kMaxPartials / 64; ++j) x[j] = at(row, (uint32_t)(lane + 64 * j) * 4u);
}

__device__ __forceinline__ void load_coef(InstDev &I, bool tile0, const float (&x)[kMaxPartials / 64])
{
    if (I.vpart == nullptr) return;
    const StepCoef c = step_coef_from_loaded(x, I.cfl_h, I.dt_max, I.dxd, I.dyd);
    I.dtd = c.dtd;
    I.cxd = c.cxd;
    I.cyd = c.cyd;
    I.cx = c.cx;
    I.cy = c.cy;
    if (tile0 && I.coef_out != nullptr && (threadIdx.x & 63) == 0) *I.coef_out = c;
}

__device__ __forceinline__ void halve_step(InstDev &I)
{
    I.cx *= 0.5f;
    I.cy *= 0.5f;
    I.cxd *= 0.5;
    I.cyd *= 0.5;
    I.dtd *= 0.5;
}


template <typename R, typename S, int LK, int VK, bool FIELD, int MODE, bool HSUM = false>
__device__ __forceinline__ void run_tile(InstDev I, int strip, int chunk, int lane, int half)
{
    constexpr bool kF64 = sizeof(R) == 8;
    constexpr bool kFD = (VK & VK_FD) != 0;   // fully discrete scheme
    constexpr int VH = VK & 1;                // the Hamiltonian
    constexpr bool kBase = MODE == MODE_HEUN2 || MODE == MODE_MID2;   // also reads the base state
    const int nx = I.nx, ny = I.ny;
    const void *s12 = MODE == MODE_FWD ? I.a12 : I.w12;
    const void *s11 = MODE == MODE_FWD ? I.a11 : I.w11;
    const void *d12 = MODE == MODE_FWD ? I.w12 : I.a12;
    const void *d11 = MODE == MODE_FWD ? I.w11 : I.a11;
    const R theta = kF64 ? R(I.thetad) : R(I.theta);
    const R V1 = R(I.V1), V2 = R(I.V2);

    const int gcol = strip * kStrip - kHalo + lane;
    int col = gcol % nx;
    if (col < 0) col += nx;
    const uint32_t off = (uint32_t)col * (uint32_t)sizeof(S);
    const uint32_t off_v = (uint32_t)col * 4u;
    const bool out_col = lane >= kHalo && lane < kHalo + kStrip && gcol < nx;
    const int k0 = chunk * I.rows;
    const int nrows = min(I.rows, ny - k0);
    const uint32_t off_st = out_col ? off : kSkip;   // halo lanes do not write

    // Iteration i (0 .. nrows; the last one only completes the y-edges)
    // handles row k0+i.  Ring slots: alpha_11 of row k0+j in y[j & 7] (rows
    // k0+i-1 .. k0+i+kAhead+1 are live), the other loads of row k0+j in
    // slot j & 3, slope and Hhat of row k0+j in slot j & 1.
    S y[8], wx_[4], b12_[4], b11_[4];
    float v0_[4];
    R sl[2], hh[2];
    R hacc = R(0);   // HSUM: this lane's sum of Hhat (FP64 fully discrete: of the
                     // node increments) over the tile's own rows
    for (int j = 0; j < 4; ++j) {
        v0_[j] = 0.0f;
        b12_[j] = b11_[j] = S(0);
    }
    float vpart[kMaxPartials / 64];   // coupled runs (HSUM): the step's inputs, first in flight
    if constexpr (HSUM) load_partials(I, vpart);
    int k = (k0 - 2) % ny;
    if (k < 0) k += ny;
    const R ym2 = R(at(row_ptr<S>(s11, k, nx), off));
    k = next_row(k, ny);
    y[7] = at(row_ptr<S>(s11, k, nx), off);
    int kprev = k;
    k = next_row(k, ny);
    y[0] = at(row_ptr<S>(s11, k, nx), off);
    sl[1] = limited_slope<LK>(ym2, R(y[7]), R(y[0]), theta);   // slope at edge k0-1/2
    hh[1] = R(0);
    // float: the carried y difference of the first row and its scaled form
    float ydm = float(R(y[0]) - R(y[7]));
    float ydms = LK == LK_SUPERBEE ? 2.0f * ydm : float(theta) * ydm;

    // Loads of the first kAhead rows.  kf: row of the next fetch (k0+i+kAhead
    // at iteration i), kf1 the row after it, kfm the row before it.
    int kfm = kprev, kf = k;
#pragma unroll
    for (int j = 0; j < kAhead; ++j) {
        const int kf1 = next_row(kf, ny);
        const bool live = j <= nrows;
        wx_[j] = at(row_ptr<S>(s12, kf, nx, live), off);
        y[j + 1] = at(row_ptr<S>(s11, kf1, nx, live), off);
        if constexpr (FIELD) v0_[j] = at(row_ptr<float>(I.v0f, kf, nx, live), off_v);
        if constexpr (kBase) {
            b12_[j] = at(row_ptr<S>(d12, kf, nx, live), off);
            b11_[j] = at(row_ptr<S>(d11, kfm, nx, live), off);
        }
        kfm = kf;
        kf = kf1;
    }
    int kf1 = next_row(kf, ny);

    // The step coefficients, with the first loads already in flight (coupled
    // runs read them from device memory).
    if constexpr (HSUM) load_coef(I, strip == 0 && chunk == 0, vpart);
    if (half) halve_step(I);
    const R cx = kF64 ? R(I.cxd) : R(I.cx);
    const R cy = kF64 ? R(I.cyd) : R(I.cy);

    auto body = [&](int it, auto phase) {
        constexpr int p = decltype(phase)::value;
        constexpr int c = p & 3, f = (p + kAhead) & 3;   // this row's and the fetched row's slots
        constexpr int h = p & 1, hp = h ^ 1;              // this row's and the previous row's slope / Hhat
        const R ym1 = R(y[(p + 7) & 7]), y0 = R(y[p]), yp1 = R(y[(p + 1) & 7]);
        const R wx = R(wx_[c]);
        const R v0 = FIELD ? R(v0_[c]) : R(I.v0);
        const R b12 = R(b12_[c]), b11 = R(b11_[c]);
        // Operands of row k0+it+kAhead.  Issued on every iteration, so the
        // wait for this row's operands never has to drain loads just issued;
        // past the tile the rows are empty (no memory is read).
        {
            const bool live = it + kAhead <= nrows;
            wx_[f] = at(row_ptr<S>(s12, kf, nx, live), off);
            y[(p + kAhead + 1) & 7] = at(row_ptr<S>(s11, kf1, nx, live), off);
            if constexpr (FIELD) v0_[f] = at(row_ptr<float>(I.v0f, kf, nx, live), off_v);
            if constexpr (kBase) {
                b12_[f] = at(row_ptr<S>(d12, kf, nx, live), off);
                b11_[f] = at(row_ptr<S>(d11, kfm, nx, live), off);
            }
            kfm = kf;
            kf = kf1;
            kf1 = next_row(kf1, ny);
        }

        // Steps 1-2 along y (alpha_11 = -w_y, slopes are odd)
        // (halving is exact, so each face value rounds once, fused or not)
        R s0;
        if constexpr (kF64) s0 = limited_slope<LK>(ym1, y0, yp1, theta);
        else s0 = y_slope_carried<LK>(ym1, y0, yp1, theta, ydm, ydms);
        const R pyp = -madd(R(-0.5), s0, y0);
        const R pym = -madd(R(0.5), sl[hp], ym1);
        sl[h] = s0;
        // Steps 1-2 along x (alpha_12 = w_x), neighbours from adjacent lanes
        const R wl = from_left(wx), wr = from_right(wx);
        const R sx = limited_slope<LK>(wl, wx, wr, theta);
        const R pxp = madd(R(-0.5), sx, wx);
        const R pxm = from_left(madd(R(0.5), sx, wx));
        // Steps 2-4
        R hv;
        if constexpr (kFD) {
            // slopes in density units: x from this lane (edge j+1/2) and the
            // left one; y of w_y = -alpha_11 above (k+1/2) and below (k-1/2)
            const R sxm = from_left(sx);
            if constexpr (kF64)   // FP64: the node increment phi^{n+1} - phi^n itself
                hv = fd_increment_ieee<VH>(wl, sxm, wx, sx, -ym1, -sl[hp], -y0, -s0, v0, V1, V2, I.dxd, I.dyd,
                                           I.dtd);
            else
                hv = fd_hamiltonian<VH>(pxm, pxp, pym, pyp, sxm, sx, -sl[hp], -s0, v0, V1, V2, cx, cy);
        } else if constexpr (kF64) {
            hv = numerical_hamiltonian_ieee<VH>(pxm, pxp, pym, pyp, v0, V1, V2);
        } else {
            hv = numerical_hamiltonian<VH>(pxm, pxp, pym, pyp, v0, V1, V2);
        }
        const R hr = from_right(hv);
        const R hprev = hh[hp];
        hh[h] = hv;
        if constexpr (HSUM) hacc += (out_col && it < nrows) ? hv : R(0);

        {   // x-edge (j+1/2, k): d(alpha_12)/dt = -(Hhat_{j+1} - Hhat_j)/dx; not on the extra row
            R nv;
            const R from = MODE == MODE_MID2 ? b12 : wx;   // the state the stage adds to
            if constexpr (kF64 && kFD) nv = from + (hr - hv) / I.dxd;   // differences of the increments
            else if constexpr (kF64) nv = from + I.dtd * (-(hr - hv) / I.dxd);
            else nv = madd(-cx, hr - hv, from);
            if constexpr (MODE == MODE_HEUN2) nv = madd(R(0.5), b12, R(0.5) * nv);
            put(row_ptr<S>(d12, k, nx, it < nrows), off_st, S(nv));
        }
        {   // y-edge (j, k-1/2): d(alpha_11)/dt = (Hhat_k - Hhat_{k-1})/dy; from the second row on
            R nv;
            const R from = MODE == MODE_MID2 ? b11 : ym1;
            if constexpr (kF64 && kFD) nv = from - (hv - hprev) / I.dyd;
            else if constexpr (kF64) nv = from + I.dtd * ((hv - hprev) / I.dyd);
            else nv = madd(cy, hv - hprev, from);
            if constexpr (MODE == MODE_HEUN2) nv = madd(R(0.5), b11, R(0.5) * nv);
            put(row_ptr<S>(d11, kprev, nx, it > 0), off_st, S(nv));
        }
        kprev = k;
        k = next_row(k, ny);
    };

    // it runs 0 .. nrows (one extra row: the Hhat row below the tile)
    for (int it = 0;; it += 8) {
        body(it, Phase<0>{});
        if (it + 1 > nrows) break;
        body(it + 1, Phase<1>{});
        if (it + 2 > nrows) break;
        body(it + 2, Phase<2>{});
        if (it + 3 > nrows) break;
        body(it + 3, Phase<3>{});
        if (it + 4 > nrows) break;
        body(it + 4, Phase<4>{});
        if (it + 5 > nrows) break;
        body(it + 5, Phase<5>{});
        if (it + 6 > nrows) break;
        body(it + 6, Phase<6>{});
        if (it + 7 > nrows) break;
        body(it + 7, Phase<7>{});
        if (it + 8 > nrows) break;
    }
    if constexpr (HSUM) {
        // fixed-order wave reduction in FP64, one partial per tile
        double v = (double)hacc;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) I.hsum[(int64_t)chunk * I.strips + strip] = v;
    }
}

// ------------------------------------------------------------ fused Heun
//
// Both Heun stages in one pass (float only, semi-discrete scheme): each wave
// runs the first stage three node rows ahead of the second and keeps the
// first stage's densities in registers, so a step reads the state (and the
// celerity field) once and writes the new state once -- 8 B per node in and
// out instead of 20 and 28 for the two unfused launches.  The second stage
// needs first-stage values two lanes and two rows beyond its outputs, so a
// wave owns 56 output columns (4 halo lanes on each side) and the first
// stage runs two rows above the tile and two (plus one unused) below.  Every value is computed with the
// same operations as in the unfused kernels (same node function, same
// updates), so the result is the same bit for bit.  Reads src, writes dst
// (distinct buffers: neighbouring tiles still read src).
constexpr int kFStrip = kFusedStrip, kFHalo = 4;
// The fused kernel's loads run kFAhead rows ahead of stage A (at most five:
// A's alpha_11 ring holds rows m-1 .. m+kFAhead+1 in eight slots).
constexpr int kFAhead = 2;
static_assert(kFAhead >= 1 && kFAhead <= 5, "fused look-ahead must fit the eight-slot rings");

template <int LK, int VK, bool FIELD, bool MID = false>
__device__ __forceinline__ void run_tile_fused(const InstDev &I, int strip, int chunk, int lane, const void *src11,
                                               const void *src12, void *dst11, void *dst12)
{
    using R = float;
    using S = float;
    const int nx = I.nx, ny = I.ny;
    const R theta = I.theta, cx = I.cx, cy = I.cy;
    // explicit midpoint: stage A advances half a step (halving is exact)
    const R cxa = MID ? 0.5f * cx : cx, cya = MID ? 0.5f * cy : cy;
    const R V1 = I.V1, V2 = I.V2;

    const int gcol = strip * kFStrip - kFHalo + lane;
    int col = gcol % nx;
    if (col < 0) col += nx;
    const uint32_t off = (uint32_t)col * 4u;
    const bool out_col = lane >= kFHalo && lane < kFHalo + kFStrip && gcol < nx;
    const int k0 = chunk * I.rows;
    const int nrows = min(I.rows, ny - k0);
    const uint32_t off_st = out_col ? off : kSkip;

    // Iteration i: the first stage ("A") at node row m = k0 - 2 + i, for
    // i = 0 .. nrows + 5, and, from i = 5 on, the second stage ("B") at node
    // row k = m - 3 (k0 .. k0 + nrows).  B lags A by three rows, one more
    // than its stencil needs, so that it reads only what A produced on
    // earlier iterations: the two node evaluations of an iteration are
    // independent and the compiler can interleave their instructions.  The
    // last iteration evaluates A on one row more than B needs, from loads
    // the range check has zeroed; nothing reads those results.  Ring slots
    // (mA0 = k0 - 2): input alpha_11 of row mA0 + j in y[j & 7] (A reads rows
    // m-1 .. m+1, loads run to m+kFAhead+1), input alpha_12 and v0 of row
    // mA0 + j in slot j & 7 (A row m, loads to m+kFAhead); for B, A's outputs
    // alpha_12 and alpha_11 of row mA0 + j in wxo[j & 3] and wyo[j & 3]
    // (written on iterations j and j + 1) and the step's initial alpha_11,
    // alpha_12 and v0 of that row in b11_[j & 3], b12_[j & 3], vb_[j & 3]
    // (copied from A's operands).
    S y[8], wx_[8], wxo[4], wyo[4], b11_[4], b12_[4];
    float v0_[8], vb_[4];
    R slA[2], hhA[2], slB[2], hhB[2];
    for (int j = 0; j < 8; ++j) v0_[j] = 0.0f;
    for (int j = 0; j < 4; ++j) vb_[j] = 0.0f;

    int k = (k0 - 4) % ny;   // A starts at node row mA0 = k0 - 2
    if (k < 0) k += ny;
    const R ym2 = R(at(row_ptr<S>(src11, k, nx), off));
    k = next_row(k, ny);
    y[7] = at(row_ptr<S>(src11, k, nx), off);
    int kf = next_row(k, ny);   // row of the next alpha_12 / v0 fetch
    y[0] = at(row_ptr<S>(src11, kf, nx), off);
    slA[1] = limited_slope<LK>(ym2, R(y[7]), R(y[0]), theta);
    hhA[1] = R(0);
    float ydmA = float(R(y[0]) - R(y[7]));
    float ydmsA = LK == LK_SUPERBEE ? 2.0f * ydmA : float(theta) * ydmA;
    float ydmB = 0.0f, ydmsB = 0.0f;   // set after the first five iterations

    const int lastA = nrows + 4;   // A's last row that B needs
    const int last = nrows + 5;    // B's last iteration
#pragma unroll
    for (int j = 0; j < kFAhead; ++j) {
        const int kf1 = next_row(kf, ny);
        wx_[j] = at(row_ptr<S>(src12, kf, nx), off);
        y[j + 1] = at(row_ptr<S>(src11, kf1, nx), off);
        if constexpr (FIELD) v0_[j] = at(row_ptr<float>(I.v0f, kf, nx), off);
        kf = kf1;
    }
    int kf1 = next_row(kf, ny);
    int kB = k0, kBprev = k0 == 0 ? ny - 1 : k0 - 1;   // B's node row and the row above it

    // The node function of both stages: Steps 1-4 at one node from the
    // alpha_11 rows above/at/below and alpha_12 of the row, with the y slope
    // carried from the previous row (as in run_tile); slhp is the slope of
    // the row above, s0 receives this row's.  T is float (one node) or F2
    // (the two stages' nodes of an iteration in lock step).
    auto node = [&](auto ym1, auto y0, auto yp1, auto wx, auto v0, auto slhp, auto &s0, auto &ydm, auto &ydms) {
        using T = decltype(ym1);
        s0 = y_slope_carried<LK>(ym1, y0, yp1, T(theta), ydm, ydms);
        const T pyp = -madd(T(-0.5f), s0, y0);
        const T pym = -madd(T(0.5f), slhp, ym1);
        const T wl = from_left(wx), wr = from_right(wx);
        const T sx = limited_slope<LK>(wl, wx, wr, T(theta));
        const T pxp = madd(T(-0.5f), sx, wx);
        const T pxm = from_left(madd(T(0.5f), sx, wx));
        return numerical_hamiltonian<VK>(pxm, pxp, pym, pyp, v0, T(V1), T(V2));
    };

    // A's outputs at ring phase p from its Hhat at row m and at the node to
    // the right: alpha_12 of row m and alpha_11 of row m-1 after stage 1.
    auto update_a = [&](auto phase, R hv, R hr, R wx, R ym1) {
        constexpr int p = decltype(phase)::value;
        constexpr int h = p & 1, hp = h ^ 1;
        const R hprev = hhA[hp];
        hhA[h] = hv;
        wxo[p & 3] = S(madd(-cxa, hr - hv, wx));
        wyo[(p + 3) & 3] = S(madd(cya, hv - hprev, ym1));
    };
    // B's outputs: alpha_12 of row kB and alpha_11 of the row above.  Heun:
    // the mean of the state and one more stage; midpoint: the state plus a
    // full step.
    auto update_b = [&](auto phase, int it, R hv, R hr, R wx, R ym1, R b12, R b11) {
        constexpr int p = decltype(phase)::value;
        constexpr int h = p & 1, hp = h ^ 1;
        const int bi = it - 5;
        const R hprev = hhB[hp];
        hhB[h] = hv;
        {
            R nv = madd(-cx, hr - hv, MID ? b12 : wx);
            if constexpr (!MID) nv = madd(R(0.5), b12, R(0.5) * nv);
            put(row_ptr<S>(dst12, kB, nx, bi < nrows), off_st, S(nv));
        }
        {
            R nv = madd(cy, hv - hprev, MID ? b11 : ym1);
            if constexpr (!MID) nv = madd(R(0.5), b11, R(0.5) * nv);
            put(row_ptr<S>(dst11, kBprev, nx, bi > 0), off_st, S(nv));
        }
        kBprev = kB;
        kB = next_row(kB, ny);
    };
    // A's operands at ring phase p, and the loads of its row m + kFAhead
    // (none past A's last useful row); the step's initial state of row m
    // (and of row m-1 for alpha_11) is kept for B.
    auto operands_a = [&](int it, auto phase, R &ym1, R &y0, R &yp1, R &wx, R &v0) {
        constexpr int p = decltype(phase)::value;
        ym1 = R(y[(p + 7) & 7]);
        y0 = R(y[p]);
        yp1 = R(y[(p + 1) & 7]);
        wx = R(wx_[p]);
        v0 = FIELD ? R(v0_[p]) : R(I.v0);
        b11_[(p + 3) & 3] = y[(p + 7) & 7];
        b12_[p & 3] = wx_[p];
        if constexpr (FIELD) vb_[p & 3] = v0_[p];
        const bool live = it + kFAhead <= lastA;
        wx_[(p + kFAhead) & 7] = at(row_ptr<S>(src12, kf, nx, live), off);
        y[(p + kFAhead + 1) & 7] = at(row_ptr<S>(src11, kf1, nx, live), off);
        if constexpr (FIELD) v0_[(p + kFAhead) & 7] = at(row_ptr<float>(I.v0f, kf, nx, live), off);
        kf = kf1;
        kf1 = next_row(kf1, ny);
    };

    // Stage A alone on iteration it (ring phase p = it & 7).
    auto stage_a = [&](int it, auto phase) {
        constexpr int p = decltype(phase)::value;
        constexpr int h = p & 1, hp = h ^ 1;
        R ym1, y0, yp1, wx, v0;
        operands_a(it, phase, ym1, y0, yp1, wx, v0);
        const R hv = node(ym1, y0, yp1, wx, v0, slA[hp], slA[h], ydmA, ydmsA);
        update_a(phase, hv, from_right(hv), wx, ym1);
    };

    // A alone on rows k0-2 .. k0+2 (iterations 0 .. 4).
    stage_a(0, Phase<0>{});
    stage_a(1, Phase<1>{});
    stage_a(2, Phase<2>{});
    stage_a(3, Phase<3>{});
    stage_a(4, Phase<4>{});
    // B's carried y slope at row k0-1, from stage-1 rows k0-2 .. k0 (slots
    // 0 .. 2), in the slot its first iteration (phase 5) reads.
    {
        const R a = R(wyo[0]), b = R(wyo[1]), c = R(wyo[2]);
        slB[0] = limited_slope<LK>(a, b, c, theta);
        ydmB = float(c - b);
        ydmsB = LK == LK_SUPERBEE ? 2.0f * ydmB : float(theta) * ydmB;
        hhB[0] = R(0);
    }
    // Iterations from 5 on: A at row m and B at row kB = m - 3, their node
    // evaluations in lock step (independent: B reads what A wrote on
    // earlier iterations).
    auto body = [&](int it, auto phase) {
        constexpr int p = decltype(phase)::value;
        constexpr int h = p & 1, hp = h ^ 1;
        R ym1a, y0a, yp1a, wxa, v0a;
        operands_a(it, phase, ym1a, y0a, yp1a, wxa, v0a);
        const R ym1b = R(wyo[p & 3]), y0b = R(wyo[(p + 1) & 3]), yp1b = R(wyo[(p + 2) & 3]);
        const R wxb = R(wxo[(p + 1) & 3]);
        const R v0b = FIELD ? R(vb_[(p + 1) & 3]) : R(I.v0);
        const R b12 = R(b12_[(p + 1) & 3]), b11 = R(b11_[p & 3]);   // the step's initial state
        F2 s0, ydm(ydmA, ydmB), ydms(ydmsA, ydmsB);
        const F2 hv = node(F2(ym1a, ym1b), F2(y0a, y0b), F2(yp1a, yp1b), F2(wxa, wxb), F2(v0a, v0b),
                           F2(slA[hp], slB[hp]), s0, ydm, ydms);
        slA[h] = s0.a;
        slB[h] = s0.b;
        ydmA = ydm.a;
        ydmsA = ydms.a;
        ydmB = ydm.b;
        ydmsB = ydms.b;
        const F2 hr = from_right(hv);
        update_a(phase, hv.a, hr.a, wxa, ym1a);
        update_b(phase, it, hv.b, hr.b, wxb, ym1b, b12, b11);
    };
    for (int it = 5;; it += 8) {
        body(it, Phase<5>{});
        if (it + 1 > last) break;
        body(it + 1, Phase<6>{});
        if (it + 2 > last) break;
        body(it + 2, Phase<7>{});
        if (it + 3 > last) break;
        body(it + 3, Phase<0>{});
        if (it + 4 > last) break;
        body(it + 4, Phase<1>{});
        if (it + 5 > last) break;
        body(it + 5, Phase<2>{});
        if (it + 6 > last) break;
        body(it + 6, Phase<3>{});
        if (it + 7 > last) break;
        body(it + 7, Phase<4>{});
        if (it + 8 > last) break;
    }
}

// Tiles are numbered row band first (tile = chunk * strips + strip), so
// consecutive waves -- the four of a block, and neighbouring blocks -- are
// side-by-side strips walking the same rows at the same time: the 128-byte
// lines shared at strip edges are fetched once and hit in cache for the
// neighbour.  Hardware places block b on XCD b % 8; each XCD gets a
// contiguous run of tiles, i.e. a band of rows across the grid.
__device__ __forceinline__ int64_t xcd_tile(int blocks_per_xcd)
{
    const int b = blockIdx.x;
    const int64_t logical = (int64_t)(b & 7) * blocks_per_xcd + (b >> 3);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    return logical * kWavesPerBlock + wave;
}

template <typename R, typename S, int LK, int VK, bool FIELD, int MODE, bool HSUM = false>
__global__ __launch_bounds__(kBlock) void stage_kernel(InstDev I, int64_t total_tiles, int blocks_per_xcd, int half)
{
    const int64_t tile = xcd_tile(blocks_per_xcd);
    if (tile >= total_tiles) return;
    const int t = (int)tile;
    run_tile<R, S, LK, VK, FIELD, MODE, HSUM>(I, t % I.strips, t / I.strips, threadIdx.x & 63, half);
}

// Batched: one launch for every tile of every instance; tile_inst maps a
// global tile to its instance.  Limiter, Hamiltonian and field presence are
// per instance and uniform over a wave.
template <typename R, typename S, int MODE, bool FD>
__global__ __launch_bounds__(kBlock) void stage_kernel_batched(const InstDev *__restrict__ insts,
                                                               const int32_t *__restrict__ tile_inst,
                                                               int64_t total_tiles, int blocks_per_xcd, int half)
{
    const int64_t tile = xcd_tile(blocks_per_xcd);
    if (tile >= total_tiles) return;
    const InstDev I = insts[tile_inst[tile]];
    const int local = (int)(tile - I.tile_begin);
    const int strip = local % I.strips, chunk = local / I.strips;
    const int lane = threadIdx.x & 63;
    with_limiter<sizeof(R) == 4>(I.limiter, [&](auto t) {
        constexpr int L = decltype(t)::value;
        if constexpr (FD) {
            if (I.vkind == VK_PRESCRIBED_FD) run_tile<R, S, L, VK_PRESCRIBED_FD, false, MODE>(I, strip, chunk, lane, half);
            else if (I.v0f != nullptr) run_tile<R, S, L, VK_LAW_FD, true, MODE>(I, strip, chunk, lane, half);
            else run_tile<R, S, L, VK_LAW_FD, false, MODE>(I, strip, chunk, lane, half);
        } else {
            if (I.vkind == VK_PRESCRIBED) run_tile<R, S, L, VK_PRESCRIBED, false, MODE>(I, strip, chunk, lane, half);
            else if (I.v0f != nullptr) run_tile<R, S, L, VK_LAW, true, MODE>(I, strip, chunk, lane, half);
            else run_tile<R, S, L, VK_LAW, false, MODE>(I, strip, chunk, lane, half);
        }
    });
}

template <typename R, typename S, int LK, int VK, bool FIELD, bool HSUM = false>
hipError_t launch_stage_t(const InstDev &I, int mode, hipStream_t s)
{
    const int64_t tiles = (int64_t)I.strips * I.chunks;
    const int64_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_xcd = (int)((blocks + 7) / 8);
    const dim3 grid(8 * per_xcd), block(kBlock);
    if constexpr ((VK & VK_FD) != 0) {   // one pass per step: forward and backward ping-pong only
        if (mode == MODE_FWD)
            hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_FWD, HSUM>), grid, block, 0, s, I, tiles,
                               per_xcd, 0);
        else if (mode == MODE_BWD)
            hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_BWD, HSUM>), grid, block, 0, s, I, tiles,
                               per_xcd, 0);
        else
            return hipErrorInvalidValue;
    } else {
        if (mode == MODE_FWD || mode == MODE_MID1)
            hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_FWD, HSUM>), grid, block, 0, s, I, tiles,
                               per_xcd, mode == MODE_MID1 ? 1 : 0);
        else if (mode == MODE_BWD)
            hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_BWD, HSUM>), grid, block, 0, s, I, tiles,
                               per_xcd, 0);
        else if (mode == MODE_MID2)
            hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_MID2, HSUM>), grid, block, 0, s, I, tiles,
                               per_xcd, 0);
        else
            hipLaunchKernelGGL((stage_kernel<R, S, LK, VK, FIELD, MODE_HEUN2, HSUM>), grid, block, 0, s, I, tiles,
                               per_xcd, 0);
    }
    return hipGetLastError();
}

// Fused Heun step: dir 0 reads the state and writes the stage buffer, dir 1
// the other way round.
template <int LK, int VK, bool FIELD, bool MID>
__global__ __launch_bounds__(kBlock) void fused_kernel(InstDev I, int64_t total_tiles, int blocks_per_xcd,
                                                       int strips, int dir)
{
    const int64_t tile = xcd_tile(blocks_per_xcd);
    if (tile >= total_tiles) return;
    const int t = (int)tile;
    const void *s11 = dir ? I.w11 : I.a11, *s12 = dir ? I.w12 : I.a12;
    void *d11 = dir ? I.a11 : I.w11, *d12 = dir ? I.a12 : I.w12;
    run_tile_fused<LK, VK, FIELD, MID>(I, t % strips, t / strips, threadIdx.x & 63, s11, s12, d11, d12);
}

// Batched fused step: one launch for the fused tiles of every instance;
// limiter, Hamiltonian and field presence are per instance (wave-uniform).
template <int DIR, bool MID>
__global__ __launch_bounds__(kBlock) void fused_kernel_batched(const InstDev *__restrict__ insts,
                                                               const int32_t *__restrict__ tile_inst,
                                                               int64_t total_tiles, int blocks_per_xcd)
{
    const int64_t tile = xcd_tile(blocks_per_xcd);
    if (tile >= total_tiles) return;
    const InstDev I = insts[tile_inst[tile]];
    const int local = (int)(tile - I.tile_begin);
    const int strip = local % I.fstrips, chunk = local / I.fstrips;
    const int lane = threadIdx.x & 63;
    const void *s11 = DIR ? I.w11 : I.a11, *s12 = DIR ? I.w12 : I.a12;
    void *d11 = DIR ? I.a11 : I.w11, *d12 = DIR ? I.a12 : I.w12;
    with_limiter<true>(I.limiter, [&](auto t) {
        constexpr int L = decltype(t)::value;
        if (I.vkind == VK_PRESCRIBED) run_tile_fused<L, VK_PRESCRIBED, false, MID>(I, strip, chunk, lane, s11, s12, d11, d12);
        else if (I.v0f != nullptr) run_tile_fused<L, VK_LAW, true, MID>(I, strip, chunk, lane, s11, s12, d11, d12);
        else run_tile_fused<L, VK_LAW, false, MID>(I, strip, chunk, lane, s11, s12, d11, d12);
    });
}

template <int LK, int VK, bool FIELD, bool MID>
hipError_t launch_fused_t(const InstDev &I, int dir, hipStream_t s)
{
    const int strips = (I.nx + kFStrip - 1) / kFStrip;
    const int64_t tiles = (int64_t)strips * tiles_along_y(I.ny, I.rows);
    const int64_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_xcd = (int)((blocks + 7) / 8);
    hipLaunchKernelGGL((fused_kernel<LK, VK, FIELD, MID>), dim3(8 * per_xcd), dim3(kBlock), 0, s, I, tiles, per_xcd,
                       strips, dir);
    return hipGetLastError();
}

// Dispatch of one instance's stage launch over limiter, Hamiltonian and
// scheme, field presence, and the coupled runs' per-tile sums of Hhat.
template <typename R, typename S>
hipError_t launch_stage_r(const InstDev &I, int mode, hipStream_t s)
{
    return with_limiter<sizeof(R) == 4>(I.limiter, [&](auto t) -> hipError_t {
        constexpr int L = decltype(t)::value;
        const bool field = I.v0f != nullptr, hsum = I.hsum != nullptr;
        switch (I.vkind) {
        case VK_PRESCRIBED: return launch_stage_t<R, S, L, VK_PRESCRIBED, false>(I, mode, s);
        case VK_PRESCRIBED_FD: return launch_stage_t<R, S, L, VK_PRESCRIBED_FD, false>(I, mode, s);
        case VK_LAW_FD:
            if (field && hsum) return launch_stage_t<R, S, L, VK_LAW_FD, true, true>(I, mode, s);
            if (field) return launch_stage_t<R, S, L, VK_LAW_FD, true>(I, mode, s);
            return launch_stage_t<R, S, L, VK_LAW_FD, false>(I, mode, s);
        default:
            if (field && hsum) return launch_stage_t<R, S, L, VK_LAW, true, true>(I, mode, s);
            if (field) return launch_stage_t<R, S, L, VK_LAW, true>(I, mode, s);
            return launch_stage_t<R, S, L, VK_LAW, false>(I, mode, s);
        }
    });
}

template <typename R, typename S>
hipError_t launch_batched_r(const InstDev *d_inst, const int32_t *d_tile_inst, int64_t total_tiles, int mode,
                            bool fd, hipStream_t s)
{
    const int64_t blocks = (total_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per_xcd = (int)((blocks + 7) / 8);
    const dim3 grid(8 * per_xcd), block(kBlock);
    if (fd) {   // its own kernels, so the semi-discrete ones keep their register budget
        if (mode == MODE_FWD)
            hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_FWD, true>), grid, block, 0, s, d_inst, d_tile_inst,
                               total_tiles, per_xcd, 0);
        else if (mode == MODE_BWD)
            hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_BWD, true>), grid, block, 0, s, d_inst, d_tile_inst,
                               total_tiles, per_xcd, 0);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (mode == MODE_FWD || mode == MODE_MID1)
        hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_FWD, false>), grid, block, 0, s, d_inst, d_tile_inst,
                           total_tiles, per_xcd, mode == MODE_MID1 ? 1 : 0);
    else if (mode == MODE_BWD)
        hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_BWD, false>), grid, block, 0, s, d_inst, d_tile_inst,
                           total_tiles, per_xcd, 0);
    else if (mode == MODE_MID2)
        hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_MID2, false>), grid, block, 0, s, d_inst, d_tile_inst,
                           total_tiles, per_xcd, 0);
    else
        hipLaunchKernelGGL((stage_kernel_batched<R, S, MODE_HEUN2, false>), grid, block, 0, s, d_inst, d_tile_inst,
                           total_tiles, per_xcd, 0);
    return hipGetLastError();
}

}  // namespace
}  // namespace fdm
