// fdm_host.hip -- host-side validation and set-up shared by the C-ABI entry
// points (declarations in fdm_host.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "fdm_host.h"

namespace fdm {
namespace host {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Host-side validation of one descriptor (no HIP call).
std::string check_desc(const fdm_transport_desc &d)
{
    if (d.nx < 1 || d.ny < 1) return "nx and ny must be >= 1";
    if ((int64_t)d.nx * d.ny >= (int64_t)1 << 31) return "nx*ny must be < 2^31";
    if (d.nx >= 1 << 27) return "nx must be < 2^27 (a row of at most 1 GiB)";
    if (!finite_pos(d.dx) || !finite_pos(d.dy)) return "dx and dy must be finite and > 0";
    if (d.limiter < FDM_LIMITER_NONE || d.limiter > FDM_LIMITER_SUPERBEE) return "unknown limiter";
    if (d.limiter == FDM_LIMITER_THETA && !(d.theta >= 1.0 && d.theta <= 2.0))
        return "theta must lie in [1, 2]";
    if (d.time_order < 0 || d.time_order > 3) return "time_order must be 1, 2 or 3";
    if (d.scheme != FDM_SCHEME_SEMIDISCRETE && d.scheme != FDM_SCHEME_FULLY_DISCRETE) return "unknown scheme";
    if (d.scheme == FDM_SCHEME_FULLY_DISCRETE && d.time_order > 1)
        return "the fully discrete scheme is one pass per step: time_order must be 0 or 1";
    if (!(std::isfinite(d.dt) && d.dt >= 0.0 && d.dt <= (double)FLT_MAX))
        return "dt must be finite (as a float) and >= 0";
    if (d.dt == 0.0 && !(d.cfl > 0.0 && d.cfl <= 1.0)) return "cfl must lie in (0, 1]";
    if (d.velocity != FDM_VELOCITY_LAW && d.velocity != FDM_VELOCITY_PRESCRIBED)
        return "unknown velocity kind";
    // the kernels take velocities as float: they must stay finite there
    const auto float_finite = [](double v) { return std::isfinite(v) && std::fabs(v) <= (double)FLT_MAX; };
    if (d.velocity == FDM_VELOCITY_LAW && d.v0_field == nullptr && !float_finite(d.v0))
        return "v0 must be finite (as a float)";
    if (d.velocity == FDM_VELOCITY_PRESCRIBED && !(float_finite(d.V[0]) && float_finite(d.V[1])))
        return "V must be finite (as a float)";
    return "";
}

// Largest float not above x (x > 0).
float round_down_float(double x)
{
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, 0.0f);
    return f;
}

// Stability bound of the step.  nu2 = dt (S1/dx + S2/dy) is the sum of the
// per-axis Courant numbers, S_i a bound on |dH/dp_i| over the grid (LAW:
// max |v0| on both axes, since |p_i| <= |p|; PRESCRIBED: |V_i|); an axis of
// one node has no differences along it and adds nothing.  Beyond nu2 = 1 the
// first-order upwind stage no longer writes each new value as a convex
// combination of old ones and is unstable in 2-D.  One forward-Euler stage
// with a limiter (time_order 1, or the fully discrete scheme) is held to
// nu2 <= 1/2, the bound of a limited (MUSCL) forward-Euler step; the paper's
// runs (Courant number 0.25 per axis, sec. 4.3-4.4) sit at exactly 1/2.
double courant_sum(const fdm_transport_desc &d, double dt, double smax_law)
{
    const double ax = d.nx > 1 ? 1.0 : 0.0, ay = d.ny > 1 ? 1.0 : 0.0;
    double s1 = smax_law, s2 = smax_law;
    if (d.velocity == FDM_VELOCITY_PRESCRIBED) {
        s1 = std::fabs((double)(float)d.V[0]);
        s2 = std::fabs((double)(float)d.V[1]);
    }
    return dt * (s1 / d.dx * ax + s2 / d.dy * ay);
}

double courant_limit(const fdm_transport_desc &d, int32_t order)
{
    return (order == 1 && d.limiter != FDM_LIMITER_NONE) ? 0.5 : 1.0;
}

// nu2 of the step a descriptor implies: a fixed dt with the given max |v0|
// (LAW), or the CFL-controlled step, for which dt max|v0| <= cfl min(dx, dy)
// whatever the celerity (LAW) and dt follows from V (PRESCRIBED).
double step_courant(const fdm_transport_desc &d, double smax_law)
{
    const double h = std::min(d.dx, d.dy);
    if (d.dt > 0.0) return courant_sum(d, (double)(float)d.dt, smax_law);
    if (d.velocity == FDM_VELOCITY_LAW) return courant_sum(d, d.cfl * h, 1.0);
    const double smax =
        std::max(std::fabs((double)(float)d.V[0]) / d.dx, std::fabs((double)(float)d.V[1]) / d.dy) * h;
    return courant_sum(d, (double)round_down_float(smax > 0.0 ? d.cfl * h / smax : d.cfl * h), 0.0);
}

// "" if the step is within the bound, else the reason.
std::string check_courant(const fdm_transport_desc &d, int32_t order, double smax_law)
{
    const double nu2 = step_courant(d, smax_law), lim = courant_limit(d, order);
    if (nu2 <= lim * (1.0 + 1e-12)) return "";
    char buf[256];
    std::snprintf(buf, sizeof(buf),
                  "dt (S1/dx + S2/dy) = %.6g exceeds %.3g (%s); lower %s", nu2, lim,
                  lim < 1.0 ? "one forward-Euler stage with a limiter" : "the 2-D Courant bound",
                  d.dt > 0.0 ? "dt" : "cfl");
    return buf;
}

// Rows per wave tile.  Each tile recomputes one extra row of Hhat and
// re-reads a few boundary rows, so long tiles are cheaper per row; but the
// launch should give every SIMD about six waves (6144 on 256 CUs x 4 SIMDs)
// to hide memory latency.  `strip_rows` is the number of (strip, row) pairs
// the launch covers (over all instances of a batched launch).  The result
// is that count / 6144 rounded up to a multiple of 4 and kept in [4, 16]
// (1024^2: 4 rows, 2048^2: 12, larger grids: 16).  The autotuner times
// fixed and SIMD-balanced heights beside it.
int pick_rows(int64_t strip_rows, int ny, int requested)
{
    if (requested > 0) return std::min(requested, ny);
    const int64_t target_waves = 256 * 4 * 6;
    int64_t rows = (strip_rows + target_waves - 1) / target_waves;
    rows = (rows + 3) / 4 * 4;
    // capped at 16: taller tiles lose on large grids (measured at 8192^2:
    // 32 rows 1.14e11, 16 rows 1.22e11, 4 rows 1.31e11 cell-updates/s; the
    // autotuner finds the last)
    rows = std::max<int64_t>(4, std::min<int64_t>(16, rows));
    return (int)std::min<int64_t>(rows, ny);
}

int64_t strip_rows_of(const fdm_transport_desc &d)
{
    return (int64_t)((d.nx + kStrip - 1) / kStrip) * d.ny;
}

double smax_uniform(const fdm_transport_desc &d)
{
    const double h = std::min(d.dx, d.dy);
    if (d.velocity == FDM_VELOCITY_PRESCRIBED)   // the float32 velocity the kernels use
        return std::max(std::fabs((double)(float)d.V[0]) / d.dx, std::fabs((double)(float)d.V[1]) / d.dy) * h;
    return std::fabs((double)(float)d.v0);
}

float step_dt(const fdm_transport_desc &d, double smax)
{
    if (d.dt > 0.0) return (float)d.dt;
    const double h = std::min(d.dx, d.dy);
    return round_down_float(smax > 0.0 ? d.cfl * h / smax : d.cfl * h);
}

void fill_inst(InstDev &I, const fdm_transport_desc &d, float dt, void *w11, void *w12)
{
    std::memset(&I, 0, sizeof(I));
    I.w11 = w11;
    I.w12 = w12;
    I.v0f = d.velocity == FDM_VELOCITY_LAW ? d.v0_field : nullptr;
    I.nx = d.nx;
    I.ny = d.ny;
    I.v0 = (float)d.v0;
    I.V1 = (float)d.V[0];
    I.V2 = (float)d.V[1];
    I.dtd = (double)dt;
    I.dxd = d.dx;
    I.dyd = d.dy;
    I.cxd = (double)dt / d.dx;
    I.cyd = (double)dt / d.dy;
    I.thetad = d.limiter == FDM_LIMITER_MINMOD ? 1.0 : d.limiter == FDM_LIMITER_MC ? 2.0 : d.theta;
    I.cx = (float)I.cxd;
    I.cy = (float)I.cyd;
    I.theta = (float)I.thetad;
    I.limiter = d.limiter;
    I.vkind = d.velocity | (d.scheme == FDM_SCHEME_FULLY_DISCRETE ? VK_FD : 0);
}

int stage_modes(int32_t order, int32_t step, int modes[2])
{
    if (order == 2) {
        modes[0] = MODE_FWD;
        modes[1] = MODE_HEUN2;
        return 2;
    }
    if (order == 3) {
        modes[0] = MODE_MID1;
        modes[1] = MODE_MID2;
        return 2;
    }
    modes[0] = (step & 1) ? MODE_BWD : MODE_FWD;
    return 1;
}

}  // namespace host
}  // namespace fdm
