// fdm_api.hip -- C ABI (include/fdm.h) of the gfx950 transport hot path.
//
// Host-side responsibilities: validate descriptors before any HIP call,
// compute the CFL-bounded step from max |v0| (a device reduction for a
// celerity field), own the per-instance stage buffers and reduction
// scratch, sequence the stage launches (two per Heun step, or one fused
// launch), replay captured HIP graphs for fdm_run, and keep a sticky error
// per context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fdm.h"
#include "fdm_host.h"
#include "fdm_internal.h"
#include "fdm_static.h"

using fdm::InstDev;
using namespace fdm::host;

struct fdm_ctx {
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;          // private stream for graph capture
    int32_t n = 0;
    int32_t time_order = 2;
    bool fd = false;   // fully discrete scheme (one pass per step)
    int32_t schedule = FDM_SCHEDULE_AUTO;
    int32_t precision = FDM_PRECISION_FP32;
    bool batched = false;
    bool fused = false;                     // fused two-stage Heun launches
    std::vector<fdm_transport_desc> desc;
    std::vector<InstDev> inst;              // host copies of the device views
    std::vector<float> dt;                  // float32 step per instance
    void *workspace = nullptr;              // all stage buffers
    InstDev *d_inst = nullptr;              // batched: device table
    InstDev *h_inst_pinned = nullptr;       // staging for table uploads
    int32_t *d_tile_inst = nullptr;         // batched: tile -> instance
    int64_t total_tiles = 0;
    fdm::StatsPartial *d_partials = nullptr;
    double *d_stats = nullptr;              // 5 doubles per instance
    double *h_stats = nullptr;              // pinned copy
    float *d_absmax = nullptr;
    bool table_valid = false;
    bool have_ref = false;
    std::vector<double> ref11, ref12;
    int64_t steps = 0;
    // graph cache for fdm_run
    hipGraphExec_t graph = nullptr;
    int32_t graph_steps = 0;
    std::vector<void *> graph_a11, graph_a12;
    std::vector<double> t_acc;              // simulated time per instance
    std::vector<float> dt_last;             // step last used per instance
    // coupled runs (single instance)
    struct {
        fdm::StaticPlan *plan = nullptr;
        fdm::StaticParams q{};
        void *tau = nullptr;                // nx*ny, state type
        void *phi = nullptr;                // nx*ny, state type (wiggly law)
        float *v0 = nullptr;                // nx*ny celerity of the run
        double *d_hsum = nullptr;           // per-tile sums of Hhat, two stages
        int64_t cap = 0;                    // tiles per stage the sums hold
        fdm::CoupledDev *d_cd = nullptr;    // step scalars on the device
        fdm::CoupledDev *h_cd = nullptr;    // pinned mirror
        double eps13 = 0.0, sigma13 = 0.0, phi_mean = 0.0, vmax = 0.0;
        bool no_graph = false;              // a chunk could not be captured as kernels only
    } cw;
    size_t elem = sizeof(float);            // bytes per state value
    int64_t tile_capacity = 0;              // entries of d_tile_inst
    int32_t requested_rows = 0;             // tile rows asked for (0: default rule)
    int64_t simds = 1024;                   // SIMDs of the device (4 per compute unit)
    bool sticky = false;
    std::string err;
};

namespace {

thread_local std::string g_init_error;

}  // namespace

void fdm::host::set_init_error(const std::string &msg) { g_init_error = msg; }

namespace {

fdm_status fail(fdm_ctx *c, fdm_status st, const std::string &msg)
{
    if (c) {
        c->err = msg;
        if (st == FDM_ERR_DEVICE) c->sticky = true;
    } else {
        g_init_error = msg;
    }
    return st;
}

#define FDM_HIP(ctx, call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            return fail((ctx), e_ == hipErrorOutOfMemory ? FDM_ERR_OUT_OF_MEMORY : FDM_ERR_DEVICE, \
                        std::string(#call) + ": " + hipGetErrorString(e_));                  \
        }                                                                                   \
    } while (0)

// A whole number of voxels: v / d within 1e-9 of an integer >= 1.
bool whole_voxels(double v, double d, int *out)
{
    if (!(std::isfinite(v) && v > 0.0)) return false;
    const double r = v / d, k = std::round(r);
    if (!(k >= 1.0 && k < 2147483647.0) || std::fabs(r - k) > 1e-9 * k) return false;
    *out = (int)k;
    return true;
}

// Host-side validation of a static descriptor; fills the internal parameters.
std::string check_static(const fdm_static_desc &d, fdm::StaticParams *q)
{
    if (d.nx < 1 || d.ny < 1) return "nx and ny must be >= 1";
    if ((int64_t)d.nx * d.ny >= (int64_t)1 << 31) return "nx*ny must be < 2^31";
    if (!finite_pos(d.dx) || !finite_pos(d.dy)) return "dx and dy must be finite and > 0";
    if (d.dx != d.dy) return "dx must equal dy (cubic voxels)";
    if (!finite_pos(d.mu)) return "mu must be finite and > 0";
    if (!(std::isfinite(d.lambda) && 3.0 * d.lambda + 2.0 * d.mu > 0.0))
        return "lambda must be finite with 3 lambda + 2 mu > 0";
    int h = 0, n3 = 0;
    if (!whole_voxels(d.layer_h, d.dx, &h)) return "layer_h must be a whole number (>= 1) of voxels of size dx";
    if (!whole_voxels(d.cell_l3, d.dx, &n3)) return "cell_l3 must be a whole number (>= 1) of voxels of size dx";
    if (h > n3) return "layer_h must not exceed cell_l3";
    if (!std::isfinite(d.eps13) || !std::isfinite(d.phi_mean)) return "eps13 and phi_mean must be finite";
    if (d.precision < FDM_PRECISION_FP32 || d.precision > FDM_PRECISION_FP64) return "unknown precision";
    if (d.reserved != 0) return "reserved must be 0";
    *q = fdm::StaticParams{d.nx, d.ny, d.dx, d.dy, d.mu, d.lambda, h, n3, d.precision == FDM_PRECISION_FP64};
    return "";
}

double static_mean_stress(const fdm_static_desc &d, const fdm::StaticParams &q)
{
    return 2.0 * d.mu * d.eps13 - d.mu * d.phi_mean * (double)q.h / (double)q.n3;
}

// Tiles (one wave64 each) of one launch: a dispatch holds fewer than 2^32
// work-items, and the grid rounds the tile count up by at most 31.
constexpr int64_t kMaxLaunchTiles = (int64_t)1 << 25;

// Tallest balanced height the autotuner tries (one round of waves over a
// 8192^2 grid needs 149 rows).
constexpr int kMaxBalancedRows = 512;

// Waves (one per tile) of the largest launch a step makes with the given
// tile height: every instance's tiles for a batched launch, the largest
// instance's for one launch per instance.
int64_t launch_waves(const fdm_ctx *c, bool fused, bool batched, int rows)
{
    int64_t total = 0, largest = 0;
    for (const fdm_transport_desc &d : c->desc) {
        const int r = std::min(rows, d.ny);
        const int w = fused ? fdm::kFusedStrip : fdm::kStrip;
        const int64_t t = (int64_t)((d.nx + w - 1) / w) * fdm::tiles_along_y(d.ny, r);
        total += t;
        largest = std::max(largest, t);
    }
    return batched ? total : largest;
}

// Smallest tile height whose launch has at most `limit` waves, or -1 if even
// one tile per strip exceeds it.  launch_waves falls as the height grows.
int balanced_rows(const fdm_ctx *c, bool fused, bool batched, int max_ny, int64_t limit)
{
    if (launch_waves(c, fused, batched, max_ny) > limit) return -1;
    int lo = 1, hi = max_ny;
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (launch_waves(c, fused, batched, mid) <= limit) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

void release(fdm_ctx *c)
{
    if (!c) return;
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->workspace) (void)hipFree(c->workspace);
    if (c->d_inst) (void)hipFree(c->d_inst);
    if (c->d_tile_inst) (void)hipFree(c->d_tile_inst);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_stats) (void)hipFree(c->d_stats);
    if (c->d_absmax) (void)hipFree(c->d_absmax);
    if (c->h_stats) (void)hipHostFree(c->h_stats);
    if (c->h_inst_pinned) (void)hipHostFree(c->h_inst_pinned);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    fdm::static_plan_destroy(c->cw.plan);
    if (c->cw.tau) (void)hipFree(c->cw.tau);
    if (c->cw.phi) (void)hipFree(c->cw.phi);
    if (c->cw.v0) (void)hipFree(c->cw.v0);
    if (c->cw.d_hsum) (void)hipFree(c->cw.d_hsum);
    if (c->cw.d_cd) (void)hipFree(c->cw.d_cd);
    if (c->cw.h_cd) (void)hipHostFree(c->cw.h_cd);
    delete c;
}

fdm_status check_ptrs(fdm_ctx *c, void *const *a11, void *const *a12)
{
    if (!a11 || !a12) return fail(c, FDM_ERR_INVALID_ARG, "alpha11/alpha12 pointer arrays must not be NULL");
    for (int i = 0; i < c->n; ++i) {
        if (!a11[i] || !a12[i]) return fail(c, FDM_ERR_INVALID_ARG, "NULL density array for instance " + std::to_string(i));
        if (a11[i] == a12[i]) return fail(c, FDM_ERR_INVALID_ARG, "alpha11 and alpha12 alias for instance " + std::to_string(i));
    }
    return FDM_OK;
}

// Point the device views at this call's arrays; re-upload the batched table
// when they changed.
fdm_status bind(fdm_ctx *c, void *const *a11, void *const *a12)
{
    bool changed = !c->table_valid;
    for (int i = 0; i < c->n; ++i) {
        if (c->inst[i].a11 != a11[i] || c->inst[i].a12 != a12[i]) changed = true;
        c->inst[i].a11 = a11[i];
        c->inst[i].a12 = a12[i];
    }
    if (c->batched && changed) {
        // the staging buffer may still feed an earlier upload
        FDM_HIP(c, hipStreamSynchronize(c->stream));
        std::memcpy(c->h_inst_pinned, c->inst.data(), sizeof(InstDev) * c->n);
        FDM_HIP(c, hipMemcpyAsync(c->d_inst, c->h_inst_pinned, sizeof(InstDev) * c->n,
                                  hipMemcpyHostToDevice, c->stream));
    }
    c->table_valid = true;
    return FDM_OK;
}

// Enqueue n_steps on stream s for the bound arrays.
fdm_status enqueue_steps(fdm_ctx *c, int32_t n_steps, hipStream_t s)
{
    if (c->fused) {   // both Heun stages per launch, ping-pong between the state and the stage buffer
        for (int32_t step = 0; step < n_steps; ++step) {
            if (c->batched)
                FDM_HIP(c, fdm::launch_fused_batched(c->d_inst, c->d_tile_inst, c->total_tiles, step & 1,
                                                     c->time_order == 3, s));
            else
                for (int i = 0; i < c->n; ++i)
                    FDM_HIP(c, fdm::launch_fused(c->inst[i], step & 1, c->time_order == 3, s));
        }
    }
    for (int32_t step = 0; step < (c->fused ? 0 : n_steps); ++step) {
        int modes[2];
        const int nm = stage_modes(c->time_order, step, modes);
        for (int m = 0; m < nm; ++m) {
            if (c->batched) {
                FDM_HIP(c, fdm::launch_stage_batched(c->d_inst, c->d_tile_inst, c->total_tiles, modes[m], c->fd,
                                                     c->precision, s));
            } else {
                for (int i = 0; i < c->n; ++i) FDM_HIP(c, fdm::launch_stage(c->inst[i], modes[m], c->precision, s));
            }
        }
    }
    // Euler and the fused Heun step ping-pong between the state and the stage
    // buffer; after an odd count the newest state sits in the stage buffer.
    if ((c->time_order == 1 || c->fused) && (n_steps & 1)) {
        for (int i = 0; i < c->n; ++i) {
            const int64_t n = (int64_t)c->inst[i].nx * c->inst[i].ny;
            FDM_HIP(c, fdm::launch_copy(c->inst[i].a11, c->inst[i].w11, n, c->precision, s));
            FDM_HIP(c, fdm::launch_copy(c->inst[i].a12, c->inst[i].w12, n, c->precision, s));
        }
    }
    return FDM_OK;
}

// Tile every instance with `requested` rows (0: the default rule) under the
// context's schedule; re-upload the batched tile map and invalidate the
// device table and the cached graph.
fdm_status retile(fdm_ctx *c, int requested)
{
    int64_t batch_strip_rows = 0;
    int max_ny = 0;
    for (int i = 0; i < c->n; ++i) {
        batch_strip_rows += strip_rows_of(c->desc[i]);
        max_ny = std::max(max_ny, c->desc[i].ny);
    }
    // The fused launch's default: the smallest height with at most five
    // waves per SIMD, so every SIMD carries the same number of tiles (the
    // autotuner's balanced heights; five per SIMD is within 1% of the best
    // at 2048^2 and 4096^2).  The unfused rule where that height is below 4
    // rows (small grids: the first stage's four extra rows would dominate)
    // or above 64.
    if (requested <= 0 && c->fused) {
        const int r = balanced_rows(c, true, c->batched, max_ny, 5 * c->simds);
        if (r >= 4 && r <= 64) requested = r;
    }
    int64_t tile = 0;
    for (int i = 0; i < c->n; ++i) {
        const fdm_transport_desc &d = c->desc[i];
        InstDev &I = c->inst[i];
        I.rows = pick_rows(c->batched ? batch_strip_rows : strip_rows_of(d), d.ny, requested);
        I.strips = (d.nx + fdm::kStrip - 1) / fdm::kStrip;
        I.fstrips = (d.nx + fdm::kFusedStrip - 1) / fdm::kFusedStrip;
        // a launch of one instance must fit one dispatch: taller tiles where
        // the height asked for would exceed it (at the default heights only
        // grids of at most three columns and more than 2^29 rows)
        const int64_t strips = c->fused ? I.fstrips : I.strips;
        while (strips * fdm::tiles_along_y(d.ny, I.rows) > kMaxLaunchTiles && I.rows < d.ny)
            I.rows = (int)std::min<int64_t>(d.ny, 2 * (int64_t)I.rows);
        I.chunks = fdm::tiles_along_y(d.ny, I.rows);
        I.tile_begin = tile;   // in the tiling of the schedule's kernel
        tile += (int64_t)(c->fused ? I.fstrips : I.strips) * I.chunks;
    }
    c->total_tiles = tile;
    c->table_valid = false;
    if (c->graph) {
        FDM_HIP(c, hipGraphExecDestroy(c->graph));
        c->graph = nullptr;
    }
    if (!c->batched) return FDM_OK;
    if (tile > kMaxLaunchTiles) return fail(c, FDM_ERR_INVALID_ARG, "too many tiles for one batched launch");
    // the map and table buffers may still feed queued work
    FDM_HIP(c, hipStreamSynchronize(c->stream));
    if (tile > c->tile_capacity) {
        if (c->d_tile_inst) FDM_HIP(c, hipFree(c->d_tile_inst));
        c->d_tile_inst = nullptr;
        c->tile_capacity = 0;
        FDM_HIP(c, hipMalloc((void **)&c->d_tile_inst, sizeof(int32_t) * tile));
        c->tile_capacity = tile;
    }
    if (!c->d_inst) FDM_HIP(c, hipMalloc((void **)&c->d_inst, sizeof(InstDev) * c->n));
    if (!c->h_inst_pinned)
        FDM_HIP(c, hipHostMalloc((void **)&c->h_inst_pinned, sizeof(InstDev) * c->n, hipHostMallocDefault));
    std::vector<int32_t> map(tile);
    for (int i = 0; i < c->n; ++i) {
        const InstDev &I = c->inst[i];
        const int64_t b = I.tile_begin, e = b + (int64_t)(c->fused ? I.fstrips : I.strips) * I.chunks;
        for (int64_t t = b; t < e; ++t) map[t] = i;
    }
    FDM_HIP(c, hipMemcpy(c->d_tile_inst, map.data(), sizeof(int32_t) * tile, hipMemcpyHostToDevice));
    return FDM_OK;
}

// Bookkeeping of n uncoupled steps.
void advance(fdm_ctx *c, int32_t n)
{
    c->steps += n;
    for (int i = 0; i < c->n; ++i) {
        c->t_acc[i] += (double)n * (double)c->dt[i];
        c->dt_last[i] = c->dt[i];
    }
}

fdm_status compute_stats(fdm_ctx *c, void *const *a11, void *const *a12, fdm_stats *out)
{
    for (int i = 0; i < c->n; ++i) {
        const int64_t n = (int64_t)c->inst[i].nx * c->inst[i].ny;
        FDM_HIP(c, fdm::launch_stats(a11[i], a12[i], n, c->precision, c->d_partials, c->d_stats + 5 * i, c->stream));
    }
    FDM_HIP(c, hipMemcpyAsync(c->h_stats, c->d_stats, sizeof(double) * 5 * c->n, hipMemcpyDeviceToHost,
                              c->stream));
    FDM_HIP(c, hipStreamSynchronize(c->stream));
    if (!c->have_ref) {
        c->ref11.resize(c->n);
        c->ref12.resize(c->n);
        for (int i = 0; i < c->n; ++i) {
            c->ref11[i] = c->h_stats[5 * i + 0];
            c->ref12[i] = c->h_stats[5 * i + 1];
        }
        c->have_ref = true;
    }
    bool bad = false;
    for (int i = 0; i < c->n; ++i) {
        const double *h = c->h_stats + 5 * i;
        fdm_stats &o = out[i];
        o.dt = c->dt_last[i];
        o.step = c->steps;
        o.t = c->t_acc[i];
        o.eps13 = c->cw.eps13;
        o.sigma13 = c->cw.sigma13;
        o.phi_mean = c->cw.phi_mean;
        o.vmax = c->cw.vmax;
        o.sum11 = h[0];
        o.sum12 = h[1];
        o.sum_abs = h[2];
        o.max_norm = h[3];
        o.nonfinite = (int64_t)h[4];
        o.drift11 = h[0] - c->ref11[i];
        o.drift12 = h[1] - c->ref12[i];
        bad |= o.nonfinite != 0;
    }
    if (bad) return fail(c, FDM_ERR_NONFINITE, "non-finite density values found");
    return FDM_OK;
}

fdm_status static_fail(fdm_ctx *c, fdm::StaticStatus st, const std::string &err)
{
    return fail(c, st == fdm::StaticStatus::OutOfMemory ? FDM_ERR_OUT_OF_MEMORY : FDM_ERR_DEVICE, err);
}

// The coupled run of one instance (see fdm_loading in include/fdm.h).
fdm_status coupled_run(fdm_ctx *c, const fdm_loading &L, void *const *a11, void *const *a12, int32_t n_steps,
                       int32_t chunk, fdm_stats *history)
{
    if (c->n != 1) return fail(c, FDM_ERR_INVALID_ARG, "coupled runs need a context of one instance");
    const fdm_transport_desc &d = c->desc[0];
    if (d.velocity != FDM_VELOCITY_LAW) return fail(c, FDM_ERR_INVALID_ARG, "coupled runs need the LAW velocity");
    if (d.dt != 0.0) return fail(c, FDM_ERR_INVALID_ARG, "coupled runs need a CFL-controlled step (dt = 0)");
    if (!(std::isfinite(L.strain_rate13) && std::isfinite(L.tau0) && L.tau0 >= 0.0 && std::isfinite(L.mobility) &&
          L.mobility >= 0.0))
        return fail(c, FDM_ERR_INVALID_ARG, "strain_rate13 must be finite, tau0 and mobility finite and >= 0");
    if (!finite_pos(L.dt_max)) return fail(c, FDM_ERR_INVALID_ARG, "dt_max must be finite and > 0");
    if (L.law != FDM_LAW_THRESHOLD && L.law != FDM_LAW_WIGGLY) return fail(c, FDM_ERR_INVALID_ARG, "unknown law");
    if (L.reserved != 0) return fail(c, FDM_ERR_INVALID_ARG, "loading.reserved must be 0");
    const bool wiggly = L.law == FDM_LAW_WIGGLY;
    if (wiggly && !(std::isfinite(L.tau_y) && L.tau_y >= 0.0 && finite_pos(L.beta)))
        return fail(c, FDM_ERR_INVALID_ARG, "the wiggly law needs tau_y finite and >= 0, beta finite and > 0");
    fdm_static_desc sd{d.nx, d.ny, d.dx, d.dy, L.mu, L.lambda, L.layer_h, L.cell_l3, L.eps13, L.phi_mean,
                       c->precision, 0};
    fdm::StaticParams q;
    const std::string m = check_static(sd, &q);
    if (!m.empty()) return fail(c, FDM_ERR_INVALID_ARG, "loading: " + m);
    fdm_status st = check_ptrs(c, a11, a12);
    if (st != FDM_OK) return st;
    if (n_steps == 0) return FDM_OK;
    st = bind(c, a11, a12);
    if (st != FDM_OK) return st;

    // workspace (kept for later calls; the plan is rebuilt when the cell changes)
    auto &w = c->cw;
    const int64_t n = (int64_t)d.nx * d.ny;
    const bool f64 = c->precision == FDM_PRECISION_FP64;
    const bool same = w.plan && w.q.nx == q.nx && w.q.ny == q.ny && w.q.dx == q.dx && w.q.mu == q.mu &&
                      w.q.lambda == q.lambda && w.q.h == q.h && w.q.n3 == q.n3 && w.q.f64 == q.f64;
    std::string err;
    if (!same) {
        fdm::static_plan_destroy(w.plan);
        w.plan = nullptr;
        const fdm::StaticStatus ss = fdm::static_plan_create(q, c->stream, &w.plan, err);
        if (ss != fdm::StaticStatus::Ok) return static_fail(c, ss, err);
        w.q = q;
    }
    if (!w.tau) FDM_HIP(c, hipMalloc(&w.tau, (f64 ? sizeof(double) : sizeof(float)) * n));
    if (wiggly && !w.phi) FDM_HIP(c, hipMalloc(&w.phi, (f64 ? sizeof(double) : sizeof(float)) * n));
    const fdm::LawParams law{wiggly, L.tau0, L.mobility, L.tau_y, L.beta, L.mobility_field};
    if (!w.v0) FDM_HIP(c, hipMalloc((void **)&w.v0, sizeof(float) * n));
    InstDev I = c->inst[0];
    if (c->fused && c->requested_rows <= 0) {
        // the stage kernels' default tiling, as on a plain context: the per-tile
        // sums then add in the same order whatever the schedule
        I.rows = pick_rows(strip_rows_of(d), d.ny, 0);
        I.chunks = fdm::tiles_along_y(d.ny, I.rows);
    }
    const int64_t tiles = (int64_t)I.strips * I.chunks;
    if (tiles > w.cap) {
        if (w.d_hsum) FDM_HIP(c, hipFree(w.d_hsum));
        w.d_hsum = nullptr;
        w.cap = 0;
        FDM_HIP(c, hipMalloc((void **)&w.d_hsum, sizeof(double) * 2 * tiles));
        w.cap = tiles;
    }
    if (!w.d_cd) FDM_HIP(c, hipMalloc((void **)&w.d_cd, sizeof(fdm::CoupledDev)));
    if (!w.h_cd) FDM_HIP(c, hipHostMalloc((void **)&w.h_cd, sizeof(fdm::CoupledDev), hipHostMallocDefault));

    // The step scalars live on the device: each step enqueues its kernels
    // without waiting (the step size by the stage kernels, the mean slip and
    // stress by the next step's pack kernel or, at a chunk end, one block);
    // the host reads them back once per chunk.
    const double h = std::min(d.dx, d.dy), mu = L.mu, frac = (double)q.h / (double)q.n3;
    FDM_HIP(c, hipStreamSynchronize(c->stream));   // the pinned mirror may feed an earlier copy
    std::memset(w.h_cd, 0, sizeof(fdm::CoupledDev));
    w.h_cd->eps13 = L.eps13;
    w.h_cd->phi_mean = L.phi_mean;
    w.h_cd->t = c->t_acc[0];
    w.h_cd->sigma_bar = 2.0 * mu * L.eps13 - mu * frac * L.phi_mean;
    FDM_HIP(c, hipMemcpyAsync(w.d_cd, w.h_cd, sizeof(fdm::CoupledDev), hipMemcpyHostToDevice, c->stream));
    w.eps13 = L.eps13;
    w.phi_mean = L.phi_mean;
    w.sigma13 = w.h_cd->sigma_bar;

    I.v0f = w.v0;
    I.vpart = c->d_absmax;
    I.nvpart = fdm::velocity_law_blocks(n);
    I.cfl_h = d.cfl * h;
    I.dt_max = L.dt_max;
    // the FP64 fully discrete stage sums node increments, the others Hhat
    const int32_t increments = c->fd && c->precision != FDM_PRECISION_FP32;
    const fdm::SlipArgs slip{w.d_cd, w.d_hsum, tiles, c->time_order, increments, L.strain_rate13, mu, frac,
                             (double)n};
    const int stages = c->time_order == 1 ? 1 : 2;
    const bool mid = c->time_order == 3;

    // One chunk of m steps on stream s.  Each step: (1) the previous step's
    // mean slip and loading, run by the first kernel of (2) the stress solve
    // of the current state; the celerity field; (3-4) one transport step with
    // v0 frozen, its step derived by the stage kernels from the velocity
    // law's max |v0| partials, and per-tile sums of Hhat.  (5) The chunk's
    // last slip update runs in a kernel of its own, ahead of the host's
    // read-back.  Only kernels: the chunk replays as a graph.
    auto enqueue_chunk = [&](int32_t m, hipStream_t s) -> fdm_status {
        InstDev J = I;
        for (int32_t j = 0; j < m; ++j) {
            const fdm::SlipArgs *ps = j > 0 ? &slip : nullptr;
            fdm::StaticStatus ss =
                wiggly ? fdm::static_plan_run_phi(w.plan, a11[0], a12[0], w.tau, w.phi, &w.d_cd->sigma_bar,
                                                  &w.d_cd->phi_mean, ps, s, err)
                       : fdm::static_plan_run(w.plan, a11[0], a12[0], w.tau, &w.d_cd->sigma_bar, ps, s, err);
            if (ss != fdm::StaticStatus::Ok) return static_fail(c, ss, err);
            ss = fdm::velocity_law(w.tau, w.phi, f64, w.v0, n, law, c->d_absmax, s, err);
            if (ss != fdm::StaticStatus::Ok) return static_fail(c, ss, err);
            J.hsum = w.d_hsum;
            J.coef_out = &w.d_cd->coef;
            FDM_HIP(c, fdm::launch_stage(J, mid ? fdm::MODE_MID1 : fdm::MODE_FWD, c->precision, s));
            J.coef_out = nullptr;
            if (stages == 2) {
                J.hsum = w.d_hsum + tiles;
                FDM_HIP(c, fdm::launch_stage(J, mid ? fdm::MODE_MID2 : fdm::MODE_HEUN2, c->precision, s));
            } else {
                FDM_HIP(c, fdm::launch_copy(J.a11, J.w11, n, c->precision, s));
                FDM_HIP(c, fdm::launch_copy(J.a12, J.w12, n, c->precision, s));
            }
        }
        FDM_HIP(c, fdm::launch_coupled_slip(slip, s));
        return FDM_OK;
    };

    // Full chunks replay one captured graph when there are at least two of
    // them (kernel nodes only; a capture that fails or records anything else
    // leaves the chunks enqueued one kernel at a time, with the same kernels).
    hipGraphExec_t gexec = nullptr;
    if (n_steps / chunk >= 2 && !w.no_graph) {
        FDM_HIP(c, hipStreamSynchronize(c->stream));
        const bool sticky0 = c->sticky;
        const std::string err0 = c->err;
        hipGraph_t g = nullptr;
        bool ok = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const fdm_status cs = enqueue_chunk(chunk, c->capture);
            ok = hipStreamEndCapture(c->capture, &g) == hipSuccess && cs == FDM_OK && g != nullptr;
        }
        size_t nn = 0;
        if (ok) ok = hipGraphGetNodes(g, nullptr, &nn) == hipSuccess;
        if (ok) {
            std::vector<hipGraphNode_t> nodes(nn);
            ok = hipGraphGetNodes(g, nodes.data(), &nn) == hipSuccess;
            for (size_t k = 0; ok && k < nn; ++k) {
                hipGraphNodeType t;
                ok = hipGraphNodeGetType(nodes[k], &t) == hipSuccess && t == hipGraphNodeTypeKernel;
            }
        }
        if (ok) ok = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {
            if (gexec) (void)hipGraphExecDestroy(gexec);
            gexec = nullptr;
            w.no_graph = true;
            (void)hipGetLastError();
            c->sticky = sticky0;
            c->err = err0;
        }
    }
    struct GraphGuard {
        hipGraphExec_t &g;
        ~GraphGuard()
        {
            if (g) (void)hipGraphExecDestroy(g);
        }
    } guard{gexec};

    int32_t rec = 0;
    for (int32_t done = 0; done < n_steps;) {
        const int32_t m = std::min(chunk, n_steps - done);
        if (m == chunk && gexec) {
            FDM_HIP(c, hipGraphLaunch(gexec, c->stream));
        } else {
            st = enqueue_chunk(m, c->stream);
            if (st != FDM_OK) return st;
        }
        done += m;
        c->steps += m;
        FDM_HIP(c, hipMemcpyAsync(w.h_cd, w.d_cd, sizeof(fdm::CoupledDev), hipMemcpyDeviceToHost, c->stream));
        FDM_HIP(c, hipStreamSynchronize(c->stream));
        if (w.h_cd->coef.nonfinite) return fail(c, FDM_ERR_NONFINITE, "non-finite celerity in the coupled run");
        c->t_acc[0] = w.h_cd->t;
        c->dt_last[0] = w.h_cd->coef.dt;
        w.eps13 = w.h_cd->eps13;
        w.phi_mean = w.h_cd->phi_mean;
        w.sigma13 = w.h_cd->sigma_bar;
        w.vmax = w.h_cd->coef.vmax;
        if (history) {
            st = compute_stats(c, a11, a12, history + rec);
            if (st != FDM_OK) return st;
            ++rec;
        }
    }
    return FDM_OK;
}

}  // namespace

extern "C" {

fdm_status fdm_transport_init(const fdm_transport_desc *descs, int32_t n_instances, const fdm_options *options,
                              void *hip_stream, fdm_ctx **out)
{
    if (!out) return fail(nullptr, FDM_ERR_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    if (!descs || n_instances < 1) return fail(nullptr, FDM_ERR_INVALID_ARG, "need at least one descriptor");
    fdm_options opt = {0, 0, 0, 0};
    if (options) opt = *options;
    if (opt.schedule < FDM_SCHEDULE_AUTO || opt.schedule > FDM_SCHEDULE_FUSED)
        return fail(nullptr, FDM_ERR_INVALID_ARG, "unknown schedule");
    if (opt.tile_rows < 0) return fail(nullptr, FDM_ERR_INVALID_ARG, "tile_rows must be >= 0");
    if (opt.fused != 0) return fail(nullptr, FDM_ERR_INVALID_ARG, "fused is reserved and must be 0");
    if (opt.precision < FDM_PRECISION_FP32 || opt.precision > FDM_PRECISION_FP64)
        return fail(nullptr, FDM_ERR_INVALID_ARG, "unknown precision");
    int32_t order = -1;
    for (int i = 0; i < n_instances; ++i) {
        const std::string m = check_desc(descs[i]);
        if (!m.empty()) return fail(nullptr, FDM_ERR_INVALID_ARG, "descriptor " + std::to_string(i) + ": " + m);
        const bool fd = descs[i].scheme == FDM_SCHEME_FULLY_DISCRETE;
        const int32_t o = descs[i].time_order == 0 ? (fd ? 1 : 2) : descs[i].time_order;
        if (order >= 0 && o != order)
            return fail(nullptr, FDM_ERR_INVALID_ARG, "all instances of a context must share time_order");
        if (descs[i].scheme != descs[0].scheme)
            return fail(nullptr, FDM_ERR_INVALID_ARG, "all instances of a context must share the scheme");
        order = o;
    }
    if (opt.schedule == FDM_SCHEDULE_FUSED &&
        !(opt.precision == FDM_PRECISION_FP32 && (order == 2 || order == 3) &&
          descs[0].scheme == FDM_SCHEME_SEMIDISCRETE))
        return fail(nullptr, FDM_ERR_INVALID_ARG,
                    "the fused schedule needs FP32 precision, time_order 2 or 3 and the semi-discrete scheme");
    // Stability bound of the step: every case but a fixed dt over a celerity
    // field is decided here, before any HIP call; that one needs the field's
    // max |v0| (after the device reduction below).
    for (int i = 0; i < n_instances; ++i) {
        const fdm_transport_desc &d = descs[i];
        if (d.velocity == FDM_VELOCITY_LAW && d.v0_field && d.dt > 0.0) continue;
        const std::string m = check_courant(d, order, std::fabs((double)(float)d.v0));
        if (!m.empty()) return fail(nullptr, FDM_ERR_CFL, "descriptor " + std::to_string(i) + ": " + m);
    }
    fdm_ctx *c = new (std::nothrow) fdm_ctx;
    if (!c) return fail(nullptr, FDM_ERR_OUT_OF_MEMORY, "host allocation failed");
    c->stream = (hipStream_t)hip_stream;
    c->n = n_instances;
    c->time_order = order;
    c->fd = descs[0].scheme == FDM_SCHEME_FULLY_DISCRETE;
    c->schedule = opt.schedule;
    c->precision = opt.precision;
    c->fused = opt.schedule == FDM_SCHEDULE_FUSED;
    c->batched = n_instances > 1 && opt.schedule != FDM_SCHEDULE_PLAIN;   // fused: one launch for all
    c->desc.assign(descs, descs + n_instances);
    c->inst.resize(n_instances);
    c->dt.resize(n_instances);
    c->t_acc.assign(n_instances, 0.0);

    auto bail = [&](fdm_status st) {
        g_init_error = c->err;
        release(c);
        return st;
    };
#define INIT_HIP(call)                                                                            \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            fail(c, e_ == hipErrorOutOfMemory ? FDM_ERR_OUT_OF_MEMORY : FDM_ERR_DEVICE,           \
                 std::string(#call) + ": " + hipGetErrorString(e_));                              \
            return bail(e_ == hipErrorOutOfMemory ? FDM_ERR_OUT_OF_MEMORY : FDM_ERR_DEVICE);       \
        }                                                                                         \
    } while (0)

    // workspace: one stage buffer (both components) per instance
    int64_t total = 0;
    for (int i = 0; i < n_instances; ++i) total += 2 * (int64_t)descs[i].nx * descs[i].ny;
    const size_t elem = opt.precision == FDM_PRECISION_FP64 ? sizeof(double) : sizeof(float);
    c->elem = elem;
    {
        int dev = 0, cus = 0;
        INIT_HIP(hipGetDevice(&dev));
        INIT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        c->simds = 4 * (int64_t)std::max(cus, 1);
    }
    INIT_HIP(hipMalloc((void **)&c->workspace, elem * total));
    INIT_HIP(hipMalloc((void **)&c->d_partials, sizeof(fdm::StatsPartial) * fdm::kStatsBlocks));
    INIT_HIP(hipMalloc((void **)&c->d_stats, sizeof(double) * 5 * n_instances));
    INIT_HIP(hipHostMalloc((void **)&c->h_stats, sizeof(double) * 5 * n_instances, hipHostMallocDefault));
    // max |v0| partials: of the celerity field at init, of the velocity law in coupled runs
    INIT_HIP(hipMalloc((void **)&c->d_absmax, sizeof(float) * std::max(fdm::kAbsmaxBlocks, fdm::kLawBlocks)));

    std::vector<float> absmax(fdm::kAbsmaxBlocks);
    int64_t off = 0;
    for (int i = 0; i < n_instances; ++i) {
        const fdm_transport_desc &d = descs[i];
        const int64_t n = (int64_t)d.nx * d.ny;
        double smax;
        if (d.velocity == FDM_VELOCITY_LAW && d.v0_field) {
            INIT_HIP(fdm::launch_absmax(d.v0_field, n, c->d_absmax, c->stream));
            INIT_HIP(hipMemcpyAsync(absmax.data(), c->d_absmax, sizeof(float) * fdm::kAbsmaxBlocks,
                                    hipMemcpyDeviceToHost, c->stream));
            INIT_HIP(hipStreamSynchronize(c->stream));
            float m = 0.0f;
            for (float v : absmax) {
                if (std::isnan(v)) {
                    fail(c, FDM_ERR_INVALID_ARG, "v0_field of descriptor " + std::to_string(i) + " is not finite");
                    return bail(FDM_ERR_INVALID_ARG);
                }
                m = std::max(m, v);
            }
            smax = m;
            if (d.dt > 0.0) {
                const std::string m2 = check_courant(d, order, smax);
                if (!m2.empty()) {
                    fail(c, FDM_ERR_CFL, "descriptor " + std::to_string(i) + ": " + m2);
                    return bail(FDM_ERR_CFL);
                }
            }
        } else {
            smax = smax_uniform(d);
        }
        const float dt = step_dt(d, smax);
        c->dt[i] = dt;
        fill_inst(c->inst[i], d, dt, static_cast<char *>(c->workspace) + elem * off,
                  static_cast<char *>(c->workspace) + elem * (off + n));
        off += 2 * n;
    }
    c->dt_last = c->dt;
    {
        c->requested_rows = opt.tile_rows;
        const fdm_status ts = retile(c, opt.tile_rows);
        if (ts != FDM_OK) return bail(ts);
    }
    INIT_HIP(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
#undef INIT_HIP
    *out = c;
    return FDM_OK;
}

fdm_status fdm_transport_step(fdm_ctx *c, void *const *alpha11, void *const *alpha12, int32_t n_steps)
{
    if (!c) return FDM_ERR_INVALID_ARG;
    if (c->sticky) return FDM_ERR_DEVICE;
    if (n_steps < 0) return fail(c, FDM_ERR_INVALID_ARG, "n_steps must be >= 0");
    fdm_status st = check_ptrs(c, alpha11, alpha12);
    if (st != FDM_OK) return st;
    if (n_steps == 0) return FDM_OK;
    st = bind(c, alpha11, alpha12);
    if (st != FDM_OK) return st;
    st = enqueue_steps(c, n_steps, c->stream);
    if (st != FDM_OK) return st;
    advance(c, n_steps);
    return FDM_OK;
}

fdm_status fdm_transport_stats(fdm_ctx *c, void *const *alpha11, void *const *alpha12, fdm_stats *out)
{
    if (!c) return FDM_ERR_INVALID_ARG;
    if (c->sticky) return FDM_ERR_DEVICE;
    if (!out) return fail(c, FDM_ERR_INVALID_ARG, "out must not be NULL");
    fdm_status st = check_ptrs(c, alpha11, alpha12);
    if (st != FDM_OK) return st;
    return compute_stats(c, alpha11, alpha12, out);
}

fdm_status fdm_static_solve(const fdm_static_desc *desc, const void *alpha11, const void *alpha12,
                            void *tau13_out, void *hip_stream)
{
    if (!desc) return fail(nullptr, FDM_ERR_INVALID_ARG, "desc must not be NULL");
    fdm::StaticParams q;
    const std::string m = check_static(*desc, &q);
    if (!m.empty()) return fail(nullptr, FDM_ERR_INVALID_ARG, m);
    if (!alpha11 || !alpha12 || !tau13_out)
        return fail(nullptr, FDM_ERR_INVALID_ARG, "alpha11, alpha12 and tau13_out must not be NULL");
    if (alpha11 == alpha12 || tau13_out == alpha11 || tau13_out == alpha12)
        return fail(nullptr, FDM_ERR_INVALID_ARG, "alpha11, alpha12 and tau13_out must be distinct");
    hipStream_t s = (hipStream_t)hip_stream;
    std::string err;
    fdm::StaticPlan *plan = nullptr;
    fdm::StaticStatus st = fdm::static_plan_create(q, s, &plan, err);
    if (st == fdm::StaticStatus::Ok) {
        const double sbar[2] = {static_mean_stress(*desc, q), desc->phi_mean};
        const hipError_t ce = hipMemcpyAsync(fdm::static_plan_scalars(plan), sbar, sizeof(sbar),
                                             hipMemcpyHostToDevice, s);
        if (ce != hipSuccess) {
            st = fdm::StaticStatus::Device;
            err = std::string("hipMemcpyAsync: ") + hipGetErrorString(ce);
        } else {
            st = fdm::static_plan_run(plan, alpha11, alpha12, tau13_out, fdm::static_plan_scalars(plan), nullptr, s,
                                      err);
        }
        const hipError_t e = hipStreamSynchronize(s);
        if (st == fdm::StaticStatus::Ok && e != hipSuccess) {
            st = fdm::StaticStatus::Device;
            err = std::string("hipStreamSynchronize: ") + hipGetErrorString(e);
        }
    }
    fdm::static_plan_destroy(plan);
    if (st == fdm::StaticStatus::Ok) return FDM_OK;
    return fail(nullptr, st == fdm::StaticStatus::OutOfMemory ? FDM_ERR_OUT_OF_MEMORY : FDM_ERR_DEVICE, err);
}

fdm_status fdm_run(fdm_ctx *c, const fdm_loading *loading, void *const *alpha11, void *const *alpha12,
                   int32_t n_steps, int32_t chunk, fdm_stats *history)
{
    if (!c) return FDM_ERR_INVALID_ARG;
    if (c->sticky) return FDM_ERR_DEVICE;
    if (n_steps < 0 || chunk < 1) return fail(c, FDM_ERR_INVALID_ARG, "need n_steps >= 0 and chunk >= 1");
    if (loading) return coupled_run(c, *loading, alpha11, alpha12, n_steps, chunk, history);
    fdm_status st = check_ptrs(c, alpha11, alpha12);
    if (st != FDM_OK) return st;
    if (n_steps == 0) return FDM_OK;
    st = bind(c, alpha11, alpha12);
    if (st != FDM_OK) return st;

    // (Re)capture a graph of `chunk` steps for these arrays.
    bool same = c->graph && c->graph_steps == chunk;
    for (int i = 0; same && i < c->n; ++i)
        same = c->graph_a11[i] == alpha11[i] && c->graph_a12[i] == alpha12[i];
    if (!same) {
        if (c->graph) {
            FDM_HIP(c, hipGraphExecDestroy(c->graph));
            c->graph = nullptr;
        }
        // the capture stream must see the table upload done by bind()
        FDM_HIP(c, hipStreamSynchronize(c->stream));
        hipGraph_t g = nullptr;
        FDM_HIP(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
        fdm_status cs = enqueue_steps(c, chunk, c->capture);
        hipError_t ee = hipStreamEndCapture(c->capture, &g);
        if (cs != FDM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return cs;
        }
        if (ee != hipSuccess) return fail(c, FDM_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ee));
        hipError_t ie = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return fail(c, FDM_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        c->graph_steps = chunk;
        c->graph_a11.assign(alpha11, alpha11 + c->n);
        c->graph_a12.assign(alpha12, alpha12 + c->n);
    }
    int32_t done = 0, rec = 0;
    while (done < n_steps) {
        const int32_t m = std::min(chunk, n_steps - done);
        if (m == chunk) {
            FDM_HIP(c, hipGraphLaunch(c->graph, c->stream));
        } else {
            st = enqueue_steps(c, m, c->stream);
            if (st != FDM_OK) return st;
        }
        done += m;
        advance(c, m);
        if (history) {
            st = compute_stats(c, alpha11, alpha12, history + (int64_t)rec * c->n);
            if (st != FDM_OK) return st;
        }
        ++rec;
    }
    if (!history) FDM_HIP(c, hipStreamSynchronize(c->stream));
    return FDM_OK;
}

int32_t fdm_tile_rows(const fdm_ctx *c, int32_t i)
{
    if (!c || i < 0 || i >= c->n) return -1;
    return c->inst[i].rows;
}

fdm_status fdm_autotune(fdm_ctx *c, void *const *alpha11, void *const *alpha12, int32_t trial_steps,
                        fdm_tune_trial *trials, int32_t max_trials, int32_t *n_trials)
{
    if (!c) return FDM_ERR_INVALID_ARG;
    if (c->sticky) return FDM_ERR_DEVICE;
    if (n_trials) *n_trials = 0;
    if (trial_steps < 1) return fail(c, FDM_ERR_INVALID_ARG, "trial_steps must be >= 1");
    if (max_trials < 0 || (max_trials > 0 && !trials))
        return fail(c, FDM_ERR_INVALID_ARG, "trials must hold max_trials >= 0 entries");
    fdm_status st = check_ptrs(c, alpha11, alpha12);
    if (st != FDM_OK) return st;

    // scratch copy of the state: the trials advance it, the caller's arrays stay
    int64_t total = 0;
    for (int i = 0; i < c->n; ++i) total += 2 * (int64_t)c->desc[i].nx * c->desc[i].ny;
    void *scratch = nullptr;
    {
        const hipError_t e = hipMalloc(&scratch, c->elem * total);
        if (e != hipSuccess)
            return fail(c, e == hipErrorOutOfMemory ? FDM_ERR_OUT_OF_MEMORY : FDM_ERR_DEVICE,
                        std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    const int64_t simds = c->simds;
    std::vector<void *> s11(c->n), s12(c->n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool was_batched = c->batched, was_fused = c->fused;
    int best_rows = -1;
    bool best_batched = was_batched, best_fused = was_fused;
    double best = 0.0;
    int32_t count = 0;
    int max_ny = 0;
    for (int i = 0; i < c->n; ++i) max_ny = std::max(max_ny, c->desc[i].ny);
    // candidate schedules: the requested one, or under AUTO batched and plain
    // (several instances) and the fused Heun launches where they apply
    std::vector<int> schedules;
    if (c->schedule == FDM_SCHEDULE_AUTO) {
        if (c->n > 1) schedules = {FDM_SCHEDULE_BATCHED, FDM_SCHEDULE_PLAIN};
        else schedules = {FDM_SCHEDULE_PLAIN};
        if (c->precision == fdm::PREC_FP32 && (c->time_order == 2 || c->time_order == 3) && !c->fd)
            schedules.push_back(FDM_SCHEDULE_FUSED);
    } else {
        schedules = {was_fused ? FDM_SCHEDULE_FUSED : was_batched ? FDM_SCHEDULE_BATCHED : FDM_SCHEDULE_PLAIN};
    }

    // Seconds per step of one launch shape on the scratch state: a warm-up
    // step, then the fastest of `reps` timed runs of trial_steps steps.
    auto time_shape = [&](int rows, bool batched, bool fused, int reps, double *out) -> fdm_status {
        c->batched = batched;
        c->fused = fused;
        fdm_status r = retile(c, rows);
        if (r != FDM_OK) return r;
        r = bind(c, s11.data(), s12.data());
        if (r != FDM_OK) return r;
        r = enqueue_steps(c, 1, c->stream);
        if (r != FDM_OK) return r;
        double best_t = 0.0;
        for (int k = 0; k < reps; ++k) {
            FDM_HIP(c, hipEventRecord(e0, c->stream));
            r = enqueue_steps(c, trial_steps, c->stream);
            if (r != FDM_OK) return r;
            FDM_HIP(c, hipEventRecord(e1, c->stream));
            FDM_HIP(c, hipEventSynchronize(e1));
            float ms = 0.0f;
            FDM_HIP(c, hipEventElapsedTime(&ms, e0, e1));
            const double t = 1e-3 * ms / trial_steps;
            if (k == 0 || t < best_t) best_t = t;
        }
        *out = best_t;
        return FDM_OK;
    };
    struct Cand {
        int rows, sched;
        bool batched, fused;
        double sec;
        int32_t slot;   // its entry in trials, or -1
    };
    std::vector<Cand> cands;
    auto run = [&]() -> fdm_status {
        int64_t off = 0;
        for (int i = 0; i < c->n; ++i) {
            const int64_t n = (int64_t)c->desc[i].nx * c->desc[i].ny;
            s11[i] = static_cast<char *>(scratch) + c->elem * off;
            s12[i] = static_cast<char *>(scratch) + c->elem * (off + n);
            off += 2 * n;
            FDM_HIP(c, hipMemcpyAsync(s11[i], alpha11[i], c->elem * n, hipMemcpyDeviceToDevice, c->stream));
            FDM_HIP(c, hipMemcpyAsync(s12[i], alpha12[i], c->elem * n, hipMemcpyDeviceToDevice, c->stream));
        }
        FDM_HIP(c, hipEventCreate(&e0));
        FDM_HIP(c, hipEventCreate(&e1));
        for (int sched : schedules) {
            const bool fused = sched == FDM_SCHEDULE_FUSED;
            const bool batched = sched == FDM_SCHEDULE_BATCHED || (fused && c->n > 1);
            // Fixed heights, then balanced ones.  A launch of at most eight
            // waves per SIMD is resident at once and its waves carry equal
            // work, so the SIMD holding the most waves sets its time: the
            // smallest height with at most k waves per SIMD (k = 1 .. 8)
            // evens the SIMDs out at the least halo work for k rounds.
            std::vector<int> heights;
            for (int rows : {4, 8, 12, 16, 24, 32, 48, 64})
                if (rows <= max_ny || rows == 4) heights.push_back(rows);
            for (int k = 1; k <= 8; ++k) {
                const int rows = balanced_rows(c, fused, batched, max_ny, k * simds);
                if (rows > 0 && rows <= kMaxBalancedRows &&
                    std::find(heights.begin(), heights.end(), rows) == heights.end())
                    heights.push_back(rows);
            }
            for (int rows : heights) {
                double sec = 0.0;
                fdm_status r = time_shape(rows, batched, fused, 2, &sec);
                if (r != FDM_OK) return r;
                if (count < max_trials) {
                    trials[count].tile_rows = rows;
                    trials[count].schedule = sched;
                    trials[count].seconds_per_step = sec;
                }
                cands.push_back({rows, sched, batched, fused, sec, count < max_trials ? count : -1});
                ++count;
            }
        }
        // Confirmation: candidates a few percent apart in one timing can
        // swap places in the next, so the three fastest are timed again,
        // interleaved, three more times each, and keep their fastest time.
        std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.sec < b.sec; });
        const size_t top = std::min<size_t>(3, cands.size());
        for (int round = 0; round < 3 && top > 1; ++round)
            for (size_t k = 0; k < top; ++k) {
                double sec = 0.0;
                fdm_status r = time_shape(cands[k].rows, cands[k].batched, cands[k].fused, 1, &sec);
                if (r != FDM_OK) return r;
                cands[k].sec = std::min(cands[k].sec, sec);
                if (cands[k].slot >= 0) trials[cands[k].slot].seconds_per_step = cands[k].sec;
            }
        for (size_t k = 0; k < top; ++k)
            if (best_rows < 0 || cands[k].sec < best) {
                best = cands[k].sec;
                best_rows = cands[k].rows;
                best_batched = cands[k].batched;
                best_fused = cands[k].fused;
            }
        return FDM_OK;
    };
    st = run();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(scratch);
    if (st == FDM_OK && best_rows > 0) {
        c->batched = best_batched;
        c->fused = best_fused;
        st = retile(c, best_rows);
        if (st == FDM_OK) c->requested_rows = best_rows;
    } else if (!c->sticky) {
        // restore the previous tiling after a non-device failure
        c->batched = was_batched;
        c->fused = was_fused;
        (void)retile(c, c->requested_rows);
    }
    c->table_valid = false;   // the table points at the scratch arrays
    if (n_trials) *n_trials = std::min(count, max_trials);
    return st;
}

double fdm_transport_dt(const fdm_ctx *c, int32_t i)
{
    if (!c || i < 0 || i >= c->n) return -1.0;
    return (double)c->dt[i];
}

void fdm_destroy(fdm_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release(c);
}

const char *fdm_status_string(fdm_status s)
{
    switch (s) {
    case FDM_OK: return "ok";
    case FDM_ERR_INVALID_ARG: return "invalid argument";
    case FDM_ERR_DEVICE: return "HIP device error";
    case FDM_ERR_OUT_OF_MEMORY: return "out of device memory";
    case FDM_ERR_CFL: return "time step above the stability bound";
    case FDM_ERR_NONFINITE: return "non-finite densities";
    case FDM_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *fdm_last_error(const fdm_ctx *c)
{
    if (!c) return g_init_error.c_str();
    return c->err.c_str();
}

}  // extern "C"
