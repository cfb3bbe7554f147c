/*
 * fdm.h -- C ABI of the MI355X (gfx950) transport hot path for the layer case
 * of field dislocation mechanics (Morin, Brenner & Suquet, arXiv:1911.03225).
 *
 * The library advances the two in-plane Nye dislocation-density components of
 * the layer case (sec. 3.2.1) with the central-upwind Godunov-type scheme of
 * sec. 3.2.2-3.2.3 on a periodic grid of pixel nodes.
 *
 * Units are the paper's dimensionless ones (sec. 3.2.1): lengths in b, times
 * in b / V_s, densities as b * alpha, celerity v0 in V_s.
 *
 * Grid and layout.  nx by ny pixel nodes x_j = j dx, y_k = k dy (sec. 3.2.3),
 * periodic in both directions; nx, ny >= 1 (ny = 1 is a 1-D problem along x).
 * Arrays are row-major, index k * nx + j, x fastest, device memory, float32
 * (double with FDM_PRECISION_FP64, see fdm_options):
 *   alpha12[k*nx + j]  alpha_12 = d1 U^p_13 on the x-edge ((j+1/2) dx, k dy);
 *   alpha11[k*nx + j]  alpha_11 = -d2 U^p_13 on the y-edge (j dx, (k+1/2) dy).
 * These are the differences of U^p_13 between neighbouring nodes, so the
 * conservative update used here is the node update of U^p_13 differenced
 * along x and y: it keeps sum(alpha_11), sum(alpha_12) and the discrete
 * div(alpha) = 0 (eq. 2) to round-off.
 *
 * Ownership.  Density arrays belong to the caller (e.g. torch tensors) and are
 * updated in place, in stream order; alpha11 and alpha12 must not alias each
 * other or another instance's arrays.  A v0 field belongs to the caller and
 * must stay valid, unchanged, for the context's lifetime.  The library owns
 * only its workspace (one stage buffer per instance, reduction partials and
 * descriptor tables), allocated in fdm_transport_init and freed in
 * fdm_destroy.
 *
 * Streams.  Every call enqueues work on the HIP stream given at init (NULL is
 * the null stream) and returns without waiting, except where stated.  One
 * context belongs to one stream; separate contexts are independent.
 *
 * Errors.  Every entry point returns an fdm_status; FDM_OK is 0.  The library
 * never aborts, throws or prints.  Arguments are validated on the host before
 * any HIP call.  A HIP failure returns FDM_ERR_DEVICE, keeps its message in
 * the context (fdm_last_error) and is sticky: every later call on that
 * context returns FDM_ERR_DEVICE until fdm_destroy.
 */
#ifndef FDM_H
#define FDM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fdm_status {
    FDM_OK = 0,
    FDM_ERR_INVALID_ARG = 1,   /* a descriptor field or pointer is invalid        */
    FDM_ERR_DEVICE = 2,        /* a HIP call failed (sticky, see fdm_last_error)  */
    FDM_ERR_OUT_OF_MEMORY = 3, /* workspace allocation failed                     */
    FDM_ERR_CFL = 4,           /* the step exceeds the stability bound (below)    */
    FDM_ERR_NONFINITE = 5,     /* a NaN or Inf was found in the densities         */
    FDM_ERR_UNSUPPORTED = 6    /* feature not available                           */
} fdm_status;

/* Step 1 limiters (sec. 3.2.2, limited second difference of U^p_13, i.e.
 * the limited slope of each density component along its own axis):
 * minmod(theta D+, (D+ + D-)/2, theta D-) with theta = 1 (MINMOD), theta = 2
 * (MC) or a given theta in [1, 2] (THETA); SUPERBEE is Roe's superbee (not in
 * the paper); NONE gives the first-order scheme. */
typedef enum fdm_limiter {
    FDM_LIMITER_NONE = 0,
    FDM_LIMITER_MINMOD = 1,
    FDM_LIMITER_MC = 2,
    FDM_LIMITER_THETA = 3,
    FDM_LIMITER_SUPERBEE = 4
} fdm_limiter;

/* Hamiltonian.  LAW: H = v0 |grad U^p_13| (eq. 52 and 56), the layer-case
 * velocity law with the celerity v0 at the nodes (a uniform value or a field;
 * v0 = 0 marks immobile nodes, e.g. eta = infinity in precipitates, sec. 5.3).
 * PRESCRIBED: H = V . grad U^p_13 with a uniform V (eq. 28 with only U^p_13
 * non-zero), for verification. */
typedef enum fdm_velocity {
    FDM_VELOCITY_LAW = 0,
    FDM_VELOCITY_PRESCRIBED = 1
} fdm_velocity;

/* Scheme.  SEMIDISCRETE: Steps 3-4 of sec. 3.2.3 taken in the limit
 * dt -> 0 (the central-upwind numerical Hamiltonian), advanced by the
 * integrator time_order.  FULLY_DISCRETE: Steps 1-4 at the step dt as the
 * paper prints them -- quadratic interpolant (eq. 42, separable along x and
 * y), values at the intermediate points x_j + a^+- dt, y_k + b^+- dt corrected
 * by -dt H of the interpolant's slope there, projection -- one pass per time
 * step (time_order must be 0 or 1).  First order in time; keeps sharp fronts
 * sharper than Heun, and overshoots smooth profiles with MC or superbee at
 * Courant numbers above about 0.25, like one forward-Euler stage. */
typedef enum fdm_scheme {
    FDM_SCHEME_SEMIDISCRETE = 0,
    FDM_SCHEME_FULLY_DISCRETE = 1
} fdm_scheme;

/* One transport problem. */
typedef struct fdm_transport_desc {
    int32_t nx, ny;          /* pixel nodes, >= 1 each; nx*ny < 2^31, nx < 2^27  */
    double dx, dy;           /* grid spacings, > 0                              */
    int32_t limiter;         /* fdm_limiter                                     */
    int32_t scheme;          /* fdm_scheme; 0 is the default; every instance of
                                a context uses the same                          */
    double theta;            /* FDM_LIMITER_THETA only, in [1, 2]               */
    int32_t time_order;      /* 1: one forward-Euler stage of the semi-discrete
                                scheme; 2: two-stage SSP Runge-Kutta (Heun),
                                the default when 0 is given; 3: explicit
                                midpoint (u + dt L(u + dt/2 L(u)), the
                                midpoint rule of sec. 3.2.2).  The fully
                                discrete scheme takes 0 or 1 (one pass)          */
    double cfl;              /* Courant number nu in (0, 1] used when dt == 0
                                (sec. 4.3: |v0| dt / dx); see the bound below   */
    double dt;               /* 0: dt = nu min(dx,dy) / s_max rounded down to a
                                float; > 0: this step (rounded to the nearest
                                float).  Either way the step must satisfy the
                                stability bound below, else FDM_ERR_CFL        */
    int32_t velocity;        /* fdm_velocity                                    */
    double v0;               /* LAW: uniform celerity when v0_field is NULL,
                                rounded to float (the kernels' and s_max's)     */
    const float *v0_field;   /* LAW: device array of nx*ny node celerities, or
                                NULL; s_max = max |v0| over the field           */
    double V[2];             /* PRESCRIBED: velocity (V1, V2), rounded to
                                float; s_max = max(|V1|/dx, |V2|/dy) min(dx,dy)  */
} fdm_transport_desc;

/* Stability bound.  nu2 = dt (S1/dx + S2/dy), the sum of the Courant numbers
 * along x and y, with S1, S2 bounds on |dH/dp1|, |dH/dp2| (LAW: max |v0| for
 * both, since |p_i| <= |p|; PRESCRIBED: |V1|, |V2|) and an axis of a single
 * node contributing 0.  fdm_transport_init rejects a descriptor with
 * FDM_ERR_CFL when
 *   nu2 > 1    (any scheme: the first-order upwind stage is unstable in 2-D
 *               beyond it), or
 *   nu2 > 1/2  for one forward-Euler stage with a limiter (time_order 1, or
 *               the fully discrete scheme): a limited Euler step grows
 *               beyond it with the compressive limiters.
 * For LAW with dt == 0 the check uses the cfl alone (dt max|v0| <=
 * cfl min(dx,dy) whatever the celerity), so on a square grid the
 * two-stage schemes take cfl <= 0.5 and a limited Euler stage cfl <= 0.25,
 * the paper's value; a 1-D problem (ny == 1) takes twice that.  With a
 * fixed dt over a celerity field the bound is checked after the device
 * reduction of max |v0|, otherwise before any HIP call. */

/* Scheduling options; pass NULL for the defaults. */
typedef enum fdm_schedule {
    FDM_SCHEDULE_AUTO = 0,     /* batched launches when n_instances > 1        */
    FDM_SCHEDULE_BATCHED = 1,  /* one launch per stage for all instances       */
    FDM_SCHEDULE_PLAIN = 2,    /* one launch per stage per instance            */
    FDM_SCHEDULE_FUSED = 3     /* one launch per step (for all instances of a
                                  context): both stages in one pass, the first
                                  stage's densities kept in registers, so a
                                  step reads and writes the state once (8 B
                                  per node each way, + 4 B read with a
                                  celerity field, against 20 + 28 B for the
                                  two stage launches).  FP32 precision,
                                  time_order 2 (Heun) or 3 (explicit
                                  midpoint), semi-discrete scheme only.  The
                                  same results bit for bit.  About 20% more
                                  arithmetic per node (halo lanes and rows of
                                  the first stage) but one launch instead of
                                  two and no stage-buffer traffic: measured
                                  faster at every size tried, 1.5x beyond the
                                  on-chip cache.  The autotuner includes it  */
} fdm_schedule;

/* Precision of the stage kernels.
 * FP32 (default): float32 densities, slopes, numerical Hamiltonian and update
 *   in float32.
 * FP64_ARITH: float32 densities; the same steps in float64 registers, results
 *   rounded once to float32 when stored.  Removes the float32 cancellations at
 *   the foot of a front that the discontinuity of the speed v0 p/|p| at p = 0
 *   amplifies (shock-dominated runs).
 * FP64: float64 densities (the arrays passed to step/stats/run are double)
 *   and float64 arithmetic.  Rounding the state to float32 after every stage
 *   is itself a perturbation the scheme amplifies over hundreds of steps, so
 *   long runs agree with a float64 evaluation of the scheme to 1e-5 only with
 *   float64 state.  A v0 field stays float32 in every mode.
 * Both float64 modes take the definition's operations in its order (IEEE
 * square root and division; for FULLY_DISCRETE the node increments of
 * phi, whose differences update the densities), so FP64 reproduces a plain
 * float64 evaluation of either scheme bit for bit. */
typedef enum fdm_precision {
    FDM_PRECISION_FP32 = 0,
    FDM_PRECISION_FP64_ARITH = 1,
    FDM_PRECISION_FP64 = 2
} fdm_precision;

typedef struct fdm_options {
    int32_t schedule;        /* fdm_schedule                                    */
    int32_t tile_rows;       /* rows per wave tile; 0 picks a default (fused:
                                at most five waves per SIMD where that gives
                                4 to 64 rows); doubled until one instance's
                                launch has at most 2^25 tiles (at the default
                                heights only grids of at most three columns
                                and over 2^29 rows need it); results do not
                                depend on it                                  */
    int32_t fused;           /* reserved, must be 0                             */
    int32_t precision;       /* fdm_precision                                   */
} fdm_options;

/* Per-instance diagnostics (FP64, deterministic: fixed-order compensated
 * reductions). */
typedef struct fdm_stats {
    double t;                /* simulated time: the sum of the steps taken      */
    double dt;               /* the float32 step last used                      */
    int64_t step;            /* steps taken since init                          */
    double sum11, sum12;     /* sum over edges of alpha_11, alpha_12            */
    double sum_abs;          /* sum over edges of |alpha_11| + |alpha_12|       */
    double max_norm;         /* max over k*nx+j of sqrt(a11^2 + a12^2)          */
    double drift11, drift12; /* sum11, sum12 minus their values at the first
                                stats evaluation of this context                */
    int64_t nonfinite;       /* number of index pairs with a NaN or Inf         */
    /* coupled runs (fdm_run with a loading); 0 otherwise */
    double eps13;            /* macroscopic shear strain                        */
    double sigma13;          /* macroscopic shear stress = mean of tau13        */
    double phi_mean;         /* mean of U^p_13 over the layer nodes             */
    double vmax;             /* max |v0| of the last step                       */
} fdm_stats;

typedef struct fdm_ctx fdm_ctx;

/* Set up n_instances >= 1 independent problems (descs[i]) on one stream.
 * Validates every descriptor on the host, computes s_max (max |v0| over the
 * node field on the device, or |v0|, or max(|V1|/dx, |V2|/dy) min(dx,dy)) and
 * dt from the Courant number (sec. 4.3: |v0| dt / dx fixed), allocates the
 * workspace and chooses tiles.  Waits for its own device work before
 * returning.  On any error *out is set to NULL and nothing is leaked. */
fdm_status fdm_transport_init(const fdm_transport_desc *descs, int32_t n_instances,
                              const fdm_options *options, void *hip_stream,
                              fdm_ctx **out);

/* Enqueue n_steps >= 0 time steps of every instance.  One step is the
 * evolution problem of the layer case (sec. 3.2.3, the 2-D form of the
 * sec. 3.2.2 scheme): at every node Step 1 limited slopes (eq. 43-44),
 * Step 2 one-sided derivatives (eq. 46) and speeds (eq. 53), Steps 3-4 the
 * numerical Hamiltonian (eq. 54-55 with the dt -> 0 limit, or at finite dt
 * for FULLY_DISCRETE), then the conservative update of the two density
 * components (the alpha form, eq. 57), once per stage of time_order.
 * alpha11[i], alpha12[i] are the device arrays of instance i (see layout
 * above; float, or double with FDM_PRECISION_FP64); they are read and
 * written in place.  The arrays are passed as void* because their element
 * type follows the context's precision.  Asynchronous: returns after
 * enqueueing. */
fdm_status fdm_transport_step(fdm_ctx *ctx, void *const *alpha11,
                              void *const *alpha12, int32_t n_steps);

/* Diagnostics of every instance's current state into out[0..n_instances-1]:
 * the summed densities, which the alpha form conserves (the Burgers vector,
 * sec. 2.1; eq. 2 keeps div alpha = 0), their drift since the first stats
 * call, the total |alpha| (the annihilation of sec. 4.3 lowers it), the
 * largest |alpha| (whose transport sec. 4.4 discusses, eq. 62) and the
 * non-finite count; see fdm_stats.  The context does not keep array
 * pointers between calls, so the arrays to measure are passed here (as in
 * fdm_transport_step).  Synchronizes the stream.  Returns
 * FDM_ERR_NONFINITE (after filling out) if any instance holds a NaN or Inf. */
fdm_status fdm_transport_stats(fdm_ctx *ctx, void *const *alpha11,
                               void *const *alpha12, fdm_stats *out);

/* Static problem (sec. 3.1.2, homogeneous Green-operator solution) in the
 * layer case (sec. 3.2.1): the layer-averaged shear stress tau_13 at the
 * layer nodes for given densities.
 *
 * Cell: the nx-by-ny layer grid, n3 = cell_l3/dx voxels along x3 (cubic
 * voxels, so dx == dy is required), homogeneous isotropic elasticity
 * (mu > 0, lambda > -2 mu / 3).  The layer is h = layer_h/dx voxels thick
 * (1 <= h <= n3, both whole numbers) and carries U^p = phi e1 (x) e3 with
 * phi the potential of the densities (alpha_12 = D1 phi, alpha_11 = -D2 phi,
 * forward differences) and mean phi_mean (the densities do not fix it).
 * The mean strain is eps13 in the 13 component, zero otherwise.  Output:
 * tau13 = mean over the layer voxels of sigma_13, whose mean over the nodes
 * is 2 mu eps13 - mu (h/n3) phi_mean. */
typedef struct fdm_static_desc {
    int32_t nx, ny;          /* layer grid (as in fdm_transport_desc)           */
    double dx, dy;           /* node spacing, dx == dy                          */
    double mu, lambda;       /* elastic constants (dimensionless: mu = 1)       */
    double layer_h;          /* layer thickness, a whole number of voxels       */
    double cell_l3;          /* cell height along x3, a whole number of voxels  */
    double eps13;            /* macroscopic shear strain                        */
    double phi_mean;         /* mean of U^p_13 over the layer nodes             */
    int32_t precision;       /* fdm_precision: FP64 = double arrays and FFTs,
                              * otherwise float arrays and FFTs               */
    int32_t reserved;        /* must be 0                                       */
} fdm_static_desc;

/* Writes tau13_out[k*nx + j] at the nodes.  alpha11/alpha12/tau13_out are
 * device arrays of nx*ny floats (doubles in FP64 precision), distinct; the
 * densities are read only.  Builds the FFT plans and the multiplier table
 * for the call, runs on hip_stream and returns after the result is complete
 * (synchronous).  Errors: FDM_ERR_INVALID_ARG (checked on the host first),
 * FDM_ERR_OUT_OF_MEMORY, FDM_ERR_DEVICE (message in fdm_last_error(NULL)). */
fdm_status fdm_static_solve(const fdm_static_desc *desc, const void *alpha11,
                            const void *alpha12, void *tau13_out, void *hip_stream);

/* Coupled run (sec. 3.1.1: the static problem solved with the current
 * plastic distortion, then the transport with the new stress; sec. 3.2.1
 * layer case).  Every step:
 *   1. tau13 = fdm_static_solve of the current densities with the current
 *      eps13 and phi_mean (elastic constants, layer_h, cell_l3 below; the
 *      descriptor's dx == dy);
 *   2. celerity at the nodes, stored as float32, with m = mobility times
 *      mobility_field (when given; 0 marks an impenetrable obstacle):
 *      FDM_LAW_THRESHOLD: v0 = -m S(tau13), S the soft threshold
 *        S(t) = sign(t) max(|t| - tau0, 0) (a Peierls-type threshold in the
 *        mobility law, the first lattice-friction approach of sec. 2.3);
 *      FDM_LAW_WIGGLY: v0 = m (tau_y cos(U^p_13 / beta) - tau13), the wiggly
 *        energy G = beta sin(U^p_13/beta) tau_y of sec. 3.2.1 (eq. 56 form),
 *        with U^p_13 = phi at the nodes recovered by the static solve's
 *        transforms (one more inverse FFT per step).  float32 cannot resolve
 *        phi / beta for the paper's beta = 1e-8: use FDM_PRECISION_FP64;
 *      v0 < 0 moves fronts so as to raise U^p_13 where the stress exceeds the
 *      friction;
 *   3. dt = the largest float <= min(cfl min(dx,dy) / max|v0|, dt_max)
 *      (dt_max when v0 = 0), cfl from the descriptor;
 *   4. one transport step (time_order) with v0 frozen;
 *   5. phi_mean -= dt * mean Hhat (Euler: of the state; Heun: the mean of
 *      the two stages' means; midpoint: of the half-step state),
 *      eps13 += strain_rate13 * dt.
 * eps13 and phi_mean give the state at the start of the call; the stats
 * records report it after each chunk. */
typedef enum fdm_law {
    FDM_LAW_THRESHOLD = 0,
    FDM_LAW_WIGGLY = 1
} fdm_law;

typedef struct fdm_loading {
    double strain_rate13;    /* macroscopic shear strain rate                   */
    double tau0;             /* FDM_LAW_THRESHOLD: threshold stress, >= 0       */
    double mobility;         /* 1 / eta (dimensionless), >= 0                   */
    double mu, lambda, layer_h, cell_l3;   /* as in fdm_static_desc           */
    double dt_max;           /* upper bound on the adaptive step, > 0           */
    double eps13;            /* macroscopic shear strain at the start           */
    double phi_mean;         /* mean of U^p_13 over the layer nodes at start    */
    int32_t law;             /* fdm_law                                         */
    int32_t reserved;        /* must be 0                                       */
    double tau_y;            /* FDM_LAW_WIGGLY: friction amplitude, >= 0        */
    double beta;             /* FDM_LAW_WIGGLY: energy period, > 0              */
    const float *mobility_field;  /* optional device array of nx*ny finite
                                     factors >= 0 on the mobility (0: an
                                     obstacle the fronts cannot enter), or NULL */
} fdm_loading;

/* Run n_steps in chunks of `chunk` steps (the last chunk may be shorter).
 * loading == NULL: uncoupled transport; each chunk is replayed from a
 * captured HIP graph and history[c] receives the stats after chunk c
 * (history needs ceil(n_steps/chunk) * n_instances records, instance-major
 * within a chunk).  history may be NULL.  Synchronizes the stream once per
 * chunk when history is given, once at the end otherwise.
 * loading != NULL: the coupled run above, for a context of one instance
 * with the LAW velocity and a CFL-controlled step (dt = 0 in its
 * descriptor) and dx == dy; the descriptor's v0 / v0_field are not used
 * during the run (they are again after it).  The step size, mean slip and
 * mean stress are computed on the device, so steps are enqueued without
 * waiting; with two full chunks or more, they are replayed from a HIP graph
 * captured once per call (where the FFT library's launches can be captured
 * as kernels; otherwise the same kernels are enqueued directly), and the
 * stream is synchronized
 * once per chunk (to read those scalars back, and for the stats record).
 * Results do not depend on the chunk length.  The first call allocates the
 * coupled workspace (FFT plans, a stress and a celerity field, per-tile
 * sums), kept until fdm_destroy. */
fdm_status fdm_run(fdm_ctx *ctx, const fdm_loading *loading, void *const *alpha11,
                   void *const *alpha12, int32_t n_steps, int32_t chunk,
                   fdm_stats *history);

/* The float32 time step of instance i (after init), or -1 on a bad argument. */
double fdm_transport_dt(const fdm_ctx *ctx, int32_t instance);

/* Rows per wave tile that instance i uses (the option, the default rule or
 * the autotuner's choice), or -1 on a bad argument. */
int32_t fdm_tile_rows(const fdm_ctx *ctx, int32_t instance);

/* One timed candidate of fdm_autotune. */
typedef struct fdm_tune_trial {
    int32_t tile_rows;       /* rows per wave tile tried (all instances)        */
    int32_t schedule;        /* FDM_SCHEDULE_BATCHED, _PLAIN or _FUSED          */
    double seconds_per_step; /* fastest timed run of trial_steps steps (two;
                                five for the three fastest candidates)        */
} fdm_tune_trial;

/* Autotuner for the launch shape (not a step of the paper's method: tiling
 * changes no result bit, only speed).  Copies the given state into scratch
 * memory, and on that copy times trial_steps (>= 1) steps for each candidate
 * tile height in {4, 8, 12, 16, 24, 32, 48, 64} (heights above the tallest
 * instance are skipped) and each balanced height: for k = 1 .. 8, the
 * smallest height (at most 512) whose largest launch has at most k waves
 * per SIMD of the device (a wave per tile; four SIMDs per compute unit),
 * so that the SIMDs carry equal work; and, for a context created with
 * FDM_SCHEDULE_AUTO,
 * for each schedule that applies: batched and plain (several instances),
 * and fused (FP32 precision, time_order 2 or 3, semi-discrete scheme).  Each
 * candidate is timed twice; the three fastest are then timed three more
 * times each, interleaved, and the context keeps the fastest of them.  alpha11/alpha12 are read, never
 * written; the step count and diagnostics baseline are unchanged.  Up to
 * max_trials measured candidates are written to trials (may be NULL when
 * max_trials is 0) and their number to *n_trials (may be NULL).  Synchronous:
 * returns after the last trial.  Allocates the scratch copy (state size) for
 * the duration of the call.  Errors: FDM_ERR_INVALID_ARG for bad arguments,
 * FDM_ERR_OUT_OF_MEMORY, FDM_ERR_DEVICE. */
fdm_status fdm_autotune(fdm_ctx *ctx, void *const *alpha11, void *const *alpha12, int32_t trial_steps,
                        fdm_tune_trial *trials, int32_t max_trials, int32_t *n_trials);

/* Allocation-free step, for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc).  It advances one
 * instance by n_steps >= 0 steps exactly as fdm_transport_init(desc, 1, NULL
 * options, hip_stream) + fdm_transport_step + fdm_destroy would -- the same
 * checks, step, kernels, default tile height and result bits -- with float32
 * density arrays (alpha11, alpha12: device arrays of nx*ny floats, read and
 * written in place, distinct), but allocates nothing: the stage buffer and
 * the max |v0| partials live in a static device array of
 * 8 * FDM_NOALLOC_MAX_NODES + 1 KiB bytes (32 MiB), which each GPU the
 * library runs on holds until the process ends.
 *   Limit: nx*ny <= FDM_NOALLOC_MAX_NODES (a 2048 x 2048 grid), else
 *   FDM_ERR_INVALID_ARG.
 *   Sharing: every call on a GPU uses that GPU's one array.  Calls on one
 *   stream are ordered; calls that overlap on one GPU (several streams or
 *   threads) race on the array and give wrong results.  Nothing in it needs
 *   to start at zero (each call writes before it reads).
 *   Synchronisation: asynchronous, except with a celerity field (v0_field),
 *   whose max |v0| is read back (the stream is synchronized once).
 *   Errors: FDM_ERR_INVALID_ARG, FDM_ERR_CFL (checked on the host before any
 *   HIP call, except the bound of a fixed dt over a field), FDM_ERR_DEVICE;
 *   the message is in fdm_last_error(NULL).  No context, nothing sticky. */
#define FDM_NOALLOC_MAX_NODES 4194304
fdm_status fdm_transport_step_noalloc(const fdm_transport_desc *desc, void *alpha11, void *alpha12,
                                      int32_t n_steps, void *hip_stream);

/* Release the context and its workspace (waits for its pending work).
 * NULL is a no-op. */
void fdm_destroy(fdm_ctx *ctx);

/* Static description of a status code. */
const char *fdm_status_string(fdm_status status);

/* Message of the last error on this context ("" if none); valid until the
 * next call on the context.  ctx == NULL gives the last error of a failed
 * fdm_transport_init on this thread. */
const char *fdm_last_error(const fdm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FDM_H */
