/*
 * fdm_oracle.c -- plain FP64 CPU reference of the layer-case transport
 * scheme of Morin, Brenner & Suquet, "Numerical simulation of model problems
 * in plasticity based on field dislocation mechanics" (arXiv:1911.03225).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU path neither
 * links it nor shares a line of code, a header or a constant with it.
 *
 * What is computed.  In the layer case (sec. 3.2.1) the plastic distortion
 * reduces to phi = U^p_13(x1, x2) and the Nye tensor to the two in-plane
 * components alpha_11 = -d2 phi and alpha_12 = d1 phi.  The evolution problem
 * is the scalar Hamilton-Jacobi equation phi_t + H(grad phi) = 0 (eq. 51/56),
 * solved by the central-upwind Godunov-type scheme of sec. 3.2.2 (1D) and
 * sec. 3.2.3 (2D).  The state held here is the gradient of phi on the edges
 * of the pixel-node grid, i.e. the density components themselves:
 *
 *     w_x(j+1/2, k) = alpha_12[k*nx + j]   ( = (phi_{j+1,k} - phi_{jk}) / dx )
 *     w_y(j, k+1/2) = -alpha_11[k*nx + j]  ( = (phi_{j,k+1} - phi_{jk}) / dy )
 *
 * The node update phi^{n+1} = phi^n - dt * Hhat, differenced along x and y,
 * is the conservative update of these components (the alpha form of the
 * transport equation, eq. 57); it keeps the summed densities and the discrete
 * div(alpha) = 0 of eq. (2) to round-off.
 *
 * Steps, in the paper's order (sec. 3.2.2 / 3.2.3):
 *   Step 1  limited second difference of phi, i.e. the limited slope of w
 *           along its own axis: the minmod family of eq. (43)-(44), with
 *           theta = 1 (minmod) and theta = 2 (monotonized central); superbee
 *           is offered as an extra limiter (not in the paper).
 *   Step 2  one-sided derivatives phi_x^+-, phi_y^+- at each node (eq. 46,
 *           applied per axis) and the one-sided local speeds a^+-, b^+- taken
 *           over all four (+-,+-) combinations (eq. 53).
 *   Step 3-4  intermediate-point solution and projection (eq. 54-55), taken
 *           in the limit dt -> 0.  This gives the semi-discrete numerical
 *           Hamiltonian
 *             Hhat = sum_{s,t} w_s v_t H(px^s, py^t)
 *                    + a+ a- /(a+ - a-) (px+ - px-)
 *                    + b+ b- /(b+ - b-) (py+ - py-)
 *           with w_- = a+/(a+ - a-), w_+ = -a-/(a+ - a-) (the 1D projection
 *           of eq. 49) and v_-+ likewise from b.  The 2D weights are the
 *           tensor product of the 1D ones: the two mixed corners of eq. (55)
 *           carry a minus sign (the printed plus signs make the four weights
 *           sum to something other than one).  When a+ = a- (nothing moves
 *           along x) the weights are 1/2 and the x viscosity term is zero.
 *   Time    time_order = 1: one forward-Euler stage of the semi-discrete
 *           scheme (the dt -> 0 form of the printed single stage);
 *           time_order = 2: two-stage SSP Runge-Kutta (Heun);
 *           time_order = 3: explicit midpoint (the "midpoint rule" the
 *           paper names for its second-order step, sec. 3.2.2).  The
 *           celerity is frozen over the whole step, as in sec. 3.2.2.
 *
 * Fully discrete variant (scheme = 1): the steps of sec. 3.2.3 at finite dt,
 * in phi form at every node: Step 1 the piecewise quadratic interpolant of
 * eq. (42) along each axis; Step 2 the speeds as above; Step 3 the
 * interpolant and its slope at the four intermediate points
 * (x_j + a^+- dt, y_k + b^+- dt), each corrected by -dt H of that slope
 * (the midpoint-rule solver); Step 4 the projection with the same
 * tensor-product weights.  The paper defers the 2-D interpolant to another
 * paper; here it is the separable one, phi_jk + X(x - x_j) + Y(y - y_k) with
 * X and Y the 1-D pieces of eq. (42) along the node's row and column.  The
 * node increments phi^{n+1} - phi^n, differenced along x and y, update the
 * densities; one such step is one time step (no Runge-Kutta stages).
 *
 * Hamiltonians:  LAW        H = v0 |p|    (eq. 52 / 56), dH/dp = v0 p/|p|,
 *                                          taken as 0 at p = 0;
 *                PRESCRIBED H = V . p     (eq. 28 with only U^p_13 nonzero,
 *                                          uniform V; used for verification).
 *
 * All arithmetic is IEEE double, evaluated in source order (built without
 * fast-math and without FMA contraction).  Loops over rows may run on
 * several OpenMP threads; every output element is written by exactly one
 * iteration and the reductions are serial, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_LIM_NONE = 0, ORC_LIM_THETA = 1, ORC_LIM_SUPERBEE = 2 };
enum { ORC_LAW = 0, ORC_PRESCRIBED = 1 };
enum { ORC_SEMIDISCRETE = 0, ORC_FULLY_DISCRETE = 1 };

typedef struct {
    int64_t nx, ny;          /* pixel nodes along x1 and x2                */
    double dx, dy;           /* grid spacings                              */
    int32_t limiter;         /* ORC_LIM_*                                  */
    int32_t vkind;           /* ORC_LAW or ORC_PRESCRIBED                  */
    double theta;            /* minmod-family parameter, in [1, 2]         */
    double v0;               /* uniform celerity when v0_field is NULL     */
    double V1, V2;           /* prescribed velocity                        */
    const double *v0_field;  /* nx*ny celerity at nodes, or NULL           */
    int32_t time_order;      /* 1, 2 (Heun) or 3 (explicit midpoint)       */
    int32_t scheme;          /* ORC_SEMIDISCRETE or ORC_FULLY_DISCRETE     */
    double dt;               /* time step                                  */
} orc_problem;

/* ---------------------------------------------------------------- Step 1 */

/* minmod of three arguments (eq. 44): the smallest if all are positive, the
 * largest if all are negative, zero otherwise. */
double orc_minmod3(double x1, double x2, double x3)
{
    if (x1 > 0.0 && x2 > 0.0 && x3 > 0.0) {
        double m = x1;
        if (x2 < m) m = x2;
        if (x3 < m) m = x3;
        return m;
    }
    if (x1 < 0.0 && x2 < 0.0 && x3 < 0.0) {
        double m = x1;
        if (x2 > m) m = x2;
        if (x3 > m) m = x3;
        return m;
    }
    return 0.0;
}

/* Limited slope of w at edge i from the three consecutive edge values
 * w_{i-1}, w_i, w_{i+1} along the edge's own axis.  This is the limited
 * second difference (Delta phi)'_{i} of eq. (43) divided by the spacing:
 * minmod(theta (w_{i+1} - w_i), (w_{i+1} - w_{i-1}) / 2, theta (w_i - w_{i-1})).
 * Superbee (Roe) is max-mod of minmod(2 D-, D+) and minmod(D-, 2 D+). */
double orc_slope(int32_t limiter, double theta, double wm, double w0, double wp)
{
    double dm = w0 - wm;   /* backward difference  */
    double dp = wp - w0;   /* forward difference   */
    if (limiter == ORC_LIM_THETA)
        return orc_minmod3(theta * dp, 0.5 * (wp - wm), theta * dm);
    if (limiter == ORC_LIM_SUPERBEE) {
        if (!(dm * dp > 0.0)) return 0.0;
        double adm = fabs(dm), adp = fabs(dp);
        double s1 = fmin(2.0 * adm, adp);
        double s2 = fmin(adm, 2.0 * adp);
        double mag = s1 > s2 ? s1 : s2;
        return dp > 0.0 ? mag : -mag;
    }
    return 0.0;
}

/* ------------------------------------------------------------ Hamiltonian */

/* H(px, py) and its partial derivatives at one node. */
void orc_hamiltonian(const orc_problem *P, double v0, double px, double py,
                     double *H, double *Hpx, double *Hpy)
{
    if (P->vkind == ORC_PRESCRIBED) {
        *H = P->V1 * px + P->V2 * py;
        *Hpx = P->V1;
        *Hpy = P->V2;
        return;
    }
    double r = sqrt(px * px + py * py);
    *H = v0 * r;
    if (r > 0.0) {
        *Hpx = v0 * px / r;
        *Hpy = v0 * py / r;
    } else {
        *Hpx = 0.0;
        *Hpy = 0.0;
    }
}

/* ------------------------------------------------------ Steps 2, 3 and 4 */

/* Semi-discrete numerical Hamiltonian at one node from its four one-sided
 * derivatives. */
double orc_hhat_node(const orc_problem *P, double v0,
                     double pxm, double pxp, double pym, double pyp)
{
    const double px[2] = {pxm, pxp};   /* index 0 is "-", 1 is "+" */
    const double py[2] = {pym, pyp};
    double H[2][2], Hx[2][2], Hy[2][2];
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t)
            orc_hamiltonian(P, v0, px[s], py[t], &H[s][t], &Hx[s][t], &Hy[s][t]);

    /* Step 2: one-sided local speeds over the four combinations. */
    double ap = 0.0, am = 0.0, bp = 0.0, bm = 0.0;
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) {
            if (Hx[s][t] > ap) ap = Hx[s][t];
            if (Hx[s][t] < am) am = Hx[s][t];
            if (Hy[s][t] > bp) bp = Hy[s][t];
            if (Hy[s][t] < bm) bm = Hy[s][t];
        }

    /* Steps 3-4 (dt -> 0): projection weights and numerical viscosity. */
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
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t)
            hhat += wx[s] * wy[t] * H[s][t];
    hhat += visc_x * (pxp - pxm) + visc_y * (pyp - pym);
    return hhat;
}

static inline int64_t wrap(int64_t i, int64_t n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

/* Work arrays of nx*ny values each, allocated once per run. */
typedef struct {
    double *sx, *sy, *h, *r11, *r12, *u11, *u12;
} orc_work;

static int work_alloc(orc_work *w, int64_t n)
{
    double **f[] = {&w->sx, &w->sy, &w->h, &w->r11, &w->r12, &w->u11, &w->u12};
    int ok = 1;
    for (size_t i = 0; i < sizeof(f) / sizeof(f[0]); ++i) {
        *f[i] = (double *)malloc(sizeof(double) * (size_t)n);
        ok &= *f[i] != NULL;
    }
    return ok;
}

static void work_free(orc_work *w)
{
    free(w->sx);
    free(w->sy);
    free(w->h);
    free(w->r11);
    free(w->r12);
    free(w->u11);
    free(w->u12);
}

/* Numerical Hamiltonian at every node (Steps 1-4); sx, sy hold the slopes. */
static void hhat_field_w(const orc_problem *P, const double *a11, const double *a12,
                         double *hhat, double *sx, double *sy)
{
    const int64_t nx = P->nx, ny = P->ny;

    /* Step 1: limited slopes of w_x = alpha_12 along x and of
     * w_y = -alpha_11 along y, one per edge. */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ny; ++k) {
        for (int64_t j = 0; j < nx; ++j) {
            double wxm = a12[k * nx + wrap(j - 1, nx)];
            double wx0 = a12[k * nx + j];
            double wxp = a12[k * nx + wrap(j + 1, nx)];
            sx[k * nx + j] = orc_slope(P->limiter, P->theta, wxm, wx0, wxp);
            double wym = -a11[wrap(k - 1, ny) * nx + j];
            double wy0 = -a11[k * nx + j];
            double wyp = -a11[wrap(k + 1, ny) * nx + j];
            sy[k * nx + j] = orc_slope(P->limiter, P->theta, wym, wy0, wyp);
        }
    }

    /* Step 2: one-sided derivatives at node (j, k); Steps 2-4: Hhat. */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ny; ++k) {
        for (int64_t j = 0; j < nx; ++j) {
            int64_t e_right = k * nx + j;              /* edge (j+1/2, k) */
            int64_t e_left = k * nx + wrap(j - 1, nx); /* edge (j-1/2, k) */
            int64_t f_up = k * nx + j;                 /* edge (j, k+1/2) */
            int64_t f_down = wrap(k - 1, ny) * nx + j; /* edge (j, k-1/2) */
            double pxp = a12[e_right] - 0.5 * sx[e_right];
            double pxm = a12[e_left] + 0.5 * sx[e_left];
            double pyp = -a11[f_up] - 0.5 * sy[f_up];
            double pym = -a11[f_down] + 0.5 * sy[f_down];
            double v0 = P->v0_field ? P->v0_field[k * nx + j] : P->v0;
            hhat[k * nx + j] = orc_hhat_node(P, v0, pxm, pxp, pym, pyp);
        }
    }
}

/* Numerical Hamiltonian at every node (Steps 1-4). hhat has nx*ny entries. */
void orc_hhat_field(const orc_problem *P, const double *a11, const double *a12,
                    double *hhat)
{
    const int64_t n = P->nx * P->ny;
    double *sx = (double *)malloc(sizeof(double) * n);
    double *sy = (double *)malloc(sizeof(double) * n);
    hhat_field_w(P, a11, a12, hhat, sx, sy);
    free(sx);
    free(sy);
}

/* Rate of the density components: d(alpha_12)/dt = -d1 Hhat and
 * d(alpha_11)/dt = +d2 Hhat, differenced across each edge (eq. 57). */
static void stage_rate_w(const orc_problem *P, const double *a11, const double *a12,
                         double *r11, double *r12, orc_work *w)
{
    const int64_t nx = P->nx, ny = P->ny;
    double *h = w->h;
    hhat_field_w(P, a11, a12, h, w->sx, w->sy);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ny; ++k) {
        for (int64_t j = 0; j < nx; ++j) {
            double h0 = h[k * nx + j];
            double hxp = h[k * nx + wrap(j + 1, nx)];
            double hyp = h[wrap(k + 1, ny) * nx + j];
            r12[k * nx + j] = -(hxp - h0) / P->dx;
            r11[k * nx + j] = (hyp - h0) / P->dy;
        }
    }
}

void orc_stage_rate(const orc_problem *P, const double *a11, const double *a12,
                    double *r11, double *r12)
{
    orc_work w;
    work_alloc(&w, P->nx * P->ny);
    stage_rate_w(P, a11, a12, r11, r12, &w);
    work_free(&w);
}

/* ------------------------------------------- fully discrete scheme (3.2.3) */

/* Step 1: the piece of the quadratic interpolant of eq. (42) that holds
 * x_j + h, as an increment over phi_j, and its slope there.  side = +1 is the
 * piece on [x_j, x_{j+1}] (used for the point x_{j+}, h >= 0), side = -1 the
 * piece on [x_{j-1}, x_j] (the point x_{j-}, h <= 0); the side is explicit so
 * that h = 0 gives that side's one-sided derivative.  D and Dp are
 * (Delta phi) and (Delta phi)' of the piece's edge, d the spacing. */
void orc_interp_piece(int32_t side, double D, double Dp, double d, double h,
                      double *val, double *slope)
{
    if (side > 0) {
        /* phi_j + D (x - x_j)/d + Dp/(2 d^2) (x - x_j)(x - x_{j+1}), x = x_j + h */
        *val = D / d * h + Dp / (2.0 * d * d) * h * (h - d);
        *slope = D / d + Dp / (2.0 * d * d) * ((h - d) + h);
    } else {
        /* phi_{j-1} + D (x - x_{j-1})/d + Dp/(2 d^2) (x - x_{j-1})(x - x_j),
         * with phi_{j-1} = phi_j - D and x - x_{j-1} = d + h */
        *val = -D + D / d * (d + h) + Dp / (2.0 * d * d) * (d + h) * h;
        *slope = D / d + Dp / (2.0 * d * d) * (h + (d + h));
    }
}

/* Steps 2-4 of the fully discrete scheme at one node: the increment
 * phi^{n+1}_jk - phi^n_jk.  Inputs: the densities on the four edges around
 * the node, as w (w_x left and right, w_y below and above), and their limited
 * slopes in the same units ((Delta phi)' divided by the spacing). */
double orc_fd_increment_node(const orc_problem *P, double v0,
                             double wxl, double sxl, double wxr, double sxr,
                             double wyd, double syd, double wyu, double syu)
{
    const double dx = P->dx, dy = P->dy, dt = P->dt;
    double unused;
    /* one-sided derivatives (eq. 46 per axis): the pieces' slopes at the node */
    double px[2], py[2];   /* index 0 is "-", 1 is "+" */
    orc_interp_piece(-1, dx * wxl, dx * sxl, dx, 0.0, &unused, &px[0]);
    orc_interp_piece(+1, dx * wxr, dx * sxr, dx, 0.0, &unused, &px[1]);
    orc_interp_piece(-1, dy * wyd, dy * syd, dy, 0.0, &unused, &py[0]);
    orc_interp_piece(+1, dy * wyu, dy * syu, dy, 0.0, &unused, &py[1]);

    /* Step 2: one-sided local speeds over the four combinations (eq. 53). */
    double ap = 0.0, am = 0.0, bp = 0.0, bm = 0.0;
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) {
            double H, Hx, Hy;
            orc_hamiltonian(P, v0, px[s], py[t], &H, &Hx, &Hy);
            if (Hx > ap) ap = Hx;
            if (Hx < am) am = Hx;
            if (Hy > bp) bp = Hy;
            if (Hy < bm) bm = Hy;
        }

    /* Step 3: interpolant and slope at x_{j-+} = x_j + a^-+ dt and
     * y_{k-+} = y_k + b^-+ dt (separable: the x piece along the row, the y
     * piece along the column). */
    double X[2], Xs[2], Y[2], Ys[2];
    orc_interp_piece(-1, dx * wxl, dx * sxl, dx, am * dt, &X[0], &Xs[0]);
    orc_interp_piece(+1, dx * wxr, dx * sxr, dx, ap * dt, &X[1], &Xs[1]);
    orc_interp_piece(-1, dy * wyd, dy * syd, dy, bm * dt, &Y[0], &Ys[0]);
    orc_interp_piece(+1, dy * wyu, dy * syu, dy, bp * dt, &Y[1], &Ys[1]);

    /* Step 4: projection onto the node, weights a+/(a+ - a-) for the "-"
     * point and -a-/(a+ - a-) for the "+" point along each axis, 1/2 each
     * when nothing moves along that axis. */
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
    for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t) {
            double H, Hx, Hy;
            orc_hamiltonian(P, v0, Xs[s], Ys[t], &H, &Hx, &Hy);
            const double phi_st = (X[s] + Y[t]) - dt * H;   /* phi^{n+1}_{j s, k t} - phi_jk */
            inc += wx[s] * wy[t] * phi_st;
        }
    return inc;
}

/* Node increments phi^{n+1} - phi^n of the fully discrete scheme at every
 * node (Steps 1-4); sx, sy hold the slopes. */
static void fd_increment_field_w(const orc_problem *P, const double *a11, const double *a12, double *inc,
                                 double *sx, double *sy)
{
    const int64_t nx = P->nx, ny = P->ny;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ny; ++k) {
        for (int64_t j = 0; j < nx; ++j) {
            sx[k * nx + j] = orc_slope(P->limiter, P->theta, a12[k * nx + wrap(j - 1, nx)], a12[k * nx + j],
                                       a12[k * nx + wrap(j + 1, nx)]);
            sy[k * nx + j] = orc_slope(P->limiter, P->theta, -a11[wrap(k - 1, ny) * nx + j], -a11[k * nx + j],
                                       -a11[wrap(k + 1, ny) * nx + j]);
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ny; ++k) {
        for (int64_t j = 0; j < nx; ++j) {
            int64_t e_right = k * nx + j, e_left = k * nx + wrap(j - 1, nx);
            int64_t f_up = k * nx + j, f_down = wrap(k - 1, ny) * nx + j;
            double v0 = P->v0_field ? P->v0_field[k * nx + j] : P->v0;
            inc[k * nx + j] = orc_fd_increment_node(P, v0, a12[e_left], sx[e_left], a12[e_right], sx[e_right],
                                                    -a11[f_down], sy[f_down], -a11[f_up], sy[f_up]);
        }
    }
}

/* Node increments phi^{n+1} - phi^n of the fully discrete scheme at every
 * node (Steps 1-4); inc has nx*ny entries. */
void orc_fd_increment_field(const orc_problem *P, const double *a11, const double *a12, double *inc)
{
    const int64_t n = P->nx * P->ny;
    double *sx = (double *)malloc(sizeof(double) * n);
    double *sy = (double *)malloc(sizeof(double) * n);
    fd_increment_field_w(P, a11, a12, inc, sx, sy);
    free(sx);
    free(sy);
}

/* One fully discrete step in place: w_x(j+1/2) += (inc_{j+1} - inc_j)/dx and
 * w_y(k+1/2) += (inc_{k+1} - inc_k)/dy, i.e. the new densities are the
 * differences of phi^{n+1}. */
static void fd_step(const orc_problem *P, double *a11, double *a12, orc_work *w)
{
    const int64_t nx = P->nx, ny = P->ny;
    double *inc = w->h;
    fd_increment_field_w(P, a11, a12, inc, w->sx, w->sy);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ny; ++k) {
        for (int64_t j = 0; j < nx; ++j) {
            double d0 = inc[k * nx + j];
            double dxp = inc[k * nx + wrap(j + 1, nx)];
            double dyp = inc[wrap(k + 1, ny) * nx + j];
            a12[k * nx + j] = a12[k * nx + j] + (dxp - d0) / P->dx;
            a11[k * nx + j] = a11[k * nx + j] - (dyp - d0) / P->dy;
        }
    }
}

/* One time step in place (w: work arrays of nx*ny values). */
static void step_w(const orc_problem *P, double *a11, double *a12, orc_work *w)
{
    if (P->scheme == ORC_FULLY_DISCRETE) {
        fd_step(P, a11, a12, w);
        return;
    }
    const int64_t n = P->nx * P->ny;
    const double dt = P->dt;
    double *r11 = w->r11, *r12 = w->r12;
    stage_rate_w(P, a11, a12, r11, r12, w);
    if (P->time_order == 1) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            a11[i] = a11[i] + dt * r11[i];
            a12[i] = a12[i] + dt * r12[i];
        }
    } else if (P->time_order == 3) {
        /* explicit midpoint: u1 = u + (dt/2) L(u);  u_new = u + dt L(u1). */
        double *u11 = w->u11, *u12 = w->u12;
        const double hdt = 0.5 * dt;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            u11[i] = a11[i] + hdt * r11[i];
            u12[i] = a12[i] + hdt * r12[i];
        }
        stage_rate_w(P, u11, u12, r11, r12, w);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            a11[i] = a11[i] + dt * r11[i];
            a12[i] = a12[i] + dt * r12[i];
        }
    } else {
        /* Heun: u1 = u + dt L(u);  u_new = u/2 + (u1 + dt L(u1))/2. */
        double *u11 = w->u11, *u12 = w->u12;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            u11[i] = a11[i] + dt * r11[i];
            u12[i] = a12[i] + dt * r12[i];
        }
        stage_rate_w(P, u11, u12, r11, r12, w);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            a11[i] = 0.5 * a11[i] + 0.5 * (u11[i] + dt * r11[i]);
            a12[i] = 0.5 * a12[i] + 0.5 * (u12[i] + dt * r12[i]);
        }
    }
}

/* One time step in place. */
void orc_step(const orc_problem *P, double *a11, double *a12)
{
    orc_work w;
    work_alloc(&w, P->nx * P->ny);
    step_w(P, a11, a12, &w);
    work_free(&w);
}

/* n_steps time steps in place (the work arrays are allocated once). */
void orc_run(const orc_problem *P, double *a11, double *a12, int64_t n_steps)
{
    orc_work w;
    work_alloc(&w, P->nx * P->ny);
    for (int64_t s = 0; s < n_steps; ++s)
        step_w(P, a11, a12, &w);
    work_free(&w);
}

/* ---------------------------------------------------------------- Time step */

/* CFL-bounded step: nu * min(dx, dy) / s_max with s_max = max |v0| (LAW) or
 * max(|V1|/dx, |V2|/dy) * min(dx, dy) (PRESCRIBED), rounded down to the
 * nearest single-precision value so both implementations step with the same
 * number.  With s_max = 0 nothing moves and the unit-speed step is used. */
double orc_cfl_dt(const orc_problem *P, double nu)
{
    double h = P->dx < P->dy ? P->dx : P->dy;
    double smax = 0.0;
    if (P->vkind == ORC_PRESCRIBED) {
        double sx = fabs(P->V1) / P->dx, sy = fabs(P->V2) / P->dy;
        smax = (sx > sy ? sx : sy) * h;
    } else if (P->v0_field) {
        for (int64_t i = 0; i < P->nx * P->ny; ++i)
            if (fabs(P->v0_field[i]) > smax) smax = fabs(P->v0_field[i]);
    } else {
        smax = fabs(P->v0);
    }
    double dt = smax > 0.0 ? nu * h / smax : nu * h;
    float f = (float)dt;
    if ((double)f > dt) f = nextafterf(f, 0.0f);
    return (double)f;
}

/* ---------------------------------------------------------------- Diagnostics */

/* Kahan-compensated running sum. */
typedef struct { double s, c; } kahan;
static inline void kahan_add(kahan *k, double x)
{
    double y = x - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/* out[0] = sum alpha_11, out[1] = sum alpha_12, out[2] = sum (|a11| + |a12|),
 * out[3] = max over index pairs of sqrt(a11^2 + a12^2), out[4] = number of
 * non-finite entries.  Serial, fixed order. */
void orc_stats(int64_t n, const double *a11, const double *a12, double *out)
{
    kahan s11 = {0, 0}, s12 = {0, 0}, sab = {0, 0};
    double mx = 0.0, nonfinite = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(a11[i]) || !isfinite(a12[i])) {
            nonfinite += 1.0;
            continue;
        }
        kahan_add(&s11, a11[i]);
        kahan_add(&s12, a12[i]);
        kahan_add(&sab, fabs(a11[i]) + fabs(a12[i]));
        double nrm = sqrt(a11[i] * a11[i] + a12[i] * a12[i]);
        if (nrm > mx) mx = nrm;
    }
    out[0] = s11.s;
    out[1] = s12.s;
    out[2] = sab.s;
    out[3] = mx;
    out[4] = nonfinite;
}

/* ---------------------------------------------------------------- Threads */

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
