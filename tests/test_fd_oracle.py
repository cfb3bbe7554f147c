"""Pins of the FP64 oracle's fully discrete scheme (arXiv:1911.03225, sec.
3.2.2 in 1-D and sec. 3.2.3 in 2-D: Steps 1-4 at a finite time step).

What fixes it, besides the oracle itself:
* the quadratic interpolant of eq. (42): it passes through the nodes, its
  slope is the derivative of its value, its curvature is
  (Delta phi)' / dx^2, it reproduces quadratics, and its slopes at the node
  are the one-sided derivatives printed in eq. (46);
* without a limiter the interpolant is piecewise linear, so every
  intermediate value is phi_j + a dt p and its slope is p: the projection then
  reduces exactly to one forward-Euler stage of the semi-discrete scheme
  (whose own pins are in test_oracle_pins.py);
* as dt -> 0 the node increment over dt tends to minus the semi-discrete
  numerical Hamiltonian, with an O(dt) error;
* for H = V . p with V >= 0 only the node itself carries weight (a- = b- = 0),
  so the step is upwinding by forward Euler;
* conservation of the summed densities, div(alpha) = 0, translation,
  mirror and transpose symmetry.
The 1-D printed scheme, re-implemented in test_oracle_pins.py, is also
compared on x-only data (the separable 2-D interpolant reduces to it).
"""
import numpy as np
import pytest

from exact_solutions import densities, half_square_dilation, l1_rel, ring_phi_exact
from paper_1911_03225_amd import workloads as W
from test_oracle_pins import _curl, _mirror_x, _printed_1d_step, _random_state


def _fd(oracle, nx, ny, **kw):
    kw.setdefault("time_order", 1)
    return oracle.Problem(nx, ny, scheme="fully_discrete", **kw)


# ------------------------------------------------------- Step 1: interpolant

@pytest.mark.parametrize("D,Dp,d", [(2.0, 0.5, 1.0), (-0.7, 1.3, 0.4), (0.3, -0.9, 2.5)])
def test_interpolant_passes_through_nodes(oracle, D, Dp, d):
    assert oracle.interp_piece(+1, D, Dp, d, 0.0)[0] == 0.0
    assert oracle.interp_piece(-1, D, Dp, d, 0.0)[0] == 0.0
    assert abs(oracle.interp_piece(+1, D, Dp, d, d)[0] - D) < 1e-15 * (abs(D) + abs(Dp))
    assert abs(oracle.interp_piece(-1, D, Dp, d, -d)[0] + D) < 1e-15 * (abs(D) + abs(Dp))


@pytest.mark.parametrize("side", [-1, 1])
def test_interpolant_slope_and_curvature(oracle, side):
    D, Dp, d = 0.8, -0.35, 0.6
    eps = 1e-6
    for h in np.linspace(0.1, 0.9, 5) * d * side:
        v_p, s_p = oracle.interp_piece(side, D, Dp, d, h + eps)
        v_m, s_m = oracle.interp_piece(side, D, Dp, d, h - eps)
        _, s0 = oracle.interp_piece(side, D, Dp, d, h)
        assert abs((v_p - v_m) / (2 * eps) - s0) < 1e-8
        assert abs((s_p - s_m) / (2 * eps) - Dp / d ** 2) < 1e-7


def test_interpolant_reproduces_quadratics(oracle):
    c2, c1, d = 0.37, -1.2, 0.5
    q = lambda x: c2 * x * x + c1 * x
    # nodes x_{j-1}, x_j = 0, x_{j+1}; second difference c2 * 2 d^2 on both edges
    Dr, Dl, Dp = q(d) - q(0.0), q(0.0) - q(-d), 2.0 * c2 * d * d
    for h in np.linspace(0.0, d, 7):
        v, s = oracle.interp_piece(+1, Dr, Dp, d, h)
        assert abs(v - q(h)) < 1e-15 and abs(s - (2 * c2 * h + c1)) < 1e-14
        v, s = oracle.interp_piece(-1, Dl, Dp, d, -h)
        assert abs(v - q(-h)) < 1e-15 and abs(s - (-2 * c2 * h + c1)) < 1e-14


def test_interpolant_slopes_at_node_are_eq46(oracle):
    D_l, Dp_l, D_r, Dp_r, d = 0.4, 0.2, -0.3, 0.5, 0.8
    assert abs(oracle.interp_piece(+1, D_r, Dp_r, d, 0.0)[1] - (D_r / d - Dp_r / (2 * d))) < 1e-15
    assert abs(oracle.interp_piece(-1, D_l, Dp_l, d, 0.0)[1] - (D_l / d + Dp_l / (2 * d))) < 1e-15


# ---------------------------------------------- reductions to known schemes

@pytest.mark.parametrize("kind", ["law_uniform", "law_field", "prescribed"])
def test_no_limiter_equals_one_euler_stage(oracle, kind):
    """sigma = 0: piecewise-linear interpolant, so the projection is exactly
    the semi-discrete Hhat times -dt; the whole step equals time_order 1."""
    nx, ny, dx, dy = 26, 22, 0.8, 1.1
    a11, a12 = _random_state(nx, ny, 21, dx, dy)
    kw = dict(dx=dx, dy=dy, limiter="none")
    if kind == "law_uniform":
        kw.update(v0=-0.9)
    elif kind == "law_field":
        kw.update(v0=W.fourier_celerity(nx, ny, np.random.default_rng(22), kmax=2).astype(np.float64))
    else:
        kw.update(vkind="prescribed", V=(0.7, -0.4))
    F = _fd(oracle, nx, ny, **kw)
    S = oracle.Problem(nx, ny, time_order=1, **kw)
    F.dt = S.dt = oracle.cfl_dt(S, 0.45)
    inc = oracle.fd_increment_field(F, a11, a12)
    hh = oracle.hhat_field(S, a11, a12)
    assert np.max(np.abs(inc + F.dt * hh)) < 1e-14 * np.max(np.abs(hh))
    b11, b12 = oracle.run(F, a11, a12, 5)
    c11, c12 = oracle.run(S, a11, a12, 5)
    scale = np.max(np.abs(c11)) + np.max(np.abs(c12))
    assert np.max(np.abs(b11 - c11)) < 1e-13 * scale and np.max(np.abs(b12 - c12)) < 1e-13 * scale


@pytest.mark.parametrize("limiter", ["minmod", "mc", "superbee"])
def test_prescribed_nonnegative_velocity_is_euler_upwind(oracle, limiter):
    """V >= 0 componentwise: a- = b- = 0, the only weighted point is the
    node itself with the left/lower derivatives, i.e. forward Euler of the
    upwind semi-discrete scheme, for any limiter."""
    nx, ny = 30, 24
    a11, a12 = _random_state(nx, ny, 23)
    kw = dict(limiter=limiter, vkind="prescribed", V=(1.0, 0.5))
    F = _fd(oracle, nx, ny, **kw)
    S = oracle.Problem(nx, ny, time_order=1, **kw)
    F.dt = S.dt = oracle.cfl_dt(S, 0.6)
    b11, b12 = oracle.run(F, a11, a12, 6)
    c11, c12 = oracle.run(S, a11, a12, 6)
    scale = np.max(np.abs(c11)) + np.max(np.abs(c12))
    assert np.max(np.abs(b11 - c11)) < 1e-13 * scale and np.max(np.abs(b12 - c12)) < 1e-13 * scale


@pytest.mark.parametrize("limiter", ["minmod", "mc", "superbee", "theta"])
@pytest.mark.parametrize("field", [False, True])
def test_small_step_limit_is_semidiscrete_hhat(oracle, limiter, field):
    """(phi^{n+1} - phi^n)/dt -> -Hhat with an O(dt) error (2-D, limiters on)."""
    nx, ny = 28, 20
    a11, a12 = _random_state(nx, ny, 24)
    v0 = W.fourier_celerity(nx, ny, np.random.default_rng(25), kmax=2).astype(np.float64) if field else -0.8
    kw = dict(limiter=limiter, theta=1.5 if limiter == "theta" else None, v0=v0)
    S = oracle.Problem(nx, ny, **kw)
    hh = oracle.hhat_field(S, a11, a12)
    errs = []
    for dt in (1e-2, 1e-4, 1e-6):
        F = _fd(oracle, nx, ny, dt=dt, **kw)
        errs.append(np.max(np.abs(-oracle.fd_increment_field(F, a11, a12) / dt - hh)))
    assert errs[0] > 0.0                  # the finite-step terms are active here
    assert errs[1] < 3e-2 * errs[0] + 1e-10
    assert errs[2] < 3e-2 * errs[1] + 1e-9
    assert errs[2] < 1e-5


@pytest.mark.parametrize("theta", [1.0, 1.5, 2.0])
@pytest.mark.parametrize("c", [-1.0, 0.7])
def test_x_only_data_matches_printed_1d_scheme(oracle, theta, c):
    """On x-only data the separable 2-D interpolant reduces to the printed 1-D
    scheme (cross-check against its independent numpy re-implementation)."""
    rng = np.random.default_rng(26)
    n, dx, dt = 96, 0.5, 0.2
    x = np.arange(n) * dx
    L = n * dx
    phi = np.sin(2 * np.pi * x / L) + 0.3 * np.abs(np.sin(6 * np.pi * x / L)) + 0.05 * rng.normal(size=n)
    new = _printed_1d_step(phi, dx, dt, theta, lambda p: c * np.abs(p), lambda p: c * np.sign(p))
    a12 = np.tile((np.roll(phi, -1) - phi) / dx, (3, 1))
    F = _fd(oracle, n, 3, dx=dx, dy=1.0, limiter="theta", theta=theta, v0=c, dt=dt)
    inc = oracle.fd_increment_field(F, np.zeros((3, n)), a12)
    for r in range(3):
        assert np.max(np.abs(inc[r] - (new - phi))) < 1e-14


@pytest.mark.parametrize("c", [-1.0, 0.7])
def test_y_only_data_matches_printed_1d_scheme(oracle, c):
    """The same along y, with dx != dy: alpha_11 = -d2 phi, so w_y = -alpha_11
    carries the 1-D profile and the y pieces use dy."""
    rng = np.random.default_rng(27)
    n, dx, dy, dt, theta = 80, 1.3, 0.6, 0.15, 1.5
    y = np.arange(n) * dy
    L = n * dy
    phi = np.cos(2 * np.pi * y / L) + 0.4 * np.abs(np.sin(4 * np.pi * y / L)) + 0.05 * rng.normal(size=n)
    new = _printed_1d_step(phi, dy, dt, theta, lambda p: c * np.abs(p), lambda p: c * np.sign(p))
    a11 = np.tile((-(np.roll(phi, -1) - phi) / dy)[:, None], (1, 3))
    F = _fd(oracle, 3, n, dx=dx, dy=dy, limiter="theta", theta=theta, v0=c, dt=dt)
    inc = oracle.fd_increment_field(F, a11, np.zeros((n, 3)))
    for col in range(3):
        assert np.max(np.abs(inc[:, col] - (new - phi))) < 1e-14


# -------------------------------------------------------------- invariants

@pytest.mark.parametrize("limiter", ["minmod", "mc", "superbee"])
def test_conservation_and_div_alpha(oracle, limiter):
    nx, ny, dx, dy = 40, 34, 0.7, 1.3
    a11, a12 = _random_state(nx, ny, 27, dx, dy)
    v0 = W.fourier_celerity(nx, ny, np.random.default_rng(28), kmax=1).astype(np.float64)
    F = _fd(oracle, nx, ny, dx=dx, dy=dy, limiter=limiter, v0=v0)
    F.dt = oracle.cfl_dt(F, 0.4)
    s0 = oracle.stats(a11, a12)
    b11, b12 = oracle.run(F, a11, a12, 150)
    s1 = oracle.stats(b11, b12)
    scale = max(s0["sum_abs"], s1["sum_abs"])
    assert abs(s1["sum11"] - s0["sum11"]) <= 1e-12 * scale
    assert abs(s1["sum12"] - s0["sum12"]) <= 1e-12 * scale
    assert np.max(np.abs(_curl(b11, b12, dx, dy))) < 1e-12 * np.max(np.abs(b12))


def test_translation_and_mirror(oracle):
    nx, ny = 32, 28
    a11, a12 = _random_state(nx, ny, 29)
    v0 = np.random.default_rng(30).uniform(-1, 1, (ny, nx))
    F = _fd(oracle, nx, ny, limiter="superbee", v0=v0, dt=0.25)
    b11, b12 = oracle.run(F, a11, a12, 10)
    sh = (5, 9)
    G = _fd(oracle, nx, ny, limiter="superbee", v0=np.roll(v0, sh, (0, 1)), dt=0.25)
    c11, c12 = oracle.run(G, np.roll(a11, sh, (0, 1)), np.roll(a12, sh, (0, 1)), 10)
    assert np.array_equal(c11, np.roll(b11, sh, (0, 1))) and np.array_equal(c12, np.roll(b12, sh, (0, 1)))
    m11, m12 = _mirror_x(a11, a12)
    M = _fd(oracle, nx, ny, limiter="superbee", v0=v0[:, (-np.arange(nx)) % nx], dt=0.25)
    d11, d12 = oracle.run(M, m11, m12, 10)
    e11, e12 = _mirror_x(b11, b12)
    scale = np.max(np.abs(b12)) + np.max(np.abs(b11))
    assert np.max(np.abs(d11 - e11)) < 1e-13 * scale and np.max(np.abs(d12 - e12)) < 1e-13 * scale


@pytest.mark.parametrize("limiter", ["minmod", "superbee"])
def test_transpose_symmetry(oracle, limiter):
    """phi'(x, y) = phi(y, x) exchanges the x and y pieces: with the x pieces
    tied to the printed 1-D scheme above, this ties the y pieces too."""
    n = 30
    a11, a12 = _random_state(n, n, 32)
    v0 = np.random.default_rng(33).uniform(-1, 1, (n, n))
    F = _fd(oracle, n, n, limiter=limiter, v0=v0, dt=0.25)
    b11, b12 = oracle.run(F, a11, a12, 10)
    G = _fd(oracle, n, n, limiter=limiter, v0=v0.T.copy(), dt=0.25)
    c11, c12 = oracle.run(G, -a12.T, -a11.T, 10)
    scale = np.max(np.abs(b12)) + np.max(np.abs(b11))
    assert np.max(np.abs(c12 + b11.T)) < 1e-13 * scale
    assert np.max(np.abs(c11 + b12.T)) < 1e-13 * scale


def test_degenerate_cases(oracle):
    F = _fd(oracle, 1, 1, limiter="mc", v0=-1.0, dt=0.5)
    b11, b12 = oracle.run(F, [[0.3]], [[-0.7]], 4)
    assert b11[0, 0] == 0.3 and b12[0, 0] == -0.7
    a11, a12 = _random_state(16, 12, 31)
    G = _fd(oracle, 16, 12, limiter="superbee", v0=np.zeros((12, 16)), dt=0.5)
    c11, c12 = oracle.run(G, a11, a12, 4)
    assert np.array_equal(c11, a11) and np.array_equal(c12, a12)
    z = np.zeros((12, 16))
    d11, d12 = oracle.run(G, z, z, 3)
    assert not np.any(d11) and not np.any(d12)


def test_one_pass_only(oracle):
    with pytest.raises(ValueError):
        oracle.Problem(8, 8, scheme="fully_discrete", time_order=2)
    with pytest.raises(ValueError):
        oracle.Problem(8, 8, scheme="upwind")


# ------------------------------------- closed forms: against the default

def test_hopf_lax_1d_annihilation_fully_discrete(oracle):
    """Sec. 4.3 set-up with the fully discrete step: the error against the
    exact dilation shrinks under refinement and the waves annihilate."""
    errs = []
    for n in (512, 1024):
        a11, a12, dx = W.half_square_waves(n)
        F = _fd(oracle, n, 1, dx=dx, dy=dx, limiter="minmod", v0=-1.0)
        F.dt = oracle.cfl_dt(F, 0.25)
        ref = np.abs(a12.astype(np.float64)).sum()
        k = int(round(74.2 / F.dt))
        b11, b12 = oracle.run(F, a11, a12, k)
        x = np.arange(n) * dx
        phi = half_square_dilation(x, k * F.dt)
        errs.append(np.abs(b12[0] - (np.roll(phi, -1) - phi) / dx).sum() / ref)
        k2 = int(round((130.0 - k * F.dt) / F.dt))
        c11, c12 = oracle.run(F, b11, b12, k2)
        assert np.abs(c12).sum() / ref < 1e-4
    assert errs[1] < errs[0] and errs[1] < 0.2


def test_hopf_lax_ring_fully_discrete(oracle):
    """Sec. 4.4.1 ring with the fully discrete step: minmod at a small Courant
    number converges under refinement without overshoot.  (The step is
    first order in time and, like a single forward-Euler stage, compressive:
    MC and superbee overshoot the Gaussian cross-section at nu >= 0.25.)"""
    L, R, sigma, t_end = 96.0, 24.0, 3.0, 16.0
    errs, peaks = [], []
    for n in (64, 128):
        dx = L / n
        a11, a12 = densities(ring_phi_exact(n, L, R, sigma, 0.0), dx, dx)
        F = _fd(oracle, n, n, dx=dx, dy=dx, limiter="minmod", v0=-1.0)
        F.dt = oracle.cfl_dt(F, 0.1)
        k = int(round(t_end / F.dt))
        b11, b12 = oracle.run(F, a11, a12, k)
        e11, e12 = densities(ring_phi_exact(n, L, R, sigma, k * F.dt), dx, dx)
        errs.append(l1_rel(b11, b12, e11, e12, a11, a12))
        peaks.append(np.max(np.hypot(b11, b12)) / np.max(np.hypot(a11, a12)))
    assert errs[1] < 0.5 * errs[0] and errs[1] < 0.12
    assert peaks[1] < 1.0


@pytest.mark.parametrize("limiter", ["minmod", "mc"])
def test_sharp_waves_against_heun(oracle, limiter):
    """The comparison with the default on the sec. 4.3 waves (sharp fronts,
    nu = 0.25, t = 74.2): the compressive one-pass step keeps the square
    profiles sharper than the Heun default, whose second stage diffuses."""
    n = 1024
    a11, a12, dx = W.half_square_waves(n)
    x = np.arange(n) * dx
    ref = np.abs(a12.astype(np.float64)).sum()
    err = {}
    for scheme, order in (("fully_discrete", 1), ("semidiscrete", 2)):
        P = oracle.Problem(n, 1, dx=dx, dy=dx, limiter=limiter, v0=-1.0, scheme=scheme, time_order=order)
        P.dt = oracle.cfl_dt(P, 0.25)
        k = int(round(74.2 / P.dt))
        b11, b12 = oracle.run(P, a11, a12, k)
        phi = half_square_dilation(x, k * P.dt)
        err[scheme] = np.abs(b12[0] - (np.roll(phi, -1) - phi) / dx).sum() / ref
    assert err["fully_discrete"] < 0.5 * err["semidiscrete"]
