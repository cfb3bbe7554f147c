"""Pins of the coupled-run oracle (oracle/coupled.py), CPU only."""
import numpy as np
import pytest

import oracle as T
from oracle import coupled as CP
from oracle import static as S
from paper_1911_03225_amd import workloads as W

KW = dict(dx=1.0, limiter="minmod", cfl=0.4, time_order=2, mu=1.0, lam=1.5, layer_h=3.0, cell_l3=24.0,
          mobility=1.0, strain_rate13=2e-3, dt_max=0.25)


@pytest.fixture(scope="module", autouse=True)
def _built():
    T.build(force=False)


def _rings(nx=48, ny=40, seed=2):
    phi, a11, a12 = W.plateau_rings(nx, ny, seed=seed, count=3, rmin=6.0, rmax=12.0)
    return phi, a11.astype(np.float64), a12.astype(np.float64)


def test_below_threshold_is_elastic_loading():
    phi, a11, a12 = _rings()
    b11, b12, hist = CP.coupled_run(a11, a12, 12, 4, tau0=1e9, eps13=0.001, phi_mean=0.03, **KW)
    assert np.array_equal(b11, a11) and np.array_equal(b12, a12)
    dt = CP.round_down_float(KW["dt_max"])
    for r in hist:
        assert r["vmax"] == 0.0 and r["dt"] == dt and r["phi_mean"] == 0.03
        t = r["step"] * dt
        assert r["t"] == pytest.approx(t, rel=1e-15)
        sig = 2 * (0.001 + KW["strain_rate13"] * t) - 0.03 * 3 / 24
        assert r["sigma13"] == pytest.approx(sig, rel=1e-13, abs=1e-15)


def test_densities_conserved_and_slip_relaxes_the_load():
    phi, a11, a12 = _rings()
    s0 = T.stats(a11, a12)
    b11, b12, hist = CP.coupled_run(a11, a12, 60, 20, tau0=0.005, eps13=0.02, phi_mean=float(phi.mean()), **KW)
    s1 = T.stats(b11, b12)
    assert abs(s1["sum11"] - s0["sum11"]) < 1e-11 and abs(s1["sum12"] - s0["sum12"]) < 1e-11
    assert not np.array_equal(b12, a12)                # fronts moved
    last = hist[-1]
    elastic = 2 * last["eps13"] - phi.mean() * 3 / 24
    assert last["phi_mean"] > phi.mean() and last["sigma13"] < elastic


def test_mean_slip_matches_the_phi_form_of_the_step():
    # Integrate phi itself with the same Hhat fields (phi^{n+1} = phi - dt/2
    # (Hhat(w^n) + Hhat(w^(1)))): its differences are the densities the
    # transport produced and its mean is the tracked mean slip.
    phi, _, _ = _rings(seed=5)
    # float64 differences of phi: exactly compatible densities (the float32
    # ones of the workload are not the gradient of any phi to 1e-13)
    ph = phi.copy()
    a12 = np.roll(ph, -1, axis=1) - ph
    a11 = -(np.roll(ph, -1, axis=0) - ph)
    eps, pm = 0.02, float(phi.mean())
    ny, nx = a11.shape
    c11, c12 = a11.copy(), a12.copy()
    for _ in range(8):
        tau = S.static_tau13(c11, c12, 1.0, 1.0, 1.0, 1.5, 3, 24, eps, pm)
        v0 = (-CP.soft_threshold(tau, 0.005)).astype(np.float32).astype(np.float64)
        vmax = np.max(np.abs(v0))
        dt = CP.round_down_float(min(0.4 / vmax, KW["dt_max"]) if vmax > 0 else KW["dt_max"])
        P = T.Problem(nx, ny, limiter="minmod", v0=v0, time_order=2, dt=dt)
        Pe = T.Problem(nx, ny, limiter="minmod", v0=v0, time_order=1, dt=dt)
        H1 = T.hhat_field(P, c11, c12)
        w11, w12 = T.run(Pe, c11, c12, 1)
        H2 = T.hhat_field(P, w11, w12)
        ph = ph - 0.5 * dt * (H1 + H2)
        c11, c12 = T.run(P, c11, c12, 1)
        pm -= dt * 0.5 * (H1.mean() + H2.mean())
        eps += KW["strain_rate13"] * dt
    d12 = np.roll(ph, -1, axis=1) - ph
    d11 = -(np.roll(ph, -1, axis=0) - ph)
    assert np.max(np.abs(d12 - c12)) < 1e-13 and np.max(np.abs(d11 - c11)) < 1e-13
    assert abs(ph.mean() - pm) < 1e-14
    # and the oracle's run tracks the same numbers
    b11, b12, hist = CP.coupled_run(a11, a12, 8, 8, tau0=0.005, eps13=0.02, phi_mean=float(phi.mean()), **KW)
    assert np.array_equal(b11, c11) and np.array_equal(b12, c12)
    assert hist[-1]["phi_mean"] == pytest.approx(pm, abs=1e-15)


def test_wiggly_without_friction_is_the_zero_threshold_law():
    phi, a11, a12 = _rings()
    kw = dict(KW, eps13=0.02, phi_mean=float(phi.mean()))
    b = CP.coupled_run(a11, a12, 10, 10, law="wiggly", tau_y=0.0, beta=1e-3, tau0=0.0, **kw)
    c = CP.coupled_run(a11, a12, 10, 10, law="threshold", tau0=0.0, **kw)
    assert np.array_equal(b[0], c[0]) and np.array_equal(b[1], c[1])
    assert b[2][-1]["phi_mean"] == c[2][-1]["phi_mean"]


def test_wiggly_friction_slows_the_slip():
    phi, a11, a12 = _rings()
    kw = dict(KW, eps13=0.02, phi_mean=float(phi.mean()))
    free = CP.coupled_run(a11, a12, 40, 40, law="wiggly", tau_y=0.0, beta=1e-3, **kw)[2][-1]["phi_mean"]
    held = CP.coupled_run(a11, a12, 40, 40, law="wiggly", tau_y=0.03, beta=1e-3, **kw)[2][-1]["phi_mean"]
    assert phi.mean() < held < free


def test_obstacles_do_not_move():
    phi, a11, a12 = _rings(seed=9)
    ny, nx = a11.shape
    X, Y = np.meshgrid(np.arange(nx), np.arange(ny))
    field = np.ones((ny, nx), np.float32)
    inside = (X - 20) ** 2 + (Y - 18) ** 2 < 8 ** 2
    field[inside] = 0.0
    b11, b12, _ = CP.coupled_run(a11, a12, 30, 30, tau0=0.002, eps13=0.03, phi_mean=float(phi.mean()),
                                 mobility_field=field, **{k: v for k, v in KW.items()})
    # an x-edge (j+1/2, k) joins nodes (j,k), (j+1,k); a y-edge (j, k+1/2) nodes (j,k), (j,k+1)
    ex = inside & np.roll(inside, -1, axis=1)
    ey = inside & np.roll(inside, -1, axis=0)
    assert ex.sum() > 100
    assert np.array_equal(b12[ex], a12[ex]) and np.array_equal(b11[ey], a11[ey])
    assert not np.array_equal(b12, a12)


def test_fully_discrete_slip_matches_the_phi_form():
    """Fully discrete scheme: phi itself advanced by the node increments has
    the transported densities as differences and the tracked mean slip as
    mean; without a limiter the run equals the one-stage semi-discrete run."""
    phi, _, _ = _rings(seed=6)
    ph = phi.copy()
    a12 = np.roll(ph, -1, axis=1) - ph
    a11 = -(np.roll(ph, -1, axis=0) - ph)
    kw = dict(KW, time_order=1, limiter="mc")
    eps, pm = 0.02, float(phi.mean())
    ny, nx = a11.shape
    c11, c12 = a11.copy(), a12.copy()
    for _ in range(6):
        tau = S.static_tau13(c11, c12, 1.0, 1.0, 1.0, 1.5, 3, 24, eps, pm)
        v0 = (-CP.soft_threshold(tau, 0.005)).astype(np.float32).astype(np.float64)
        vmax = np.max(np.abs(v0))
        dt = CP.round_down_float(min(0.4 / vmax, KW["dt_max"]) if vmax > 0 else KW["dt_max"])
        P = T.Problem(nx, ny, limiter="mc", v0=v0, time_order=1, dt=dt, scheme="fully_discrete")
        inc = T.fd_increment_field(P, c11, c12)
        ph = ph + inc
        c11, c12 = T.run(P, c11, c12, 1)
        pm += inc.mean()
        eps += KW["strain_rate13"] * dt
    d12 = np.roll(ph, -1, axis=1) - ph
    d11 = -(np.roll(ph, -1, axis=0) - ph)
    assert np.max(np.abs(d12 - c12)) < 1e-13 and np.max(np.abs(d11 - c11)) < 1e-13
    b11, b12, hist = CP.coupled_run(a11, a12, 6, 6, tau0=0.005, eps13=0.02, phi_mean=float(phi.mean()),
                                    scheme="fully_discrete", **kw)
    assert np.array_equal(b11, c11) and np.array_equal(b12, c12)
    assert hist[-1]["phi_mean"] == pytest.approx(pm, abs=1e-14)
    kn = dict(kw, limiter="none")
    f = CP.coupled_run(a11, a12, 6, 6, tau0=0.005, eps13=0.02, phi_mean=pm, scheme="fully_discrete", **kn)
    e = CP.coupled_run(a11, a12, 6, 6, tau0=0.005, eps13=0.02, phi_mean=pm, **kn)
    assert np.max(np.abs(f[0] - e[0])) < 1e-13 and np.max(np.abs(f[1] - e[1])) < 1e-13
    assert f[2][-1]["phi_mean"] == pytest.approx(e[2][-1]["phi_mean"], abs=1e-13)


def test_explicit_midpoint_slip_matches_the_phi_form():
    """Explicit midpoint: phi^{n+1} = phi - dt Hhat(u + dt/2 L(u)).  Its
    differences are the densities the midpoint transport produced, and its
    mean is the tracked mean slip."""
    phi, _, _ = _rings(seed=7)
    ph = phi.copy()
    a12 = np.roll(ph, -1, axis=1) - ph
    a11 = -(np.roll(ph, -1, axis=0) - ph)
    eps, pm = 0.02, float(phi.mean())
    ny, nx = a11.shape
    c11, c12 = a11.copy(), a12.copy()
    for _ in range(6):
        tau = S.static_tau13(c11, c12, 1.0, 1.0, 1.0, 1.5, 3, 24, eps, pm)
        v0 = (-CP.soft_threshold(tau, 0.005)).astype(np.float32).astype(np.float64)
        vmax = np.max(np.abs(v0))
        dt = CP.round_down_float(min(0.4 / vmax, KW["dt_max"]) if vmax > 0 else KW["dt_max"])
        P = T.Problem(nx, ny, limiter="minmod", v0=v0, time_order=3, dt=dt)
        Ph = T.Problem(nx, ny, limiter="minmod", v0=v0, time_order=1, dt=0.5 * dt)
        h11, h12 = T.run(Ph, c11, c12, 1)
        H = T.hhat_field(P, h11, h12)
        ph = ph - dt * H
        c11, c12 = T.run(P, c11, c12, 1)
        pm -= dt * H.mean()
        eps += KW["strain_rate13"] * dt
    d12 = np.roll(ph, -1, axis=1) - ph
    d11 = -(np.roll(ph, -1, axis=0) - ph)
    assert np.max(np.abs(d12 - c12)) < 1e-13 and np.max(np.abs(d11 - c11)) < 1e-13
    kw = dict(KW, time_order=3)
    b11, b12, hist = CP.coupled_run(a11, a12, 6, 6, tau0=0.005, eps13=0.02, phi_mean=float(phi.mean()), **kw)
    assert np.array_equal(b11, c11) and np.array_equal(b12, c12)
    assert hist[-1]["phi_mean"] == pytest.approx(pm, abs=1e-15)


@pytest.mark.parametrize("law", ["threshold", "wiggly"])
def test_celerity_of_a_density_free_layer(law):
    """No densities: tau13 is the mean stress 2 mu eps13 - mu (h/L3) <phi>
    everywhere and phi = <phi> at every node, so the celerity is the law
    evaluated by hand (threshold: -m S(tau); wiggly: m (tau_y cos(phi/beta)
    - tau)), the step min(cfl dx / max|v0|, dt_max) rounded down to float32,
    and nothing moves."""
    import math
    ny, nx = 6, 8
    z = np.zeros((ny, nx))
    mu, eps, pm, m = 0.8, 0.013, 0.02, 0.7
    kw = dict(KW, mu=mu, lam=1.2, mobility=m, dt_max=100.0)
    tau = 2 * mu * eps - mu * pm * 3 / 24
    if law == "wiggly":
        v = m * (0.03 * math.cos(pm / 0.007) - tau)
        run = CP.coupled_run(z, z, 1, 1, law="wiggly", tau_y=0.03, beta=0.007, eps13=eps, phi_mean=pm, **kw)
    else:
        v = -m * math.copysign(max(abs(tau) - 0.004, 0.0), tau)
        run = CP.coupled_run(z, z, 1, 1, tau0=0.004, eps13=eps, phi_mean=pm, **kw)
    b11, b12, hist = run
    vmax = abs(float(np.float32(v)))
    assert vmax > 0.0
    r = hist[-1]
    assert r["vmax"] == vmax
    dt = float(np.float32(0.4 / vmax))
    if dt > 0.4 / vmax:
        dt = float(np.nextafter(np.float32(dt), np.float32(0)))
    assert r["dt"] == dt and dt <= 0.4 / vmax and r["t"] == dt
    assert np.all(b11 == 0.0) and np.all(b12 == 0.0) and r["phi_mean"] == pm
    assert r["eps13"] == pytest.approx(eps + KW["strain_rate13"] * dt, rel=1e-15)
    assert r["sigma13"] == pytest.approx(2 * mu * r["eps13"] - mu * pm * 3 / 24, rel=1e-14)
