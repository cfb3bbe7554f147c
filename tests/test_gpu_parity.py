"""GPU (HIP, gfx950) path against the FP64 oracle, through the C ABI.

Tolerance: relative L1 over both components, normalised by the initial L1
norm, at most 1e-5 per started block of 1000 steps, checked at every
snapshot (the FP32 path against the FP64 scheme on the same float32 inputs).
Relative L-infinity is reported in the assertion messages but not gated: at
shocks FP32 rounding moves a front sample by one ulp of the jump.
"""
import numpy as np
import pytest

from gpu_util import compare_run, gpu_run, oracle_problem, rel_l1, state_dtype, to_dev, tolerance
from exact_solutions import densities, ring_phi_exact
from paper_1911_03225_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fdm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_03225_amd import fdm as F
    F.load_library()
    return F


def _assert_report(report, n_total):
    for s, e1, einf in report:
        assert e1 <= tolerance(s), "step %d: rel L1 %.3e (rel Linf %.3e)" % (s, e1, einf)


# -------------------------------------------------- colliding pulses, 64^2

@pytest.mark.parametrize("limiter", ["minmod", "mc", "superbee"])
def test_colliding_pulses(fdm, oracle, limiter):
    """64x64, opposite Gaussian pulses, LAW v0 = -1, Courant 0.5, 400 steps."""
    a11, a12 = W.colliding_pulses(64)
    dt, rep, g, o = compare_run(oracle, a11, a12, 400, every=100, limiter=limiter, cfl=0.5, v0=-1.0)
    assert dt == 0.5
    _assert_report(rep, 400)
    assert not np.any(g[0])                      # alpha_11 stays exactly 0


@pytest.mark.parametrize("ny,V", [(1, (1.0, 0.5)), (64, (1.0, 0.0))])
def test_exact_period(fdm, oracle, ny, V):
    """First order, one stage, Courant number 1 along x on x-only data:
    exact return after 64 steps.  The run is explicitly one-dimensional: a
    single row with V = (1, 0.5) (the y axis has no differences), or the
    64 x 64 grid with V = (1, 0).  V = (1, 0.5) on the 64 x 64 grid at
    dt = 1 is rejected (2-D Courant number 1.5, unstable for general data)."""
    a11, a12 = W.exact_period_profile(64)
    a11, a12 = np.ascontiguousarray(a11[:ny]), np.ascontiguousarray(a12[:ny])
    dt, rep, g, o = compare_run(oracle, a11, a12, 64, every=16, limiter="none", time_order=1,
                                velocity="prescribed", V=V, cfl=1.0)
    assert dt == 1.0
    _assert_report(rep, 64)
    assert np.max(np.abs(g[1] - a12)) <= 1e-6 * np.max(np.abs(a12))


@pytest.mark.parametrize("steps", [7, 8])
def test_single_stage_odd_even(fdm, oracle, steps):
    a11, a12 = W.ring(96, 80, R=20.0, sigma=3.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, steps, limiter="minmod", time_order=1, cfl=0.25, v0=-1.0)
    _assert_report(rep, steps)


# ------------------------------------------------------------- expanding loop

@pytest.mark.parametrize("limiter", ["superbee", "mc"])
def test_ring_1000_steps(fdm, oracle, limiter):
    """The expanding loop at 256^2 (R = 50, sigma = 6), Courant 0.4, 1000 steps."""
    a11, a12 = W.ring(256, 256, R=50.0, sigma=6.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 1000, every=100, limiter=limiter, cfl=0.4, v0=-1.0)
    assert dt == float(np.nextafter(np.float32(0.4), np.float32(0)))
    _assert_report(rep, 1000)


@pytest.mark.parametrize("limiter", ["superbee", "mc"])
def test_loop_2048_short(fdm, oracle, limiter):
    """The loop at its full size (2048^2, R = 300, sigma = 6) for 12 steps, full grid."""
    a11, a12 = W.ring(2048, 2048, R=300.0, sigma=6.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 12, every=6, limiter=limiter, cfl=0.4, v0=-1.0)
    _assert_report(rep, 12)


def _both_precisions(oracle, a11, a12, snaps, **kw):
    """GPU runs in float64-state and FP32 modes against one oracle run."""
    runs = {}
    for prec in ("fp64", "fp32"):
        dt, out = gpu_run(a11, a12, snaps[-1], snapshots=snaps, options={"precision": prec}, **dict(kw))
        runs[prec] = out
    ny, nx = a11.shape
    P = oracle_problem(oracle, nx, ny, dt, **kw)
    o11, o12 = a11.astype(np.float64), a12.astype(np.float64)
    done, rows = 0, []
    for k, s in enumerate(snaps):
        o11, o12 = oracle.run(P, o11, o12, s - done)
        done = s
        e = {p: rel_l1(runs[p][k][1], runs[p][k][2], o11, o12, a11, a12) for p in runs}
        rows.append((s, e["fp64"], e["fp32"]))
    return rows


@pytest.mark.timeout(300)
def test_loop_2048_500_steps(fdm, oracle):
    """The 2048^2 loop for 500 steps: float64 state within 1e-5, FP32 within
    its float32-state bound."""
    a11, a12 = W.ring(2048, 2048, R=300.0, sigma=6.0)
    rows = _both_precisions(oracle, a11, a12, [100, 250, 500], limiter="superbee", cfl=0.4, v0=-1.0)
    for s, e64, e32 in rows:
        assert e64 <= tolerance(s), (s, e64, e32)
        assert e32 <= fp32_loop_bound(s), (s, e64, e32)


@pytest.mark.timeout(300)
def test_loop_1024_full_length(fdm, oracle):
    """The loop scaled to 1024^2 (R = 150) for the full 2000 steps: the loop meets
    its periodic images near step 905 and annihilates along the cell edges."""
    a11, a12 = W.ring(1024, 1024, R=150.0, sigma=6.0)
    rows = _both_precisions(oracle, a11, a12, [500, 1000, 1500, 2000], limiter="mc", cfl=0.4, v0=-1.0)
    for s, e64, e32 in rows:
        assert e64 <= tolerance(s), (s, e64, e32)
        assert e32 <= fp32_loop_bound(s), (s, e64, e32)


def _mean_radius(a11, a12, n):
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x)
    r = np.hypot(X - n / 2, Y - n / 2)
    w = np.hypot(a11, a12)
    return float((w * r).sum() / w.sum())


def test_loop_2048_full_length_properties(fdm):
    """The 2048^2 loop for its full 2000 steps (t ~ 800, past the collision with the
    periodic images at t ~ 724): finite, conserved totals, the loop's radius
    follows R + |v0| t and its peak density is kept (no damping, sec. 4.4.1)
    before the collision."""
    from paper_1911_03225_amd import fdm as F
    import torch
    n, R, sigma = 2048, 300.0, 6.0
    a11, a12 = W.ring(n, n, R=R, sigma=sigma)
    t11, t12 = to_dev(a11), to_dev(a12)
    ctx = F.fdm_transport_init(F.desc(n, n, limiter="superbee", cfl=0.4, v0=-1.0))
    s0 = F.fdm_transport_stats(ctx, t11, t12)[0]
    F.fdm_transport_step(ctx, t11, t12, 1000)
    s1 = F.fdm_transport_stats(ctx, t11, t12)[0]
    dt = F.fdm_transport_dt(ctx)
    g11, g12 = t11.cpu().numpy().astype(np.float64), t12.cpu().numpy().astype(np.float64)
    e11, e12 = densities(ring_phi_exact(n, float(n), R, sigma, 1000 * dt), 1.0, 1.0)
    r_num, r_exact = _mean_radius(g11, g12, n), _mean_radius(e11, e12, n)
    peak = np.max(np.hypot(g11, g12)) / np.max(np.hypot(a11, a12))
    F.fdm_transport_step(ctx, t11, t12, 1000)
    s2 = F.fdm_transport_stats(ctx, t11, t12)[0]
    torch.cuda.synchronize()
    F.fdm_destroy(ctx)
    assert s2["nonfinite"] == 0 and s2["step"] == 2000
    for s in (s1, s2):
        assert abs(s["drift11"]) <= 1e-5 * s0["sum_abs"] and abs(s["drift12"]) <= 1e-5 * s0["sum_abs"]
    assert abs(r_num - r_exact) < 1.0, (r_num, r_exact)
    # superbee over-compresses smooth profiles: the Gaussian cross-section
    # steepens and its peak rises a little (about 12% by t = 400)
    assert 0.95 < peak < 1.2, peak


# ------------------------------------------------------ varying celerity

def test_bands_field_shape_parity(fdm, oracle):
    """Diagonal bands + Fourier celerity field, the 4096^2 recipe scaled to 512^2
    (wave vectors |k| <= 8 per 4096 cells become |k| <= 1), minmod, Courant
    0.45, 300 steps."""
    rng = np.random.default_rng(3)
    a11, a12 = W.diagonal_bands(512, 512, rng, n_bands=16)
    v0 = W.fourier_celerity(512, 512, rng, kmax=1)
    dt, rep, g, o = compare_run(oracle, a11, a12, 300, every=100, limiter="minmod", cfl=0.45,
                                v0_field=v0)
    _assert_report(rep, 300)


def test_bands_field_4096_short(fdm, oracle):
    """Bands under a celerity field at full size (4096^2) for 4 steps, full grid."""
    a11, a12, v0 = W.bands_and_celerity(4096, seed=3)
    dt, rep, g, o = compare_run(oracle, a11, a12, 4, every=2, limiter="minmod", cfl=0.45, v0_field=v0)
    assert dt <= 0.45 / np.abs(v0).max()
    _assert_report(rep, 4)


# ------------------------------------------------------------ edge cases

ODD = [(1, 1), (1, 9), (9, 1), (3, 5), (65, 3), (1000, 3), (7, 130), (61, 61), (121, 67), (60, 4), (120, 2)]


def _odd_state(nx, ny, seed):
    # node differences of a random phi plus a uniform density (curl-free,
    # non-zero even on a 1 x 1 grid)
    rng = np.random.default_rng(seed)
    phi = rng.normal(size=(ny, nx))
    phi = phi + np.roll(phi, 1, 0) + np.roll(phi, 1, 1)
    a11, a12 = densities(phi, 1.0, 1.0)
    return (a11 + 0.3).astype(np.float32), (a12 - 0.2).astype(np.float32)


@pytest.mark.parametrize("nx,ny", ODD)
@pytest.mark.parametrize("limiter", ["superbee", "mc", "minmod"])
def test_odd_sizes(fdm, oracle, nx, ny, limiter):
    a11, a12 = _odd_state(nx, ny, nx * 1000 + ny)
    dt, rep, g, o = compare_run(oracle, a11, a12, 20, every=10, limiter=limiter, cfl=0.4, v0=-0.8)
    _assert_report(rep, 20)


@pytest.mark.parametrize("nx,ny", [(3, 5), (65, 3), (121, 67), (300, 200)])
def test_odd_sizes_smooth_field(fdm, oracle, nx, ny):
    """A celerity field that varies over the whole cell (one Fourier mode
    per axis), minmod."""
    a11, a12 = _odd_state(nx, ny, 7 * nx + ny)
    x = np.arange(nx)[None, :] / nx
    y = np.arange(ny)[:, None] / ny
    v0 = (0.9 * np.cos(2 * np.pi * x) * np.ones((ny, 1)) + 0.1 * np.sin(2 * np.pi * y)).astype(np.float32)
    dt, rep, g, o = compare_run(oracle, a11, a12, 20, every=10, limiter="minmod", cfl=0.4, v0_field=v0)
    _assert_report(rep, 20)


def test_zero_and_immobile(fdm):
    z = np.zeros((33, 70), np.float32)
    dt, out = gpu_run(z, z, 10, limiter="superbee", v0=-1.0)
    assert not np.any(out[-1][1]) and not np.any(out[-1][2])
    rng = np.random.default_rng(1)
    a11, a12 = (x.astype(np.float32) for x in densities(rng.normal(size=(33, 70)), 1.0, 1.0))
    dt, out = gpu_run(a11, a12, 10, limiter="mc", v0_field=np.zeros((33, 70), np.float32))
    assert np.array_equal(out[-1][1], a11) and np.array_equal(out[-1][2], a12)


# ---------------------------------------------------- GPU self-consistency

def test_translation_invariance_bitwise(fdm):
    """Integer periodic shifts commute with the step, bit for bit (catches
    tile-edge and halo mistakes: the strip/chunk boundaries move)."""
    rng = np.random.default_rng(5)
    ny, nx = 130, 150
    a11, a12 = (x.astype(np.float32) for x in densities(rng.normal(size=(ny, nx)), 1.0, 1.0))
    _, base = gpu_run(a11, a12, 25, limiter="superbee", v0=-0.7, options={"tile_rows": 8})
    for sh in [(1, 0), (0, 1), (37, 61), (129, 149)]:
        _, moved = gpu_run(np.roll(a11, sh, (0, 1)), np.roll(a12, sh, (0, 1)), 25, limiter="superbee",
                           v0=-0.7, options={"tile_rows": 8})
        assert np.array_equal(moved[-1][1], np.roll(base[-1][1], sh, (0, 1)))
        assert np.array_equal(moved[-1][2], np.roll(base[-1][2], sh, (0, 1)))


def test_tile_rows_bitwise(fdm):
    a11, a12 = W.ring(200, 170, R=40.0, sigma=4.0)
    outs = [gpu_run(a11, a12, 30, limiter="mc", v0=-1.0, options={"tile_rows": r})[1][-1] for r in (1, 3, 16, 64)]
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])


# Every row of a tile is computed by one of eight unrolled copies of the row
# loop, chosen by the row's offset in its tile; a boundary row's Hhat is
# computed by both tiles.  Results may not depend on the tile height, for
# any limiter, velocity kind or precision (a copy that rounded differently,
# e.g. by fusing another product, showed up only with a celerity field).
@pytest.mark.parametrize("precision", ["fp32", "fp64_arith", "fp64"])
@pytest.mark.parametrize("limiter,kind", [("minmod", "field"), ("superbee", "field"), ("mc", "uniform"),
                                          ("minmod", "uniform"), ("none", "uniform"),
                                          ("superbee", "prescribed")])
def test_tile_rows_bitwise_all_kernels(fdm, limiter, kind, precision):
    rng = np.random.default_rng(5)
    nx, ny = 310, 270
    a11, a12 = W.diagonal_bands(nx, ny, rng, n_bands=6)
    kw = dict(limiter=limiter, cfl=0.4)
    if kind == "field":
        kw["v0_field"] = W.fourier_celerity(nx, ny, rng, kmax=2)
    elif kind == "prescribed":
        kw.update(velocity="prescribed", V=(1.0, -0.5))
    else:
        kw["v0"] = -1.0
    outs = [gpu_run(a11, a12, 24, options={"tile_rows": r, "precision": precision}, **dict(kw))[1][-1]
            for r in (1, 3, 4, 8, 12, 16, 64)]
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])


def test_deterministic(fdm):
    a11, a12, v0 = W.bands_and_celerity(512, seed=7)
    r1 = gpu_run(a11, a12, 50, limiter="minmod", cfl=0.45, v0_field=v0)[1][-1]
    r2 = gpu_run(a11, a12, 50, limiter="minmod", cfl=0.45, v0_field=v0)[1][-1]
    assert np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])


# -------------------------------------------------------------- reductions

def test_stats_match_oracle(fdm, oracle):
    from paper_1911_03225_amd import fdm as F
    a11, a12, v0 = W.bands_and_celerity(1024, seed=11)
    t11, t12 = to_dev(a11), to_dev(a12)
    vf = to_dev(v0)
    ctx = F.fdm_transport_init(F.desc(1024, 1024, limiter="minmod", cfl=0.45, v0_field=vf), keep=[vf])
    for k in range(3):
        s = F.fdm_transport_stats(ctx, t11, t12)[0]
        o = oracle.stats(t11.cpu().numpy(), t12.cpu().numpy())
        assert s["sum11"] == pytest.approx(o["sum11"], rel=1e-14, abs=1e-9)
        assert s["sum12"] == pytest.approx(o["sum12"], rel=1e-14, abs=1e-9)
        assert s["sum_abs"] == pytest.approx(o["sum_abs"], rel=1e-14)
        assert s["max_norm"] == o["max_norm"]
        assert s["nonfinite"] == 0
        F.fdm_transport_step(ctx, t11, t12, 40)
    F.fdm_destroy(ctx)


# ------------------------------------------------- batched, graphs, errors

def _mixed_instances():
    rng = np.random.default_rng(21)
    cases = []
    for (nx, ny), lim, kind in [((64, 64), "minmod", "field"), ((130, 70), "superbee", "uniform"),
                                ((1, 33), "mc", "uniform"), ((256, 128), "minmod", "field"),
                                ((61, 59), "superbee", "uniform"), ((200, 200), "mc", "uniform")]:
        a11, a12 = W.ring(nx, ny, R=max(2.0, min(nx, ny) / 4), sigma=2.0)
        if kind == "field":
            a11, a12 = W.diagonal_bands(nx, ny, rng, n_bands=4)
        v0f = W.fourier_celerity(nx, ny, rng, kmax=1) if kind == "field" else None
        cases.append(dict(nx=nx, ny=ny, a11=a11, a12=a12, limiter=lim, v0_field=v0f,
                          v0=float(rng.choice([-1.0, 1.0]))))
    return cases


def _run_many(F, cases, schedule, n_steps, use_run=False, precision="fp32"):
    import torch
    keep, descs, t11, t12 = [], [], [], []
    for c in cases:
        vf = to_dev(c["v0_field"]) if c["v0_field"] is not None else None
        if vf is not None:
            keep.append(vf)
        descs.append(F.desc(c["nx"], c["ny"], limiter=c["limiter"], cfl=0.4, v0=c["v0"], v0_field=vf))
        t11.append(to_dev(c["a11"], state_dtype({"precision": precision})))
        t12.append(to_dev(c["a12"], state_dtype({"precision": precision})))
    ctx = F.fdm_transport_init(descs, options={"schedule": schedule, "precision": precision}, keep=keep)
    if use_run:
        F.fdm_run(ctx, t11, t12, n_steps, 10)
    else:
        F.fdm_transport_step(ctx, t11, t12, n_steps)
    torch.cuda.synchronize()
    dts = [F.fdm_transport_dt(ctx, i) for i in range(len(cases))]
    F.fdm_destroy(ctx)
    return dts, [(x.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)) for x, y in zip(t11, t12)]


@pytest.mark.parametrize("precision", ["fp32", "fp64_arith", "fp64"])
def test_batched_equals_plain_bitwise_and_oracle(fdm, oracle, precision):
    from paper_1911_03225_amd import fdm as F
    cases = _mixed_instances()
    dts, plain = _run_many(F, cases, "plain", 40, precision=precision)
    dts2, batched = _run_many(F, cases, "batched", 40, precision=precision)
    assert dts == dts2
    # FP32 arithmetic on shock-dominated fronts: see test_shock_dominated_fp32
    bound = FP32_SHOCK_BOUND if precision == "fp32" else tolerance(40)
    for c, p, b, dt in zip(cases, plain, batched, dts):
        assert np.array_equal(p[0], b[0]) and np.array_equal(p[1], b[1])
        P = oracle_problem(oracle, c["nx"], c["ny"], dt, limiter=c["limiter"], v0=c["v0"], v0_field=c["v0_field"])
        o11, o12 = oracle.run(P, c["a11"], c["a12"], 40)
        assert rel_l1(b[0], b[1], o11, o12, c["a11"], c["a12"]) <= bound


# Shock-dominated runs: fronts that collide (annihilation, sec. 4.3) or
# collapse.  Float32 cancellations at the foot of a front leave ~1e-9
# absolute noise in one-sided derivatives that should be ~1e-10; the speed
# v0 p/|p| is discontinuous at p = 0, so the noisy sign of such a corner
# gradient changes a+- by O(|v0|) and Hhat by O(a dp).  FP64 arithmetic (the
# state stays float32) removes it; FP32 arithmetic is held to an empirical
# bound (worst seen 3.4e-4 over 500 steps of the batched recipe's band
# instances, with a margin).
FP32_SHOCK_BOUND = 2e-3


# Float32 *state*: rounding the densities to float32 after every stage is a
# relative perturbation of 6e-8 that the scheme amplifies over hundreds of
# steps (through the same discontinuity); the oracle itself, run with float32
# storage between stages, drifts from its float64 run by 8e-5 (superbee),
# 9e-6 (MC), 5e-5 (minmod) after 600 steps of a 512^2 loop.  The FP32 path is
# held to 1e-6 per step (worst measured: 4.7e-4 after 1000 steps of the
# 2048^2 loop); the float64-state mode to the 1e-5 per 1000 steps bar.
def fp32_loop_bound(n_steps):
    return max(tolerance(n_steps), 1e-6 * n_steps)


FP32_LOOP_BOUND = fp32_loop_bound(100)


def _shock_cases():
    cases = []
    for inst in W.batched_instances():
        if inst.nx == 64 and inst.init == "bands" and inst.velocity == "uniform" and len(cases) < 3:
            a11, a12, _ = inst.make()
            cases.append(("c5-bands-%s" % inst.limiter, a11, a12, inst.limiter, inst.v0, 500))
    a11, a12 = W.ring(130, 70, R=17.5, sigma=2.0)
    cases.append(("ring-collision", a11, a12, "superbee", -1.0, 60))
    a11, a12 = W.ring(200, 200, R=50.0, sigma=2.0)
    cases.append(("ring-collapse", a11, a12, "mc", 1.0, 150))
    return cases


@pytest.mark.parametrize("precision", ["fp64_arith", "fp64"])
@pytest.mark.parametrize("case", range(5))
def test_shock_dominated_fp64(fdm, oracle, case, precision):
    name, a11, a12, lim, v0, steps = _shock_cases()[case]
    dt, rep, g, o = compare_run(oracle, a11, a12, steps, every=max(1, steps // 5),
                                options={"precision": precision}, limiter=lim, cfl=0.4, v0=v0)
    _assert_report(rep, steps)


@pytest.mark.parametrize("case", range(5))
def test_shock_dominated_fp32(fdm, oracle, case):
    name, a11, a12, lim, v0, steps = _shock_cases()[case]
    dt, rep, g, o = compare_run(oracle, a11, a12, steps, every=max(1, steps // 5), limiter=lim, cfl=0.4, v0=v0)
    for s, e1, einf in rep:
        assert e1 <= FP32_SHOCK_BOUND, (name, s, e1)


def test_run_graph_equals_step(fdm):
    from paper_1911_03225_amd import fdm as F
    cases = _mixed_instances()
    _, stepped = _run_many(F, cases, "batched", 45)
    _, ran = _run_many(F, cases, "batched", 45, use_run=True)
    for a, b in zip(stepped, ran):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_run_history(fdm, oracle):
    from paper_1911_03225_amd import fdm as F
    a11, a12 = W.ring(128, 128, R=30.0, sigma=3.0)
    t11, t12 = to_dev(a11), to_dev(a12)
    ctx = F.fdm_transport_init(F.desc(128, 128, limiter="mc", cfl=0.4, v0=-1.0))
    hist = F.fdm_run(ctx, t11, t12, 55, 20)
    assert len(hist) == 3 and [h[0]["step"] for h in hist] == [20, 40, 55]
    dt = F.fdm_transport_dt(ctx)
    assert hist[-1][0]["t"] == pytest.approx(55 * dt)
    o = oracle.stats(t11.cpu().numpy(), t12.cpu().numpy())
    assert hist[-1][0]["sum_abs"] == pytest.approx(o["sum_abs"], rel=1e-14)
    F.fdm_destroy(ctx)


def test_error_paths(fdm):
    from paper_1911_03225_amd import fdm as F
    a11, a12 = W.ring(64, 64, R=16.0, sigma=2.0)
    # a fixed dt above the stability bound
    with pytest.raises(F.FdmError) as e:
        F.fdm_transport_init(F.desc(64, 64, v0=-2.0, dt=0.6))
    assert e.value.status == F.FDM_ERR_CFL
    # ... over a celerity field: checked after the device reduction of max |v0|
    field = to_dev(np.full((64, 64), 0.5, np.float32))
    F.fdm_destroy(F.fdm_transport_init(F.desc(64, 64, v0_field=field, dt=1.0)))     # nu2 = 1
    with pytest.raises(F.FdmError) as e:
        F.fdm_transport_init(F.desc(64, 64, v0_field=field, dt=1.01))
    assert e.value.status == F.FDM_ERR_CFL and "2-D Courant" in F.fdm_last_error(None)
    with pytest.raises(F.FdmError) as e:
        F.fdm_transport_init(F.desc(64, 64, v0_field=field, dt=0.6, time_order=1))
    assert e.value.status == F.FDM_ERR_CFL and "forward-Euler" in F.fdm_last_error(None)
    # a non-finite celerity field
    bad = np.ones((64, 64), np.float32)
    bad[3, 5] = np.nan
    with pytest.raises(F.FdmError) as e:
        F.fdm_transport_init(F.desc(64, 64, v0_field=to_dev(bad)))
    assert e.value.status == F.FDM_ERR_INVALID_ARG
    # NaN in the densities is reported by the diagnostics
    ctx = F.fdm_transport_init(F.desc(64, 64, v0=-1.0))
    t11, t12 = to_dev(a11), to_dev(a12)
    t12[10, 10] = float("nan")
    with pytest.raises(F.FdmError) as e:
        F.fdm_transport_stats(ctx, t11, t12)
    assert e.value.status == F.FDM_ERR_NONFINITE
    s = F.fdm_transport_stats(ctx, t11, t12, allow_nonfinite=True)[0]
    assert s["nonfinite"] == 1
    # aliasing arrays
    with pytest.raises(F.FdmError) as e:
        F.fdm_transport_step(ctx, t11, t11, 1)
    assert e.value.status == F.FDM_ERR_INVALID_ARG
    F.fdm_destroy(ctx)


# ---------------------------------------------------------- batched workload

def _batched_subset():
    """One instance per (size, velocity, limiter) of the batched recipe."""
    seen, out = set(), []
    for inst in W.batched_instances():
        key = (inst.nx, inst.ny, inst.velocity, inst.limiter)
        if key not in seen:
            seen.add(key)
            out.append(inst)
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_subset(fdm, oracle, precision):
    """fp64: float64 state, 1e-5 for every instance.  fp32: the FP32 bar for
    the instance kind (see FP32_LOOP_BOUND and FP32_SHOCK_BOUND)."""
    import torch
    from paper_1911_03225_amd import fdm as F
    steps = 100
    insts = _batched_subset()
    arrays = [i.make() for i in insts]
    keep, descs, t11, t12 = [], [], [], []
    for i, (a11, a12, v) in zip(insts, arrays):
        vf = to_dev(v) if v is not None else None
        if vf is not None:
            keep.append(vf)
        descs.append(F.desc(i.nx, i.ny, limiter=i.limiter, cfl=0.4, v0=i.v0, v0_field=vf))
        t11.append(to_dev(a11, state_dtype({"precision": precision})))
        t12.append(to_dev(a12, state_dtype({"precision": precision})))
    ctx = F.fdm_transport_init(descs, options={"schedule": "batched", "precision": precision}, keep=keep)
    F.fdm_run(ctx, t11, t12, steps, 50, history=False)
    torch.cuda.synchronize()
    dts = [F.fdm_transport_dt(ctx, k) for k in range(len(insts))]
    F.fdm_destroy(ctx)
    failures = []
    for i, (a11, a12, v), g11, g12, dt in zip(insts, arrays, t11, t12, dts):
        P = oracle_problem(oracle, i.nx, i.ny, dt, limiter=i.limiter, v0=i.v0, v0_field=v)
        o11, o12 = oracle.run(P, a11, a12, steps)
        e = rel_l1(g11.cpu().numpy().astype(np.float64), g12.cpu().numpy().astype(np.float64), o11, o12, a11, a12)
        smooth = i.init == "ring" and i.velocity == "uniform"
        bound = tolerance(steps) if precision == "fp64" else (FP32_LOOP_BOUND if smooth else FP32_SHOCK_BOUND)
        if not e <= bound:
            failures.append((i.nx, i.ny, i.velocity, i.limiter, i.init, e))
    assert not failures, failures


# ------------------------------------------- FP64 mode: bit-for-bit oracle

def _bitwise_cases():
    cases = []
    a11, a12 = W.colliding_pulses(64)
    cases.append(("c1-collision", a11, a12, dict(limiter="minmod", cfl=0.5, v0=-1.0), 100))
    a11, a12 = W.ring(130, 70, R=17.5, sigma=2.0)
    cases.append(("ring-collision", a11, a12, dict(limiter="superbee", cfl=0.4, v0=-1.0), 60))
    for inst in W.batched_instances():
        if inst.nx == 128 and inst.init == "bands" and inst.velocity == "uniform" and inst.limiter == "mc":
            a11, a12, _ = inst.make()
            cases.append(("c5-bands-mc", a11, a12, dict(limiter="mc", cfl=0.4, v0=inst.v0), 100))
            break
    rng = np.random.default_rng(3)
    a11, a12 = W.diagonal_bands(96, 80, rng, n_bands=6)
    v0 = W.fourier_celerity(96, 80, rng, kmax=1)
    cases.append(("bands-field", a11, a12, dict(limiter="theta", theta=1.5, cfl=0.45, v0_field=v0), 80))
    a11, a12 = W.ring(61, 67, R=12.0, sigma=3.0)
    cases.append(("euler-prescribed", a11, a12, dict(limiter="superbee", time_order=1, velocity="prescribed",
                                                     V=(0.7, -0.4), cfl=0.3), 31))
    a11, a12 = W.ring(110, 90, R=20.0, sigma=2.5)
    cases.append(("midpoint-ring", a11, a12, dict(limiter="superbee", time_order=3, cfl=0.4, v0=-1.0), 70))
    rng = np.random.default_rng(4)
    a11, a12 = W.diagonal_bands(88, 72, rng, n_bands=5)
    v0 = W.fourier_celerity(88, 72, rng, kmax=1)
    cases.append(("midpoint-field", a11, a12, dict(limiter="minmod", time_order=3, cfl=0.45, v0_field=v0), 60))
    return cases


@pytest.mark.parametrize("case", range(7))
def test_fp64_state_matches_oracle_bitwise(fdm, oracle, case):
    """FDM_PRECISION_FP64 evaluates the oracle's operations in the oracle's
    order with IEEE arithmetic: the results agree bit for bit."""
    name, a11, a12, kw, steps = _bitwise_cases()[case]
    dt, out = gpu_run(a11, a12, steps, options={"precision": "fp64"}, **dict(kw))
    ny, nx = a11.shape
    P = oracle_problem(oracle, nx, ny, dt, **kw)
    o11, o12 = oracle.run(P, a11, a12, steps)
    g11, g12 = out[-1][1], out[-1][2]
    d = max(np.max(np.abs(g11 - o11)), np.max(np.abs(g12 - o12)))
    assert d == 0.0, (name, d, rel_l1(g11, g12, o11, o12, a11, a12))


# ------------------------------------------------------- explicit midpoint

def test_midpoint_fp32_matches_oracle(fdm, oracle):
    """time_order 3 (explicit midpoint) on the ring, MC, 600 steps: the
    float32 path is held to the same loop bound as Heun."""
    a11, a12 = W.ring(256, 256, R=60.0, sigma=4.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 600, every=200, limiter="mc", cfl=0.4, v0=-1.0, time_order=3)
    for s_, e1, einf in rep:
        assert e1 <= fp32_loop_bound(s_), (s_, e1, einf)


def test_midpoint_smooth_meets_tolerance(fdm, oracle):
    (a11, a12), dx = W.smooth_sine(128, L=128.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 300, every=100, limiter="minmod", cfl=0.4,
                                velocity="prescribed", V=(1.0, 0.5), time_order=3)
    for s_, e1, einf in rep:
        assert e1 <= tolerance(s_), (s_, e1, einf)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_midpoint_tile_rows_schedules_and_graph_bitwise(fdm, precision):
    from paper_1911_03225_amd import fdm as F
    rng = np.random.default_rng(6)
    a11, a12 = W.diagonal_bands(150, 130, rng, n_bands=5)
    v0 = W.fourier_celerity(150, 130, rng, kmax=1)
    kw = dict(limiter="superbee", time_order=3, cfl=0.4, v0_field=v0)
    outs = [gpu_run(a11, a12, 20, options={"tile_rows": r, "precision": precision}, **dict(kw))[1][-1]
            for r in (1, 5, 12, 64)]
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])
    cases = _mixed_instances()
    for c in cases:
        c["limiter"] = "mc"
    import torch
    res = {}
    for sched, use_run in (("plain", False), ("batched", False), ("batched", True)):
        keep, descs, t11, t12 = [], [], [], []
        for c in cases:
            vf = to_dev(c["v0_field"]) if c["v0_field"] is not None else None
            if vf is not None:
                keep.append(vf)
            descs.append(F.desc(c["nx"], c["ny"], limiter="mc", cfl=0.4, v0=c["v0"], v0_field=vf, time_order=3))
            t11.append(to_dev(c["a11"], state_dtype({"precision": precision})))
            t12.append(to_dev(c["a12"], state_dtype({"precision": precision})))
        ctx = F.fdm_transport_init(descs, options={"schedule": sched, "precision": precision}, keep=keep)
        if use_run:
            F.fdm_run(ctx, t11, t12, 20, 10)
        else:
            F.fdm_transport_step(ctx, t11, t12, 20)
        torch.cuda.synchronize()
        res[(sched, use_run)] = [(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(t11, t12)]
        F.fdm_destroy(ctx)
    ref = res[("plain", False)]
    for k, v in res.items():
        for (a, b), (c_, d) in zip(v, ref):
            assert np.array_equal(a, c_) and np.array_equal(b, d), k


# ------------------------------------------------------------- step size

STEP_CASES = [
    dict(nx=32, ny=24, dx=1.0, dy=1.0, cfl=0.4, v0=-1.0),
    dict(nx=32, ny=24, dx=0.7, dy=1.9, cfl=0.45, v0=2.3),
    dict(nx=40, ny=16, dx=1.3, dy=0.6, cfl=0.5, velocity="prescribed", V=(0.7, -0.4)),
    dict(nx=40, ny=16, dx=1.3, dy=0.6, cfl=0.3, velocity="prescribed", V=(-0.2, 0.9)),
    dict(nx=40, ny=16, dx=0.9, dy=0.9, cfl=0.6, velocity="prescribed", V=(1.0, 0.5)),
    dict(nx=40, ny=1, dx=0.9, dy=0.9, cfl=1.0, velocity="prescribed", V=(1.0, 0.5)),
    dict(nx=64, ny=48, dx=1.1, dy=0.8, cfl=0.45, field=True),
    dict(nx=8, ny=8, dx=1.0, dy=1.0, cfl=0.4, v0=0.0),
]


@pytest.mark.parametrize("case", STEP_CASES)
def test_step_size_equals_oracle(fdm, oracle, case):
    """The CFL step (the largest float32 not above nu min(dx, dy) / s_max,
    s_max per axis for a prescribed velocity, max |v0| of a celerity field
    by a device reduction) is the oracle's, bit for bit."""
    kw = dict(case)
    nx, ny = kw.pop("nx"), kw.pop("ny")
    field = None
    if kw.pop("field", False):
        field = W.fourier_celerity(nx, ny, np.random.default_rng(17), kmax=2).astype(np.float32)
        kw["v0_field"] = to_dev(field)
    ctx = fdm.fdm_transport_init(fdm.desc(nx, ny, **kw), keep=[kw["v0_field"]] if field is not None else [])
    dt = fdm.fdm_transport_dt(ctx)
    fdm.fdm_destroy(ctx)
    vkind = "prescribed" if kw.get("velocity") == "prescribed" else "law"
    f32 = lambda x: float(np.float32(x))   # the library takes velocities as float32
    P = oracle.Problem(nx, ny, dx=kw["dx"], dy=kw["dy"], vkind=vkind, V=tuple(map(f32, kw.get("V", (0.0, 0.0)))),
                       v0=field.astype(np.float64) if field is not None else f32(kw.get("v0", -1.0)))
    assert dt == oracle.cfl_dt(P, kw["cfl"])


@pytest.mark.parametrize("nx,ny,offset,where", [(37, 23, 0, "last"), (37, 23, 1, "last"), (64, 48, 1, "first"),
                                                (64, 48, 0, "middle"), (257, 129, 3, "last"), (256, 64, 0, "last")])
def test_field_max_reduction_layouts(fdm, oracle, nx, ny, offset, where):
    """max |v0| of a celerity field is reduced on the device with vector
    loads where the field is 16-byte aligned and a scalar loop for the rest:
    fields whose size is not a multiple of four, or that start 4, 8 or 12
    bytes past an aligned address, with the largest magnitude at the first,
    a middle or the last node, give the oracle's CFL step bit for bit, and a
    NaN at that node is refused."""
    import torch
    rng = np.random.default_rng(7 * nx + offset)
    field = rng.uniform(-1.0, 1.0, (ny, nx)).astype(np.float32)
    idx = {"first": 0, "middle": nx * ny // 2, "last": nx * ny - 1}[where]
    field.flat[idx] = -3.5
    buf = torch.zeros(nx * ny + 4, dtype=torch.float32, device="cuda:0")
    view = buf[offset:offset + nx * ny].view(ny, nx)
    assert view.data_ptr() % 16 == 4 * offset
    view.copy_(torch.from_numpy(field))
    ctx = fdm.fdm_transport_init(fdm.desc(nx, ny, cfl=0.45, v0_field=view), keep=[buf])
    dt = fdm.fdm_transport_dt(ctx)
    fdm.fdm_destroy(ctx)
    P = oracle.Problem(nx, ny, dx=1.0, dy=1.0, vkind="law", V=(0.0, 0.0), v0=field.astype(np.float64))
    assert dt == oracle.cfl_dt(P, 0.45)
    view.view(-1)[idx] = float("nan")
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_init(fdm.desc(nx, ny, cfl=0.45, v0_field=view), keep=[buf])
    assert e.value.status == fdm.FDM_ERR_INVALID_ARG


# ------------------------------------------------------ extreme aspect ratios

def _long_bands(nx, ny, seed):
    """Node differences of a random periodic phi, smoothed along both axes."""
    rng = np.random.default_rng(seed)
    phi = rng.normal(size=(ny, nx))
    for _ in range(3):
        phi = (phi + np.roll(phi, 1, 0) + np.roll(phi, 1, 1)) / 3.0
    a12 = (np.roll(phi, -1, 1) - phi).astype(np.float32)
    a11 = (-(np.roll(phi, -1, 0) - phi)).astype(np.float32)
    return a11, a12


@pytest.mark.parametrize("nx,ny", [(1 << 20, 3), (5, 1 << 19), (70001, 33)])
def test_extreme_aspect_ratios(fdm, oracle, nx, ny):
    """Rows of a million nodes and columns of half a million (32-bit byte
    offsets near 4 MB, hundreds of thousands of tiles): the FP64 mode equals
    the oracle bit for bit, and FP32 on the plain and fused schedules agrees
    with it to the 1e-5 bar, bit for bit with each other."""
    a11, a12 = _long_bands(nx, ny, nx + ny)
    kw = dict(limiter="mc", cfl=0.4, v0=-1.0)
    dt, f64 = gpu_run(a11, a12, 4, options={"precision": "fp64"}, **kw)
    P = oracle_problem(oracle, nx, ny, dt, **kw)
    o11, o12 = oracle.run(P, a11, a12, 4)
    assert np.array_equal(f64[-1][1], o11) and np.array_equal(f64[-1][2], o12)
    _, plain = gpu_run(a11, a12, 4, options={"schedule": "plain"}, **kw)
    _, fused = gpu_run(a11, a12, 4, options={"schedule": "fused"}, **kw)
    assert np.array_equal(plain[-1][1], fused[-1][1]) and np.array_equal(plain[-1][2], fused[-1][2])
    assert rel_l1(plain[-1][1], plain[-1][2], o11, o12, a11, a12) <= tolerance(4)


@pytest.mark.parametrize("schedule", ["plain", "fused"])
def test_over_4gib_arrays_tile_periodically(fdm, schedule):
    """A 36000^2 grid, 5.2 GB per density array (row offsets beyond 32 bits),
    made of 18 x 18 copies of a 2000^2 loop.  The scheme is local and the
    same at every node, so after 3 steps every copy equals the 2000^2 run
    bit for bit."""
    import torch
    t, m = 2000, 18
    a11, a12 = W.ring(t, t, R=500.0, sigma=6.0)
    kw = dict(limiter="superbee", cfl=0.4, v0=-1.0)
    dt_small, small = gpu_run(a11, a12, 3, options={"schedule": schedule}, **kw)
    s11 = torch.from_numpy(small[-1][1].astype(np.float32)).cuda()
    s12 = torch.from_numpy(small[-1][2].astype(np.float32)).cuda()
    n = t * m
    b11 = to_dev(a11).repeat(m, m)
    b12 = to_dev(a12).repeat(m, m)
    ctx = fdm.fdm_transport_init(fdm.desc(n, n, **kw), options={"schedule": schedule})
    assert fdm.fdm_transport_dt(ctx) == dt_small
    fdm.fdm_transport_step(ctx, b11, b12, 3)
    torch.cuda.synchronize()
    big_stats = fdm.fdm_transport_stats(ctx, b11, b12)[0]
    fdm.fdm_destroy(ctx)
    for big, ref in ((b11, s11), (b12, s12)):
        same = torch.equal(big.view(m, t, m, t), ref.view(1, t, 1, t).expand(m, t, m, t))
        assert same
    # the diagnostics over 1.3e9 nodes: compensated sums of m^2 equal copies
    ctx = fdm.fdm_transport_init(fdm.desc(t, t, **kw))
    small_stats = fdm.fdm_transport_stats(ctx, s11, s12)[0]
    fdm.fdm_destroy(ctx)
    assert big_stats["max_norm"] == small_stats["max_norm"] and big_stats["nonfinite"] == 0
    assert big_stats["sum_abs"] == pytest.approx(m * m * small_stats["sum_abs"], rel=1e-13)
    for k in ("sum11", "sum12"):
        assert abs(big_stats[k] - m * m * small_stats[k]) <= 1e-13 * big_stats["sum_abs"]
    del b11, b12
    torch.cuda.empty_cache()
