"""GPU (HIP, gfx950) path of the fully discrete scheme (sec. 3.2.3, the
paper's finite-step form) against the FP64 oracle, through the C ABI.

Same bar as the semi-discrete scheme: relative L1 over both components,
normalised by the initial L1 norm, at most 1e-5 per started block of 1000
steps.  The cases run at Courant number 0.25, the paper's value: like one
forward-Euler stage, the one-pass step amplifies rounding-size input changes
chaotically at 0.4-0.5 with MC or superbee (a 1e-7 relative perturbation of
the inputs moves the FP64 oracle's own result by 1e-3 to 1e-1 there, against
5e-7 at 0.25), so no float32 evaluation can follow it there.
"""
import numpy as np
import pytest

from gpu_util import compare_run, gpu_run, oracle_problem, rel_l1, to_dev, tolerance
from paper_1911_03225_amd import workloads as W

pytestmark = pytest.mark.gpu

FD = dict(scheme="fully_discrete", time_order=1)


@pytest.fixture(scope="module")
def fdm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_03225_amd import fdm as F
    F.load_library()
    return F


def _assert_report(report):
    for s, e1, einf in report:
        assert e1 <= tolerance(s), "step %d: rel L1 %.3e (rel Linf %.3e)" % (s, e1, einf)


@pytest.mark.parametrize("precision", ["fp32", "fp64_arith", "fp64"])
@pytest.mark.parametrize("limiter", ["minmod", "mc", "superbee"])
def test_fd_colliding_pulses(fdm, oracle, limiter, precision):
    """64x64 opposite Gaussian pulses, LAW v0 = -1, 400 steps."""
    a11, a12 = W.colliding_pulses(64)
    dt, rep, g, o = compare_run(oracle, a11, a12, 400, every=100, options={"precision": precision},
                                limiter=limiter, cfl=0.25, v0=-1.0, **FD)
    _assert_report(rep)
    assert not np.any(g[0])                      # alpha_11 stays exactly 0
    if precision == "fp64":
        assert rep[-1][1] < 1e-12


@pytest.mark.parametrize("limiter", ["minmod", "mc", "superbee", "none"])
def test_fd_ring(fdm, oracle, limiter):
    """A loop expanding (v0 = -1), 300 steps, FP32."""
    a11, a12 = W.ring(160, 144, R=40.0, sigma=4.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 300, every=100, limiter=limiter, cfl=0.25, v0=-1.0, **FD)
    _assert_report(rep)


def test_fd_theta_nonsquare_spacing(fdm, oracle):
    a11, a12 = W.ring(120, 100, R=30.0, sigma=3.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 200, every=100, limiter="theta", theta=1.5, dx=0.8, dy=1.25,
                                cfl=0.25, v0=-1.0, **FD)
    _assert_report(rep)


@pytest.mark.parametrize("V,limiter", [((1.0, 0.5), "mc"), ((-0.7, 0.9), "minmod"), ((0.3, -1.0), "minmod")])
def test_fd_prescribed(fdm, oracle, V, limiter):
    """H = V . p: the step is forward-Euler upwinding.  With MC and a
    velocity against the grid diagonal it is anti-diffusive: a 1e-7 input
    change moves the oracle's own result by 3.4e-6 after 200 steps (V =
    (-0.7, 0.9)), against 2e-7 to 7e-7 with minmod, so MC runs on one case."""
    a11, a12 = W.ring(96, 80, R=20.0, sigma=3.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 200, every=100, limiter=limiter, velocity="prescribed", V=V,
                                cfl=0.25, **FD)
    _assert_report(rep)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_fd_celerity_field(fdm, oracle, precision):
    """A Fourier-mode celerity field of one sign (expansion everywhere),
    diagonal bands, 200 steps."""
    nx, ny = 192, 128
    v0 = -(1.0 + 0.5 * W.fourier_celerity(nx, ny, np.random.default_rng(3))).astype(np.float32)
    a11, a12 = W.diagonal_bands(nx, ny, np.random.default_rng(4), n_bands=12)
    dt, rep, g, o = compare_run(oracle, a11, a12, 200, every=50, options={"precision": precision},
                                limiter="minmod", v0_field=v0, cfl=0.25, **FD)
    _assert_report(rep)


@pytest.mark.parametrize("precision,steps", [("fp64_arith", 20), ("fp64", 100)])
def test_fd_sign_changing_celerity(fdm, oracle, precision, steps):
    """A celerity field that changes sign (fronts pile up and annihilate
    where it does), on bands with exactly empty gaps.  There the fully
    discrete step is ill-conditioned:
    * in the oracle alone a 1e-7 relative change of the inputs moves the
      result by 9e-5 after 50 steps and 2e-2 after 200 (one Euler stage of the
      semi-discrete scheme: 1.3e-7);
    * float32 arithmetic departs by 7e-5 within 10 steps: a float32 numpy
      emulation of the kernel's operations gives 7.5e-5 where the GPU gives
      7.4e-5 -- rounding residues where the scheme has exact zeros change
      one-sided speeds by O(v0);
    * float64 arithmetic on float32 state (FP64_ARITH) follows it for 20
      steps (7.9e-7; 2.8e-5 by step 50).
    So this case runs in FP64_ARITH over 20 steps and in FP64 over 100."""
    nx, ny = 192, 128
    v0 = W.fourier_celerity(nx, ny, np.random.default_rng(3))
    a11, a12 = W.diagonal_bands(nx, ny, np.random.default_rng(4), n_bands=12)
    dt, rep, g, o = compare_run(oracle, a11, a12, steps, every=steps // 2, options={"precision": precision},
                                limiter="minmod", v0_field=v0, cfl=0.25, **FD)
    _assert_report(rep)


def _fd_bitwise_cases():
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    cases = []
    a11, a12 = W.ring(160, 144, R=40.0, sigma=4.0)
    cases.append(("ring-superbee", a11, a12, dict(limiter="superbee", cfl=0.25, v0=-1.0), 300))
    a11, a12 = W.ring(120, 100, R=30.0, sigma=3.0)
    cases.append(("theta-nonsquare-spacing", a11, a12,
                  dict(limiter="theta", theta=1.5, dx=0.8, dy=1.25, cfl=0.25, v0=-1.0), 200))
    a11, a12 = W.ring(96, 80, R=20.0, sigma=3.0)
    cases.append(("prescribed-mc", a11, a12, dict(limiter="mc", velocity="prescribed", V=(-0.7, 0.9), cfl=0.25),
                  200))
    nx, ny = 192, 128
    v0 = f32(W.fourier_celerity(nx, ny, np.random.default_rng(3)))
    a11, a12 = W.diagonal_bands(nx, ny, np.random.default_rng(4), n_bands=12)
    cases.append(("sign-changing-field", a11, a12, dict(limiter="minmod", v0_field=v0, cfl=0.25), 200))
    a11, a12 = W.colliding_pulses(64)
    cases.append(("colliding-pulses-mc", a11, a12, dict(limiter="mc", cfl=0.25, v0=-1.0), 400))
    rng = np.random.default_rng(6503)
    phi = rng.normal(size=(3, 65))
    phi = phi + np.roll(phi, 1, 0) + np.roll(phi, 1, 1)
    cases.append(("odd-65x3", -(np.roll(phi, -1, 0) - phi) - 0.2, np.roll(phi, -1, 1) - phi + 0.3,
                  dict(limiter="superbee", cfl=0.25, v0=-0.8), 20))
    return [(n, f32(x), f32(y), kw, st) for n, x, y, kw, st in cases]


@pytest.mark.parametrize("case", range(6))
def test_fd_fp64_state_matches_oracle_bitwise(fdm, oracle, case):
    """FDM_PRECISION_FP64 evaluates the fully discrete step in the
    definition's form -- the node increments of Steps 1-4 with IEEE
    operations in the oracle's order, the densities updated by their
    differences -- so it follows the oracle bit for bit, also where the
    scheme amplifies rounding-size changes (the sign-changing field)."""
    name, a11, a12, kw, steps = _fd_bitwise_cases()[case]
    dt, out = gpu_run(a11, a12, steps, options={"precision": "fp64"}, **FD, **dict(kw))
    ny, nx = a11.shape
    o11, o12 = oracle.run(oracle_problem(oracle, nx, ny, dt, **FD, **kw), a11, a12, steps)
    g11, g12 = out[-1][1], out[-1][2]
    d = max(np.max(np.abs(g11 - o11)), np.max(np.abs(g12 - o12)))
    assert d == 0.0, (name, d, rel_l1(g11, g12, o11, o12, a11, a12))


ODD = [(1, 1), (1, 9), (9, 1), (3, 5), (65, 3), (61, 61), (121, 67), (120, 2)]


@pytest.mark.parametrize("nx,ny", ODD)
def test_fd_odd_sizes(fdm, oracle, nx, ny):
    rng = np.random.default_rng(nx * 100 + ny)
    phi = rng.normal(size=(ny, nx))
    phi = phi + np.roll(phi, 1, 0) + np.roll(phi, 1, 1)
    a12 = (np.roll(phi, -1, 1) - phi + 0.3).astype(np.float32)
    a11 = (-(np.roll(phi, -1, 0) - phi) - 0.2).astype(np.float32)
    dt, rep, g, o = compare_run(oracle, a11, a12, 20, every=10, limiter="superbee", cfl=0.25, v0=-0.8, **FD)
    _assert_report(rep)


def test_fd_default_time_order_is_one_pass(fdm, oracle):
    """time_order 0 selects the one-pass step for the fully discrete scheme."""
    a11, a12 = W.ring(64, 64, R=16.0, sigma=2.0)
    _, a = gpu_run(a11, a12, 9, limiter="mc", cfl=0.25, scheme="fully_discrete", time_order=0)
    _, b = gpu_run(a11, a12, 9, limiter="mc", cfl=0.25, **FD)
    assert np.array_equal(a[-1][1], b[-1][1]) and np.array_equal(a[-1][2], b[-1][2])


def test_fd_tile_heights_bitwise(fdm):
    """The result does not depend on the tile height (FP32, bit for bit)."""
    a11, a12 = W.ring(200, 150, R=50.0, sigma=4.0)
    outs = []
    for rows in (3, 8, 13, 40):
        _, out = gpu_run(a11, a12, 11, options={"tile_rows": rows}, limiter="superbee", cfl=0.25, **FD)
        outs.append(out[-1])
    for o in outs[1:]:
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])


def _one_sign_field(nx, ny):
    return -(1.0 + 0.5 * W.fourier_celerity(nx, ny, np.random.default_rng(9))).astype(np.float32)


def test_fd_batched_equals_plain(fdm, oracle):
    """Three instances of different sizes, limiters and celerities: batched and
    plain launches agree bit for bit, and each follows the oracle."""
    import torch
    shapes = [(64, 48), (130, 70), (33, 257)]
    lims = ["minmod", "superbee", "mc"]
    states, descs, keep = [], [], []
    for i, ((nx, ny), lim) in enumerate(zip(shapes, lims)):
        a11, a12 = W.ring(nx, ny, R=min(nx, ny) / 4, sigma=2.0)
        v0f = None
        if i == 1:   # a single-sign field (a sign-changing one is ill-conditioned here)
            v0f = to_dev(_one_sign_field(nx, ny))
            keep.append(v0f)
        states.append((a11, a12))
        descs.append(fdm.desc(nx, ny, limiter=lim, cfl=0.25, v0=-1.0, v0_field=v0f, **FD))
    results = {}
    for sched in ("batched", "plain"):
        t = [(to_dev(a), to_dev(b)) for a, b in states]
        ctx = fdm.fdm_transport_init(descs, options={"schedule": sched}, keep=keep)
        fdm.fdm_transport_step(ctx, [x[0] for x in t], [x[1] for x in t], 25)
        torch.cuda.synchronize()
        results[sched] = [(x.cpu().numpy(), y.cpu().numpy()) for x, y in t]
        dts = [fdm.fdm_transport_dt(ctx, i) for i in range(3)]
        fdm.fdm_destroy(ctx)
    for (b11, b12), (p11, p12) in zip(results["batched"], results["plain"]):
        assert np.array_equal(b11, p11) and np.array_equal(b12, p12)
    from gpu_util import oracle_problem
    for i, ((a11, a12), (nx, ny)) in enumerate(zip(states, shapes)):
        v0f = _one_sign_field(nx, ny) if i == 1 else None
        P = oracle_problem(oracle, nx, ny, dts[i], limiter=lims[i], v0=-1.0, v0_field=v0f, **FD)
        o11, o12 = oracle.run(P, a11, a12, 25)
        g11, g12 = results["batched"][i]
        assert rel_l1(g11, g12, o11, o12, a11, a12) <= tolerance(25)


@pytest.mark.parametrize("rows", [9, 16])
def test_fd_loop_2048_short(fdm, oracle, rows):
    """The benchmark's fully discrete leg at full size: the 2048^2 loop,
    superbee, Courant 0.25, 10 steps, at a SIMD-balanced tile height (9) and
    the default rule's (16)."""
    a11, a12 = W.ring(2048, 2048, R=300.0, sigma=6.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 10, every=5, options={"tile_rows": rows},
                                limiter="superbee", cfl=0.25, v0=-1.0, **FD)
    _assert_report(rep)
