"""The fused Heun schedule (both stages in one launch per step, first-stage
densities kept in registers) against the unfused launches and the oracle.

The fused kernel evaluates every node with the same operations as the two
unfused stage kernels, so results must agree bit for bit, whatever the grid
size, tile height, step count (odd counts end in the stage buffer and are
copied back) and schedule path (direct steps or graph-replayed chunks).
"""
import numpy as np
import pytest

from gpu_util import compare_run, gpu_run, to_dev, tolerance
from paper_1911_03225_amd import workloads as W

pytestmark = pytest.mark.gpu

FUSED = {"schedule": "fused"}


@pytest.fixture(scope="module")
def fdm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_03225_amd import fdm as F
    F.load_library()
    return F


def _same(a, b):
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


CASES = [
    dict(limiter="superbee", v0=-1.0),
    dict(limiter="mc", v0=0.8),
    dict(limiter="minmod", v0=-0.6),
    dict(limiter="theta", theta=1.4, v0=-1.0),
    dict(limiter="none", v0=-1.0),
    dict(limiter="mc", velocity="prescribed", V=(0.7, -0.4)),
]


@pytest.mark.parametrize("kw", CASES)
@pytest.mark.parametrize("steps", [1, 6, 7])
def test_fused_equals_unfused_bitwise(fdm, kw, steps):
    a11, a12 = W.ring(150, 130, R=35.0, sigma=3.0)
    _, f = gpu_run(a11, a12, steps, options=FUSED, cfl=0.4, **dict(kw))
    _, u = gpu_run(a11, a12, steps, options={"schedule": "plain"}, cfl=0.4, **dict(kw))
    _same(f[-1], u[-1])


@pytest.mark.parametrize("kw", [CASES[0], CASES[2], CASES[5]])
@pytest.mark.parametrize("steps", [1, 6, 7])
def test_fused_midpoint_equals_unfused_bitwise(fdm, kw, steps):
    """The explicit midpoint (time_order 3) fused the same way: stage A takes
    half a step, stage B a full one from the step's initial state."""
    a11, a12 = W.ring(150, 130, R=35.0, sigma=3.0)
    _, f = gpu_run(a11, a12, steps, options=FUSED, cfl=0.4, time_order=3, **dict(kw))
    _, u = gpu_run(a11, a12, steps, options={"schedule": "plain"}, cfl=0.4, time_order=3, **dict(kw))
    _same(f[-1], u[-1])


def test_fused_midpoint_batched_and_oracle(fdm, oracle):
    import torch
    nx, ny = 192, 128
    v0 = W.fourier_celerity(nx, ny, np.random.default_rng(3))
    a11, a12 = W.diagonal_bands(nx, ny, np.random.default_rng(4), n_bands=12)
    dt, rep, g, o = compare_run(oracle, a11, a12, 200, every=100, options=FUSED, limiter="minmod", cfl=0.4,
                                v0_field=v0, time_order=3)
    for s, e1, einf in rep:
        assert e1 <= tolerance(s), (s, e1, einf)
    field = to_dev(v0)
    descs = [fdm.desc(nx, ny, limiter="minmod", cfl=0.4, v0_field=field, time_order=3),
             fdm.desc(70, 90, limiter="superbee", cfl=0.4, v0=-1.0, time_order=3)]
    states = [(a11, a12), W.ring(70, 90, R=20.0, sigma=2.0)]
    res = {}
    for sched in ("fused", "plain"):
        t = [(to_dev(a), to_dev(b)) for a, b in states]
        ctx = fdm.fdm_transport_init(descs, options={"schedule": sched}, keep=[field])
        fdm.fdm_transport_step(ctx, [x[0] for x in t], [x[1] for x in t], 9)
        torch.cuda.synchronize()
        res[sched] = [(x.cpu().numpy(), y.cpu().numpy()) for x, y in t]
        fdm.fdm_destroy(ctx)
    for (f11, f12), (p11, p12) in zip(res["fused"], res["plain"]):
        assert np.array_equal(f11, p11) and np.array_equal(f12, p12)


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 3), (3, 5), (55, 9), (56, 2), (57, 3), (113, 67), (119, 9), (120, 2),
                                   (121, 3), (200, 1), (239, 7), (241, 5), (1, 40)])
def test_fused_odd_sizes_bitwise(fdm, nx, ny):
    rng = np.random.default_rng(nx * 1000 + ny)
    phi = rng.normal(size=(ny, nx))
    phi = phi + np.roll(phi, 1, 0) + np.roll(phi, 1, 1)
    a12 = (np.roll(phi, -1, 1) - phi + 0.3).astype(np.float32)
    a11 = (-(np.roll(phi, -1, 0) - phi) - 0.2).astype(np.float32)
    kw = dict(limiter="superbee", cfl=0.4, v0=-0.8)
    _, f = gpu_run(a11, a12, 5, options=FUSED, **kw)
    _, u = gpu_run(a11, a12, 5, options={"schedule": "plain"}, **kw)
    _same(f[-1], u[-1])


@pytest.mark.parametrize("rows", [1, 3, 12, 64])
def test_fused_tile_heights_bitwise(fdm, rows):
    a11, a12 = W.ring(190, 170, R=45.0, sigma=4.0)
    kw = dict(limiter="superbee", cfl=0.4, v0=-1.0)
    _, f = gpu_run(a11, a12, 9, options={"schedule": "fused", "tile_rows": rows}, **kw)
    _, u = gpu_run(a11, a12, 9, options={"schedule": "plain"}, **kw)
    _same(f[-1], u[-1])


def test_fused_celerity_field_bitwise_and_oracle(fdm, oracle):
    nx, ny = 192, 128
    v0 = W.fourier_celerity(nx, ny, np.random.default_rng(3))
    a11, a12 = W.diagonal_bands(nx, ny, np.random.default_rng(4), n_bands=12)
    _, f = gpu_run(a11, a12, 40, options=FUSED, limiter="minmod", cfl=0.4, v0_field=v0)
    _, u = gpu_run(a11, a12, 40, options={"schedule": "plain"}, limiter="minmod", cfl=0.4, v0_field=v0)
    _same(f[-1], u[-1])
    dt, rep, g, o = compare_run(oracle, a11, a12, 200, every=100, options=FUSED, limiter="minmod", cfl=0.45,
                                v0_field=v0)
    for s, e1, einf in rep:
        assert e1 <= tolerance(s), (s, e1, einf)


def test_fused_ring_oracle_parity(fdm, oracle):
    a11, a12 = W.ring(256, 256, R=60.0, sigma=6.0)
    dt, rep, g, o = compare_run(oracle, a11, a12, 500, every=100, options=FUSED, limiter="superbee", cfl=0.4,
                                v0=-1.0)
    for s, e1, einf in rep:
        assert e1 <= tolerance(s), (s, e1, einf)


def test_loop_2048_fused_balanced_heights(fdm, oracle):
    """The 2048^2 loop (superbee, Courant 0.4) in the launch
    shapes the benchmark runs: the fused schedule at the SIMD-balanced tile
    heights 15 and 19 (graph-replayed chunks), 12 steps against the oracle,
    and bit for bit equal to each other."""
    from gpu_util import oracle_problem, rel_l1
    a11, a12 = W.ring(2048, 2048, R=300.0, sigma=6.0)
    runs = []
    for rows in (15, 19):
        runs.append(_run_chunks(fdm, a11, a12, 12, 6, {"schedule": "fused", "tile_rows": rows},
                                limiter="superbee", cfl=0.4, v0=-1.0))
    (dt, g11, g12), (dt2, h11, h12) = runs
    assert dt == dt2
    assert np.array_equal(g11, h11) and np.array_equal(g12, h12)
    P = oracle_problem(oracle, 2048, 2048, dt, limiter="superbee", cfl=0.4, v0=-1.0)
    o11, o12 = oracle.run(P, a11.astype(np.float64), a12.astype(np.float64), 12)
    e1 = rel_l1(g11, g12, o11, o12, a11, a12)
    assert e1 <= tolerance(12), e1


def test_bands_field_4096_fused_equals_plain(fdm):
    """The celerity-field workload at full size (4096^2 bands under a
    Fourier celerity, minmod, Courant 0.45) in the benchmark's launch shape:
    the fused schedule at 50-row tiles gives the plain schedule's bits after
    an odd number of steps (the last copied back from the stage buffer)."""
    import torch
    a11, a12, v0 = W.bands_and_celerity(4096, seed=3)
    tv = to_dev(v0)
    out = []
    for opts in ({"schedule": "fused", "tile_rows": 50}, {"schedule": "plain"}):
        t11, t12 = to_dev(a11), to_dev(a12)
        ctx = fdm.fdm_transport_init(fdm.desc(4096, 4096, limiter="minmod", cfl=0.45, v0_field=tv),
                                     options=opts, keep=[tv])
        fdm.fdm_run(ctx, t11, t12, 3, 3)
        torch.cuda.synchronize()
        out.append((t11.cpu().numpy(), t12.cpu().numpy()))
        fdm.fdm_destroy(ctx)
        del t11, t12
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("n", [256, 2048, 4096])
def test_fused_default_tile_height(fdm, n):
    """Without a height asked for, a fused context tiles at the smallest
    height with at most five waves (one per 56-column tile) per SIMD, or by
    the unfused rule where that height is below 4 or above 64 rows; the
    results do not depend on it (the bitwise tests above)."""
    import torch
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    strips = -(-n // 56)
    r = next(r for r in range(1, n + 1) if strips * -(-n // r) <= 5 * simds)
    if not 4 <= r <= 64:   # the unfused rule: (strip, row) pairs / 6144, up to a multiple of 4, in [4, 16]
        rows = -(-(-(-n // 60) * n) // 6144)
        r = min(16, max(4, -(-rows // 4) * 4), n)
    ctx = fdm.fdm_transport_init(fdm.desc(n, n, limiter="superbee", cfl=0.4, v0=-1.0), options=FUSED)
    assert fdm.fdm_tile_rows(ctx, 0) == r
    fdm.fdm_destroy(ctx)


def _run_chunks(F, a11, a12, steps, chunk, options, **kw):
    import torch
    ny, nx = a11.shape
    t11, t12 = to_dev(a11), to_dev(a12)
    ctx = F.fdm_transport_init(F.desc(nx, ny, **kw), options=options)
    assert F.fdm_tile_rows(ctx, 0) == options["tile_rows"]
    F.fdm_run(ctx, t11, t12, steps, chunk)
    torch.cuda.synchronize()
    dt = F.fdm_transport_dt(ctx)
    F.fdm_destroy(ctx)
    return dt, t11.cpu().numpy().astype(np.float64), t12.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("chunk", [5, 8])
def test_fused_graph_chunks_bitwise(fdm, chunk):
    """fdm_run replays captured chunks (odd chunks end with the copy back)."""
    import torch
    a11, a12 = W.ring(160, 120, R=30.0, sigma=3.0)
    outs = []
    for opts in (FUSED, {"schedule": "plain"}):
        t11, t12 = to_dev(a11), to_dev(a12)
        ctx = fdm.fdm_transport_init(fdm.desc(160, 120, limiter="mc", cfl=0.4, v0=-1.0), options=opts)
        hist = fdm.fdm_run(ctx, t11, t12, 3 * chunk, chunk)
        torch.cuda.synchronize()
        outs.append((t11.cpu().numpy(), t12.cpu().numpy(), [h[0]["sum_abs"] for h in hist]))
        fdm.fdm_destroy(ctx)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


@pytest.mark.parametrize("schedule", ["fused", "plain"])
def test_graph_replays_each_equal_direct_steps(fdm, schedule):
    """fdm_run keeps one captured graph per chunk length and array set: call
    it four times for one chunk each (one capture, three replays), with
    eager device work, a host copy and a synchronisation between calls, and
    compare every replay bitwise with the same steps enqueued directly."""
    import torch
    a11, a12 = W.ring(150, 110, R=28.0, sigma=3.0)
    opts = {"schedule": schedule}
    ctxs, states = [], []
    for _ in range(2):
        ctxs.append(fdm.fdm_transport_init(fdm.desc(150, 110, limiter="superbee", cfl=0.4, v0=-1.0),
                                           options=opts))
        states.append((to_dev(a11), to_dev(a12)))
    (g11, g12), (e11, e12) = states
    chunk = 6
    for rep in range(4):
        assert fdm.fdm_run(ctxs[0], g11, g12, chunk, chunk, history=False) is None
        fdm.fdm_transport_step(ctxs[1], e11, e12, chunk)
        torch.cuda.synchronize()
        assert np.array_equal(g11.cpu().numpy(), e11.cpu().numpy()), rep
        assert np.array_equal(g12.cpu().numpy(), e12.cpu().numpy()), rep
        assert fdm.fdm_transport_stats(ctxs[0], g11, g12) == fdm.fdm_transport_stats(ctxs[1], e11, e12)
        # eager work of the caller's own on the device between replays
        scratch = (g11 * 2.0 + e12).sum()
        torch.cuda.synchronize()
        assert np.isfinite(float(scratch))
    for c in ctxs:
        fdm.fdm_destroy(c)


def test_fused_several_instances_equal_batched(fdm):
    """Several instances: one batched fused launch per step for all of them
    (different sizes, limiters, a celerity field, a prescribed velocity)."""
    import torch
    shapes = [(64, 48), (130, 70), (33, 257), (200, 9)]
    lims = ["minmod", "superbee", "mc", "superbee"]
    states = [W.ring(nx, ny, R=min(nx, ny) / 4, sigma=2.0) for nx, ny in shapes]
    field = to_dev(W.fourier_celerity(130, 70, np.random.default_rng(9)))
    descs = [fdm.desc(64, 48, limiter="minmod", cfl=0.4, v0=-1.0),
             fdm.desc(130, 70, limiter="superbee", cfl=0.4, v0_field=field),
             fdm.desc(33, 257, limiter="mc", cfl=0.4, v0=0.7),
             fdm.desc(200, 9, limiter="superbee", cfl=0.4, velocity="prescribed", V=(-0.6, 0.8))]
    res = {}
    for sched in ("fused", "batched", "plain"):
        t = [(to_dev(a), to_dev(b)) for a, b in states]
        ctx = fdm.fdm_transport_init(descs, options={"schedule": sched}, keep=[field])
        fdm.fdm_transport_step(ctx, [x[0] for x in t], [x[1] for x in t], 11)
        torch.cuda.synchronize()
        res[sched] = [(x.cpu().numpy(), y.cpu().numpy()) for x, y in t]
        fdm.fdm_destroy(ctx)
    for other in ("batched", "plain"):
        for (f11, f12), (b11, b12) in zip(res["fused"], res[other]):
            assert np.array_equal(f11, b11) and np.array_equal(f12, b12)


def test_autotune_tries_the_fused_schedule(fdm):
    """AUTO on an FP32 Heun context also times the fused launches; the tuned
    context gives the same bits as an untuned one."""
    import torch
    a11, a12 = W.ring(256, 256, R=60.0, sigma=4.0)
    t11, t12 = to_dev(a11), to_dev(a12)
    ctx = fdm.fdm_transport_init(fdm.desc(256, 256, limiter="superbee", cfl=0.4, v0=-1.0))
    trials = fdm.fdm_autotune(ctx, [t11], [t12], trial_steps=2)
    assert {t["schedule"] for t in trials} == {"plain", "fused"}
    fdm.fdm_transport_step(ctx, t11, t12, 7)
    torch.cuda.synchronize()
    fdm.fdm_destroy(ctx)
    _, u = gpu_run(a11, a12, 7, options={"schedule": "plain"}, limiter="superbee", cfl=0.4, v0=-1.0)
    assert np.array_equal(t11.cpu().numpy(), u[-1][1]) and np.array_equal(t12.cpu().numpy(), u[-1][2])
    # FP64 contexts do not offer it
    ctx = fdm.fdm_transport_init(fdm.desc(64, 64, limiter="mc", cfl=0.4, v0=-1.0),
                                 options={"precision": "fp64_arith"})
    s11, s12 = to_dev(a11[:64, :64]), to_dev(a12[:64, :64])
    trials = fdm.fdm_autotune(ctx, [s11], [s12], trial_steps=1)
    assert {t["schedule"] for t in trials} == {"plain"}
    fdm.fdm_destroy(ctx)


def test_coupled_run_on_a_fused_context(fdm):
    """A context created with the fused schedule still runs coupled steps
    (they use the stage kernels with their per-tile Hhat sums), with the same
    bits as a plain context."""
    import torch
    phi, a11, a12 = W.plateau_rings(96, 80, seed=2, count=4, rmin=8.0, rmax=20.0)
    out = []
    for sched in ("fused", "plain"):
        t11, t12 = to_dev(a11), to_dev(a12)
        ctx = fdm.fdm_transport_init(fdm.desc(96, 80, limiter="minmod", cfl=0.4, v0=-1.0),
                                     options={"schedule": sched})
        L = fdm.loading(strain_rate13=2e-3, tau0=0.005, mobility=1.0, mu=1.0, lam=1.5, layer_h=3.0,
                        cell_l3=24.0, dt_max=0.25, eps13=0.02, phi_mean=float(phi.mean()))
        hist = fdm.fdm_run(ctx, t11, t12, 20, 10, loading=L)
        fdm.fdm_transport_step(ctx, t11, t12, 3)      # and uncoupled steps after it
        torch.cuda.synchronize()
        out.append((t11.cpu().numpy(), t12.cpu().numpy(), [h[0]["phi_mean"] for h in hist]))
        fdm.fdm_destroy(ctx)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
