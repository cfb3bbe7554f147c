"""The launch-shape autotuner (fdm_autotune) through the C ABI.

Tiling changes no result bit, so after tuning a context must produce exactly
what an untuned one produces, and the caller's state must not be touched by
the trials.
"""
import numpy as np
import pytest

from gpu_util import state_dtype, to_dev
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


def _cases():
    rng = np.random.default_rng(33)
    cases = []
    for (nx, ny), lim, kind in [((96, 64), "minmod", "field"), ((128, 128), "superbee", "uniform"),
                                ((61, 200), "mc", "uniform")]:
        a11, a12 = W.ring(nx, ny, R=max(2.0, min(nx, ny) / 4), sigma=2.0)
        v0f = None
        if kind == "field":
            a11, a12 = W.diagonal_bands(nx, ny, rng, n_bands=4)
            v0f = W.fourier_celerity(nx, ny, rng, kmax=1)
        cases.append(dict(nx=nx, ny=ny, a11=a11, a12=a12, limiter=lim, v0_field=v0f,
                          v0=float(rng.choice([-1.0, 1.0]))))
    return cases


def _setup(F, cases, schedule, precision="fp32"):
    keep, descs, t11, t12 = [], [], [], []
    for c in cases:
        vf = to_dev(c["v0_field"]) if c["v0_field"] is not None else None
        if vf is not None:
            keep.append(vf)
        descs.append(F.desc(c["nx"], c["ny"], limiter=c["limiter"], cfl=0.4, v0=c["v0"], v0_field=vf))
        t11.append(to_dev(c["a11"], state_dtype({"precision": precision})))
        t12.append(to_dev(c["a12"], state_dtype({"precision": precision})))
    ctx = F.fdm_transport_init(descs, options={"schedule": schedule, "precision": precision}, keep=keep)
    return ctx, t11, t12


FIXED = {4, 8, 12, 16, 24, 32, 48, 64}


def _simds():
    import torch
    return 4 * torch.cuda.get_device_properties(0).multi_processor_count


def _balanced_heights(cases, fused, batched, simds):
    """For k = 1..8 the smallest tile height whose largest launch has at most
    k waves (one per tile) per SIMD, by trying every height."""
    width = 56 if fused else 60
    max_ny = max(c["ny"] for c in cases)

    def waves(rows):
        t = [-(-c["nx"] // width) * -(-c["ny"] // min(rows, c["ny"])) for c in cases]
        return sum(t) if batched else max(t)
    out = set()
    for k in range(1, 9):
        fits = [r for r in range(1, max_ny + 1) if waves(r) <= k * simds]
        if fits and fits[0] <= 512:
            out.add(fits[0])
    return out


def _expected_heights(cases, schedule):
    max_ny = max(c["ny"] for c in cases)
    fixed = {r for r in FIXED if r <= max_ny or r == 4}
    fused = schedule == "fused"
    batched = schedule == "batched" or (fused and len(cases) > 1)
    return fixed | _balanced_heights(cases, fused, batched, _simds())


def test_balanced_heights_of_a_large_grid():
    """The helper itself on 2048^2 (no device call): one, two, ... waves per
    SIMD of 1024 SIMDs at the smallest height that fits."""
    case = [dict(nx=2048, ny=2048)]
    assert _balanced_heights(case, True, False, 1024) == {76, 38, 25, 19, 15, 13, 11, 10}
    assert _balanced_heights(case, False, False, 1024) == {71, 36, 24, 18, 15, 12, 11, 9}


def _host(ts):
    return [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_autotune_single_instance(fdm, precision):
    import torch
    a11, a12 = W.ring(256, 192, R=50, sigma=3.0)
    case = [dict(nx=256, ny=192, a11=a11, a12=a12, limiter="mc", v0_field=None, v0=-1.0)]
    ctx, t11, t12 = _setup(fdm, case, "auto", precision)
    before = _host(t11) + _host(t12)
    trials = fdm.fdm_autotune(ctx, t11, t12, trial_steps=3)
    torch.cuda.synchronize()
    after = _host(t11) + _host(t12)
    assert all(np.array_equal(x, y) for x, y in zip(before, after)), "autotune wrote the caller's state"
    # FP32 Heun contexts also time the fused launches
    assert {t["schedule"] for t in trials} == ({"plain", "fused"} if precision == "fp32" else {"plain"})
    for sched in {t["schedule"] for t in trials}:
        assert {t["tile_rows"] for t in trials if t["schedule"] == sched} == _expected_heights(case, sched)
    best = min(trials, key=lambda t: t["seconds_per_step"])
    assert fdm.fdm_tile_rows(ctx, 0) == best["tile_rows"]
    assert all(t["seconds_per_step"] > 0 for t in trials)
    fdm.fdm_run(ctx, t11, t12, 40, 20)
    torch.cuda.synchronize()
    tuned = _host(t11) + _host(t12)
    assert fdm.fdm_transport_stats(ctx, t11, t12)[0]["step"] == 40
    fdm.fdm_destroy(ctx)

    ctx, u11, u12 = _setup(fdm, case, "auto", precision)
    fdm.fdm_transport_step(ctx, u11, u12, 40)
    torch.cuda.synchronize()
    ref = _host(u11) + _host(u12)
    fdm.fdm_destroy(ctx)
    assert all(np.array_equal(x, y) for x, y in zip(tuned, ref))


def test_autotune_batched_schedules(fdm):
    import torch
    cases = _cases()
    ctx, t11, t12 = _setup(fdm, cases, "auto")
    trials = fdm.fdm_autotune(ctx, t11, t12, trial_steps=2)
    assert {t["schedule"] for t in trials} == {"batched", "plain", "fused"}
    # fixed candidates above the tallest instance (200 rows) are skipped
    for sched in ("batched", "plain", "fused"):
        assert {t["tile_rows"] for t in trials if t["schedule"] == sched} == _expected_heights(cases, sched)
    assert max(t["tile_rows"] for t in trials) <= 200
    best = min(trials, key=lambda t: t["seconds_per_step"])
    for i, c in enumerate(cases):
        assert fdm.fdm_tile_rows(ctx, i) == min(best["tile_rows"], c["ny"])
    fdm.fdm_transport_step(ctx, t11, t12, 30)
    fdm.fdm_run(ctx, t11, t12, 20, 10)
    torch.cuda.synchronize()
    tuned = _host(t11) + _host(t12)
    fdm.fdm_destroy(ctx)

    ctx, u11, u12 = _setup(fdm, cases, "plain")
    fdm.fdm_transport_step(ctx, u11, u12, 50)
    torch.cuda.synchronize()
    ref = _host(u11) + _host(u12)
    fdm.fdm_destroy(ctx)
    assert all(np.array_equal(x, y) for x, y in zip(tuned, ref))


def test_autotune_fixed_schedule_kept(fdm):
    cases = _cases()
    ctx, t11, t12 = _setup(fdm, cases, "batched")
    trials = fdm.fdm_autotune(ctx, t11, t12, trial_steps=1, max_trials=3)
    assert len(trials) == 3 and all(t["schedule"] == "batched" for t in trials)
    fdm.fdm_destroy(ctx)


def test_autotune_rejects_bad_arguments(fdm):
    a11, a12 = W.ring(64, 64, R=16, sigma=2.0)
    case = [dict(nx=64, ny=64, a11=a11, a12=a12, limiter="minmod", v0_field=None, v0=-1.0)]
    ctx, t11, t12 = _setup(fdm, case, "auto")
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_autotune(ctx, t11, t12, trial_steps=0)
    assert e.value.status == fdm.FDM_ERR_INVALID_ARG
    rows = fdm.fdm_tile_rows(ctx, 0)
    assert rows > 0 and fdm.fdm_tile_rows(ctx, 1) == -1
    fdm.fdm_destroy(ctx)
