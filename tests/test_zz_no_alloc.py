"""fdm_transport_step_noalloc (no device allocation; stage buffer in a static
device array) against the context entry points fdm_transport_init +
fdm_transport_step on the same inputs: the same bits, on two calls in a
row, the second on a smaller grid, for every integrator, the fully
discrete scheme, a celerity field and a prescribed velocity."""
import numpy as np
import pytest

from gpu_util import to_dev
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


CASES = [
    ("heun-superbee", dict(limiter="superbee", cfl=0.4, v0=-1.0)),
    ("midpoint-mc", dict(limiter="mc", cfl=0.4, v0=-1.0, time_order=3)),
    ("euler-minmod", dict(limiter="minmod", cfl=0.25, v0=1.0, time_order=1)),
    ("fully-discrete", dict(limiter="superbee", cfl=0.25, v0=-1.0, time_order=1, scheme="fully_discrete")),
    ("prescribed", dict(limiter="mc", velocity="prescribed", V=(0.7, -0.4), cfl=0.4)),
    ("field", dict(limiter="theta", theta=1.5, cfl=0.45, field=True)),
    ("field-fixed-dt", dict(limiter="minmod", dt=0.3, field=True)),
]


def _inputs(nx, ny, field, seed):
    rng = np.random.default_rng(seed)
    if field:
        a11, a12 = W.diagonal_bands(nx, ny, rng, n_bands=6)
        return a11, a12, W.fourier_celerity(nx, ny, rng, kmax=1)
    a11, a12 = W.ring(nx, ny, R=min(nx, ny) / 4.0, sigma=3.0)
    return a11, a12, None


def _context_run(F, a11, a12, steps, v0f, kw):
    import torch
    ny, nx = a11.shape
    t11, t12 = to_dev(a11), to_dev(a12)
    ctx = F.fdm_transport_init(F.desc(nx, ny, v0_field=v0f, **kw), keep=[v0f] if v0f is not None else [])
    F.fdm_transport_step(ctx, t11, t12, steps)
    torch.cuda.synchronize()
    F.fdm_destroy(ctx)
    return t11.cpu().numpy(), t12.cpu().numpy()


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_context_step(fdm, name, kw):
    import torch
    kw = dict(kw)
    field = kw.pop("field", False)
    for (nx, ny, steps, seed) in ((288, 288, 11, 1), (96, 96, 7, 2)):   # the second call: a smaller input
        a11, a12, v0 = _inputs(nx, ny, field, seed)
        v0f = to_dev(v0) if v0 is not None else None
        print("noalloc case %s %dx%d %d steps" % (name, nx, ny, steps), flush=True)
        r11, r12 = _context_run(fdm, a11, a12, steps, v0f, kw)
        t11, t12 = to_dev(a11), to_dev(a12)
        fdm.fdm_transport_step_noalloc(fdm.desc(nx, ny, v0_field=v0f, **kw), t11, t12, steps)
        torch.cuda.synchronize()
        g11, g12 = t11.cpu().numpy(), t12.cpu().numpy()
        assert np.array_equal(g11, r11) and np.array_equal(g12, r12), (name, nx, ny)
        assert not np.array_equal(g12, a12)   # it moved


def test_noalloc_largest_grid_and_limit(fdm):
    """A grid of exactly the maximum size runs (a 2048^2 loop, two Heun
    steps, equal to the context path); one node more is rejected on the
    host."""
    import torch
    n = 2048
    assert n * n == fdm.NOALLOC_MAX_NODES
    a11, a12 = W.ring(n, n, R=300.0, sigma=6.0)
    kw = dict(limiter="superbee", cfl=0.4, v0=-1.0)
    r11, r12 = _context_run(fdm, a11, a12, 2, None, kw)
    t11, t12 = to_dev(a11), to_dev(a12)
    fdm.fdm_transport_step_noalloc(fdm.desc(n, n, **kw), t11, t12, 2)
    torch.cuda.synchronize()
    assert np.array_equal(t11.cpu().numpy(), r11) and np.array_equal(t12.cpu().numpy(), r12)
    b11, b12 = to_dev(np.zeros((1, n * n + 1), np.float32)), to_dev(np.zeros((1, n * n + 1), np.float32))
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_step_noalloc(fdm.desc(n * n + 1, 1, **kw), b11, b12, 1)
    assert e.value.status == fdm.FDM_ERR_INVALID_ARG
    assert "maximum" in fdm.fdm_last_error(None)
