"""GPU static solve (fdm_static_solve: rocFFT + the multiplier kernels)
against the FP64 oracle of oracle/static.py, on the same float32 (or
float64) densities.

Bars: FP64 precision matches the oracle to 1e-12 (relative L2); FP32
(single-precision FFTs, float32 multiplier) to 1e-5 relative L2 and 1e-4 of
max|tau| pointwise -- a radix-2 FFT of N points loses about log2(N) ulps of
the field's RMS, 2e-6 at 512^2.
"""
import numpy as np
import pytest

from gpu_util import to_dev
from oracle import static as S
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


def _solve(fdm, a11, a12, precision, **kw):
    ny, nx = a11.shape
    dt = np.float64 if precision == "fp64" else np.float32
    t11, t12 = to_dev(a11, dt), to_dev(a12, dt)
    d = fdm.static_desc(nx, ny, precision=precision, **kw)
    tau = fdm.fdm_static_solve(d, t11, t12)
    return tau.cpu().numpy().astype(np.float64), (t11, t12)


def _oracle(a11, a12, dx=1.0, mu=1.0, lam=1.5, layer_h=4.0, cell_l3=512.0, eps13=0.0, phi_mean=0.0):
    h, n3 = int(round(layer_h / dx)), int(round(cell_l3 / dx))
    return S.static_tau13(np.asarray(a11, np.float64), np.asarray(a12, np.float64), dx, dx, mu, lam, h, n3,
                          eps13, phi_mean)


def _errors(g, o):
    rel_l2 = np.linalg.norm(g - o) / np.linalg.norm(o)
    rel_inf = np.max(np.abs(g - o)) / np.max(np.abs(o))
    return rel_l2, rel_inf


@pytest.mark.parametrize("precision", ["fp32", "fp64_arith", "fp64"])
def test_coupled_workload_rings(fdm, precision):
    phi, a11, a12 = W.plateau_rings(512, 512, seed=4)
    kw = dict(layer_h=4.0, cell_l3=512.0, eps13=0.003, phi_mean=float(phi.mean()))
    g, _ = _solve(fdm, a11, a12, precision, **kw)
    o = _oracle(a11, a12, **kw)
    l2, linf = _errors(g, o)
    if precision == "fp64":
        assert l2 < 1e-12 and linf < 1e-12, (l2, linf)
    else:
        assert l2 < 1e-5 and linf < 1e-4, (l2, linf)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_odd_grid_thin_layer_non_unit_spacing(fdm, precision):
    rng = np.random.default_rng(8)
    nx, ny, dx = 97, 64, 0.5
    x = np.arange(nx)[None, :] / nx
    y = np.arange(ny)[:, None] / ny
    phi = 0.1 + 0.2 * np.sin(2 * np.pi * (3 * x + y)) + 0.05 * rng.normal(size=(ny, nx))
    a11, a12 = W.densities_from_phi(phi, dx, dx)
    kw = dict(dx=dx, mu=0.7, lam=0.4, layer_h=0.5, cell_l3=16.5, eps13=-0.01, phi_mean=0.1)
    g, _ = _solve(fdm, a11, a12, precision, **kw)
    o = _oracle(a11, a12, **kw)
    l2, linf = _errors(g, o)
    bound = 1e-12 if precision == "fp64" else 1e-5
    assert l2 < bound and linf < 10 * bound, (l2, linf)


def test_full_thickness_band_closed_form(fdm):
    # phi(x2) through the whole cell: tau13 = mu (2 eps - phi) (antiplane shear)
    n, mu, eps = 128, 1.0, 0.004
    phi1 = 0.2 * np.tanh((np.arange(n) - n / 2) / 4.0) + 0.03
    phi = np.tile(phi1[:, None], (1, n))
    a11, a12 = W.densities_from_phi(phi)
    phi32 = S.phi_from_alpha(a11, a12, 1.0, 1.0, float(phi.mean()))   # the potential of the rounded densities
    g, _ = _solve(fdm, a11, a12, "fp64", mu=mu, layer_h=8.0, cell_l3=8.0, eps13=eps, phi_mean=float(phi.mean()))
    assert np.max(np.abs(g - mu * (2 * eps - phi32))) < 1e-13


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_mean_is_the_macroscopic_stress_and_densities_untouched(fdm, precision):
    import torch
    phi, a11, a12 = W.plateau_rings(256, 192, seed=11, count=8, rmin=10, rmax=40)
    kw = dict(layer_h=3.0, cell_l3=96.0, eps13=0.002, phi_mean=0.05)
    dt = np.float64 if precision == "fp64" else np.float32
    g, (t11, t12) = _solve(fdm, a11, a12, precision, **kw)
    assert np.array_equal(t11.cpu().numpy(), a11.astype(dt)) and np.array_equal(t12.cpu().numpy(), a12.astype(dt))
    sbar = 2 * 1.0 * 0.002 - 1.0 * 0.05 * 3 / 96
    assert abs(g.mean() - sbar) < (1e-13 if precision == "fp64" else 1e-7)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("nx,ny", [(4096, 2048), (1009, 503), (2048, 3)])
def test_large_and_prime_sizes(fdm, precision, nx, ny):
    """FFT lengths beyond one pass (4096 x 2048), prime lengths (1009 x 503)
    and a thin strip (2048 x 3), on a thin cell (L3 = 16 voxels, h = 4) so
    the oracle's sum over the x3 modes stays short; same bars as above."""
    rng = np.random.default_rng(nx + ny)
    x = np.arange(nx)[None, :] / nx
    y = np.arange(ny)[:, None] / ny
    phi = 0.2 * np.sin(2 * np.pi * (5 * x + 2 * y)) + 0.05 * rng.normal(size=(ny, nx))
    a11, a12 = W.densities_from_phi(phi)
    kw = dict(layer_h=4.0, cell_l3=16.0, eps13=0.002, phi_mean=float(phi.mean()))
    g, _ = _solve(fdm, a11, a12, precision, **kw)
    o = _oracle(a11, a12, **kw)
    l2, linf = _errors(g, o)
    if precision == "fp64":
        assert l2 < 1e-12 and linf < 1e-12, (l2, linf)
    else:
        assert l2 < 1e-5 and linf < 1e-4, (l2, linf)
