"""Pins of the static-problem oracle (oracle/static.py), CPU only.

The folded 2-D layer multiplier is checked against the literal 3-D Green
operator solution of sec. 3.1.2 (4th-order tensors, a matrix inverse per
frequency) on small voxel cells, and both against closed forms: antiplane
shear of a full-thickness band, equilibrium (xi . sigma^ = 0), compatibility
of the total strain (inc eps = 0) and the mean stress of the prescribed mean
strain.
"""
import numpy as np
import pytest

from oracle import static as S


def _smooth_phi(nx, ny, seed, modes=4):
    rng = np.random.default_rng(seed)
    x = np.arange(nx)[None, :] / nx
    y = np.arange(ny)[:, None] / ny
    phi = np.zeros((ny, nx))
    for _ in range(modes):
        k1, k2 = rng.integers(-3, 4, size=2)
        phi += rng.uniform(-0.3, 0.3) * np.cos(2 * np.pi * (k1 * x + k2 * y) + rng.uniform(0, 2 * np.pi))
    return phi


def _alpha(phi, dx=1.0, dy=1.0):
    a12 = (np.roll(phi, -1, axis=1) - phi) / dx
    a11 = -(np.roll(phi, -1, axis=0) - phi) / dy
    return a11, a12


def test_phi_round_trip():
    phi = _smooth_phi(24, 18, 1) + 0.37
    phi += np.random.default_rng(2).normal(0, 0.05, phi.shape)   # rough too
    a11, a12 = _alpha(phi, 0.5, 0.25)
    back = S.phi_from_alpha(a11, a12, 0.5, 0.25, phi.mean())
    assert np.max(np.abs(back - phi)) < 1e-13


def test_full_thickness_band_along_x1_is_antiplane_shear():
    # phi(x2) through the whole cell: u cannot relax it, sigma13 = mu (2 eps - phi)
    ny, nx, mu = 32, 8, 1.3
    phi = np.tile(np.tanh((np.arange(ny) - ny / 2) / 3.0)[:, None] * 0.2 + 0.05, (1, nx))
    a11, a12 = _alpha(phi)
    tau = S.static_tau13(a11, a12, 1.0, 1.0, mu, 0.9, h=6, n3=6, eps13=0.01, phi_mean=phi.mean())
    assert np.max(np.abs(tau - mu * (2 * 0.01 - phi))) < 1e-13


def test_full_thickness_band_along_x2_is_stress_free():
    # phi(x1): u3(x1) takes it up, only the mean stress remains
    ny, nx, mu = 6, 40, 0.8
    phi = np.tile(0.2 * np.sin(2 * np.pi * np.arange(nx) / nx)[None, :] + 0.1, (ny, 1))
    a11, a12 = _alpha(phi)
    tau = S.static_tau13(a11, a12, 1.0, 1.0, mu, 1.2, h=5, n3=5, eps13=-0.02, phi_mean=phi.mean())
    assert np.max(np.abs(tau - mu * (2 * -0.02 - phi.mean()))) < 1e-13


@pytest.mark.parametrize("nx,ny,h,n3,mu,lam,d", [(10, 8, 2, 6, 1.0, 1.5, 1.0), (8, 12, 3, 8, 0.7, 0.4, 1.0),
                                                 (9, 7, 1, 5, 1.0, 3.0, 1.0), (8, 6, 2, 7, 1.0, 1.5, 0.35),
                                                 # thin layers, as in the coupled workload (4 of 512 voxels)
                                                 (32, 32, 4, 64, 1.0, 1.5, 1.0), (24, 20, 2, 128, 1.0, 1.5, 1.0)])
def test_layer_multiplier_matches_3d_green_operator(nx, ny, h, n3, mu, lam, d):
    phi = _smooth_phi(nx, ny, nx * ny) + np.random.default_rng(3).normal(0, 0.02, (ny, nx))
    a11, a12 = _alpha(phi, d, d)
    eps = 0.003
    sigma, sig_hat, eps_hat, xi = S.static_3d(phi, d, d, mu, lam, h, n3, eps)
    tau3d = S.layer_average(sigma[0, 2], h)
    tau2d = S.static_tau13(a11, a12, d, d, mu, lam, h, n3, eps, phi.mean())
    assert np.max(np.abs(tau3d - tau2d)) < 1e-13
    # symmetric stress
    assert np.max(np.abs(sigma - sigma.transpose(1, 0, 2, 3, 4))) < 1e-14


def test_3d_solution_is_in_equilibrium_compatible_and_has_the_prescribed_mean():
    nx, ny, h, n3, mu, lam, eps = 8, 6, 2, 6, 1.0, 1.5, 0.004
    phi = _smooth_phi(nx, ny, 9)
    sigma, sig_hat, eps_hat, xi = S.static_3d(phi, 1.0, 1.0, mu, lam, h, n3, eps)
    scale = np.max(np.abs(sig_hat))
    # div sigma = 0: xi_j sigma^_ij = 0 at every xi != 0 (the xi = 0 term is zero anyway)
    div = np.einsum("jabc,ijabc->iabc", xi, sig_hat)
    assert np.max(np.abs(div)) < 1e-12 * scale * np.max(np.abs(xi))
    # total strain is a symmetric gradient: inc(eps)^ = e_ikl e_jmn xi_k xi_m eps^_ln = 0
    e = np.zeros((3, 3, 3))
    for i, j, k in [(0, 1, 2), (1, 2, 0), (2, 0, 1)]:
        e[i, j, k], e[i, k, j] = 1.0, -1.0
    inc = np.einsum("ikl,jmn,kabc,mabc,lnabc->ijabc", e, e, xi, xi, eps_hat)
    assert np.max(np.abs(inc)) < 1e-12 * np.max(np.abs(eps_hat)) * np.max(np.abs(xi)) ** 2
    # mean stress of the prescribed mean strain
    sbar = S.mean_stress13(mu, eps, phi.mean(), h, n3)
    assert abs(sigma[0, 2].mean() - sbar) < 1e-14
    assert abs(sigma[0, 2].mean() - (2 * mu * eps - mu * phi.mean() * h / n3)) < 1e-14
    # the layer average keeps that mean
    a11, a12 = _alpha(phi)
    tau = S.static_tau13(a11, a12, 1.0, 1.0, mu, lam, h, n3, eps, phi.mean())
    assert abs(tau.mean() - sbar) < 1e-14


def test_multiplier_bounds_and_symmetry():
    nu = S.poisson_ratio(1.0, 1.5)
    K = S.layer_multiplier(16, 12, 1.0, 1.0, nu, 4, 32)
    # a weighted mean (weights (n3/h)|chi^|^2 sum to 1) of G in [0, 1 + 1/(2(1-nu))]
    assert np.isclose((32 / 4) * S.chi_hat_sq(32, 4).sum(), 1.0)
    assert K.min() >= 0.0 and K.max() <= 1.0 + 1.0 / (2 * (1 - nu)) + 1e-15
    assert np.allclose(K, np.roll(K[:, ::-1], 1, axis=1)) and np.allclose(K, np.roll(K[::-1, :], 1, axis=0))
    # full thickness: K = xi2^2 / |xi|^2, independent of nu
    Kf = S.layer_multiplier(16, 12, 1.0, 1.0, 0.1, 8, 8)
    x1 = 2 * np.pi * np.fft.fftfreq(16)
    x2 = 2 * np.pi * np.fft.fftfreq(12)
    X1, X2 = np.meshgrid(x1, x2)
    s = X1 ** 2 + X2 ** 2
    s[0, 0] = 1.0
    ref = X2 ** 2 / s
    ref[0, 0] = 0.0
    assert np.max(np.abs(Kf - ref)) < 1e-15
