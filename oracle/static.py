"""FP64 oracle of the static problem in the layer case (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this module; the GPU library shares no code with it.  Plain
numpy in float64.

Problem (arXiv:1911.03225, sec. 3.1.2 and 3.2.1).  A periodic cell
``nx*dx x ny*dy x n3*dx`` of homogeneous isotropic elasticity (mu, lambda)
holds a layer of ``h`` voxels (thickness ``h*dx``) in which the plastic
distortion is ``U^p = phi(x1, x2) e1 (x) e3``; outside the layer it is zero.
For xi != 0 the stress follows the homogeneous Green-operator solution of
sec. 3.1.2, ``sigma^ = (C:Gamma^ - I):C:U^p^`` with
``Gamma^ = [xi (x) (xi.C.xi)^-1 (x) xi]^(s)``; the mean stress is that of the
prescribed mean strain, ``sigma_bar = C:(eps_bar - <U^p>)``.  The output is the
layer average ``tau13 = (1/h) int_layer sigma13 dx3`` (sec. 3.2.1) at the
nodes of the layer grid.

Two routes:

* ``static_3d`` builds the 3-D voxel field and applies the operator above
  literally (4th-order tensors, matrix inverse per frequency): slow, for
  small cells.
* ``static_tau13`` folds x3 analytically.  For the layer ansatz the xi-space
  solution is ``sigma13^ = -mu phi^ chi^(xi3) G(xi)`` with
  ``G = xi2^2/|xi|^2 + 2/(1-nu) xi1^2 xi3^2/|xi|^4`` (chi the layer's indicator,
  nu = lambda/(2(lambda+mu))), so the layer average is a 2-D multiplier,
  ``tau13^ = -mu K phi^`` with ``K = (n3/h) sum_m3 |chi^[m3]|^2 G``.  The tests
  pin it to ``static_3d``.

``phi`` comes from the densities: ``alpha12 = D1 phi`` and
``alpha11 = -D2 phi`` are forward differences on the staggered grid (sec.
3.2.1), inverted exactly in Fourier space (least squares, exact for
compatible densities); its mean, which the densities do not fix, is an
input.  Frequencies are the continuous ones of the discrete Fourier modes,
``xi = 2 pi m / L`` with ``m`` in ``[-n/2, n/2)``.
"""
from __future__ import annotations

import functools

import numpy as np


def poisson_ratio(mu: float, lam: float) -> float:
    return lam / (2.0 * (lam + mu))


def _xi(n: int, d: float) -> np.ndarray:
    return 2.0 * np.pi * np.fft.fftfreq(n, d)


def phi_from_alpha(a11, a12, dx: float, dy: float, phi_mean: float) -> np.ndarray:
    """Node values of phi = U^p_13 whose staggered forward differences are
    (alpha12, -alpha11), with the given mean (exact inverse of the difference
    operators on compatible densities, least squares otherwise)."""
    a11 = np.asarray(a11, dtype=np.float64)
    a12 = np.asarray(a12, dtype=np.float64)
    ny, nx = a11.shape
    d1 = (np.exp(2j * np.pi * np.fft.fftfreq(nx)) - 1.0) / dx      # symbol of D1
    d2 = (np.exp(2j * np.pi * np.fft.fftfreq(ny)) - 1.0) / dy      # symbol of D2
    D1, D2 = np.meshgrid(d1, d2)
    A11, A12 = np.fft.fft2(a11), np.fft.fft2(a12)
    den = np.abs(D1) ** 2 + np.abs(D2) ** 2
    den[0, 0] = 1.0
    P = (np.conj(D1) * A12 - np.conj(D2) * A11) / den
    P[0, 0] = phi_mean * nx * ny
    return np.real(np.fft.ifft2(P))


def chi_hat_sq(n3: int, h: int) -> np.ndarray:
    """|chi^[m3]|^2 of the indicator of h consecutive voxels out of n3 (DFT
    normalised by 1/n3), m3 = 0 .. n3-1."""
    chi = np.zeros(n3)
    chi[:h] = 1.0
    return np.abs(np.fft.fft(chi) / n3) ** 2


@functools.lru_cache(maxsize=16)
def layer_multiplier(nx: int, ny: int, dx: float, dy: float, nu: float, h: int, n3: int) -> np.ndarray:
    """K[m2, m1] of tau13^ = -mu K phi^ (m != 0); K[0, 0] = 0.  A pure
    function of the cell, so it is computed once per cell and kept
    (read-only) for the steps of a coupled run."""
    x1, x2, x3 = _xi(nx, dx), _xi(ny, dy), _xi(n3, dx)
    c2 = chi_hat_sq(n3, h)
    K = np.zeros((ny, nx))
    X1, X2 = np.meshgrid(x1, x2)
    for m3 in range(n3):
        if c2[m3] == 0.0:
            continue
        s = X1 ** 2 + X2 ** 2 + x3[m3] ** 2
        s[s == 0.0] = np.inf                      # the xi = 0 mode is the mean
        G = X2 ** 2 / s + 2.0 / (1.0 - nu) * X1 ** 2 * x3[m3] ** 2 / s ** 2
        K += c2[m3] * G
    K *= n3 / h
    K[0, 0] = 0.0
    K.setflags(write=False)
    return K


def mean_stress13(mu: float, eps13: float, phi_mean: float, h: int, n3: int) -> float:
    """sigma_bar_13 = 2 mu (eps_bar_13 - <sym U^p>_13), <sym U^p>_13 = phi_mean (h/n3) / 2."""
    return 2.0 * mu * eps13 - mu * phi_mean * h / n3


def static_tau13(a11, a12, dx: float, dy: float, mu: float, lam: float, h: int, n3: int,
                 eps13: float, phi_mean: float) -> np.ndarray:
    """Layer-averaged tau13 at the nodes, through the folded multiplier."""
    phi = phi_from_alpha(a11, a12, dx, dy, phi_mean)
    ny, nx = phi.shape
    K = layer_multiplier(nx, ny, dx, dy, poisson_ratio(mu, lam), h, n3)
    T = -mu * K * np.fft.fft2(phi)
    T[0, 0] = mean_stress13(mu, eps13, phi_mean, h, n3) * nx * ny
    return np.real(np.fft.ifft2(T))


def stiffness(mu: float, lam: float) -> np.ndarray:
    """Isotropic C_ijkl = lambda d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def green_operator(xi: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Gamma^_ijkl(xi) = [xi_j N_ik xi_l]^(s), N = (xi.C.xi)^-1, symmetrised over
    (i,j) and (k,l) (the pairs are already exchanged by C's symmetry)."""
    A = np.einsum("j,ijkl,l->ik", xi, C, xi)
    N = np.linalg.inv(A)
    G = np.einsum("j,ik,l->ijkl", xi, N, xi)
    G = 0.5 * (G + G.transpose(1, 0, 2, 3))
    G = 0.5 * (G + G.transpose(0, 1, 3, 2))
    return G


def static_3d(phi, dx: float, dy: float, mu: float, lam: float, h: int, n3: int, eps13: float):
    """Full 3-D solve on a voxel cell (small sizes only).  Returns (sigma,
    sigma_hat, eps_hat, xi): sigma[i, j] of shape (3, 3, n3, ny, nx) in real
    space, the transforms and the frequency grid (3, n3, ny, nx).  The layer
    occupies voxels x3 = 0 .. h-1."""
    phi = np.asarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    C = stiffness(mu, lam)
    chi = np.zeros(n3)
    chi[:h] = 1.0
    Up = np.zeros((3, 3, n3, ny, nx))
    Up[0, 2] = chi[:, None, None] * phi[None, :, :]
    Up_hat = np.fft.fftn(Up, axes=(2, 3, 4))
    x1, x2, x3 = _xi(nx, dx), _xi(ny, dy), _xi(n3, dx)
    X3, X2, X1 = np.meshgrid(x3, x2, x1, indexing="ij")
    sig_hat = np.zeros_like(Up_hat)
    eps_hat = np.zeros_like(Up_hat)
    I4 = 0.5 * (np.einsum("ik,jl->ijkl", np.eye(3), np.eye(3)) + np.einsum("il,jk->ijkl", np.eye(3), np.eye(3)))
    for a in range(n3):
        for b in range(ny):
            for c in range(nx):
                if a == 0 and b == 0 and c == 0:
                    continue
                xi = np.array([X1[a, b, c], X2[a, b, c], X3[a, b, c]])
                Gm = green_operator(xi, C)
                T = np.einsum("klmn,mn->kl", C, Up_hat[:, :, a, b, c])         # C:U^p^
                e = np.einsum("ijkl,kl->ij", Gm, T)                              # Gamma^:C:U^p^
                eps_hat[:, :, a, b, c] = e
                sig_hat[:, :, a, b, c] = np.einsum("ijkl,kl->ij", C, e) - T      # (C:Gamma^ - I):C:U^p^
    # mean: sigma_bar = C:(eps_bar - <sym U^p>), eps_bar = eps13 (e1e3 + e3e1)
    eps_bar = np.zeros((3, 3))
    eps_bar[0, 2] = eps_bar[2, 0] = eps13
    up_mean = np.einsum("ijkl,kl->ij", I4, Up.mean(axis=(2, 3, 4)))
    npts = n3 * ny * nx
    sig_hat[:, :, 0, 0, 0] = np.einsum("ijkl,kl->ij", C, eps_bar - up_mean) * npts
    eps_hat[:, :, 0, 0, 0] = eps_bar * npts
    sigma = np.real(np.fft.ifftn(sig_hat, axes=(2, 3, 4)))
    return sigma, sig_hat, eps_hat, np.stack([X1, X2, X3])


def layer_average(field3d, h: int) -> np.ndarray:
    """Mean over the layer voxels x3 = 0 .. h-1 of a (n3, ny, nx) field."""
    return np.asarray(field3d)[:h].mean(axis=0)
