"""Seeded synthetic inputs shaped like the paper's model problems.

This module builds initial density fields and celerity fields only; it holds
none of the transport scheme's arithmetic.  Both the GPU path and the FP64
oracle are fed from here, with every array rounded to float32 once so that
both sides see the same bits (the oracle promotes them exactly to float64).

Layout (arXiv:1911.03225, sec. 3.2.1): arrays have shape (ny, nx);
``alpha12[k, j]`` is alpha_12 = d1 phi on the x-edge (j+1/2, k) and
``alpha11[k, j]`` is alpha_11 = -d2 phi on the y-edge (j, k+1/2), with
phi = U^p_13 given at the pixel nodes (j dx, k dy).  Building the densities as
node differences of one nodal phi makes the discrete div(alpha) vanish
(eq. 2) up to the float32 rounding of the stored values.

The paper's own runs (sec. 4.3 annihilation of two half-square waves, sec.
4.4.1 expansion of a smooth loop, sec. 4.4.2 polygonal loops) have no data
files; their shapes are reproduced here from the text.  Amplitudes are O(1)
where the paper uses 1e-2: the Hamiltonian is 1-homogeneous in grad phi, so
the solution scales linearly with the amplitude.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import gcd, pi, sqrt

import numpy as np
from scipy.special import erf as _verf, erfc as _verfc

__all__ = [
    "densities_from_phi", "colliding_pulses", "exact_period_profile", "smooth_sine",
    "ring", "square_loop", "half_square_waves", "diagonal_bands",
    "fourier_celerity", "bands_and_celerity", "Instance", "batched_instances",
]

def densities_from_phi(phi: np.ndarray, dx: float = 1.0, dy: float = 1.0):
    """(alpha11, alpha12) as float32 node differences of a periodic nodal phi."""
    phi = np.asarray(phi, dtype=np.float64)
    a12 = (np.roll(phi, -1, axis=1) - phi) / dx
    a11 = -(np.roll(phi, -1, axis=0) - phi) / dy
    return a11.astype(np.float32), a12.astype(np.float32)


def _step_profile(xi: np.ndarray, sigma: float) -> np.ndarray:
    """-sigma*sqrt(pi/2)*erfc(xi/(sigma*sqrt2)): its derivative is the unit Gaussian."""
    return -sigma * sqrt(pi / 2.0) * _verfc(xi / (sigma * sqrt(2.0)))


def colliding_pulses(n: int = 64, sigma: float = 4.0, x_neg: float = 20.0, x_pos: float = 44.0):
    """Two opposite-sign Gaussian pulses of alpha_12 (amplitude 1) on an n x n grid.

    phi(x) = sum over images of [Psi(x - x_pos) - Psi(x - x_neg)]: a well that a
    negative celerity fills, so the pulses meet.  alpha_11 = 0 (x-only data,
    the paper's 1D case of sec. 4.3 laid on a 2-D grid).
    """
    x = np.arange(n, dtype=np.float64)
    phi1 = np.zeros(n)
    for m in range(-2, 3):
        phi1 += _step_profile(x - x_pos + n * m, sigma) - _step_profile(x - x_neg + n * m, sigma)
    phi = np.broadcast_to(phi1, (n, n))
    return densities_from_phi(phi)


def exact_period_profile(n: int = 64):
    """x-only data for the exact-return check of the first-order scheme."""
    return colliding_pulses(n)


def smooth_sine(n: int, L: float = 1.0):
    """phi = (L/2pi) [sin(2pi x/L) + 1/2 sin(2pi (x+y)/L)] at n x n nodes over [0, L)^2."""
    dx = L / n
    x = np.arange(n) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    phi = (L / (2 * pi)) * (np.sin(2 * pi * X / L) + 0.5 * np.sin(2 * pi * (X + Y) / L))
    return densities_from_phi(phi, dx, dx), dx


def ring(nx: int, ny: int, R: float, sigma: float, A: float = 1.0,
         center=None, dx: float = 1.0):
    """Circular loop: phi = sum over images of A sigma sqrt(pi/2) erfc((r - R)/(sigma sqrt2)).

    |grad phi| is a Gaussian cross-section of height A at radius R and phi > 0
    inside the loop (the slipped area), so a negative celerity expands it.
    """
    Lx, Ly = nx * dx, ny * dx
    cx, cy = center if center is not None else (Lx / 2.0, Ly / 2.0)
    x = np.arange(nx) * dx
    y = np.arange(ny) * dx
    X, Y = np.meshgrid(x, y, indexing="xy")
    phi = np.zeros((ny, nx))
    for mx in (-1, 0, 1):
        for my in (-1, 0, 1):
            r = np.hypot(X - cx - mx * Lx, Y - cy - my * Ly)
            z = (r - R) / (sigma * sqrt(2.0))
            close = z < 30.0           # erfc underflows beyond this
            phi[close] += A * sigma * sqrt(pi / 2.0) * _verfc(z[close])
    return densities_from_phi(phi, dx, dx)


def plateau_rings(nx: int, ny: int, seed: int = 4, count: int = 20, rmin: float = 20.0, rmax: float = 80.0,
                  plateau: float = 0.2, sigma: float = 2.0, dx: float = 1.0):
    """Seeded loops for the coupled workload: phi = sum over loops of
    +-plateau * erfc((r - R)/(sigma sqrt2)) / 2 (a plateau inside each loop,
    erfc edges, periodic images), centres uniform, radii uniform in
    [rmin, rmax], signs random.  Returns (phi, alpha11, alpha12): phi float64
    at the nodes, the densities float32."""
    rng = np.random.default_rng(seed)
    Lx, Ly = nx * dx, ny * dx
    X, Y = np.meshgrid(np.arange(nx) * dx, np.arange(ny) * dx, indexing="xy")
    phi = np.zeros((ny, nx))
    for _ in range(count):
        cx, cy = rng.uniform(0, Lx), rng.uniform(0, Ly)
        R = rng.uniform(rmin, rmax)
        A = plateau * rng.choice([-1.0, 1.0])
        for mx in (-1, 0, 1):
            for my in (-1, 0, 1):
                z = (np.hypot(X - cx - mx * Lx, Y - cy - my * Ly) - R) / (sigma * sqrt(2.0))
                close = z < 30.0
                phi[close] += 0.5 * A * _verfc(z[close])
    a11, a12 = densities_from_phi(phi, dx, dx)
    return phi, a11, a12


def ring_phi_profile(r, R: float, sigma: float, A: float = 1.0):
    """The radial plateau Phi(r) used by ``ring`` (for exact solutions)."""
    r = np.asarray(r, dtype=np.float64)
    return A * sigma * sqrt(pi / 2.0) * _verfc((r - R) / (sigma * sqrt(2.0)))


def _smooth_box(x: np.ndarray, x0: float, x1: float, s: float) -> np.ndarray:
    return 0.5 * (_verf((x - x0) / (s * sqrt(2.0))) - _verf((x - x1) / (s * sqrt(2.0))))


def square_loop(n: int, side: float, edge_sigma: float, A: float = 1.0, dx: float = 1.0):
    """Polygonal (square) loop: phi = A * box(x) * box(y) with erf edges.

    The square of the given side is centred in the n x n cell (sec. 4.4.2).
    """
    L = n * dx
    x = np.arange(n) * dx
    bx = _smooth_box(x, L / 2 - side / 2, L / 2 + side / 2, edge_sigma)
    phi = A * np.outer(bx, bx)
    return densities_from_phi(phi, dx, dx)


def half_square_waves(n: int, L: float = 320.0, width: float = 10.0,
                      gap: float = 210.0, amplitude: float = 1.0):
    """Two half-square waves of alpha_12 of opposite sign (sec. 4.3), 1-D (ny = 1).

    The negative wave sits left of the centre, the positive one right of it;
    their inner fronts are ``gap`` apart (L/2 -+ gap/2).  Built from the
    exact piecewise-linear phi at the nodes, so the cell averages are exact.
    """
    dx = L / n
    x = np.arange(n) * dx
    phi = half_square_phi(x, L, width, gap, amplitude)
    a12 = (np.roll(phi, -1) - phi) / dx
    return np.zeros((1, n), np.float32), a12.astype(np.float32)[None, :], dx


def half_square_phi(x, L: float = 320.0, width: float = 10.0, gap: float = 210.0,
                    amplitude: float = 1.0):
    """Nodal phi of ``half_square_waves``: 0 outside, a well of depth width*amplitude."""
    x = np.asarray(x, dtype=np.float64) % L
    left_in, right_in = L / 2 - gap / 2, L / 2 + gap / 2
    left_out, right_out = left_in - width, right_in + width
    phi = np.zeros_like(x)
    phi = np.where((x > left_out) & (x < left_in), -(x - left_out) * amplitude, phi)
    phi = np.where((x >= left_in) & (x <= right_in), -width * amplitude, phi)
    phi = np.where((x > right_in) & (x < right_out), -(right_out - x) * amplitude, phi)
    return phi


def diagonal_bands(nx: int, ny: int, rng: np.random.Generator, n_bands: int = 64,
                   wmin: int = 8, wmax: int = 32, amin: float = 0.5, amax: float = 1.0):
    """Diagonal band pattern: alpha_12 = b(m), alpha_11 = -b(m), m = (j + k) mod P.

    P = gcd-compatible period along the diagonal (nx when nx == ny).  Bands of
    alternating sign with widths U{wmin..wmax} and |amplitude| U[amin, amax],
    separated by random gaps filling the rest of the period.  The pattern is
    exactly curl-free and need not have zero mean.
    """
    P = gcd(nx, ny) if nx != ny else nx
    widths = rng.integers(wmin, wmax + 1, size=n_bands)
    while widths.sum() > P:           # small grids: shrink the band count
        n_bands -= 1
        widths = widths[:n_bands]
    amps = rng.uniform(amin, amax, size=n_bands)
    signs = np.where(np.arange(n_bands) % 2 == 0, 1.0, -1.0)
    free = P - int(widths.sum())
    cuts = np.sort(rng.integers(0, free + 1, size=n_bands))
    gaps = np.diff(np.concatenate([[0], cuts]))
    b = np.zeros(P)
    pos = 0
    for i in range(n_bands):
        pos += int(gaps[i])
        b[pos:pos + int(widths[i])] = signs[i] * amps[i]
        pos += int(widths[i])
    j = np.arange(nx)[None, :]
    k = np.arange(ny)[:, None]
    m = (j + k) % P
    band = b[m]
    return (-band).astype(np.float32), band.astype(np.float32)


def fourier_celerity(nx: int, ny: int, rng: np.random.Generator, v0: float = 1.0,
                     n_modes: int = 16, kmax: int = 8, tau0: float = 0.5):
    """v0 tanh(tau/tau0) at the nodes, tau a unit-RMS sum of Fourier modes.

    tau = sum_i a_i cos(2 pi (k_i . x)/N + psi_i) with distinct integer wave
    vectors 1 <= |k_i|_inf <= kmax, a_i ~ U[0.5, 1], psi_i ~ U[0, 2 pi).
    Sign changes of the celerity drive bands into each other (annihilation).
    """
    n_modes = min(n_modes, ((2 * kmax + 1) ** 2 - 1) // 2)   # sign-distinct vectors
    ks = set()
    while len(ks) < n_modes:
        k = tuple(int(v) for v in rng.integers(-kmax, kmax + 1, size=2))
        if max(abs(k[0]), abs(k[1])) >= 1 and (-k[0], -k[1]) not in ks:
            ks.add(k)
    ks = sorted(ks)
    a = rng.uniform(0.5, 1.0, size=n_modes)
    psi = rng.uniform(0.0, 2 * pi, size=n_modes)
    x = np.arange(nx, dtype=np.float64)[None, :] / nx
    y = np.arange(ny, dtype=np.float64)[:, None] / ny
    tau = np.zeros((ny, nx))
    for (kx, ky), ai, pi_ in zip(ks, a, psi):
        tau += ai * np.cos(2 * pi * (kx * x + ky * y) + pi_)
    tau /= np.sqrt(np.mean(tau ** 2))
    return (v0 * np.tanh(tau / tau0)).astype(np.float32)


def bands_and_celerity(n: int = 4096, seed: int = 3):
    """Spatially varying celerity workload: diagonal bands + Fourier celerity."""
    rng = np.random.default_rng(seed)
    a11, a12 = diagonal_bands(n, n, rng)
    v0 = fourier_celerity(n, n, rng)
    return a11, a12, v0


@dataclass
class Instance:
    """One independent transport problem of the batched workload."""
    nx: int
    ny: int
    limiter: str
    velocity: str            # "uniform" or "fourier"
    v0: float                # uniform celerity (+-1) when velocity == "uniform"
    init: str                # "ring" or "bands"
    seed: int
    arrays: dict = field(default_factory=dict, repr=False)

    def make(self):
        """(alpha11, alpha12, v0_field or None), float32, generated on demand."""
        rng = np.random.default_rng(self.seed)
        if self.init == "ring":
            m = min(self.nx, self.ny)
            a11, a12 = ring(self.nx, self.ny, R=m / 4.0, sigma=max(2.0, m / 64.0))
        else:
            a11, a12 = diagonal_bands(self.nx, self.ny, rng)
        v0f = None
        if self.velocity == "fourier":
            # the 4096^2 field's wave vectors (|k| <= 8 per 4096 cells) scaled
            # to this grid
            kmax = max(1, int(round(8 * min(self.nx, self.ny) / 4096)))
            v0f = fourier_celerity(self.nx, self.ny, rng, kmax=kmax)
        return a11, a12, v0f


BATCH_SIZES = ((64, 64), (128, 128), (256, 512), (512, 512), (1024, 1024), (1024, 2048))
BATCH_COUNTS = (128, 96, 64, 48, 32, 16)


def batched_instances(seed: int = 5, counts=BATCH_COUNTS, sizes=BATCH_SIZES):
    """The batched workload: 384 instances of six sizes (weights 8:6:4:3:2:1).

    Per instance, drawn in order from default_rng(seed): limiter in
    {minmod, superbee, mc}, velocity in {uniform +-1, Fourier field},
    initial state in {ring, diagonal bands}, independently.  Sizes are
    (nx, ny).  The Fourier fields keep the 4096^2 field's wave vectors
    scaled to the grid, so they change sign on scales of hundreds of cells,
    where every limiter is stable.
    """
    rng = np.random.default_rng(seed)
    out = []
    for (nx, ny), c in zip(sizes, counts):
        for _ in range(c):
            lim = ("minmod", "superbee", "mc")[int(rng.integers(0, 3))]
            vel = ("uniform", "fourier")[int(rng.integers(0, 2))]
            v0 = float(rng.choice([-1.0, 1.0]))
            init = ("ring", "bands")[int(rng.integers(0, 2))]
            s = int(rng.integers(0, 2**31 - 1))
            out.append(Instance(nx, ny, lim, vel, v0, init, s))
    return out


def stratified_subset(instances, large_nodes=None):
    """One instance per (size, velocity, limiter) class, in workload order.
    Sizes of more than large_nodes nodes (when given) keep only their first
    instance, so that an oracle pass over the subset stays short."""
    seen, sizes, out = set(), set(), []
    for inst in instances:
        key = (inst.nx, inst.ny, inst.velocity, inst.limiter)
        if key in seen:
            continue
        if large_nodes is not None and inst.nx * inst.ny > large_nodes and (inst.nx, inst.ny) in sizes:
            continue
        seen.add(key)
        sizes.add((inst.nx, inst.ny))
        out.append(inst)
    return out
