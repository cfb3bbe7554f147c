"""FP64 oracle of the coupled run of the layer case (test infrastructure).

Only the test-suite uses this module; the GPU library shares no code with
it.  It alternates, per step, the static problem and the transport as in
arXiv:1911.03225 sec. 3.1.1 (the static problem solved with the current
plastic distortion, then the transport with the new stress), in the layer
case of sec. 3.2.1:

1. tau13, the layer-averaged shear stress of the current densities and the
   current mean strain and mean slip (``oracle.static``);
2. the celerity with m = mobility times an optional node factor (0 marks
   an obstacle, the precipitates of sec. 5), rounded to float32 (the library
   takes node celerities as float32, like every other input):
   threshold law  v0 = -m S(tau13), S the soft threshold
                  S(t) = sign(t) max(|t| - tau0, 0) (sec. 2.3, first approach);
   wiggly law     v0 = m (tau_y cos(phi / beta) - tau13), the energy
                  G = beta sin(phi/beta) tau_y of sec. 3.2.1, phi at the nodes
                  recovered from the densities and their mean;
3. dt = the largest float not above min(cfl min(dx,dy) / max|v0|, dt_max);
4. one step of the FP64 transport oracle with v0 frozen over the step;
5. the mean of phi = U^p_13, which the densities do not carry, follows
   phi_{n+1} = phi_n - dt Hhat (Euler), the Heun average of the two stages'
   Hhat, or Hhat of the half-step state (explicit midpoint), so its mean
   moves by -dt times the mean of that Hhat; with the fully discrete scheme
   of sec. 3.2.3 it moves by the mean of the node increments.  The mean
   strain moves by strain_rate13 * dt.
"""
from __future__ import annotations

import numpy as np

import oracle as T
from oracle import static as S


def round_down_float(x: float) -> float:
    f = np.float32(x)
    if float(f) > x:
        f = np.nextafter(f, np.float32(0.0))
    return float(f)


def soft_threshold(t, t0: float):
    return np.sign(t) * np.maximum(np.abs(t) - t0, 0.0)


def coupled_run(a11, a12, n_steps: int, chunk: int, *, dx: float = 1.0, limiter: str = "minmod",
                theta=None, cfl: float = 0.4, time_order: int = 2, mu: float = 1.0, lam: float = 1.5,
                layer_h: float = 4.0, cell_l3: float = 512.0, tau0: float = 0.01, mobility: float = 1.0,
                strain_rate13: float = 1e-3, dt_max: float = 0.05, eps13: float = 0.0, phi_mean: float = 0.0,
                law: str = "threshold", tau_y: float = 0.0, beta: float = 1.0, mobility_field=None,
                scheme: str = "semidiscrete"):
    """Returns (alpha11, alpha12, history); history holds one dict per chunk
    (after its last step): t, dt, step, eps13, sigma13, phi_mean, vmax and
    the density sums."""
    a11 = np.array(a11, dtype=np.float64)
    a12 = np.array(a12, dtype=np.float64)
    ny, nx = a11.shape
    h, n3 = int(round(layer_h / dx)), int(round(cell_l3 / dx))
    eps, phi, t = float(eps13), float(phi_mean), 0.0
    history = []
    for step in range(n_steps):
        tau = S.static_tau13(a11, a12, dx, dx, mu, lam, h, n3, eps, phi)
        m = mobility if mobility_field is None else mobility * np.asarray(mobility_field, np.float32).astype(np.float64)
        if law == "wiggly":
            nodes = S.phi_from_alpha(a11, a12, dx, dx, phi)
            v0 = m * (tau_y * np.cos(nodes / beta) - tau)
        else:
            v0 = -(m * soft_threshold(tau, tau0))
        v0 = v0.astype(np.float32).astype(np.float64)
        vmax = float(np.max(np.abs(v0)))
        dt = round_down_float(min(cfl * dx / vmax, dt_max) if vmax > 0.0 else dt_max)
        P = T.Problem(nx, ny, dx, dx, limiter=limiter, theta=theta, v0=v0, time_order=time_order, dt=dt,
                      scheme=scheme)
        if scheme == "fully_discrete":   # phi_{n+1} - phi_n: the node increments of the step
            hmean = -float(np.mean(T.fd_increment_field(P, a11, a12))) / dt
        else:
            hmean = float(np.mean(T.hhat_field(P, a11, a12)))
        if scheme == "fully_discrete":
            pass
        elif time_order == 2:       # Heun: phi - dt/2 (Hhat(u) + Hhat(u + dt L(u)))
            Pe = T.Problem(nx, ny, dx, dx, limiter=limiter, theta=theta, v0=v0, time_order=1, dt=dt)
            w11, w12 = T.run(Pe, a11, a12, 1)
            hmean = 0.5 * (hmean + float(np.mean(T.hhat_field(P, w11, w12))))
        elif time_order == 3:     # midpoint: phi - dt Hhat(u + dt/2 L(u))
            Ph = T.Problem(nx, ny, dx, dx, limiter=limiter, theta=theta, v0=v0, time_order=1, dt=0.5 * dt)
            w11, w12 = T.run(Ph, a11, a12, 1)
            hmean = float(np.mean(T.hhat_field(P, w11, w12)))
        a11, a12 = T.run(P, a11, a12, 1)
        phi -= dt * hmean
        eps += strain_rate13 * dt
        t += dt
        if (step + 1) % chunk == 0 or step + 1 == n_steps:
            rec = T.stats(a11, a12)
            rec.update(t=t, dt=dt, step=step + 1, eps13=eps, phi_mean=phi, vmax=vmax,
                       sigma13=S.mean_stress13(mu, eps, phi, h, n3))
            history.append(rec)
    return a11, a12, history
