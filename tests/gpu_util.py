"""Helpers for the GPU tests: run the HIP path through the C ABI and compare
with the FP64 oracle on the same float32 inputs."""
from __future__ import annotations

import numpy as np


def to_dev(a, dtype=np.float32):
    """Device copy; float64 copies hold the float32-rounded values exactly."""
    import torch
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32), dtype=dtype)
    return torch.from_numpy(a).to("cuda:0")


def state_dtype(options):
    return np.float64 if (options or {}).get("precision") == "fp64" else np.float32


def gpu_run(a11, a12, n_steps, snapshots=None, options=None, **desc_kw):
    """Run the HIP path; returns (dt, [(step, a11, a12) ...]) in float64 numpy.

    snapshots: list of step counts at which to copy the state back (the last
    one must be n_steps); defaults to [n_steps].
    """
    import torch
    from paper_1911_03225_amd import fdm

    ny, nx = a11.shape
    keep = []
    v0f = desc_kw.pop("v0_field", None)
    if v0f is not None:
        v0f = to_dev(v0f)
        keep.append(v0f)
    t11, t12 = to_dev(a11, state_dtype(options)), to_dev(a12, state_dtype(options))
    ctx = fdm.fdm_transport_init(fdm.desc(nx, ny, v0_field=v0f, **desc_kw), options=options, keep=keep)
    dt = fdm.fdm_transport_dt(ctx)
    out, done = [], 0
    for s in (snapshots or [n_steps]):
        fdm.fdm_transport_step(ctx, t11, t12, s - done)
        done = s
        torch.cuda.synchronize()
        out.append((s, t11.cpu().numpy().astype(np.float64), t12.cpu().numpy().astype(np.float64)))
    fdm.fdm_destroy(ctx)
    return dt, out


def oracle_problem(oracle, nx, ny, dt, dx=1.0, dy=1.0, limiter="minmod", theta=1.0, time_order=2,
                   velocity="law", v0=-1.0, v0_field=None, V=(0.0, 0.0), scheme="semidiscrete", **_):
    v = v0 if v0_field is None else np.asarray(v0_field, dtype=np.float64)
    return oracle.Problem(nx, ny, dx=dx, dy=dy, limiter=limiter, theta=theta, vkind=velocity,
                          v0=float(np.float32(v)) if np.ndim(v) == 0 else v,
                          V=tuple(float(np.float32(x)) for x in V), time_order=time_order, dt=dt,
                          scheme=scheme)


def rel_l1(g11, g12, o11, o12, ref11, ref12):
    """||gpu - oracle||_1 over both components / ||initial||_1."""
    den = np.abs(ref11).sum() + np.abs(ref12).sum()
    return float((np.abs(g11 - o11).sum() + np.abs(g12 - o12).sum()) / den)


def rel_linf(g11, g12, o11, o12, ref11, ref12):
    den = max(np.abs(ref11).max(), np.abs(ref12).max())
    return float(max(np.abs(g11 - o11).max(), np.abs(g12 - o12).max()) / den)


def tolerance(n_steps):
    """Relative L1 bound: 1e-5 per started block of 1000 steps."""
    return 1e-5 * max(1, -(-n_steps // 1000))


def compare_run(oracle, a11, a12, n_steps, every=None, options=None, **kw):
    """GPU vs oracle on the same inputs, checked every `every` steps."""
    every = every or n_steps
    snaps = list(range(every, n_steps + 1, every))
    if snaps[-1] != n_steps:
        snaps.append(n_steps)
    dt, gsnaps = gpu_run(a11, a12, n_steps, snapshots=snaps, options=options, **dict(kw))
    ny, nx = a11.shape
    P = oracle_problem(oracle, nx, ny, dt, **kw)
    o11, o12 = a11.astype(np.float64), a12.astype(np.float64)
    done = 0
    report = []
    for s, g11, g12 in gsnaps:
        o11, o12 = oracle.run(P, o11, o12, s - done)
        done = s
        e1 = rel_l1(g11, g12, o11, o12, a11, a12)
        einf = rel_linf(g11, g12, o11, o12, a11, a12)
        report.append((s, e1, einf))
    return dt, report, (g11, g12), (o11, o12)
