"""FP64 CPU oracle of the layer-case FDM transport scheme (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The GPU library never calls it and shares
no code with it.  The arithmetic lives in ``fdm_oracle.c`` (plain C, IEEE
double, no fast-math, no FMA contraction); this module only builds that file
with gcc and marshals numpy arrays to it.

Conventions (arXiv:1911.03225, sec. 3.2.1): ``alpha12[k*nx + j]`` is
alpha_12 = d1 U^p_13 on the x-edge (j+1/2, k) and ``alpha11[k*nx + j]`` is
alpha_11 = -d2 U^p_13 on the y-edge (j, k+1/2) of a periodic nx-by-ny grid of
pixel nodes.  Arrays are 2-D numpy arrays of shape (ny, nx).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdm_oracle.c")
_LIB = os.path.join(_HERE, "libfdm_oracle.so")

LIMITERS = ("none", "minmod", "mc", "theta", "superbee")
_LIM_NONE, _LIM_THETA, _LIM_SUPERBEE = 0, 1, 2
_LAW, _PRESCRIBED = 0, 1
SCHEMES = ("semidiscrete", "fully_discrete")


def build(force: bool = True) -> str:
    """Compile ``fdm_oracle.c`` into ``libfdm_oracle.so`` with gcc + OpenMP."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-std=c11", "-fno-fast-math", "-ffp-contract=off",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("vkind", ctypes.c_int32),
        ("theta", ctypes.c_double),
        ("v0", ctypes.c_double), ("V1", ctypes.c_double), ("V2", ctypes.c_double),
        ("v0_field", ctypes.c_void_p),
        ("time_order", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("dt", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        d, p, i64 = ctypes.c_double, ctypes.c_void_p, ctypes.c_int64
        P = ctypes.POINTER(_Problem)
        lib.orc_minmod3.argtypes = [d, d, d]
        lib.orc_minmod3.restype = d
        lib.orc_slope.argtypes = [ctypes.c_int32, d, d, d, d]
        lib.orc_slope.restype = d
        lib.orc_hamiltonian.argtypes = [P, d, d, d, p, p, p]
        lib.orc_hamiltonian.restype = None
        lib.orc_hhat_node.argtypes = [P, d, d, d, d, d]
        lib.orc_hhat_node.restype = d
        lib.orc_hhat_field.argtypes = [P, p, p, p]
        lib.orc_hhat_field.restype = None
        lib.orc_stage_rate.argtypes = [P, p, p, p, p]
        lib.orc_stage_rate.restype = None
        lib.orc_step.argtypes = [P, p, p]
        lib.orc_step.restype = None
        lib.orc_run.argtypes = [P, p, p, i64]
        lib.orc_run.restype = None
        lib.orc_cfl_dt.argtypes = [P, d]
        lib.orc_cfl_dt.restype = d
        lib.orc_interp_piece.argtypes = [ctypes.c_int32, d, d, d, d, p, p]
        lib.orc_interp_piece.restype = None
        lib.orc_fd_increment_node.argtypes = [P, d, d, d, d, d, d, d, d, d]
        lib.orc_fd_increment_node.restype = d
        lib.orc_fd_increment_field.argtypes = [P, p, p, p]
        lib.orc_fd_increment_field.restype = None
        lib.orc_stats.argtypes = [i64, p, p, p]
        lib.orc_stats.restype = None
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


class Problem:
    """Scheme parameters for one grid (mirrors the C ``orc_problem``).

    limiter: "none" | "minmod" (theta=1) | "mc" (theta=2) | "theta" | "superbee"
    vkind:   "law" (H = v0 |p|) | "prescribed" (H = V . p)
    v0:      uniform celerity, or an (ny, nx) array of node celerities
    scheme:  "semidiscrete" (Steps 3-4 in the limit dt -> 0, with the
             integrator time_order) | "fully_discrete" (Steps 1-4 of sec.
             3.2.3 at the step dt; one pass per step, time_order must be 1)
    """

    def __init__(self, nx, ny, dx=1.0, dy=1.0, limiter="minmod", theta=None,
                 vkind="law", v0=-1.0, V=(0.0, 0.0), time_order=2, dt=None, scheme="semidiscrete"):
        self.nx, self.ny = int(nx), int(ny)
        self.dx, self.dy = float(dx), float(dy)
        if limiter not in LIMITERS:
            raise ValueError("unknown limiter %r" % (limiter,))
        self.limiter = limiter
        if limiter == "minmod":
            theta = 1.0
        elif limiter == "mc":
            theta = 2.0
        self.theta = float(theta) if theta is not None else 1.0
        if vkind not in ("law", "prescribed"):
            raise ValueError("unknown vkind %r" % (vkind,))
        self.vkind = vkind
        if np.ndim(v0) == 0:
            self.v0, self.v0_field = float(v0), None
        else:
            f = np.ascontiguousarray(v0, dtype=np.float64)
            if f.shape != (self.ny, self.nx):
                raise ValueError("v0 field must have shape (ny, nx)")
            self.v0, self.v0_field = 0.0, f
        self.V = (float(V[0]), float(V[1]))
        self.time_order = int(time_order)
        self.dt = None if dt is None else float(dt)
        if scheme not in SCHEMES:
            raise ValueError("unknown scheme %r" % (scheme,))
        if scheme == "fully_discrete" and self.time_order != 1:
            raise ValueError("the fully discrete scheme is a one-pass step: time_order must be 1")
        self.scheme = scheme

    def _c(self) -> _Problem:
        lim = {"none": _LIM_NONE, "superbee": _LIM_SUPERBEE}.get(self.limiter, _LIM_THETA)
        c = _Problem()
        c.nx, c.ny, c.dx, c.dy = self.nx, self.ny, self.dx, self.dy
        c.limiter = lim
        c.vkind = _LAW if self.vkind == "law" else _PRESCRIBED
        c.theta = self.theta
        c.v0, c.V1, c.V2 = self.v0, self.V[0], self.V[1]
        c.v0_field = self.v0_field.ctypes.data if self.v0_field is not None else None
        c.time_order = self.time_order
        c.scheme = SCHEMES.index(self.scheme)
        c.dt = self.dt if self.dt is not None else 0.0
        return c


def _arr(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def minmod3(x1, x2, x3) -> float:
    return _load().orc_minmod3(float(x1), float(x2), float(x3))


def slope(limiter, wm, w0, wp, theta=None) -> float:
    """Step 1: limited slope at an edge from three consecutive edge values."""
    pb = Problem(1, 1, limiter=limiter, theta=theta)
    lim = {"none": _LIM_NONE, "superbee": _LIM_SUPERBEE}.get(limiter, _LIM_THETA)
    return _load().orc_slope(lim, pb.theta, float(wm), float(w0), float(wp))


def hamiltonian(prob: Problem, px, py, v0=None):
    """(H, dH/dpx, dH/dpy) at one node."""
    c = prob._c()
    out = (ctypes.c_double * 3)()
    base = ctypes.addressof(out)
    _load().orc_hamiltonian(ctypes.byref(c), prob.v0 if v0 is None else float(v0),
                            float(px), float(py), base, base + 8, base + 16)
    return out[0], out[1], out[2]


def hhat_node(prob: Problem, pxm, pxp, pym, pyp, v0=None) -> float:
    """Steps 2-4: semi-discrete numerical Hamiltonian from one-sided derivatives."""
    c = prob._c()
    return _load().orc_hhat_node(ctypes.byref(c), prob.v0 if v0 is None else float(v0),
                                 float(pxm), float(pxp), float(pym), float(pyp))


def hhat_field(prob: Problem, alpha11, alpha12) -> np.ndarray:
    shape = (prob.ny, prob.nx)
    a11, a12 = _arr(alpha11, shape), _arr(alpha12, shape)
    out = np.empty(shape)
    c = prob._c()
    _load().orc_hhat_field(ctypes.byref(c), a11.ctypes.data, a12.ctypes.data, out.ctypes.data)
    return out


def stage_rate(prob: Problem, alpha11, alpha12):
    """(d alpha_11/dt, d alpha_12/dt) of the semi-discrete scheme."""
    shape = (prob.ny, prob.nx)
    a11, a12 = _arr(alpha11, shape), _arr(alpha12, shape)
    r11, r12 = np.empty(shape), np.empty(shape)
    c = prob._c()
    _load().orc_stage_rate(ctypes.byref(c), a11.ctypes.data, a12.ctypes.data,
                           r11.ctypes.data, r12.ctypes.data)
    return r11, r12


def interp_piece(side: int, D, Dp, d, h):
    """Fully discrete Step 1: (increment over phi_j, slope) of the quadratic
    interpolant piece on the side's interval at x_j + h."""
    out = (ctypes.c_double * 2)()
    base = ctypes.addressof(out)
    _load().orc_interp_piece(int(side), float(D), float(Dp), float(d), float(h), base, base + 8)
    return out[0], out[1]


def fd_increment_node(prob: Problem, wxl, sxl, wxr, sxr, wyd, syd, wyu, syu, v0=None) -> float:
    """Fully discrete Steps 2-4 at one node: phi^{n+1} - phi^n at step prob.dt."""
    c = prob._c()
    return _load().orc_fd_increment_node(ctypes.byref(c), prob.v0 if v0 is None else float(v0),
                                         *(float(x) for x in (wxl, sxl, wxr, sxr, wyd, syd, wyu, syu)))


def fd_increment_field(prob: Problem, alpha11, alpha12) -> np.ndarray:
    """Node increments phi^{n+1} - phi^n of one fully discrete step."""
    if prob.dt is None:
        raise ValueError("Problem.dt must be set (use cfl_dt)")
    shape = (prob.ny, prob.nx)
    a11, a12 = _arr(alpha11, shape), _arr(alpha12, shape)
    out = np.empty(shape)
    c = prob._c()
    _load().orc_fd_increment_field(ctypes.byref(c), a11.ctypes.data, a12.ctypes.data, out.ctypes.data)
    return out


def cfl_dt(prob: Problem, nu: float) -> float:
    c = prob._c()
    return _load().orc_cfl_dt(ctypes.byref(c), float(nu))


def run(prob: Problem, alpha11, alpha12, n_steps: int):
    """Advance copies of (alpha11, alpha12) by n_steps; returns the new pair."""
    if prob.dt is None:
        raise ValueError("Problem.dt must be set (use cfl_dt)")
    shape = (prob.ny, prob.nx)
    a11, a12 = _arr(alpha11, shape).copy(), _arr(alpha12, shape).copy()
    c = prob._c()
    _load().orc_run(ctypes.byref(c), a11.ctypes.data, a12.ctypes.data, int(n_steps))
    return a11, a12


def stats(alpha11, alpha12) -> dict:
    a11 = _arr(alpha11).ravel()
    a12 = _arr(alpha12).ravel()
    out = np.empty(5)
    _load().orc_stats(a11.size, a11.ctypes.data, a12.ctypes.data, out.ctypes.data)
    return {"sum11": out[0], "sum12": out[1], "sum_abs": out[2],
            "max_norm": out[3], "nonfinite": int(out[4])}


def max_threads() -> int:
    return _load().orc_max_threads()


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))
