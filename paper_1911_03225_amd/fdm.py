"""ctypes binding of ``libfdm.so`` (C ABI in include/fdm.h), same entry-point names.

Argument marshalling only: every step of the transport runs in the library's
HIP kernels.  torch supplies device memory (float32 CUDA tensors) and the
stream; it is imported before the library is loaded so that both use the same
HIP runtime.  There is no CPU fallback: if the library is missing or a call
fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # noqa: F401  (must be loaded before libfdm.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdm.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fdm.h")

FDM_OK, FDM_ERR_INVALID_ARG, FDM_ERR_DEVICE, FDM_ERR_OUT_OF_MEMORY = 0, 1, 2, 3
FDM_ERR_CFL, FDM_ERR_NONFINITE, FDM_ERR_UNSUPPORTED = 4, 5, 6
LIMITERS = {"none": 0, "minmod": 1, "mc": 2, "theta": 3, "superbee": 4}
VELOCITIES = {"law": 0, "prescribed": 1}
SCHEDULES = {"auto": 0, "batched": 1, "plain": 2, "fused": 3}
PRECISIONS = {"fp32": 0, "fp64_arith": 1, "fp64": 2}
SCHEMES = {"semidiscrete": 0, "fully_discrete": 1}


class fdm_transport_desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("scheme", ctypes.c_int32), ("theta", ctypes.c_double),
        ("time_order", ctypes.c_int32), ("cfl", ctypes.c_double), ("dt", ctypes.c_double),
        ("velocity", ctypes.c_int32), ("v0", ctypes.c_double),
        ("v0_field", ctypes.c_void_p), ("V", ctypes.c_double * 2),
    ]


class fdm_options(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("precision", ctypes.c_int32)]


class fdm_stats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("dt", ctypes.c_double), ("step", ctypes.c_int64),
        ("sum11", ctypes.c_double), ("sum12", ctypes.c_double),
        ("sum_abs", ctypes.c_double), ("max_norm", ctypes.c_double),
        ("drift11", ctypes.c_double), ("drift12", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
        ("eps13", ctypes.c_double), ("sigma13", ctypes.c_double),
        ("phi_mean", ctypes.c_double), ("vmax", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class fdm_tune_trial(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("seconds_per_step", ctypes.c_double)]


class fdm_static_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("mu", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("layer_h", ctypes.c_double), ("cell_l3", ctypes.c_double),
                ("eps13", ctypes.c_double), ("phi_mean", ctypes.c_double),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class fdm_loading(ctypes.Structure):
    _fields_ = [("strain_rate13", ctypes.c_double), ("tau0", ctypes.c_double),
                ("mobility", ctypes.c_double), ("mu", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("layer_h", ctypes.c_double),
                ("cell_l3", ctypes.c_double), ("dt_max", ctypes.c_double),
                ("eps13", ctypes.c_double), ("phi_mean", ctypes.c_double),
                ("law", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tau_y", ctypes.c_double), ("beta", ctypes.c_double),
                ("mobility_field", ctypes.c_void_p)]


LAWS = {"threshold": 0, "wiggly": 1}


def loading(strain_rate13: float = 1e-3, tau0: float = 0.01, mobility: float = 1.0, mu: float = 1.0,
            lam: float = 1.5, layer_h: float = 4.0, cell_l3: float = 512.0, dt_max: float = 0.05,
            eps13: float = 0.0, phi_mean: float = 0.0, law="threshold", tau_y: float = 0.0, beta: float = 1.0,
            mobility_field=None) -> fdm_loading:
    """mobility_field: optional float32 CUDA tensor (ny, nx) of factors on the mobility (keep it alive)."""
    mf = None
    if mobility_field is not None:
        mf = _ptr(mobility_field, None, "mobility_field")
    return fdm_loading(float(strain_rate13), float(tau0), float(mobility), float(mu), float(lam), float(layer_h),
                       float(cell_l3), float(dt_max), float(eps13), float(phi_mean),
                       LAWS[law] if isinstance(law, str) else int(law), 0, float(tau_y), float(beta), mf)


class FdmError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__("%s failed: %s (%s)" % (where, fdm_status_string(status), message))


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfdm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libfdm.so not found at %s; build it with "
                           "`python -m paper_1911_03225_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P, i32, vp = ctypes.POINTER, ctypes.c_int32, ctypes.c_void_p
    fpp = P(ctypes.c_void_p)
    lib.fdm_transport_init.argtypes = [P(fdm_transport_desc), i32, P(fdm_options), vp, P(vp)]
    lib.fdm_transport_step.argtypes = [vp, fpp, fpp, i32]
    lib.fdm_transport_stats.argtypes = [vp, fpp, fpp, P(fdm_stats)]
    lib.fdm_transport_step_noalloc.argtypes = [P(fdm_transport_desc), vp, vp, i32, vp]
    lib.fdm_static_solve.argtypes = [P(fdm_static_desc), vp, vp, vp, vp]
    lib.fdm_run.argtypes = [vp, P(fdm_loading), fpp, fpp, i32, i32, P(fdm_stats)]
    lib.fdm_transport_dt.argtypes = [vp, i32]
    lib.fdm_transport_dt.restype = ctypes.c_double
    lib.fdm_tile_rows.argtypes = [vp, i32]
    lib.fdm_tile_rows.restype = i32
    lib.fdm_autotune.argtypes = [vp, fpp, fpp, i32, P(fdm_tune_trial), i32, P(i32)]
    lib.fdm_destroy.argtypes = [vp]
    lib.fdm_destroy.restype = None
    lib.fdm_status_string.argtypes = [ctypes.c_int]
    lib.fdm_status_string.restype = ctypes.c_char_p
    lib.fdm_last_error.argtypes = [vp]
    lib.fdm_last_error.restype = ctypes.c_char_p
    for name in ("fdm_transport_init", "fdm_transport_step", "fdm_transport_stats",
                 "fdm_static_solve", "fdm_run", "fdm_autotune", "fdm_transport_step_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/fdm.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdm_\w+)\s*\(", text)))


def fdm_status_string(status: int) -> str:
    return load_library().fdm_status_string(int(status)).decode()


def fdm_last_error(ctx=None) -> str:
    h = ctx.handle if isinstance(ctx, Context) else ctx
    return load_library().fdm_last_error(h).decode()


def _check(status: int, where: str, ctx=None):
    if status != FDM_OK:
        raise FdmError(status, where, fdm_last_error(ctx))


def desc(nx, ny, dx=1.0, dy=1.0, limiter="minmod", theta=1.0, time_order=2, cfl=0.4,
         dt=0.0, velocity="law", v0=-1.0, v0_field=None, V=(0.0, 0.0),
         scheme="semidiscrete") -> fdm_transport_desc:
    """Build an fdm_transport_desc; v0_field is a float32 CUDA tensor of shape (ny, nx)."""
    d = fdm_transport_desc()
    d.nx, d.ny, d.dx, d.dy = int(nx), int(ny), float(dx), float(dy)
    d.limiter = LIMITERS[limiter] if isinstance(limiter, str) else int(limiter)
    d.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    d.theta, d.time_order, d.cfl, d.dt = float(theta), int(time_order), float(cfl), float(dt)
    d.velocity = VELOCITIES[velocity] if isinstance(velocity, str) else int(velocity)
    d.v0 = float(v0)
    d.v0_field = _ptr(v0_field, (ny, nx), "v0_field") if v0_field is not None else None
    d.V[0], d.V[1] = float(V[0]), float(V[1])
    return d


def _ptr(t, shape, what, dtype=torch.float32):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % what)
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s CUDA tensor" % (what, str(dtype).replace("torch.", "")))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (what, tuple(shape), tuple(t.shape)))
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        if not torch.cuda.is_available():
            return ctypes.c_void_p(0)          # null stream; the library reports the missing device
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream) if hasattr(stream, "cuda_stream") else ctypes.c_void_p(stream)


class Context:
    """An fdm_ctx handle plus the Python objects it must keep alive."""

    def __init__(self, handle, descs, keep, precision=0):
        self.handle = handle
        self.descs = descs
        self._keep = keep
        self.precision = precision
        self.dtype = torch.float64 if precision == PRECISIONS["fp64"] else torch.float32

    @property
    def n(self):
        return len(self.descs)

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                fdm_destroy(self)
            except Exception:
                pass


def fdm_transport_init(descs, options=None, stream=None, keep=()):
    """descs: one fdm_transport_desc or a list; options: fdm_options or dict."""
    lib = load_library()
    if isinstance(descs, fdm_transport_desc):
        descs = [descs]
    arr = (fdm_transport_desc * len(descs))(*descs)
    opt = None
    if options is not None:
        if isinstance(options, dict):
            o = fdm_options()
            o.schedule = SCHEDULES.get(options.get("schedule", "auto"), 0) \
                if isinstance(options.get("schedule", "auto"), str) else int(options["schedule"])
            o.tile_rows = int(options.get("tile_rows", 0))
            o.fused = int(options.get("fused", 0))
            prec = options.get("precision", "fp32")
            o.precision = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
            options = o
        opt = ctypes.byref(options)
    h = ctypes.c_void_p()
    st = lib.fdm_transport_init(arr, len(descs), opt, _stream_handle(stream), ctypes.byref(h))
    _check(st, "fdm_transport_init", None)
    return Context(h, list(descs), keep, options.precision if options is not None else 0)


def _ptr_arrays(ctx, alpha11, alpha12):
    if isinstance(alpha11, torch.Tensor):
        alpha11, alpha12 = [alpha11], [alpha12]
    if len(alpha11) != ctx.n or len(alpha12) != ctx.n:
        raise ValueError("need one alpha11 and one alpha12 tensor per instance")
    p11 = (ctypes.c_void_p * ctx.n)()
    p12 = (ctypes.c_void_p * ctx.n)()
    for i, (a, b, d) in enumerate(zip(alpha11, alpha12, ctx.descs)):
        p11[i] = _ptr(a, (d.ny, d.nx), "alpha11[%d]" % i, ctx.dtype)
        p12[i] = _ptr(b, (d.ny, d.nx), "alpha12[%d]" % i, ctx.dtype)
    return p11, p12


def fdm_transport_step(ctx, alpha11, alpha12, n_steps: int) -> None:
    p11, p12 = _ptr_arrays(ctx, alpha11, alpha12)
    _check(load_library().fdm_transport_step(ctx.handle, p11, p12, int(n_steps)),
           "fdm_transport_step", ctx)


NOALLOC_MAX_NODES = 4194304


def fdm_transport_step_noalloc(desc_, alpha11, alpha12, n_steps: int, stream=None) -> None:
    """Allocation-free step of one float32 instance (no context)."""
    shape = (desc_.ny, desc_.nx)
    st = load_library().fdm_transport_step_noalloc(ctypes.byref(desc_), _ptr(alpha11, shape, "alpha11"),
                                                   _ptr(alpha12, shape, "alpha12"), int(n_steps),
                                                   _stream_handle(stream))
    _check(st, "fdm_transport_step_noalloc", None)


def fdm_transport_stats(ctx, alpha11, alpha12, allow_nonfinite: bool = False):
    p11, p12 = _ptr_arrays(ctx, alpha11, alpha12)
    out = (fdm_stats * ctx.n)()
    st = load_library().fdm_transport_stats(ctx.handle, p11, p12, out)
    if not (allow_nonfinite and st == FDM_ERR_NONFINITE):
        _check(st, "fdm_transport_stats", ctx)
    return [o.as_dict() for o in out]


def fdm_run(ctx, alpha11, alpha12, n_steps: int, chunk: int, loading=None, history: bool = True):
    p11, p12 = _ptr_arrays(ctx, alpha11, alpha12)
    n_chunks = (int(n_steps) + int(chunk) - 1) // int(chunk) if n_steps > 0 else 0
    hist = (fdm_stats * max(1, n_chunks * ctx.n))() if history else None
    st = load_library().fdm_run(ctx.handle, ctypes.byref(loading) if loading is not None else None,
                                p11, p12, int(n_steps), int(chunk), hist)
    _check(st, "fdm_run", ctx)
    if not history:
        return None
    return [[hist[c * ctx.n + i].as_dict() for i in range(ctx.n)] for c in range(n_chunks)]


def static_desc(nx: int, ny: int, dx: float = 1.0, dy: float = None, mu: float = 1.0, lam: float = 1.5,
                layer_h: float = 4.0, cell_l3: float = 512.0, eps13: float = 0.0, phi_mean: float = 0.0,
                precision="fp32") -> fdm_static_desc:
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return fdm_static_desc(int(nx), int(ny), float(dx), float(dx if dy is None else dy), float(mu), float(lam),
                           float(layer_h), float(cell_l3), float(eps13), float(phi_mean), p, 0)


def fdm_static_solve(desc_, alpha11, alpha12, tau13_out=None, stream=None):
    """tau13 (layer-averaged shear stress at the nodes) for the densities;
    allocates tau13_out when not given.  Synchronous."""
    dtype = torch.float64 if desc_.precision == PRECISIONS["fp64"] else torch.float32
    shape = (desc_.ny, desc_.nx)
    if tau13_out is None:
        tau13_out = torch.empty(shape, dtype=dtype, device=alpha11.device)
    st = load_library().fdm_static_solve(ctypes.byref(desc_), _ptr(alpha11, shape, "alpha11", dtype),
                                         _ptr(alpha12, shape, "alpha12", dtype),
                                         _ptr(tau13_out, shape, "tau13_out", dtype), _stream_handle(stream))
    _check(st, "fdm_static_solve", None)
    return tau13_out


def fdm_tile_rows(ctx, instance: int = 0) -> int:
    return int(load_library().fdm_tile_rows(ctx.handle, int(instance)))


def fdm_autotune(ctx, alpha11, alpha12, trial_steps: int = 10, max_trials: int = 64):
    """Time the candidate tilings on a copy of the state and keep the
    fastest; returns the list of measured trials (dicts) in the order run."""
    p11, p12 = _ptr_arrays(ctx, alpha11, alpha12)
    arr = (fdm_tune_trial * max_trials)()
    n = ctypes.c_int32(0)
    _check(load_library().fdm_autotune(ctx.handle, p11, p12, int(trial_steps), arr, int(max_trials),
                                       ctypes.byref(n)), "fdm_autotune", ctx)
    names = {v: k for k, v in SCHEDULES.items()}
    return [{"tile_rows": arr[i].tile_rows, "schedule": names.get(arr[i].schedule, arr[i].schedule),
             "seconds_per_step": arr[i].seconds_per_step} for i in range(n.value)]


def fdm_transport_dt(ctx, instance: int = 0) -> float:
    return load_library().fdm_transport_dt(ctx.handle, int(instance))


def fdm_destroy(ctx) -> None:
    if ctx.handle:
        load_library().fdm_destroy(ctx.handle)
        ctx.handle = None
