"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function include/fdm.h declares, and
reject invalid descriptors on the host before any HIP call.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fdm():
    from paper_1911_03225_amd import fdm as F
    if not os.path.exists(F.LIB_PATH):
        from paper_1911_03225_amd import build
        build.build()
    F.load_library()
    return F


def test_exports_every_declared_function(fdm):
    names = fdm.header_functions()
    assert {"fdm_transport_init", "fdm_transport_step", "fdm_static_solve", "fdm_run"} <= set(names)
    lib = fdm.load_library()
    for n in names:
        assert hasattr(lib, n), n


def test_header_enums_match_binding(fdm):
    text = open(os.path.join(ROOT, "include", "fdm.h")).read()
    vals = dict((k, int(v)) for k, v in re.findall(r"\b(FDM_\w+)\s*=\s*(\d+)", text))
    assert vals["FDM_OK"] == fdm.FDM_OK
    assert vals["FDM_ERR_INVALID_ARG"] == fdm.FDM_ERR_INVALID_ARG
    assert vals["FDM_ERR_DEVICE"] == fdm.FDM_ERR_DEVICE
    assert vals["FDM_ERR_CFL"] == fdm.FDM_ERR_CFL
    assert vals["FDM_ERR_NONFINITE"] == fdm.FDM_ERR_NONFINITE
    assert vals["FDM_ERR_UNSUPPORTED"] == fdm.FDM_ERR_UNSUPPORTED
    for name, v in fdm.LIMITERS.items():
        assert vals["FDM_LIMITER_" + name.upper()] == v
    assert vals["FDM_VELOCITY_LAW"] == fdm.VELOCITIES["law"]
    assert vals["FDM_VELOCITY_PRESCRIBED"] == fdm.VELOCITIES["prescribed"]
    for name, v in fdm.SCHEMES.items():
        assert vals["FDM_SCHEME_" + name.upper()] == v
    for name, v in fdm.SCHEDULES.items():
        assert vals["FDM_SCHEDULE_" + name.upper()] == v


def test_struct_offsets_match_the_header(fdm, tmp_path):
    """Every field offset of the binding's structs equals the C compiler's."""
    import ctypes
    import subprocess
    structs = [fdm.fdm_transport_desc, fdm.fdm_stats, fdm.fdm_loading, fdm.fdm_options,
               fdm.fdm_tune_trial, fdm.fdm_static_desc]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fdm.h"', "int main(void) {"]
    expect = []
    for st in structs:
        name = st.__name__
        lines.append('printf("%%zu\\n", sizeof(%s));' % name)
        expect.append(ctypes.sizeof(st))
        for f in st._fields_:
            cname = f[0].rstrip("_")          # Python keywords carry a trailing underscore
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (name, cname))
            expect.append(getattr(st, f[0]).offset)
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == expect


def test_struct_sizes_match_c_layout(fdm):
    import ctypes
    # int32 + pad before each double, pointer-aligned field: the C layout
    assert ctypes.sizeof(fdm.fdm_transport_desc) == 104
    assert ctypes.sizeof(fdm.fdm_stats) == 112
    assert ctypes.sizeof(fdm.fdm_loading) == 112
    assert ctypes.sizeof(fdm.fdm_options) == 16
    assert ctypes.sizeof(fdm.fdm_tune_trial) == 16
    assert ctypes.sizeof(fdm.fdm_static_desc) == 80


def test_status_strings(fdm):
    for st in range(7):
        assert fdm.fdm_status_string(st)
    assert fdm.fdm_status_string(99) == "unknown status"


BAD = [
    (dict(nx=0), "nx and ny"),
    (dict(ny=-3), "nx and ny"),
    (dict(nx=65536, ny=65536), "2^31"),
    (dict(nx=1 << 27, ny=1), "2^27"),
    (dict(dx=0.0), "dx and dy"),
    (dict(dy=float("nan")), "dx and dy"),
    (dict(limiter=7), "limiter"),
    (dict(limiter="theta", theta=2.5), "theta"),
    (dict(limiter="theta", theta=0.9), "theta"),
    (dict(time_order=4), "time_order"),
    (dict(time_order=-1), "time_order"),
    (dict(cfl=0.0), "cfl"),
    (dict(cfl=1.5), "cfl"),
    (dict(dt=-1.0), "dt"),
    (dict(dt=1e39, v0=0.0), "dt"),
    (dict(velocity=5), "velocity"),
    (dict(v0=float("inf")), "v0"),
    (dict(velocity="prescribed", V=(float("nan"), 0.0)), "V"),
    (dict(v0=1e39), "v0"),
    (dict(velocity="prescribed", V=(0.5, -4e38)), "V"),
    (dict(scheme=5), "scheme"),
    (dict(scheme="fully_discrete", time_order=2), "one pass per step"),
    (dict(scheme="fully_discrete", time_order=3), "one pass per step"),
]


@pytest.mark.parametrize("kw,msg", BAD)
def test_invalid_descriptor_rejected_on_host(fdm, kw, msg):
    args = dict(nx=16, ny=16)
    args.update(kw)
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_init(fdm.desc(**args))
    assert e.value.status == fdm.FDM_ERR_INVALID_ARG
    assert msg in fdm.fdm_last_error(None)


# The stability bound nu2 = dt (S1/dx + S2/dy) <= 1 (1/2 for one limited
# forward-Euler stage), decided on the host for every case but a fixed dt
# over a celerity field.
COURANT_BAD = [
    (dict(cfl=0.6), "2-D Courant"),                                   # LAW, Heun, square grid: nu2 = 1.2
    (dict(cfl=0.8, dx=0.5), "2-D Courant"),                           # nu2 = 0.8 * 0.5 * (1/0.5 + 1/1) = 1.2
    (dict(cfl=0.26, time_order=1), "forward-Euler"),                  # limited Euler stage: nu2 = 0.52
    (dict(cfl=0.3, time_order=1, scheme="fully_discrete"), "forward-Euler"),
    (dict(limiter="none", time_order=1, velocity="prescribed", V=(1.0, 0.5), cfl=1.0), "2-D Courant"),
    (dict(dt=0.6, v0=-1.0), "2-D Courant"),                           # fixed dt, uniform celerity
    (dict(dt=0.3, v0=-1.0, time_order=1, limiter="superbee"), "forward-Euler"),
    (dict(dt=0.6, velocity="prescribed", V=(0.9, 0.9)), "2-D Courant"),
    (dict(nx=1, ny=64, cfl=1.0, time_order=1), "forward-Euler"),      # 1-D along y
]


@pytest.mark.parametrize("kw,msg", COURANT_BAD)
def test_courant_bound_rejected_on_host(fdm, kw, msg):
    args = dict(nx=16, ny=16)
    args.update(kw)
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_init(fdm.desc(**args))
    assert e.value.status == fdm.FDM_ERR_CFL
    assert msg in fdm.fdm_last_error(None)


COURANT_OK = [
    dict(cfl=0.5),                                                    # nu2 = 1: the colliding-pulse runs
    dict(cfl=0.25, time_order=1),                                     # the paper's Courant number
    dict(cfl=0.25, time_order=1, scheme="fully_discrete"),
    dict(ny=1, cfl=1.0),                                              # 1-D: one axis
    dict(ny=1, cfl=0.5, time_order=1, limiter="superbee"),
    dict(ny=1, limiter="none", time_order=1, velocity="prescribed", V=(1.0, 0.5), cfl=1.0),
    dict(limiter="none", time_order=1, velocity="prescribed", V=(1.0, 0.0), dt=1.0),
    dict(limiter="none", time_order=1, cfl=0.5),
    dict(dt=0.5, v0=-1.0),
    dict(dt=1.0, v0=-1.0, dx=2.0, dy=2.0),
    dict(velocity="prescribed", V=(0.7, -0.4), dx=1.3, dy=0.6, cfl=0.5),
]


@pytest.mark.parametrize("kw", COURANT_OK)
def test_courant_bound_accepts_stable_steps(fdm, kw):
    """Within the bound the descriptor passes the host checks (and, with no
    GPU, fails only at the first HIP call)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    args = dict(nx=16, ny=16)
    args.update(kw)
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_init(fdm.desc(**args))
    assert e.value.status == fdm.FDM_ERR_DEVICE, fdm.fdm_last_error(None)


def test_mixed_schemes_rejected(fdm):
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_init([fdm.desc(8, 8, time_order=1),
                                fdm.desc(8, 8, time_order=1, scheme="fully_discrete")])
    assert e.value.status == fdm.FDM_ERR_INVALID_ARG
    assert "scheme" in fdm.fdm_last_error(None)


def test_mixed_time_orders_rejected(fdm):
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_init([fdm.desc(8, 8, time_order=1), fdm.desc(8, 8, time_order=2)])
    assert e.value.status == fdm.FDM_ERR_INVALID_ARG


def test_null_arguments(fdm):
    lib = fdm.load_library()
    import ctypes
    h = ctypes.c_void_p()
    assert lib.fdm_transport_init(None, 1, None, None, ctypes.byref(h)) == fdm.FDM_ERR_INVALID_ARG
    assert lib.fdm_transport_init(None, 1, None, None, None) == fdm.FDM_ERR_INVALID_ARG
    assert lib.fdm_transport_step(None, None, None, 1) == fdm.FDM_ERR_INVALID_ARG
    assert lib.fdm_run(None, None, None, None, 1, 1, None) == fdm.FDM_ERR_INVALID_ARG
    assert fdm.load_library().fdm_transport_dt(None, 0) == -1.0
    assert lib.fdm_tile_rows(None, 0) == -1
    assert lib.fdm_autotune(None, None, None, 1, None, 0, None) == fdm.FDM_ERR_INVALID_ARG
    lib.fdm_destroy(None)   # no-op


STATIC_BAD = [
    (dict(nx=0), "nx and ny"),
    (dict(dx=1.0, dy=0.5), "dx must equal dy"),
    (dict(mu=0.0), "mu"),
    (dict(lam=-1.0), "lambda"),
    (dict(layer_h=2.5), "layer_h"),
    (dict(layer_h=0.0), "layer_h"),
    (dict(cell_l3=3.0, layer_h=4.0), "must not exceed"),
    (dict(cell_l3=float("inf")), "cell_l3"),
    (dict(eps13=float("nan")), "eps13"),
    (dict(precision=5), "precision"),
]


@pytest.mark.parametrize("kw,msg", STATIC_BAD)
def test_static_solve_rejects_bad_descriptors_on_host(fdm, kw, msg):
    import ctypes
    lib = fdm.load_library()
    args = dict(nx=16, ny=16, cell_l3=16.0)
    args.update(kw)
    d = fdm.static_desc(**args)
    assert lib.fdm_static_solve(ctypes.byref(d), None, None, None, None) == fdm.FDM_ERR_INVALID_ARG
    assert msg in fdm.fdm_last_error(None)


def test_static_solve_null_and_aliased_arrays(fdm):
    import ctypes
    lib = fdm.load_library()
    d = fdm.static_desc(16, 16, cell_l3=16.0)
    assert lib.fdm_static_solve(None, None, None, None, None) == fdm.FDM_ERR_INVALID_ARG
    assert lib.fdm_static_solve(ctypes.byref(d), None, None, None, None) == fdm.FDM_ERR_INVALID_ARG
    assert "NULL" in fdm.fdm_last_error(None)
    p = ctypes.c_void_p(4096)
    assert lib.fdm_static_solve(ctypes.byref(d), p, p, ctypes.c_void_p(8192), None) == fdm.FDM_ERR_INVALID_ARG
    assert "distinct" in fdm.fdm_last_error(None)
    d.reserved = 1
    assert lib.fdm_static_solve(ctypes.byref(d), p, ctypes.c_void_p(8), ctypes.c_void_p(16), None) == \
        fdm.FDM_ERR_INVALID_ARG


def test_valid_descriptor_without_gpu_fails_cleanly(fdm):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_init(fdm.desc(16, 16))
    assert e.value.status == fdm.FDM_ERR_DEVICE


def test_invalid_options_rejected(fdm):
    for opts in ({"precision": 7}, {"schedule": 9}, {"tile_rows": -1}, {"fused": 1}):
        with pytest.raises(fdm.FdmError) as e:
            fdm.fdm_transport_init(fdm.desc(16, 16), options=opts)
        assert e.value.status == fdm.FDM_ERR_INVALID_ARG


@pytest.mark.parametrize("kw,opts", [
    (dict(), {"schedule": "fused", "precision": "fp64"}),
    (dict(), {"schedule": "fused", "precision": "fp64_arith"}),
    (dict(time_order=1), {"schedule": "fused"}),
    (dict(time_order=1, scheme="fully_discrete"), {"schedule": "fused"}),
])
def test_fused_schedule_needs_fp32_two_stage_semidiscrete(fdm, kw, opts):
    with pytest.raises(fdm.FdmError) as e:
        fdm.fdm_transport_init(fdm.desc(16, 16, **kw), options=opts)
    assert e.value.status == fdm.FDM_ERR_INVALID_ARG
    assert "fused" in fdm.fdm_last_error(None)


def test_missing_library_fails_loudly(fdm, monkeypatch, tmp_path):
    """No fallback path: without libfdm.so the binding raises."""
    monkeypatch.setattr(fdm, "_lib", None)
    with pytest.raises(RuntimeError, match="not found"):
        fdm.load_library(str(tmp_path / "libfdm.so"))


def test_noalloc_step_rejects_on_host(fdm):
    """The allocation-free step validates before any HIP call: a grid above
    its maximum, a bad descriptor, NULL or aliased arrays, a step above the
    stability bound."""
    import ctypes
    lib = fdm.load_library()
    p, q = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    n = fdm.NOALLOC_MAX_NODES
    cases = [
        (fdm.desc(n + 1, 1), p, q, fdm.FDM_ERR_INVALID_ARG, "maximum"),
        (fdm.desc(2049, 2048), p, q, fdm.FDM_ERR_INVALID_ARG, "maximum"),
        (fdm.desc(0, 16), p, q, fdm.FDM_ERR_INVALID_ARG, "nx and ny"),
        (fdm.desc(16, 16), None, q, fdm.FDM_ERR_INVALID_ARG, "NULL"),
        (fdm.desc(16, 16), p, p, fdm.FDM_ERR_INVALID_ARG, "alias"),
        (fdm.desc(16, 16, cfl=0.6), p, q, fdm.FDM_ERR_CFL, "2-D Courant"),
        (fdm.desc(16, 16, cfl=0.3, time_order=1), p, q, fdm.FDM_ERR_CFL, "forward-Euler"),
    ]
    for d, a, b, st, msg in cases:
        assert lib.fdm_transport_step_noalloc(ctypes.byref(d), a, b, 1, None) == st, msg
        assert msg in fdm.fdm_last_error(None)
    assert lib.fdm_transport_step_noalloc(None, p, q, 1, None) == fdm.FDM_ERR_INVALID_ARG
    assert lib.fdm_transport_step_noalloc(ctypes.byref(fdm.desc(16, 16)), p, q, -1, None) == fdm.FDM_ERR_INVALID_ARG
    # zero steps: validated, then nothing to do (no HIP call)
    assert lib.fdm_transport_step_noalloc(ctypes.byref(fdm.desc(n, 1)), p, q, 0, None) == fdm.FDM_OK
