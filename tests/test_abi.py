"""The C-ABI library loads, exports every declared entry point, and rejects
invalid arguments on the host before touching HIP (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2606_13259_amd import das
    if not os.path.exists(das.LIB_PATH):
        from paper_2606_13259_amd import build
        build.build()
    return das, das.lib()


def test_header_symbols_are_exported():
    das, L = _lib()
    hdr = open(os.path.join(ROOT, "include", "das.h")).read()
    names = sorted(set(re.findall(r"^(?:das_status|const char\s*\*|int32_t)\s+(das_\w+)\s*\(", hdr, re.M)))
    assert "das_forward" in names and "das_adjoint" in names and "das_plan_create" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in das.h but not exported"


def _cfg(**over):
    das, L = _lib()
    cfg, keep = das.make_config(synth.cfg1())
    for k, v in over.items():
        setattr(cfg, k, v)
    return das, L, cfg, keep


@pytest.mark.parametrize("field,value", [
    ("num_samples", 1), ("num_elements", 0), ("num_tx", 0), ("max_batch", 0),
    ("sound_speed", 0.0), ("sound_speed", float("nan")), ("fs", -1.0), ("apod", 7),
    ("storage", 4), ("storage", -1), ("algo", 9),
])
def test_plan_create_rejects_bad_config(field, value):
    das, L, cfg, keep = _cfg(**{field: value})
    h = ctypes.c_void_p()
    st = L.das_plan_create(ctypes.byref(h), ctypes.byref(cfg), 0)
    assert st == das.DAS_ERR_INVALID_ARG
    assert not h.value
    assert len(L.das_last_error()) > 0


def test_plan_create_rejects_bad_grid_and_tx():
    das, L, cfg, keep = _cfg()
    cfg.grid.dims[1] = 0
    h = ctypes.c_void_p()
    assert L.das_plan_create(ctypes.byref(h), ctypes.byref(cfg), 0) == das.DAS_ERR_INVALID_ARG
    das, L, cfg, keep = _cfg()
    cfg.grid.spacing[2] = -1e-4
    assert L.das_plan_create(ctypes.byref(h), ctypes.byref(cfg), 0) == das.DAS_ERR_INVALID_ARG
    das, L, cfg, keep = _cfg()
    keep[2][0].vec[2] = 2.0                   # plane-wave direction not unit
    assert L.das_plan_create(ctypes.byref(h), ctypes.byref(cfg), 0) == das.DAS_ERR_INVALID_ARG
    das, L, cfg, keep = _cfg()
    keep[2][0].kind = 5
    assert L.das_plan_create(ctypes.byref(h), ctypes.byref(cfg), 0) == das.DAS_ERR_INVALID_ARG
    das, L, cfg, keep = _cfg(apod=1, f_number=0.0)
    assert L.das_plan_create(ctypes.byref(h), ctypes.byref(cfg), 0) == das.DAS_ERR_INVALID_ARG
    assert L.das_plan_create(None, ctypes.byref(cfg), 0) == das.DAS_ERR_INVALID_ARG
    assert L.das_plan_create(ctypes.byref(h), None, 0) == das.DAS_ERR_INVALID_ARG


def test_null_plan_and_pointers_are_rejected():
    das, L = _lib()
    P = ctypes.c_void_p
    assert L.das_forward(None, P(1), 1, P(1), None) == das.DAS_ERR_INVALID_ARG
    assert L.das_prepare(None, P(1), 0, 1, 1, P(1), None) == das.DAS_ERR_INVALID_ARG
    assert L.das_adjoint(None, P(1), 1, P(1), None) == das.DAS_ERR_INVALID_ARG
    assert L.das_grad_sound_speed(None, P(1), P(1), 1, P(1), None) == das.DAS_ERR_INVALID_ARG
    assert L.das_plan_set_sound_speed(None, 1500.0) == das.DAS_ERR_INVALID_ARG
    assert L.das_autotune(None, 1, None) == das.DAS_ERR_INVALID_ARG
    assert L.das_debug_delays(None, 0, 0, 1, 0, 1, P(1), None) == das.DAS_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert L.das_workspace_bytes(None, 1, ctypes.byref(n)) == das.DAS_ERR_INVALID_ARG
    assert L.das_forward_batched(0, None, None, None, None, None) == das.DAS_ERR_INVALID_ARG
    assert L.das_plan_destroy(None) == das.DAS_OK
    assert L.das_status_string(das.DAS_ERR_HIP) == b"DAS_ERR_HIP"
    dims = (ctypes.c_int32 * 3)()
    for i in range(L.das_num_tile_shapes()):
        assert L.das_tile_shape(i, dims) == das.DAS_OK
        assert dims[0] * dims[1] * dims[2] == 256
    assert L.das_tile_shape(99, dims) == das.DAS_ERR_INVALID_ARG


def test_clutter_filter_argument_checks():
    """The clutter filter validates sizes, component ranges and pointers on
    the host (no pointer is dereferenced before the checks pass)."""
    das, L = _lib()
    n = ctypes.c_size_t()
    assert L.das_clutter_workspace_bytes(0, ctypes.byref(n)) == das.DAS_ERR_INVALID_ARG
    assert L.das_clutter_workspace_bytes(513, ctypes.byref(n)) == das.DAS_ERR_INVALID_ARG
    assert L.das_clutter_workspace_bytes(256, None) == das.DAS_ERR_INVALID_ARG
    assert L.das_clutter_workspace_bytes(256, ctypes.byref(n)) == das.DAS_OK
    assert n.value >= 2 * 256 * 256 * 8
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails its checks
    cases = [
        ((None, 64, 100, 3, 64), das.DAS_ERR_INVALID_ARG),     # x NULL
        ((fake, 0, 100, 0, 1), das.DAS_ERR_INVALID_ARG),       # T = 0
        ((fake, 64, 0, 3, 64), das.DAS_ERR_INVALID_ARG),       # N = 0
        ((fake, 64, 100, 5, 5), das.DAS_ERR_INVALID_ARG),      # empty band
        ((fake, 64, 100, 3, 65), das.DAS_ERR_INVALID_ARG),     # k_hi > T
        ((fake, 64, 100, -1, 10), das.DAS_ERR_INVALID_ARG),    # k_lo < 0
        ((fake, 256, 100, 100, 200), das.DAS_ERR_UNSUPPORTED),  # 100 kept, 156 removed: > 64
    ]
    for (x, T, N, lo, hi), want in cases:
        st = L.das_clutter_filter(x, T, N, lo, hi, fake, fake, None, fake, None)
        assert st == want, (T, N, lo, hi, st)
