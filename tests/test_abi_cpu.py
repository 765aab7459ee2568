"""The C ABI library loads and exports every symbol the header declares, and
argument validation answers without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2209_11606_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2209_11606_amd import vorohip
    return vorohip


def test_exports_every_declared_symbol():
    v = _lib()
    header = open(os.path.join(ROOT, "include", "vorohip.h")).read()
    declared = set(re.findall(r"^\s*(?:vc_status|void|const char \*)\s*(vc_\w+)\s*\(", header, re.M))
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(v.lib(), name), name
    assert declared == set(v.EXPORTED)


def test_argument_validation_without_gpu():
    v = _lib()
    L = v.lib()
    o = v.vc_options()
    lo = (ctypes.c_double * 3)(0, 0, 0)
    hi = (ctypes.c_double * 3)(1, 1, 1)
    pe = (ctypes.c_int * 3)(0, 0, 0)
    assert L.vc_options_init(None, 3, lo, hi, pe) == v.VC_E_ARG
    assert L.vc_options_init(ctypes.byref(o), 4, lo, hi, pe) == v.VC_E_ARG
    assert "dim" in v.vc_last_error()
    assert L.vc_options_init(ctypes.byref(o), 3, lo, hi, pe) == v.VC_OK
    assert o.n_opt == 5.0 and o.precision == v.VC_FP64
    h = ctypes.c_void_p()
    x = np.zeros((4, 3))
    # n < 1, null positions, null out: rejected before any device call
    assert L.vc_container_create(x.ctypes.data, 0, ctypes.byref(o), None, ctypes.byref(h)) == v.VC_E_ARG
    assert L.vc_container_create(None, 4, ctypes.byref(o), None, ctypes.byref(h)) == v.VC_E_ARG
    assert L.vc_container_create(x.ctypes.data, 4, ctypes.byref(o), None, None) == v.VC_E_ARG
    bad = v.vc_options_init(3, [0, 0, 0], [1, 1, 1], [0, 0, 0])
    bad.hi[1] = 0.0
    assert L.vc_container_create(x.ctypes.data, 4, ctypes.byref(bad), None, ctypes.byref(h)) == v.VC_E_ARG
    bad = v.vc_options_init(3, [0, 0, 0], [1, 1, 1], [0, 0, 0])
    bad.precision = 7
    assert L.vc_container_create(x.ctypes.data, 4, ctypes.byref(bad), None, ctypes.byref(h)) == v.VC_E_ARG
    bad = v.vc_options_init(3, [0, 0, 0], [1, 1, 1], [0, 0, 0])
    bad.slots = 3
    assert L.vc_container_create(x.ctypes.data, 4, ctypes.byref(bad), None, ctypes.byref(h)) == v.VC_E_ARG
    assert L.vc_result_create(None, v.VC_ALL, ctypes.byref(h)) == v.VC_E_ARG
    assert L.vc_compute(None, None, None) == v.VC_E_ARG
    assert L.vc_compute_subset(None, None, None, 0, None) == v.VC_E_ARG
    bad = v.vc_options_init(3, [0, 0, 0], [1, 1, 1], [0, 0, 0])
    bad.clip = -1.0
    assert L.vc_container_create(x.ctypes.data, 4, ctypes.byref(bad), None, ctypes.byref(h)) == v.VC_E_ARG
    assert "clip" in v.vc_last_error()
    assert L.vc_result_get(None, 0, None, None) == v.VC_E_ARG
    assert L.vc_result_kernel_ms(None, None) == v.VC_E_ARG
    t = ctypes.c_double()
    assert L.vc_device_fma_rate(v.VC_FP64, 3, None, None) == v.VC_E_ARG
    assert L.vc_device_fma_rate(v.VC_FP64, 0, None, ctypes.byref(t)) == v.VC_E_ARG
    assert L.vc_device_fma_rate(5, 3, None, ctypes.byref(t)) == v.VC_E_ARG
    assert v.vc_version().startswith("vorohip")
    # the chunked form: dimension, chunk and halo counts, mask
    o2 = v.vc_options_init(2, [0, 0], [1, 1], [0, 0])
    S = L.vc_tessellate_slabs
    assert S(x.ctypes.data, 4, ctypes.byref(o2), v.VC_VOLUME, 2, 1, None, ctypes.byref(h)) == v.VC_E_ARG
    assert "3D" in v.vc_last_error()
    assert S(x.ctypes.data, 4, ctypes.byref(o), v.VC_VOLUME, 0, 1, None, ctypes.byref(h)) == v.VC_E_ARG
    assert S(x.ctypes.data, 4, ctypes.byref(o), v.VC_VOLUME, 2, 0, None, ctypes.byref(h)) == v.VC_E_ARG
    assert S(x.ctypes.data, 0, ctypes.byref(o), v.VC_VOLUME, 2, 1, None, ctypes.byref(h)) == v.VC_E_ARG
    assert S(None, 4, ctypes.byref(o), v.VC_VOLUME, 2, 1, None, ctypes.byref(h)) == v.VC_E_ARG
    assert S(x.ctypes.data, 4, ctypes.byref(o), v.VC_VOLUME, 2, 1, None, None) == v.VC_E_ARG
    for m in (v.VC_NEIGHBORS, v.VC_WEINBERG, v.VC_PERIMETER, 1 << 12):
        assert S(x.ctypes.data, 4, ctypes.byref(o), v.VC_VOLUME | m, 2, 1, None, ctypes.byref(h)) == v.VC_E_ARG
    assert "per-cell fields only" in v.vc_last_error()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib.util
    from paper_2209_11606_amd import vorohip
    spec = importlib.util.spec_from_file_location("vorohip_copy", vorohip.__file__)
    mod = importlib.util.module_from_spec(spec)
    monkeypatch.setattr(os.path, "exists", lambda p: False if p.endswith("libvorohip.so") else True)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_grid_rule_host():
    """The library's grid sizing (section 2.1.4, ceiling rule) on the host,
    against the plain formula."""
    import math
    v = _lib()
    for dim, n, side, nopt in [(3, 1000, 1.0, 5.0), (3, 1_000_000, 100.0, 5.0), (2, 10_000_000, 1.0, 5.0),
                               (3, 102_400_000, 1.0, 5.0), (3, 10, 1.0, 5.0), (2, 100_000, 1.0, 3.4),
                               (3, 100_000_000, 1.0, 4.6)]:
        o = v.vc_options_init(dim, [0.0] * dim, [side] * dim, [1] * dim, n_opt=nopt)
        g = v.vc_grid_size(o, n)
        lam = (n / (nopt * side ** dim)) ** (1.0 / dim)
        want = [max(1, math.ceil(lam * side))] * dim + [1] * (3 - dim)
        assert g == want, (dim, n, g, want)
    o = v.vc_options_init(3, [0, 0, 0], [2.0, 1.0, 0.5], [0, 0, 0], grid=[7, 3, 2])
    assert v.vc_grid_size(o, 12345) == [7, 3, 2]
    o = v.vc_options_init(3, [0, 0, 0], [4.0, 1.0, 0.5], [0, 0, 0])
    assert v.vc_grid_size(o, 2000) == [math.ceil((2000 / 10) ** (1 / 3) * s) for s in (4.0, 1.0, 0.5)]
