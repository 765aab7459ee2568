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
    assert L.vc_result_get(None, 0, None, None) == v.VC_E_ARG
    assert L.vc_result_kernel_ms(None, None) == v.VC_E_ARG
    assert v.vc_version().startswith("vorohip")


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib.util
    from paper_2209_11606_amd import vorohip
    spec = importlib.util.spec_from_file_location("vorohip_copy", vorohip.__file__)
    mod = importlib.util.module_from_spec(spec)
    monkeypatch.setattr(os.path, "exists", lambda p: False if p.endswith("libvorohip.so") else True)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)
