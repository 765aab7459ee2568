"""Thin Python binding of the vorohip C ABI (include/vorohip.h).

Argument marshalling only: every step of the cell computation runs in the HIP
library.  Functions keep the C names.  PyTorch provides device memory and the
stream; results are copied out with vc_result_copy.  If the library has not
been built the import fails loudly -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VOROHIP_PHASE_CLOCKS=1 loads the build with the grouped cell kernel's phase
# profile (python -m paper_2209_11606_amd.build --phase-clocks); VOROHIP_LIB
# names another build of the library to load (A/B measurements)
LIB_PATH = os.environ.get("VOROHIP_LIB") or os.path.join(
    _HERE, "libvorohip_phase.so" if os.environ.get("VOROHIP_PHASE_CLOCKS") == "1" else "libvorohip.so")

VC_OK, VC_E_ARG, VC_E_RANGE, VC_E_DUPLICATE, VC_E_NOMEM, VC_E_HIP, VC_E_CAPACITY, VC_E_STATE = 0, -1, -2, -3, -4, -5, -6, -7
VC_FORCE_RECHECK, VC_FORCE_EXACT = 1, 2
VC_CELL_OK, VC_CELL_SPILLED, VC_CELL_CAPACITY, VC_CELL_DUPLICATE, VC_CELL_SKIPPED, VC_CELL_EMPTY = 0, 1, 2, 3, 4, 5
VC_CELL_FO_OVERFLOW = 64  # flag bit on a complete cell with a face of 32 or more edges
VC_CELL_RANGE = 6  # vc_tessellate_noalloc: a coordinate outside the box
VC_FP64, VC_F32_FILTER = 0, 1
VC_VOLUME, VC_CENTROID, VC_COUNTS, VC_FACE_ORDERS, VC_NEIGHBORS, VC_NEIGHBOR_COUNT, VC_DIAG = 1, 2, 4, 8, 16, 32, 64
VC_ALL = 127
VC_PERIMETER = 128
VC_WEINBERG = 256
(VC_F_VOLUME, VC_F_CENTROID, VC_F_NV, VC_F_NE, VC_F_NF, VC_F_FACE_ORDERS, VC_F_NBR_OFFSETS, VC_F_NBR_IDS,
 VC_F_NBR_SHIFTS, VC_F_STATUS, VC_F_DIAG, VC_F_PERIMETER, VC_F_WB_OFFSETS, VC_F_WB_CODES, VC_F_WB_SYM,
 VC_F_WB_CHIRAL) = range(16)
VC_FO_LEN = 32
VC_DIAG_LEN = 32
DIAG_NAMES = ["candidates", "tests", "cuts", "new_vertices", "exact", "recheck", "spilled", "blocks", "fallback",
              "shells", "loaded", "recomputed"]
PHASE_NAMES = ["new", "gather", "batch", "test", "cut", "stats", "test_iterations", "control"]
_FIELD_DTYPE = {VC_F_VOLUME: np.float64, VC_F_CENTROID: np.float64, VC_F_NV: np.int32, VC_F_NE: np.int32,
                VC_F_NF: np.int32, VC_F_FACE_ORDERS: np.uint8, VC_F_NBR_OFFSETS: np.int64, VC_F_NBR_IDS: np.int32,
                VC_F_NBR_SHIFTS: np.uint8, VC_F_STATUS: np.uint8, VC_F_DIAG: np.uint64, VC_F_PERIMETER: np.float64,
                VC_F_WB_OFFSETS: np.int64, VC_F_WB_CODES: np.uint8, VC_F_WB_SYM: np.int32, VC_F_WB_CHIRAL: np.uint8}


class vc_options(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("periodic", ctypes.c_int * 3), ("n_opt", ctypes.c_double), ("grid", ctypes.c_int * 3),
                ("precision", ctypes.c_int), ("slots", ctypes.c_int), ("waves", ctypes.c_int),
                ("chunk", ctypes.c_int), ("cells_per_wave", ctypes.c_int), ("clip", ctypes.c_double),
                ("capacity", ctypes.c_int), ("force", ctypes.c_int)]


class vc_tuning(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int), ("waves", ctypes.c_int), ("chunk", ctypes.c_int),
                ("cells_per_wave", ctypes.c_int), ("ms", ctypes.c_float), ("capacity", ctypes.c_int)]


class VcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vorohip error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"vorohip: {LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, U32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32
    sig = {
        "vc_options_init": (I32, [P, I32, P, P, P]),
        "vc_container_create": (I32, [P, I64, P, P, P]),
        "vc_container_rebin": (I32, [P, P, P]),
        "vc_container_set_radii": (I32, [P, P, P]),
        "vc_batch_set_radii": (I32, [P, P, P]),
        "vc_result_create": (I32, [P, U32, P]),
        "vc_grid_size": (I32, [P, I64, P]),
        "vc_container_blocks": (I32, [P, P, P, P]),
        "vc_compute": (I32, [P, P, P]),
        "vc_compute_subset": (I32, [P, P, P, I64, P]),
        "vc_result_get": (I32, [P, I32, P, P]),
        "vc_result_copy": (I32, [P, I32, P, I64]),
        "vc_result_destroy": (None, [P]),
        "vc_container_destroy": (None, [P]),
        "vc_batch_create": (I32, [P, P, I64, P, P, P]),
        "vc_batch_rebin": (I32, [P, P, P]),
        "vc_batch_result_create": (I32, [P, U32, P]),
        "vc_batch_compute": (I32, [P, P, I32, P]),
        "vc_batch_tune": (I32, [P, P, P, P]),
        "vc_batch_tune_members": (I32, [P, P, P, I64, P, P]),
        "vc_batch_destroy": (None, [P]),
        "vc_result_kernel_ms": (I32, [P, P]),
        "vc_last_error": (ctypes.c_char_p, []),
        "vc_version": (ctypes.c_char_p, []),
        "vc_device_fma_rate": (I32, [I32, I32, P, P]),
        "vc_tessellate_noalloc": (I32, [P, I64, P, P, P, P, P, P, P, P, P]),
        "vc_tessellate_slabs": (I32, [P, I64, P, U32, I32, I32, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = ["vc_options_init", "vc_container_create", "vc_container_rebin", "vc_container_set_radii",
            "vc_batch_set_radii", "vc_grid_size", "vc_container_blocks",
            "vc_result_create", "vc_compute", "vc_compute_subset",
            "vc_result_get", "vc_result_copy", "vc_result_kernel_ms", "vc_result_destroy", "vc_container_destroy", "vc_batch_create",
            "vc_batch_rebin", "vc_batch_result_create", "vc_batch_compute", "vc_batch_tune", "vc_batch_tune_members",
            "vc_batch_destroy",
            "vc_last_error", "vc_version", "vc_device_fma_rate", "vc_tessellate_noalloc", "vc_tessellate_slabs"]


def lib():
    return _lib


def vc_last_error():
    return _lib.vc_last_error().decode()


def vc_version():
    return _lib.vc_version().decode()


def _check(code):
    if code != VC_OK:
        raise VcError(code, vc_last_error())


def vc_device_fma_rate(precision=VC_FP64, reps=3, stream=None):
    """Measured vector FMA rate of the current device in TFLOP/s (an FMA
    counts as 2): FP64 for VC_FP64, unpacked FP32 for VC_F32_FILTER."""
    out = ctypes.c_double(0.0)
    _check(_lib.vc_device_fma_rate(precision, reps, _stream_ptr(stream), ctypes.byref(out)))
    return out.value


def vc_options_init(dim, lo, hi, periodic, **kw):
    o = vc_options()
    lo_a = (ctypes.c_double * 3)(*[float(v) for v in lo])
    hi_a = (ctypes.c_double * 3)(*[float(v) for v in hi])
    pe_a = (ctypes.c_int * 3)(*[int(bool(v)) for v in periodic])
    _check(_lib.vc_options_init(ctypes.byref(o), dim, lo_a, hi_a, pe_a))
    names = {f for f, _ in vc_options._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"vc_options has no field {k!r}")
        if k == "grid":
            for d, g in enumerate(v):
                o.grid[d] = int(g)
        else:
            setattr(o, k, v)
    return o


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def vc_container_create(xyz, opts, stream=None):
    """xyz: a contiguous float64 torch tensor (n x dim) on the GPU, or a numpy
    array on the host.  Returns the container handle (c_void_p)."""
    n = xyz.shape[0]
    ptr = xyz.data_ptr() if hasattr(xyz, "data_ptr") else xyz.ctypes.data
    h = ctypes.c_void_p()
    _check(_lib.vc_container_create(ctypes.c_void_p(ptr), n, ctypes.byref(opts), ctypes.c_void_p(_stream_ptr(stream)),
                                    ctypes.byref(h)))
    return h


def vc_tessellate_slabs(xyz, opts, mask, nslab, halo, stream=None):
    """The chunked form for one large 3D set (positions as for
    vc_container_create): returns a new result handle of n cells by input
    index, computed in nslab chunks of layers along z with `halo` more
    layers on each side."""
    n = xyz.shape[0]
    if not hasattr(xyz, "data_ptr"):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    ptr = xyz.data_ptr() if hasattr(xyz, "data_ptr") else xyz.ctypes.data
    h = ctypes.c_void_p()
    _check(_lib.vc_tessellate_slabs(ctypes.c_void_p(ptr), n, ctypes.byref(opts), mask, int(nslab), int(halo),
                                    ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h)))
    return h


def vc_container_rebin(c, xyz, stream=None):
    ptr = xyz.data_ptr() if hasattr(xyz, "data_ptr") else xyz.ctypes.data
    _check(_lib.vc_container_rebin(c, ctypes.c_void_p(ptr), ctypes.c_void_p(_stream_ptr(stream))))


def _radii_ptr(radii):
    if radii is None:
        return None, None
    if hasattr(radii, "data_ptr"):
        import torch
        if radii.dtype != torch.float64 or not radii.is_contiguous():
            raise ValueError("radii must be a contiguous float64 tensor")
        return radii, radii.data_ptr()
    a = np.ascontiguousarray(radii, dtype=np.float64)
    return a, a.ctypes.data


def vc_container_set_radii(c, radii, stream=None):
    """radii: n float64 values by input index (numpy array, or torch tensor on
    the host or the GPU), or None for the plain Voronoi tessellation."""
    keep, ptr = _radii_ptr(radii)
    _check(_lib.vc_container_set_radii(c, ctypes.c_void_p(ptr), ctypes.c_void_p(_stream_ptr(stream))))
    del keep


def vc_batch_set_radii(b, radii, stream=None):
    keep, ptr = _radii_ptr(radii)
    _check(_lib.vc_batch_set_radii(b, ctypes.c_void_p(ptr), ctypes.c_void_p(_stream_ptr(stream))))
    del keep


def vc_grid_size(opts, n):
    g = (ctypes.c_int * 3)()
    _check(_lib.vc_grid_size(ctypes.byref(opts), int(n), g))
    return list(g)


def vc_container_blocks(c, n):
    nb = ctypes.c_int64()
    _check(_lib.vc_container_blocks(c, None, None, ctypes.byref(nb)))
    start = np.empty(nb.value + 1, np.int32)
    ids = np.empty(n, np.int32)
    _check(_lib.vc_container_blocks(c, start.ctypes.data, ids.ctypes.data, None))
    return start, ids


def vc_result_create(c, mask):
    h = ctypes.c_void_p()
    _check(_lib.vc_result_create(c, mask, ctypes.byref(h)))
    return h


def vc_compute(c, r, stream=None):
    _check(_lib.vc_compute(c, r, ctypes.c_void_p(_stream_ptr(stream))))


def vc_compute_subset(c, r, ids, stream=None):
    """ids: int64 input indices, a numpy array (host) or a torch tensor
    (host or device)."""
    if hasattr(ids, "data_ptr"):
        if ids.dtype != __import__("torch").int64 or not ids.is_contiguous():
            raise ValueError("vc_compute_subset: ids must be a contiguous int64 tensor")
        ptr, m = ids.data_ptr(), ids.numel()
    else:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        ptr, m = ids.ctypes.data, ids.size
    _check(_lib.vc_compute_subset(c, r, ctypes.c_void_p(ptr), int(m), ctypes.c_void_p(_stream_ptr(stream))))


def vc_result_get(r, field):
    p = ctypes.c_void_p()
    k = ctypes.c_int64()
    _check(_lib.vc_result_get(r, field, ctypes.byref(p), ctypes.byref(k)))
    return p.value, k.value


def vc_result_copy(r, field):
    _, k = vc_result_get(r, field)
    out = np.empty(k, dtype=_FIELD_DTYPE[field])
    _check(_lib.vc_result_copy(r, field, out.ctypes.data, out.nbytes))
    return out


def vc_result_kernel_ms(r):
    ms = ctypes.c_float()
    _check(_lib.vc_result_kernel_ms(r, ctypes.byref(ms)))
    return ms.value


def vc_result_destroy(r):
    _lib.vc_result_destroy(r)


def vc_container_destroy(c):
    _lib.vc_container_destroy(c)


def vc_batch_create(xyz, offsets, opts_list, stream=None):
    """xyz: all positions back to back (torch tensor on the GPU or numpy);
    offsets: n_tess + 1 particle offsets; opts_list: one vc_options each."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    arr = (vc_options * len(opts_list))(*opts_list)
    ptr = xyz.data_ptr() if hasattr(xyz, "data_ptr") else xyz.ctypes.data
    h = ctypes.c_void_p()
    _check(_lib.vc_batch_create(ctypes.c_void_p(ptr), off.ctypes.data, len(opts_list), arr,
                                ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h)))
    return h


def vc_batch_rebin(b, xyz, stream=None):
    ptr = xyz.data_ptr() if hasattr(xyz, "data_ptr") else xyz.ctypes.data
    _check(_lib.vc_batch_rebin(b, ctypes.c_void_p(ptr), ctypes.c_void_p(_stream_ptr(stream))))


def vc_batch_result_create(b, mask):
    h = ctypes.c_void_p()
    _check(_lib.vc_batch_result_create(b, mask, ctypes.byref(h)))
    return h


def vc_batch_compute(b, r, graph=False, stream=None):
    _check(_lib.vc_batch_compute(b, r, int(bool(graph)), ctypes.c_void_p(_stream_ptr(stream))))


def _tuning(t):
    return dict(slots=t.slots, waves=t.waves, chunk=t.chunk, cells_per_wave=t.cells_per_wave, ms=t.ms,
                capacity=t.capacity)


def vc_batch_tune(b, r, stream=None):
    t = vc_tuning()
    _check(_lib.vc_batch_tune(b, r, ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(t)))
    return _tuning(t)


def vc_batch_tune_members(b, r, members, stream=None):
    """Tune on the cells of the listed tessellations only (a class of input)."""
    m = np.ascontiguousarray(np.asarray(members, dtype=np.int64))
    t = vc_tuning()
    _check(_lib.vc_batch_tune_members(b, r, m.ctypes.data, len(m), ctypes.c_void_p(_stream_ptr(stream)),
                                      ctypes.byref(t)))
    return _tuning(t)


def vc_tessellate_noalloc(xyz, opts, out, stream=None):
    """The allocation-free tessellation: xyz a contiguous float64 device
    tensor (n x dim); out a dict of preallocated device tensors by field name
    (nf: int32[n] and status: uint8[n] required; vol: float64[n],
    cen: float64[n, 3], nv, ne: int32[n], fo: uint8[n, 32] optional)."""
    def ptr(key):
        t = out.get(key)
        return None if t is None else ctypes.c_void_p(t.data_ptr())
    _check(_lib.vc_tessellate_noalloc(ctypes.c_void_p(xyz.data_ptr()), int(xyz.shape[0]), ctypes.byref(opts),
                                      ptr("vol"), ptr("cen"), ptr("nv"), ptr("ne"), ptr("nf"), ptr("fo"),
                                      ptr("status"), ctypes.c_void_p(_stream_ptr(stream))))


def vc_batch_destroy(b):
    _lib.vc_batch_destroy(b)


def fetch(r, mask, n, dim=3):
    """Copy every field of a result that the mask produced into numpy arrays."""
    out = {"status": vc_result_copy(r, VC_F_STATUS), "nf": vc_result_copy(r, VC_F_NF)}
    if mask & VC_VOLUME:
        out["vol"] = vc_result_copy(r, VC_F_VOLUME)
    if mask & VC_CENTROID:
        out["cen"] = vc_result_copy(r, VC_F_CENTROID).reshape(n, 3)[:, :dim]
    if mask & VC_PERIMETER:
        out["perim"] = vc_result_copy(r, VC_F_PERIMETER)
    if mask & VC_COUNTS:
        out["nv"] = vc_result_copy(r, VC_F_NV)
        out["ne"] = vc_result_copy(r, VC_F_NE)
    if mask & VC_FACE_ORDERS:
        out["fo"] = vc_result_copy(r, VC_F_FACE_ORDERS).reshape(n, VC_FO_LEN).astype(np.int32)
    if mask & VC_NEIGHBORS:
        off = vc_result_copy(r, VC_F_NBR_OFFSETS)
        ids = vc_result_copy(r, VC_F_NBR_IDS)
        sh = vc_result_copy(r, VC_F_NBR_SHIFTS)
        out["nbr_off"], out["nbr_ids"], out["nbr_sh"] = off, ids, sh
    if mask & VC_WEINBERG:
        out["wb_off"] = vc_result_copy(r, VC_F_WB_OFFSETS)
        out["wb_codes"] = vc_result_copy(r, VC_F_WB_CODES)
        out["wb_sym"] = vc_result_copy(r, VC_F_WB_SYM)
        out["wb_chiral"] = vc_result_copy(r, VC_F_WB_CHIRAL)
    d = vc_result_copy(r, VC_F_DIAG)
    out["diag"] = dict(zip(DIAG_NAMES, d[:len(DIAG_NAMES)].tolist()))
    return out


def phase_profile(r):
    """Per-phase shader-clock cycles and run counts of the grouped cell
    kernel (only a library built with --phase-clocks writes them)."""
    d = vc_result_copy(r, VC_F_DIAG)
    return {"cycles": dict(zip(PHASE_NAMES, d[16:24].tolist())), "runs": dict(zip(PHASE_NAMES, d[24:32].tolist()))}


def weinberg_codes(res):
    """Per-cell Weinberg codes (uint8 arrays) from the CSR fields of fetch()."""
    off, codes = res["wb_off"], res["wb_codes"]
    return [codes[off[i]:off[i + 1]] for i in range(len(off) - 1)]


def neighbor_lists(res):
    """Per-cell sorted (label, image) arrays from the CSR fields of fetch()."""
    off, ids, sh = res["nbr_off"], res["nbr_ids"], res["nbr_sh"]
    return [np.stack([ids[off[i]:off[i + 1]].astype(np.int64), sh[off[i]:off[i + 1]].astype(np.int64)], 1)
            for i in range(len(off) - 1)]


def tessellate(xyz, lo, hi, periodic, mask=VC_ALL, stream=None, radii=None, **opts):
    """Create a container from device positions, compute all cells, fetch the
    results to the host, and free everything.  Convenience for tests.
    radii (n values) makes it the radical tessellation."""
    dim = xyz.shape[1]
    o = vc_options_init(dim, lo, hi, periodic, **opts)
    c = vc_container_create(xyz, o, stream)
    try:
        if radii is not None:
            vc_container_set_radii(c, radii, stream)
        r = vc_result_create(c, mask)
        try:
            vc_compute(c, r, stream)
            return fetch(r, mask, xyz.shape[0], dim)
        finally:
            vc_result_destroy(r)
    finally:
        vc_container_destroy(c)
