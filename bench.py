"""Benchmark: 3D Voronoi cells/s on one MI355X, FP32-filter vs FP64 plain.

Workload: 1,000,000 i.i.d. uniform particles in the periodic cube of side 100
(density 1), full statistics (volume, centroid, V/E/F, face orders, CSR
neighbour lists).  One step = the whole hot path on positions already resident
in HBM: binning (count, scan, scatter, in-block order), every cell, the
large-capacity spill pass and the neighbour compaction.

Variants: the plain form (one container, FP64 or FP32-filter side tests) and
the batched form (vc_batch: autotuned launch parameters, compute replayed
from a hipGraph).  `value` is the fastest variant.  --workload batch4096
measures the 4,096-tessellation set instead.

Prints one JSON line.  The roofline object covers the dominant kernel (the
cell kernel): its algorithmic FP64 flops per launch -- the oracle's operation
counts on a sample of the same workload, weighted (every candidate's distance
test 9, vertex side test 6, new vertex 12, fan tetrahedron 28), scaled to the
cells of one launch -- over its HIP-event duration, against the FP64 vector
peak.  Each entry of `variants` carries the same fraction for its own cell
kernel (roofline_frac), so the plain FP64 and the FP32-filter forms are
both placed against the peak.
The cpu_baseline object times the oracle on the host cores on a bounded
sample of the same workload (with the CPU model and core counts);
cpu_serial times it on one thread.  Each variant's `parity` compares that
variant's own outputs of the timed run with the oracle's cells of the
sample: volume and centroid errors (max, mean) and mismatch counts of the
counts, face orders, overflow flags and neighbour lists.
binning_roofline is the rebin alone (HIP events) against the HBM peak, with
56 algorithmic bytes per particle (what the library moves is reported beside
it); end_to_end is one pass from positions in pinned host memory to every
result field in host memory (PCIe included), reported beside `value`, never
as it.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COUNTERS = os.path.join(ROOT, "profiles", "cells_periodic1M_counters.md")
KERNEL_SOURCES = ["cell3d.hip", "cell3d_group.hip", "cell_common.h", "vc_internal.h"]
HBM_PEAK = 8.0e12  # B/s
# binning of one particle, algorithmic: its position read (24 B), its
# block-sorted record written (24 B of position and 4 B of id) and its block
# count (4 B): 56 B
BIN_BYTES_PER_PARTICLE = 56
# what the library's rebin moves per particle: device copy of the positions
# (24 B read + 24 B written), block count (24 B read, 8 B written),
# provisional slot (12 B read, 4 B written), rank by id and final scatter
# (24 B of position, 16 B of index, block and range, ~20 B of the block's ids
# read; 32 B written)
BIN_BYTES_IMPLEMENTATION = 188
FP64_VECTOR_PEAK = 78.6e12  # FLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FLOP_WEIGHTS = dict(candidates=9, vertex_tests=6, new_vertices=12, fan_triangles=28)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--cpu-sample", type=int, default=500_000,
                   help="oracle cells timed on the host (about 20 s of core time for the 1M set)")
    p.add_argument("--cpu-serial-sample", type=int, default=100_000, help="oracle cells timed on one thread")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--calibration-copy-mib", type=int, default=0,
                   help="first copy a device buffer of this size (reference for HBM byte counters)")
    p.add_argument("--variants", default="all", help="comma list of variants to run (default all)")
    p.add_argument("--phase-clocks", action="store_true",
                   help="load the library built with the grouped cell kernel's phase profile "
                        "(python -m paper_2209_11606_amd.build --phase-clocks) and report cycles per phase")
    p.add_argument("--slabs", type=int, default=None,
                   help="also time the chunked form with this many container-block chunks along z "
                        "(default: 8 for periodic102m, none otherwise)")
    p.add_argument("--halo", type=int, default=3, help="layers of blocks on each side of a chunk")
    p.add_argument("--workload", default="periodic1m",
                   choices=["periodic1m", "batch4096", "fcc10m", "periodic2d10m", "periodic102m",
                            "localized10m", "localized10m_unclipped", "localized100k_unclipped", "localized2d10m", "clustered10m",
                            "clustered2d100m", "polydisperse1m", "vorotop1m"],
                   help="periodic1m: the metric's configuration (default); the others measure the remaining sets")
    return p.parse_args()


def kernel_key(precision_name, tuned):
    """Which cell kernel a variant ran: cells per wave and slots per lane."""
    cpw = tuned.get("cells_per_wave", 1) if tuned else 1
    slots = tuned.get("slots", 2) if tuned else 2
    return f"{precision_name},cpw={cpw}" + (f",slots={slots}" if cpw == 1 else "")


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2209_11606_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def committed_counters(key):
    """The committed counter summary's entry for this kernel (traffic, VALU
    busy fraction, waiting fraction), or None when it has none or was taken
    on other kernel sources."""
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    i = text.find("```json")
    if i < 0:
        return None
    data = json.loads(text[i + 7:text.index("```", i + 7)])
    e = data.get("kernels", {}).get(key)
    if not e or data.get("source_sha256") != sources_sha256():
        return None
    return e


def committed_traffic(key):
    """HBM bytes per launch of the cell kernel, from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, each divided by what the
    counter reads for a device copy of known size).  None when the summary
    has no entry for this kernel or was taken on other kernel sources."""
    e = committed_counters(key)
    return e["traffic_bytes"] if e else None


def _timed(torch, stream, steps, step_fn):
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        step_fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def options(v, w, **kw):
    """vc_options of a workload: its box, and its grid and clip side if set."""
    extra = {}
    if w.get("grid"):
        extra["grid"] = w["grid"]
    if w.get("clip"):
        extra["clip"] = w["clip"]
    extra.update(kw)
    return v.vc_options_init(len(w["lo"]), w["lo"], w["hi"], w["periodic"], **extra)


def time_variant(v, torch, xt, w, precision, steps, warmup, mask, sample=None):
    """Plain form: one container; step = rebin + compute."""
    stream = torch.cuda.current_stream()
    o = options(v, w, precision=precision)
    c = v.vc_container_create(xt, o, stream)
    if w.get("radii") is not None:
        v.vc_container_set_radii(c, w["radii"], stream)
    r = v.vc_result_create(c, mask)
    kms = []

    def step():
        v.vc_container_rebin(c, xt, stream)
        v.vc_compute(c, r, stream)
        kms.append(v.vc_result_kernel_ms(r))
    try:
        for _ in range(warmup):
            step()
        kms.clear()
        ms = _timed(torch, stream, steps, step)
        out = _summary(v, r, ms, float(np.mean(kms)), sample)
    finally:
        v.vc_result_destroy(r)
        v.vc_container_destroy(c)
    return out


def time_chunked(v, torch, xt, w, precision, steps, warmup, mask, nslab, halo, sample=None, launch=None):
    """Chunked form (vc_tessellate_slabs): step = every cell of the set, in
    nslab container-block chunks along z with `halo` layers on each side,
    each chunk binned on its own with the set's grid."""
    stream = torch.cuda.current_stream()
    kw = dict(precision=precision)
    if launch:
        kw.update({k: launch[k] for k in ("cells_per_wave", "slots", "waves", "chunk", "capacity")})
    o = options(v, w, **kw)
    held = []

    def step():
        while held:
            v.vc_result_destroy(held.pop())
        held.append(v.vc_tessellate_slabs(xt, o, mask, nslab, halo, stream))
    try:
        for _ in range(warmup):
            step()
        ms = _timed(torch, stream, steps, step)
        out = _summary(v, held[0], ms, v.vc_result_kernel_ms(held[0]), sample)
        out["tuned"] = dict(launch or {}, chunks=nslab, halo=halo)
    finally:
        while held:
            v.vc_result_destroy(held.pop())
    return out


def time_binning(v, torch, xt, w, steps):
    """Binning alone: vc_container_rebin on HBM-resident positions (copy,
    count, scan, scatter, in-block order, range check), HIP events."""
    stream = torch.cuda.current_stream()
    o = options(v, w)
    c = v.vc_container_create(xt, o, stream)
    try:
        ms = _timed(torch, stream, steps, lambda: v.vc_container_rebin(c, xt, stream))
    finally:
        v.vc_container_destroy(c)
    n = xt.shape[0]
    achieved = n * BIN_BYTES_PER_PARTICLE / (ms / 1e3)
    return dict(ms=ms, bytes_per_particle=BIN_BYTES_PER_PARTICLE, achieved_GBps=achieved / 1e9,
                peak_GBps=HBM_PEAK / 1e9, frac=achieved / HBM_PEAK, bound="hbm",
                implementation_bytes_per_particle=BIN_BYTES_IMPLEMENTATION,
                implementation_GBps=n * BIN_BYTES_IMPLEMENTATION / (ms / 1e3) / 1e9)


def end_to_end(v, torch, xyz, w, precision, mask, reps=3, launch=None):
    """Positions in pinned host memory to results in host memory: rebin from
    the host pointer (PCIe copy + binning), compute, copy every produced
    field back.  The container and result exist beforehand.  launch: the
    tuner's choice for this set (cells per wave, slots, waves, chunk), else
    two cells per wave in 3D."""
    import time as _t
    stream = torch.cuda.current_stream()
    host = torch.from_numpy(xyz).pin_memory()
    n, dim = xyz.shape
    if launch:
        form = {k: int(launch[k]) for k in ("cells_per_wave", "slots", "waves", "chunk", "capacity")}
    else:
        form = dict(cells_per_wave=2 if dim == 3 else 0)
    o = options(v, w, precision=precision, **form)
    c = v.vc_container_create(host, o, stream)
    if w.get("radii") is not None:
        v.vc_container_set_radii(c, w["radii"], stream)
    r = v.vc_result_create(c, mask)
    try:
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t = _t.perf_counter()
            v.vc_container_rebin(c, host, stream)
            v.vc_compute(c, r, stream)
            v.fetch(r, mask, n, dim)
            torch.cuda.synchronize()
            ms = (_t.perf_counter() - t) * 1e3
            best = ms if best is None else min(best, ms)
    finally:
        v.vc_result_destroy(r)
        v.vc_container_destroy(c)
    return dict(ms=best, cells_per_s=n / (best / 1e3),
                includes="H2D of positions from pinned memory, binning, cells, compaction, D2H of every field")


def time_batched(v, torch, xt, offsets, opts, steps, warmup, mask, radii=None, sample=None, classes=None):
    """Batched form: autotuned launch parameters, compute replayed from a
    hipGraph; step = rebin + graph launch.  The cell-kernel duration for the
    roofline comes from eager launches with the same parameters."""
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    b = v.vc_batch_create(xt, offsets, opts, stream)
    if radii is not None:
        v.vc_batch_set_radii(b, radii, stream)
    r = v.vc_batch_result_create(b, mask)
    try:
        per_class = None
        if classes:
            # the launch form each input class would take on its own (the
            # batch runs in one launch with the whole-batch choice below)
            per_class = {k: v.vc_batch_tune_members(b, r, ms, stream) for k, ms in sorted(classes.items())}
        tuned = v.vc_batch_tune(b, r, stream)
        kms = []
        for _ in range(max(1, warmup)):
            v.vc_batch_compute(b, r, False, stream)
            kms.append(v.vc_result_kernel_ms(r))

        def step():
            v.vc_batch_rebin(b, xt, stream)
            v.vc_batch_compute(b, r, True, stream)
        for _ in range(warmup):
            step()
        ms = _timed(torch, stream, steps, step)
        for _ in range(3):
            v.vc_batch_compute(b, r, False, stream)
            kms.append(v.vc_result_kernel_ms(r))
        out = _summary(v, r, ms, float(np.median(kms)), sample)
        out["tuned"] = tuned
        if per_class:
            out["tuned_per_class"] = per_class
        if os.environ.get("VOROHIP_PHASE_CLOCKS") == "1":
            out["phases"] = v.phase_profile(r)
    finally:
        v.vc_result_destroy(r)
        v.vc_batch_destroy(b)
    return out


def _summary(v, r, ms, kernel_ms, sample=None):
    """Timing, status and counters of a variant; with `sample` (input
    indices), the variant's own output fields on those cells, kept for the
    parity check against the oracle."""
    status = v.vc_result_copy(r, v.VC_F_STATUS)
    diag = dict(zip(v.DIAG_NAMES, v.vc_result_copy(r, v.VC_F_DIAG)[:len(v.DIAG_NAMES)].tolist()))
    base = status & ~np.uint8(v.VC_CELL_FO_OVERFLOW)
    ok = (base <= v.VC_CELL_SPILLED) | (base == v.VC_CELL_EMPTY)
    out = dict(ms_per_step=ms, kernel_ms=kernel_ms, status_ok=bool(np.all(ok)), diag=diag,
               empty_cells=int(np.sum(base == v.VC_CELL_EMPTY)))
    if sample is not None:
        n = len(status)

        def get(field):
            try:
                return v.vc_result_copy(r, field)
            except v.VcError:  # not in the statistics mask
                return None
        f = {"status": status[sample]}
        for key, field in (("vol", v.VC_F_VOLUME), ("nv", v.VC_F_NV), ("ne", v.VC_F_NE), ("nf", v.VC_F_NF)):
            a = get(field)
            f[key] = None if a is None else a[sample]
        a = get(v.VC_F_CENTROID)
        f["cen"] = None if a is None else a.reshape(n, 3)[sample]
        a = get(v.VC_F_FACE_ORDERS)
        f["fo"] = None if a is None else a.reshape(n, v.VC_FO_LEN)[sample].astype(np.int32)
        off, ids, sh = get(v.VC_F_NBR_OFFSETS), get(v.VC_F_NBR_IDS), get(v.VC_F_NBR_SHIFTS)
        f["nbr"] = None if ids is None else [
            np.stack([ids[off[i]:off[i + 1]].astype(np.int64), sh[off[i]:off[i + 1]].astype(np.int64)], 1)
            for i in sample[:NBR_SAMPLE]]
        out["fields"] = f
    return out


NBR_SAMPLE = 20_000  # sample cells whose neighbour lists are compared


def parity(fields, ref, ref_nbr, offsets_of_sample):
    """Errors of a variant's own outputs against the oracle on the sample:
    max and mean relative volume error, max centroid error over V^(1/3)
    (V^(1/2) in 2D), and mismatch counts of the topology fields (counts,
    face orders, status flags) and of the sorted neighbour lists."""
    vol_r = ref["vol"]
    out = dict(cells=int(len(vol_r)))
    dim = ref["cen"].shape[1]
    if fields["vol"] is not None:
        live = vol_r > 0
        rel = np.abs(fields["vol"] - vol_r)[live] / vol_r[live]
        out.update(vol_rel_err_max=float(rel.max()), vol_rel_err_mean=float(rel.mean()))
        if fields["cen"] is not None:
            scale = vol_r[live] ** (1.0 / dim)
            cerr = np.abs(fields["cen"][live][:, :dim] - ref["cen"][live]).max(1) / scale
            out.update(centroid_err_max=float(cerr.max()), centroid_err_mean=float(cerr.mean()))
    mism = {}
    for key in ("nv", "ne", "nf"):
        if (dim == 2 and key == "ne") or fields[key] is None:
            continue
        mism[key] = int(np.sum(fields[key] != ref[key]))
    if fields.get("fo") is not None and dim == 3:
        mism["fo"] = int(np.sum(np.any(fields["fo"] != ref["fo"], 1)))
    flag = 64
    mism["fo_overflow_flag"] = int(np.sum(((fields["status"] & flag) != 0) != ((ref["status"] & flag) != 0)))
    bad = 0
    for t, lab in enumerate(ref_nbr if fields["nbr"] is not None else []):
        got = fields["nbr"][t].copy()
        base = offsets_of_sample[t]
        got[got[:, 0] >= 0, 0] -= base  # batch ids are global
        order = np.lexsort((got[:, 1], got[:, 0]))
        bad += not np.array_equal(got[order], lab)
    mism["nbr"] = int(bad)
    out["mismatches"] = mism
    out["nbr_cells"] = len(ref_nbr) if fields["nbr"] is not None else 0
    out["all_equal"] = all(v_ == 0 for v_ in mism.values())
    return out


def host_description():
    """CPU model, and the logical and physical cores usable by this process."""
    cpus = sorted(os.sched_getaffinity(0))
    model, phys, cur = None, set(), {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if cur.get("processor") is not None and int(cur["processor"]) in cpus:
                    phys.add((cur.get("physical id", "0"), cur.get("core id", cur["processor"])))
                cur = {}
                continue
            k, val = [x.strip() for x in line.split(":", 1)]
            cur[k] = val
            if k == "model name" and model is None:
                model = val
        if cur.get("processor") is not None and int(cur["processor"]) in cpus:
            phys.add((cur.get("physical id", "0"), cur.get("core id", cur["processor"])))
    except OSError:
        pass
    return dict(cpu_model=model, logical_cores=len(cpus), physical_cores=len(phys) or None)


def sample_cells(members, sample):
    """The oracle sample: the first cells of each member in member order, up
    to `sample` cells; returns (member, local indices, global indices)."""
    out, done, base = [], 0, 0
    for t, m in enumerate(members):
        if done >= sample:
            break
        k = min(sample - done, len(m["xyz"]))
        idx = np.arange(k, dtype=np.int64)
        out.append((t, idx, base + idx))
        done += k
        base += len(m["xyz"])
    return out


def cpu_baseline(members, sample):
    """The oracle on the host cores: the first `sample` cells of the
    workload (in member order), OpenMP dynamic schedule over cells.  Also
    returns the oracle's cells (untimed neighbour lists for the first
    NBR_SAMPLE of them), for the parity of every GPU variant."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    done, secs = 0, 0.0
    tot = {}
    ref = {k: [] for k in ("vol", "cen", "nv", "ne", "nf", "fo", "status")}
    ref_nbr, nbr_base = [], []
    offsets = np.cumsum([0] + [len(m["xyz"]) for m in members])
    for t, idx, _ in sample_cells(members, sample):
        m = members[t]
        o = oracle.Oracle(m["xyz"], m["lo"], m["hi"], m["periodic"], grid=m.get("grid"), clip=m.get("clip", 0.0),
                          radii=m.get("radii"))
        k = len(idx)
        if m.get("weinberg"):
            # cells and their Weinberg codes (the VoroTop pipeline); the
            # statistics pass runs untimed, for the operation counts
            t0 = time.perf_counter()
            o.weinberg(idx, nthreads=cores)
            secs += time.perf_counter() - t0
            r = o.cells(idx, nthreads=cores, neighbors=False)
        else:
            t0 = time.perf_counter()
            r = o.cells(idx, nthreads=cores, neighbors=False)
            secs += time.perf_counter() - t0
        done += k
        for key, val in r["counters"].items():
            tot[key] = tot.get(key, 0) + val
        for key in ref:
            ref[key].append(r[key])
        need = NBR_SAMPLE - len(ref_nbr)
        if need > 0:
            ref_nbr += o.cells(idx[:need], nthreads=cores)["nbr"]
            nbr_base += [int(offsets[t])] * min(need, k)
    ref = {key: np.concatenate(val) for key, val in ref.items()}
    # every candidate's distance test is counted (9 flops each); the reading
    # without the candidates the radius bound rejects is reported beside it
    rest = (FLOP_WEIGHTS["vertex_tests"] * tot["vertex_tests"]
            + FLOP_WEIGHTS["new_vertices"] * tot["new_vertices"]
            + FLOP_WEIGHTS["fan_triangles"] * tot["fan_triangles"])
    flops = (FLOP_WEIGHTS["candidates"] * tot["candidates"] + rest) / done
    flops_in_range = (FLOP_WEIGHTS["candidates"] * (tot["candidates"] - tot["radius_rejects"]) + rest) / done
    per_cell = {k: val / done for k, val in tot.items()}
    per_cell["flops_without_radius_rejects"] = flops_in_range
    cpu = dict(value=done / secs, unit="cells/s", cores=cores, kind="oracle", seconds=secs)
    cpu.update(host_description())
    return cpu, flops, per_cell, (ref, ref_nbr, np.array(nbr_base, np.int64))


def cpu_serial(members, sample):
    """The oracle on one host thread: the first `sample` cells of the first
    member (the paper's serial timings are per cell, one core)."""
    import oracle
    m = members[0]
    k = min(sample, len(m["xyz"]))
    o = oracle.Oracle(m["xyz"], m["lo"], m["hi"], m["periodic"], grid=m.get("grid"), clip=m.get("clip", 0.0),
                      radii=m.get("radii"))
    t = time.perf_counter()
    o.cells(np.arange(k, dtype=np.int64), nthreads=1, neighbors=False)
    secs = time.perf_counter() - t
    return dict(value=k / secs, unit="cells/s", cores=1, kind="oracle", seconds=secs,
                sample=f"first {k} cells, one thread")


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {a.gpus}); "
              "sharding over several GPUs is designed but not launched.", file=sys.stderr)
        sys.exit(2)
    if a.phase_clocks:
        os.environ["VOROHIP_PHASE_CLOCKS"] = "1"
    import torch
    from paper_2209_11606_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB_PHASE if a.phase_clocks else hipbuild.LIB):
        raise SystemExit("bench.py: the library is not built; run __graft_entry__.build() first")
    from paper_2209_11606_amd import vorohip as v
    from paper_2209_11606_amd import workloads as W

    if a.workload == "periodic1m":
        w = W.periodic_1m()
        members = [w]
        desc = ("periodic_uniform_1M: 1,000,000 uniform particles, periodic cube side 100, full statistics")
        sample_desc = "first {} cells of the same 1M-particle periodic set"
    elif a.workload == "fcc10m":
        members = [W.fcc_10m()]
        desc = "fcc_perturbed_10M: perturbed FCC (sigma 1e-3 a), 10,000,000 particles, periodic, full statistics"
        sample_desc = "first {} cells of the perturbed FCC set"
    elif a.workload == "periodic2d10m":
        members = [W.periodic_2d_10m()]
        desc = "periodic_uniform_2d_10M: 10,000,000 uniform particles, periodic unit square, full statistics"
        sample_desc = "first {} cells of the 2D set"
    elif a.workload == "periodic102m":
        members = [W.periodic_102m()]
        desc = ("periodic_uniform_102M: 102,400,000 uniform particles, periodic unit cube, "
                "face-order vector and neighbour count only")
        sample_desc = "first {} cells of the 102.4M set"
    elif a.workload == "localized10m":
        w = W.localized(100_000_000)
        # N_opt 5 over the occupied central cube (volume 0.1)
        w["grid"] = [int(math.ceil((len(w["xyz"]) / (5.0 * 0.1)) ** (1.0 / 3.0)))] * 3
        members = [w]
        desc = ("localized_clipped_10M: 10^8 uniform points in the walled unit cube, the ~10^7 inside the "
                "central cube of volume 0.1 kept, each cell clipped by the cube of side 1.5*sqrt(3)*1e-8^(1/3) "
                "(section 3.1.3), full statistics")
        sample_desc = "first {} cells of the localized set"
    elif a.workload == "localized10m_unclipped":
        w = W.localized(100_000_000)
        w["clip"] = 0.0
        members = [w]
        desc = ("localized_unclipped_10M: 10^8 uniform points in the walled unit cube, the ~10^7 inside the "
                "central cube of volume 0.1 kept, no clipping, the paper's N_opt 49 grid (126^3; section 3.1), "
                "full statistics")
        sample_desc = "first {} cells of the localized set"
    elif a.workload == "localized100k_unclipped":
        w = W.localized(1_000_000)
        w["clip"] = 0.0
        members = [w]
        desc = ("localized_unclipped_100k: 10^6 uniform points in the walled unit cube, the ~10^5 inside the "
                "central cube of volume 0.1 kept, no clipping, the paper's N_opt 49 grid (27^3; section 3.1), "
                "full statistics")
        sample_desc = "first {} cells of the localized set"
    elif a.workload == "localized2d10m":
        members = [W.localized(100_000_000, dim=2)]
        desc = ("localized_2d_10M: 10^8 uniform points in the walled unit square, the ~10^7 inside the central "
                "square of area 0.1 kept, the paper's N_opt 30 grid (1825^2; section 3.1), full statistics")
        sample_desc = "first {} cells of the 2D localized set"
    elif a.workload == "clustered2d100m":
        members = [W.clustered(100_000_000, dim=2)]
        desc = ("extreme_clustering_2d_100M: 10^8 points with coordinates 1/2 + 4 (X - 1/2)^3, walled unit "
                "square, N_opt 0.5 grid (14142^2; section 3.1), full statistics")
        sample_desc = "first {} cells of the 2D clustered set"
    elif a.workload == "clustered10m":
        members = [W.clustered(10_000_000)]
        desc = ("extreme_clustering_10M: 10^7 points with coordinates 1/2 + 4 (X - 1/2)^3, walled unit cube, "
                "N_opt 0.5 grid (section 3.1), full statistics")
        sample_desc = "first {} cells of the clustered set"
    elif a.workload == "vorotop1m":
        members = [W.vorotop(1_000_000)]
        desc = ("vorotop_1M: 1,000,000 uniform particles in the periodic unit cube, full statistics and every "
                "cell's Weinberg code (the VoroTop workload of section 5)")
        sample_desc = "first {} cells and Weinberg codes of the same set"
    elif a.workload == "polydisperse1m":
        members = [W.polydisperse(1_000_000, 3)]
        desc = ("polydisperse_radical_1M: radical tessellation of 1,000,000 uniform particles in the periodic "
                "unit cube, radii uniform on [0, 0.6 n^(-1/3)) (section 2.1.1), full statistics")
        sample_desc = "first {} cells of the polydisperse set"
    else:
        members = W.batch(4096)
        desc = ("batch_4096: 4,096 independent 3D tessellations, sizes log-uniform in [100, 100000], "
                "periodic/walled x uniform/perturbed BCC, full statistics")
        sample_desc = "first {} cells of the batch in tessellation order"
    offsets = np.zeros(len(members) + 1, np.int64)
    for t, m in enumerate(members):
        offsets[t + 1] = offsets[t] + len(m["xyz"])
    n = int(offsets[-1])
    xyz = members[0]["xyz"] if len(members) == 1 else np.concatenate([m["xyz"] for m in members])
    xt = torch.from_numpy(xyz).to("cuda:0")
    if a.calibration_copy_mib > 0:
        src = torch.ones(a.calibration_copy_mib << 17, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        del src, dst
    torch.cuda.synchronize()
    res = {}
    variants = []
    dim = xyz.shape[1]
    mask = v.VC_FACE_ORDERS | v.VC_NEIGHBOR_COUNT if a.workload == "periodic102m" else v.VC_ALL
    if members[0].get("weinberg"):
        mask |= v.VC_WEINBERG
    if len(members) == 1:
        variants += [("fp64", v.VC_FP64, False), ("f32_filter", v.VC_F32_FILTER, False)]
    if dim == 3:
        variants += [("fp64_batched", v.VC_FP64, True), ("f32_filter_batched", v.VC_F32_FILTER, True)]
    nslab = a.slabs if a.slabs is not None else (8 if a.workload == "periodic102m" else 0)
    if nslab > 0 and dim == 3 and len(members) == 1:
        variants += [("fp64_chunked", v.VC_FP64, "chunked")]
    if a.variants != "all":
        keep = set(a.variants.split(","))
        variants = [x for x in variants if x[0] in keep]
    sample = None
    if not a.no_cpu_baseline:
        sample = np.concatenate([g for _, _, g in sample_cells(members, a.cpu_sample)])
    for name, prec, batched in variants:
        if batched == "chunked":
            tuned = res.get("fp64_batched", {}).get("tuned")
            res[name] = time_chunked(v, torch, xt, members[0], prec, a.steps, a.warmup, mask, nslab, a.halo,
                                     sample, launch=tuned)
        elif batched:
            opts = [options(v, m, precision=prec) for m in members]
            radii = None
            if members[0].get("radii") is not None:
                radii = np.concatenate([m["radii"] for m in members])
            classes = None
            if len(members) > 1 and members[0].get("kind"):
                classes = {}
                for t, m in enumerate(members):
                    classes.setdefault(m["kind"], []).append(t)
            res[name] = time_batched(v, torch, xt, offsets, opts, a.steps, a.warmup, mask, radii, sample, classes)
        else:
            res[name] = time_variant(v, torch, xt, members[0], prec, a.steps, a.warmup, mask, sample)
        print(f"# {name}: {res[name]['ms_per_step']:.3f} ms/step, cell kernel {res[name]['kernel_ms']:.3f} ms, "
              f"tuned {res[name].get('tuned')}, diag {res[name]['diag']}", file=sys.stderr, flush=True)
    binning = e2e = None
    if len(members) == 1:
        binning = time_binning(v, torch, xt, members[0], a.steps)
        if a.workload != "periodic102m":
            tuned = res.get("fp64_batched", {}).get("tuned") if dim == 3 else None
            e2e = end_to_end(v, torch, xyz, members[0], v.VC_FP64, mask, launch=tuned)
        print(f"# binning: {binning['ms']:.3f} ms, end-to-end: {e2e and round(e2e['ms'], 3)} ms",
              file=sys.stderr, flush=True)
    serial = None
    if a.no_cpu_baseline:
        cpu, flops_per_cell = None, None
    else:
        cpu, flops_per_cell, per_cell, (ref, ref_nbr, nbr_base) = cpu_baseline(members, a.cpu_sample)
        for name in res:
            f = res[name].pop("fields", None)
            if f is not None:
                res[name]["parity"] = parity(f, ref, ref_nbr, nbr_base)
                print(f"# {name} parity: {res[name]['parity']}", file=sys.stderr, flush=True)
        if dim == 2:
            flops_per_cell = None  # the flop model is the 3D one
        cpu["sample"] = sample_desc.format(min(a.cpu_sample, n)) + ", OpenMP dynamic,64 over cells"
        print(f"# oracle: {cpu['value']:.0f} cells/s on {cpu['cores']} cores; per cell {per_cell}",
              file=sys.stderr, flush=True)
        serial = cpu_serial(members, a.cpu_serial_sample)
    best = max(res, key=lambda k: n / res[k]["ms_per_step"])
    b = res[best]
    value = n / (b["ms_per_step"] / 1e3)
    roof = None
    if flops_per_cell is not None:
        achieved = n * flops_per_cell / (b["kernel_ms"] / 1e3)
        key = kernel_key("fp64" if best.startswith("fp64") else "f32_filter", b.get("tuned"))
        traffic = committed_traffic(key) if a.workload == "periodic1m" else None
        ctr = committed_counters(key) if a.workload == "periodic1m" else None
        # the published peak, confirmed on this device by an FMA microbenchmark
        measured = {"fp64": v.vc_device_fma_rate(v.VC_FP64), "fp32_unpacked": v.vc_device_fma_rate(v.VC_F32_FILTER)}
        roof = dict(bound="alu", achieved=achieved / 1e12, peak=FP64_VECTOR_PEAK / 1e12, unit="TFLOP/s",
                    frac=achieved / FP64_VECTOR_PEAK, traffic=traffic,
                    kernel="cell construction (" + key + ")", flops_per_cell=flops_per_cell,
                    flops_per_cell_reading="every candidate's distance test counted (9), vertex side tests (6), "
                                           "new vertices (12), fan tetrahedra (28), from the oracle's counts",
                    flops_per_cell_without_radius_rejects=per_cell.get("flops_without_radius_rejects"),
                    kernel_ms=b["kernel_ms"], measured_fma_peak=measured,
                    # issue-side utilisation from the same counter runs: the
                    # kernel is bound by instruction issue and latency
                    valu_busy=ctr and ctr.get("valu_busy"), wait_frac=ctr and ctr.get("wait_frac"))
    out = {
        "metric": ("3D" if dim == 3 else "2D") + (" radical" if members[0].get("radii") is not None else "")
                  + " Voronoi cells/s on 1 MI355X, FP32-filter vs FP64 plain; "
                  "oracle-exact topology",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": b["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if best.startswith("fp64") else "f32-filter+f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "tessellations": len(members), "variant": best},
        "variants": {k: dict(cells_per_s=n / (r["ms_per_step"] / 1e3), ms_per_step=r["ms_per_step"],
                             cell_kernel_ms=r["kernel_ms"], all_cells_ok=r["status_ok"],
                             empty_cells=r["empty_cells"], tuned=r.get("tuned"),
                             roofline_frac=(None if flops_per_cell is None else
                                            n * flops_per_cell / (r["kernel_ms"] / 1e3) / FP64_VECTOR_PEAK),
                             tuned_per_class=r.get("tuned_per_class"),
                             diag=r["diag"], phases=r.get("phases"), parity=r.get("parity"))
                     for k, r in res.items()},
        "roofline": roof,
        "binning_roofline": binning,
        "end_to_end": e2e,
        "cpu_baseline": cpu,
        "oracle_work_per_cell": None if a.no_cpu_baseline else per_cell,
        "cpu_serial": serial,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
