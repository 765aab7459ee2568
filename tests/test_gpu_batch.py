"""The batched form: many independent tessellations in one persistent launch.

Each tessellation's cells must be bitwise identical to the same tessellation
computed alone (the work queue and launch parameters never change a cell),
match the oracle, and stay identical across hipGraph replays and after the
autotuner picks its launch parameters.
"""
import numpy as np
import pytest

import oracle
from paper_2209_11606_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FIELDS = ("vol", "cen", "nv", "ne", "nf", "fo", "status")


@pytest.fixture(scope="module")
def v():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_11606_amd import vorohip
    return vorohip


def make_batch(count, seed, hi):
    members = W.batch(count, seed, 100, hi)
    offsets = np.zeros(count + 1, np.int64)
    for t, m in enumerate(members):
        offsets[t + 1] = offsets[t] + len(m["xyz"])
    xyz = np.concatenate([m["xyz"] for m in members])
    return members, offsets, xyz


def batch_run(v, members, offsets, xyz, graph_replays=0, tune=False, precision=0):
    opts = [v.vc_options_init(3, m["lo"], m["hi"], m["periodic"], precision=precision) for m in members]
    s = torch.cuda.Stream()
    xt = torch.from_numpy(xyz).to("cuda:0")
    torch.cuda.synchronize()
    b = v.vc_batch_create(xt, offsets, opts, s)
    r = v.vc_batch_result_create(b, v.VC_ALL)
    try:
        tuned = v.vc_batch_tune(b, r, s) if tune else None
        v.vc_batch_compute(b, r, False, s)
        eager = v.fetch(r, v.VC_ALL, len(xyz))
        replays = []
        for k in range(graph_replays):
            # eager work between replays on the same stream and on the default one
            with torch.cuda.stream(s):
                junk = torch.randn(1 << 16, device="cuda:0").sum()
            v.vc_batch_compute(b, r, True, s)
            s.synchronize()
            replays.append(v.fetch(r, v.VC_ALL, len(xyz)))
            float(junk)
        return eager, replays, tuned
    finally:
        v.vc_result_destroy(r)
        v.vc_batch_destroy(b)


def split(res, offsets, t):
    a, e = offsets[t], offsets[t + 1]
    out = {k: res[k][a:e] for k in FIELDS}
    off = res["nbr_off"]
    out["nbr"] = [np.stack([res["nbr_ids"][off[i]:off[i + 1]].astype(np.int64),
                            res["nbr_sh"][off[i]:off[i + 1]].astype(np.int64)], 1) for i in range(a, e)]
    return out


def test_batch_equals_single_and_oracle(v):
    members, offsets, xyz = make_batch(24, 2024, 3000)
    eager, _, _ = batch_run(v, members, offsets, xyz)
    assert np.all(eager["status"] <= 1)
    for t, m in enumerate(members):
        xt = torch.from_numpy(np.ascontiguousarray(m["xyz"])).to("cuda:0")
        one = v.tessellate(xt, m["lo"], m["hi"], m["periodic"], v.VC_ALL)
        part = split(eager, offsets, t)
        for k in FIELDS:
            assert np.array_equal(part[k], one[k]), (t, m["kind"], k)
        nb1 = v.neighbor_lists(one)
        # neighbour ids in the batch are global (offset by the tessellation start)
        for i in range(len(nb1)):
            got = part["nbr"][i].copy()
            got[got[:, 0] >= 0, 0] -= offsets[t]
            assert np.array_equal(got, nb1[i])
        if t % 6 == 0:
            r = oracle.Oracle(m["xyz"], m["lo"], m["hi"], m["periodic"]).cells()
            assert np.array_equal(one["nf"], r["nf"]) and np.array_equal(one["fo"], r["fo"])
            assert np.max(np.abs(one["vol"] - r["vol"]) / r["vol"]) <= 1e-12
            for i in range(len(nb1)):
                assert np.array_equal(nb1[i], r["nbr"][i])


def test_graph_replays_and_tuner(v):
    members, offsets, xyz = make_batch(40, 77, 5000)
    eager, replays, _ = batch_run(v, members, offsets, xyz, graph_replays=3)
    for rep in replays:
        for k in FIELDS + ("nbr_off", "nbr_ids", "nbr_sh"):
            assert np.array_equal(rep[k], eager[k]), k
    tuned_eager, tuned_replays, tuned = batch_run(v, members, offsets, xyz, graph_replays=2, tune=True)
    assert tuned["slots"] in (2, 4) and tuned["chunk"] in (1, 4, 16, 64) and tuned["ms"] > 0
    assert tuned["cells_per_wave"] in (1, 2, 4)
    for res in [tuned_eager] + tuned_replays:
        # the tuned form may lay vertices out differently: same cells to rounding
        for k in ("nv", "ne", "nf", "fo", "status", "nbr_off", "nbr_ids", "nbr_sh"):
            assert np.array_equal(res[k], eager[k]), k
        assert np.max(np.abs(res["vol"] - eager["vol"]) / eager["vol"]) <= 1e-13
    for res in tuned_replays:
        for k in FIELDS + ("nbr_off", "nbr_ids", "nbr_sh"):
            assert np.array_equal(res[k], tuned_eager[k]), k


def test_batch_f32_filter_bitwise(v):
    members, offsets, xyz = make_batch(16, 5, 4000)
    a, _, _ = batch_run(v, members, offsets, xyz)
    b, _, _ = batch_run(v, members, offsets, xyz, precision=1)
    for k in FIELDS + ("nbr_off", "nbr_ids", "nbr_sh"):
        assert np.array_equal(a[k], b[k]), k


def test_batch_argument_errors(v):
    members, offsets, xyz = make_batch(3, 9, 500)
    opts = [v.vc_options_init(3, m["lo"], m["hi"], m["periodic"]) for m in members]
    bad = offsets.copy()
    bad[2] = bad[1]
    with pytest.raises(v.VcError) as e:
        v.vc_batch_create(xyz, bad, opts)
    assert e.value.code == v.VC_E_ARG


def test_full_size_periodic_1m_bench_path(v):
    """The benchmark's own launch path on its workload: the 1M periodic set
    as a one-member batch, tuned, computed eagerly and by two graph
    replays, in both precisions.  Every replay equals the eager result bit
    for bit; sampled cells equal the oracle; the volumes tile the box."""
    import math
    from test_gpu_parity import assert_parity
    w = W.periodic_1m()
    x = np.ascontiguousarray(w["xyz"])
    n = len(x)
    offsets = np.array([0, n], np.int64)
    idx = np.random.default_rng(11).choice(n, 1000, replace=False)
    r = oracle.Oracle(x, w["lo"], w["hi"], w["periodic"]).cells(idx, nthreads=oracle.num_threads())
    for precision in (v.VC_FP64, v.VC_F32_FILTER):
        eager, replays, tuned = batch_run(v, [w], offsets, x, graph_replays=2, tune=True, precision=precision)
        print("bench path", precision, tuned, flush=True)
        for res in replays:
            for k in ("vol", "cen", "nv", "ne", "nf", "fo", "status", "nbr_off", "nbr_ids", "nbr_sh"):
                assert np.array_equal(res[k], eager[k]), k
        # a tuned capacity below the kernel's own may send cells to the
        # spill pass (status SPILLED); nothing else may fail.  At full
        # capacity the grouped forms leave only the cells with a side
        # decision in the exact predicate's band to the one-cell kernel
        # (about 16 in this set)
        assert np.all(eager["status"] <= v.VC_CELL_SPILLED)
        if tuned["capacity"] == 0:
            assert np.sum(eager["status"] == v.VC_CELL_SPILLED) <= 100
        assert math.fsum(eager["vol"]) == pytest.approx(100.0 ** 3, rel=1e-12)
        eager["nbr"] = v.neighbor_lists(eager)
        assert_parity(eager, r, idx)


def _member_nbr(res, offsets, t, cells):
    """Sorted (label, image) lists of some cells of member t, labels made
    local to the member (walls stay negative)."""
    off, ids, sh = res["nbr_off"], res["nbr_ids"], res["nbr_sh"]
    out = []
    for i in cells:
        g = offsets[t] + i
        lab = ids[off[g]:off[g + 1]].astype(np.int64)
        lab[lab >= 0] -= offsets[t]
        out.append(np.stack([lab, sh[off[g]:off[g + 1]].astype(np.int64)], 1))
    return out


def _symmetric(res, offsets, t):
    """Neighbour symmetry inside member t: (i -> j, s) pairs with (j -> i, -s)."""
    a, e = int(offsets[t]), int(offsets[t + 1])
    off = res["nbr_off"]
    ids = res["nbr_ids"][off[a]:off[e]].astype(np.int64)
    sh = res["nbr_sh"][off[a]:off[e]].astype(np.int64)
    src = np.repeat(np.arange(a, e, dtype=np.int64), np.diff(off[a:e + 1]))
    keep = ids >= 0
    src, ids, sh = src[keep], ids[keep], sh[keep]
    s = np.stack([sh % 5 - 2, (sh // 5) % 5 - 2, sh // 25 - 2], 1)
    negc = 25 * (-s[:, 2] + 2) + 5 * (-s[:, 1] + 2) + (-s[:, 0] + 2)
    fwd = np.sort(src * (1 << 40) + ids * 128 + sh)
    bwd = np.sort(ids * (1 << 40) + src * 128 + negc)
    return np.array_equal(fwd, bwd)


@pytest.mark.timeout(900)
def test_full_size_batch4096(v):
    """The 4,096-tessellation batch at its own size (5.85e7 cells; sizes
    log-uniform in [100, 1e5]; periodic / walled x uniform / perturbed BCC),
    tuned and replayed from a hipGraph as the benchmark runs it.  The replay
    equals the eager launch bit for bit.  On every member: the volumes tile
    the box, Euler's V - E + F = 2 and the face-order sums hold for every
    cell.  Neighbour symmetry on the 20 largest members and 4 per class.
    Element-wise parity with the oracle (counts, face orders, neighbour
    lists, volume, centroid) on 60 cells of 8 members of each class and on
    50 cells of each of the 20 largest members."""
    import math
    from test_gpu_parity import assert_parity
    members = W.batch(4096)
    count = len(members)
    offsets = np.zeros(count + 1, np.int64)
    for t, m in enumerate(members):
        offsets[t + 1] = offsets[t] + len(m["xyz"])
    n = int(offsets[-1])
    xyz = np.concatenate([m["xyz"] for m in members])
    opts = [v.vc_options_init(3, m["lo"], m["hi"], m["periodic"]) for m in members]
    s = torch.cuda.Stream()
    xt = torch.from_numpy(xyz).to("cuda:0")
    torch.cuda.synchronize()
    b = v.vc_batch_create(xt, offsets, opts, s)
    r = v.vc_batch_result_create(b, v.VC_ALL)
    try:
        tuned = v.vc_batch_tune(b, r, s)
        print("batch4096 tuned", tuned, flush=True)
        v.vc_batch_compute(b, r, False, s)
        s.synchronize()
        eager = v.fetch(r, v.VC_ALL, n)
        v.vc_batch_compute(b, r, True, s)  # capture and replay
        v.vc_batch_compute(b, r, True, s)  # replay again
        s.synchronize()
        rep = v.fetch(r, v.VC_ALL, n)
        for k in ("vol", "cen", "nv", "ne", "nf", "fo", "status", "nbr_off", "nbr_ids", "nbr_sh"):
            assert np.array_equal(rep[k], eager[k]), k
        del rep
    finally:
        v.vc_result_destroy(r)
        v.vc_batch_destroy(b)
    g = eager
    print("batch4096 diag", g["diag"], flush=True)
    assert np.all(g["status"] <= 1)
    assert np.all(g["nv"] - g["ne"] + g["nf"] == 2)
    assert np.all(g["fo"].sum(1) == g["nf"])
    assert np.all((g["fo"] * np.arange(32)).sum(1) == 2 * g["ne"])
    for t, m in enumerate(members):
        box = float(np.prod(np.asarray(m["hi"]) - np.asarray(m["lo"])))
        assert math.fsum(g["vol"][offsets[t]:offsets[t + 1]]) == pytest.approx(box, rel=1e-12), t
    sizes = np.diff(offsets)
    largest = np.argsort(sizes)[-20:]
    rng = np.random.default_rng(4096)
    by_kind = {}
    for t, m in enumerate(members):
        by_kind.setdefault(m["kind"], []).append(t)
    assert sorted(by_kind) == ["periodic_bcc", "periodic_uniform", "walled_bcc", "walled_uniform"]
    picks = [(int(t), 50) for t in largest]
    for kind, ts in sorted(by_kind.items()):
        sel = rng.choice(ts, 8, replace=False)
        picks += [(int(t), 60) for t in sel]
        for t in list(sel[:4]):
            assert _symmetric(g, offsets, int(t)), (kind, t)
    for t in largest:
        assert _symmetric(g, offsets, int(t)), t
    checked = 0
    for t, k in picks:
        m = members[t]
        nt = int(sizes[t])
        cells = np.sort(rng.choice(nt, min(k, nt), replace=False))
        ref = oracle.Oracle(m["xyz"], m["lo"], m["hi"], m["periodic"]).cells(cells, nthreads=oracle.num_threads())
        a = int(offsets[t])
        part = {key: g[key][a + cells] for key in ("vol", "cen", "nv", "ne", "nf", "fo", "status")}
        part["nbr"] = _member_nbr(g, offsets, t, cells)
        assert_parity(part, ref, np.arange(len(cells)))
        checked += len(cells)
    print(f"batch4096: {checked} cells of {len(picks)} members equal the oracle", flush=True)


def test_tuner_per_class_and_capacity(v):
    """Tuning on one class of members (the periodic ones) picks a valid
    launch form, including the vertex capacity before the spill pass; the
    tuned batch still gives the same cells; a member index outside the
    batch is rejected."""
    members, offsets, xyz = make_batch(24, 31, 3000)
    opts = [v.vc_options_init(3, m["lo"], m["hi"], m["periodic"]) for m in members]
    s = torch.cuda.Stream()
    xt = torch.from_numpy(xyz).to("cuda:0")
    torch.cuda.synchronize()
    b = v.vc_batch_create(xt, offsets, opts, s)
    r = v.vc_batch_result_create(b, v.VC_ALL)
    try:
        v.vc_batch_compute(b, r, False, s)
        base = v.fetch(r, v.VC_ALL, len(xyz))
        per = [t for t, m in enumerate(members) if m["kind"].startswith("periodic")]
        t = v.vc_batch_tune_members(b, r, per, s)
        print("periodic members tuned", t, flush=True)
        assert t["cells_per_wave"] in (1, 2, 4) and t["ms"] > 0
        full = {1: 64 * t["slots"], 2: 64, 4: 64}[t["cells_per_wave"]]
        assert t["capacity"] in (0, full * 3 // 4)
        v.vc_batch_compute(b, r, False, s)
        got = v.fetch(r, v.VC_ALL, len(xyz))
        for k in ("nv", "ne", "nf", "fo", "nbr_off", "nbr_ids", "nbr_sh"):
            assert np.array_equal(got[k], base[k]), k
        # a smaller capacity sends more cells through the spill pass: only
        # the SPILLED code may change, to or from OK
        def norm(st):
            st = st.copy()
            st[(st & 63) == v.VC_CELL_SPILLED] &= ~np.uint8(63)
            return st
        assert np.array_equal(norm(got["status"]), norm(base["status"]))
        if t["capacity"]:
            assert np.count_nonzero((got["status"] & 63) == v.VC_CELL_SPILLED) >= \
                np.count_nonzero((base["status"] & 63) == v.VC_CELL_SPILLED)
        assert np.max(np.abs(got["vol"] - base["vol"]) / base["vol"]) <= 1e-13
        with pytest.raises(v.VcError) as e:
            v.vc_batch_tune_members(b, r, [0, len(members)], s)
        assert e.value.code == v.VC_E_RANGE
    finally:
        v.vc_result_destroy(r)
        v.vc_batch_destroy(b)
