"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Topology (vertex, edge, face counts, face-order vectors, sorted neighbour
lists) must be identical; volumes within 1e-12 relative and centroids within
1e-12 * vol^(1/3) (the tolerance the target states for FP64).  The FP32-filter
form must be bitwise identical to the FP64 form: its filter only ever defers
to FP64 inside a band that covers the FP32 rounding error.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_2209_11606_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def v():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_11606_amd import vorohip
    return vorohip


def run(v, x, lo, hi, per, **opt):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    out = v.tessellate(xt, lo, hi, per, v.VC_ALL, **opt)
    out["nbr"] = v.neighbor_lists(out)
    return out


def assert_parity(g, r, idx=None, vol_tol=1e-12):
    idx = np.arange(len(g["vol"])) if idx is None else np.asarray(idx)
    st = g["status"][idx].astype(np.int64)
    assert np.all((st & ~64) <= 1), np.unique(st)
    # the face-order overflow flag (a face of 32 or more edges) as the oracle's
    assert np.array_equal((st & 64) != 0, (np.asarray(r["status"]) & 64) != 0)
    for key in ("nv", "ne", "nf"):
        bad = np.nonzero(g[key][idx] != r[key])[0]
        assert len(bad) == 0, (key, idx[bad[:5]], g[key][idx][bad[:5]], r[key][bad[:5]])
    assert np.array_equal(g["fo"][idx], r["fo"])
    for t, i in enumerate(idx):
        assert np.array_equal(g["nbr"][i], r["nbr"][t]), (i, g["nbr"][i].tolist(), r["nbr"][t].tolist())
    rel = np.abs(g["vol"][idx] - r["vol"]) / r["vol"]
    assert rel.max() <= vol_tol, rel.max()
    scale = r["vol"] ** (1.0 / 3.0)
    cerr = np.abs(g["cen"][idx] - r["cen"]).max(1) / scale
    assert cerr.max() <= 1e-12, cerr.max()


def same_bits(a, b):
    for k in ("vol", "cen", "nv", "ne", "nf", "fo", "status", "nbr_off", "nbr_ids", "nbr_sh"):
        assert np.array_equal(a[k], b[k]), k


def test_walled_1k_all_cells(v):
    w = W.walled_1k()
    g = run(v, w["xyz"], w["lo"], w["hi"], w["periodic"])
    r = oracle.Oracle(w["xyz"], w["lo"], w["hi"], w["periodic"]).cells()
    assert_parity(g, r)


@pytest.mark.parametrize("n,per,seed", [(30, [0, 0, 0], 7), (24, [1, 1, 1], 8), (20, [1, 0, 1], 11)])
def test_tiny_against_exact_brute_force(v, n, per, seed):
    x = W.uniform(n, 3, 1.0, seed)
    g = run(v, x, [0] * 3, [1] * 3, per)
    for i in range(n):
        b = brute.cell(x, i, [0] * 3, [1] * 3, per)
        assert g["nv"][i] == b["nv"] and g["ne"][i] == b["ne"] and g["nf"][i] == b["nf"]
        assert list(g["fo"][i]) == b["fo"]
        assert [tuple(t) for t in g["nbr"][i].tolist()] == b["nbr"]
        assert abs(g["vol"][i] - float(b["vol"])) <= 1e-13 * float(b["vol"])


@pytest.mark.parametrize("n", [1, 2, 7])
def test_ragged_small_counts(v, n):
    x = W.uniform(n, 3, 1.0, 100 + n)
    for per in ([0, 0, 0], [1, 1, 1]):
        g = run(v, x, [0] * 3, [1] * 3, per)
        r = oracle.Oracle(x, [0] * 3, [1] * 3, per).cells()
        assert_parity(g, r)
        assert math.fsum(g["vol"]) == pytest.approx(1.0, rel=1e-13)


def test_nonunit_offset_box(v):
    lo, hi = [-1.5, 2.0, 0.25], [0.5, 2.75, 1.75]
    u = W.uniform(500, 3, 1.0, 21)
    x = np.array(lo) + u * (np.array(hi) - np.array(lo))
    x = np.minimum(x, np.nextafter(np.array(hi), -np.inf))
    per = [1, 0, 1]
    g = run(v, x, lo, hi, per)
    r = oracle.Oracle(x, lo, hi, per).cells()
    assert_parity(g, r)


@pytest.mark.parametrize("a", [1.0, 2.0])
def test_lattices_degenerate(v, a):
    """Exact lattices: every degenerate contact is an exact zero; the GPU
    merges split vertices and drops zero-area faces like the oracle."""
    for (x, hi), V, E, F, vol in [(W.sc(5, a), 8, 12, 6, a ** 3), (W.bcc(4, a), 24, 36, 14, a ** 3 / 2),
                                  (W.fcc((3, 3, 4), a), 14, 24, 12, a ** 3 / 4)]:
        g = run(v, x, [0] * 3, hi, [1, 1, 1])
        assert set(g["nv"]) == {V} and set(g["ne"]) == {E} and set(g["nf"]) == {F}
        assert np.allclose(g["vol"], vol, rtol=1e-13)
        r = oracle.Oracle(x, [0] * 3, hi, [1, 1, 1]).cells()
        assert_parity(g, r)
    x, hi = W.sc(4, a)
    g = run(v, x, [0] * 3, hi, [0, 0, 0])
    r = oracle.Oracle(x, [0] * 3, hi, [0, 0, 0]).cells()
    assert_parity(g, r)


def test_periodic_20k_all_cells_and_f32_bitwise(v):
    side = 20000 ** (1 / 3)
    x = W.uniform(20000, 3, side, 31)
    g = run(v, x, [0] * 3, [side] * 3, [1, 1, 1])
    r = oracle.Oracle(x, [0] * 3, [side] * 3, [1, 1, 1]).cells(nthreads=oracle.num_threads())
    assert_parity(g, r)
    f = run(v, x, [0] * 3, [side] * 3, [1, 1, 1], precision=v.VC_F32_FILTER)
    same_bits(g, f)
    assert f["diag"]["recheck"] > 0
    g2 = run(v, x, [0] * 3, [side] * 3, [1, 1, 1])
    same_bits(g, g2)  # run-to-run determinism


def test_perturbed_fcc_near_degenerate(v):
    x, hi = W.fcc((8, 8, 8), 1.0, 1e-3, seed=3)
    g = run(v, x, [0] * 3, hi, [1, 1, 1])
    r = oracle.Oracle(x, [0] * 3, hi, [1, 1, 1]).cells(nthreads=oracle.num_threads())
    assert_parity(g, r)
    f = run(v, x, [0] * 3, hi, [1, 1, 1], precision=v.VC_F32_FILTER)
    same_bits(g, f)


def same_cells(a, b, tol=1e-13):
    """Same topology and neighbour lists; volumes and centroids to rounding
    (different launch forms lay the vertices out differently, so the fan sums
    run in a different order)."""
    for k in ("nv", "ne", "nf", "fo", "status", "nbr_off", "nbr_ids", "nbr_sh"):
        assert np.array_equal(a[k], b[k]), k
    assert np.max(np.abs(a["vol"] - b["vol"]) / a["vol"]) <= tol
    assert np.max(np.abs(a["cen"] - b["cen"]).max(1) / a["vol"] ** (1 / 3)) <= tol


def test_launch_forms_agree(v):
    """Slots, chunk, waves and cells per wave never change a cell; within one
    form the FP32 filter is bitwise identical to FP64."""
    side = 3000 ** (1 / 3)
    x = W.uniform(3000, 3, side, 41)
    base = run(v, x, [0] * 3, [side] * 3, [1, 1, 1])
    for opt in (dict(slots=4), dict(chunk=1), dict(chunk=64), dict(waves=7)):
        same_bits(base, run(v, x, [0] * 3, [side] * 3, [1, 1, 1], **opt))
    r = oracle.Oracle(x, [0] * 3, [side] * 3, [1, 1, 1]).cells()
    for cpw in (2, 4):
        g = run(v, x, [0] * 3, [side] * 3, [1, 1, 1], cells_per_wave=cpw)
        same_cells(base, g)
        assert_parity(g, r)
        f = run(v, x, [0] * 3, [side] * 3, [1, 1, 1], cells_per_wave=cpw, precision=v.VC_F32_FILTER, chunk=1)
        same_bits(g, f)


@pytest.mark.parametrize("cpw", [2, 4])
def test_grouped_forms_on_hard_inputs(v, cpw):
    """Several cells per wave on the walled 1k set, exact lattices and the
    near-degenerate perturbed FCC."""
    w = W.walled_1k()
    g = run(v, w["xyz"], w["lo"], w["hi"], w["periodic"], cells_per_wave=cpw)
    assert_parity(g, oracle.Oracle(w["xyz"], w["lo"], w["hi"], w["periodic"]).cells())
    for (x, hi) in [W.sc(5, 1.0), W.bcc(4, 2.0), W.fcc((3, 3, 4), 2.0), W.fcc((6, 6, 6), 1.0, 1e-3, seed=3)]:
        g = run(v, x, [0] * 3, hi, [1, 1, 1], cells_per_wave=cpw)
        assert_parity(g, oracle.Oracle(x, [0] * 3, hi, [1, 1, 1]).cells())


def test_full_size_periodic_1m(v):
    """The 1M-particle periodic workload of the benchmark in a plain
    container (two cells per wave): sampled cells against the oracle,
    invariants over all (the batched, tuned path of the benchmark is tested
    in test_gpu_batch.py)."""
    w = W.periodic_1m()
    x = w["xyz"]
    g = run(v, x, w["lo"], w["hi"], w["periodic"])
    n = len(x)
    assert np.all(g["status"] == 0)
    assert math.fsum(g["vol"]) == pytest.approx(100.0 ** 3, rel=1e-12)
    assert np.all(g["nv"] - g["ne"] + g["nf"] == 2)
    assert np.all(2 * g["ne"] == 3 * g["nv"])
    assert np.all(g["fo"].sum(1) == g["nf"])
    assert np.all((g["fo"] * np.arange(32)).sum(1) == 2 * g["ne"])
    # neighbour symmetry over the CSR arrays: (i -> j, s) pairs with (j -> i, -s)
    off, ids, sh = g["nbr_off"], g["nbr_ids"].astype(np.int64), g["nbr_sh"].astype(np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    s = np.stack([sh % 5 - 2, (sh // 5) % 5 - 2, sh // 25 - 2], 1)
    negc = 25 * (-s[:, 2] + 2) + 5 * (-s[:, 1] + 2) + (-s[:, 0] + 2)
    fwd = np.sort(src * (n * 128) + ids * 128 + sh)
    bwd = np.sort(ids * (n * 128) + src * 128 + negc)
    assert np.array_equal(fwd, bwd)
    ef = 2 + 48 * math.pi ** 2 / 35
    assert abs(g["nf"].mean() - ef) < 0.02
    idx = np.random.default_rng(0).choice(n, 1500, replace=False)
    r = oracle.Oracle(x, w["lo"], w["hi"], w["periodic"]).cells(idx, nthreads=oracle.num_threads())
    assert_parity(g, r, idx)


def test_errors(v):
    x = W.uniform(100, 3, 1.0, 5)
    x[3, 1] = 1.5
    xt = torch.from_numpy(x).to("cuda:0")
    with pytest.raises(v.VcError) as e:
        v.tessellate(xt, [0] * 3, [1] * 3, [0, 0, 0])
    assert e.value.code == v.VC_E_RANGE
    x = W.uniform(100, 3, 1.0, 5)
    x[7] = x[8]
    g = run(v, x, [0] * 3, [1] * 3, [0, 0, 0])
    assert g["status"][7] == 3 and g["status"][8] == 3


@pytest.mark.parametrize("form", [dict(), dict(cells_per_wave=2), dict(cells_per_wave=4), dict(slots=4)])
def test_face_order_overflow(v, form):
    """Two cells with two 40-gon faces each: every launch form reports the
    overflow flag on exactly those cells, face orders without the 40-gons,
    and otherwise the oracle's cells."""
    x = W.ring_face(40)
    g = run(v, x, [0] * 3, [1] * 3, [0, 0, 0], **form)
    r = oracle.Oracle(x, [0] * 3, [1] * 3, [0, 0, 0]).cells()
    assert np.array_equal(g["status"] & 64, np.array([64, 64] + [0] * 40, np.uint8))
    assert np.all(g["fo"][:2].sum(1) == g["nf"][:2] - 2)
    assert_parity(g, r)


@pytest.mark.parametrize("form", [dict(), dict(cells_per_wave=2), dict(cells_per_wave=4)])
def test_forced_spill_walled_1k(v, form):
    """Capacity 3 sends every cell to the large-capacity spill pass at its
    first cut (a polyhedron has at least four vertices): all 1,000 cells are
    re-run there (status SPILLED, the spill counter equal to n) and still
    equal the oracle's cells."""
    w = W.walled_1k()
    g = run(v, w["xyz"], w["lo"], w["hi"], w["periodic"], capacity=3, **form)
    n = len(w["xyz"])
    assert np.all(g["status"] == v.VC_CELL_SPILLED) and g["diag"]["spilled"] == n
    assert_parity(g, oracle.Oracle(w["xyz"], w["lo"], w["hi"], w["periodic"]).cells())


def test_forced_spill_periodic_20k(v):
    """Every cell of the periodic 20k set through the spill pass (two cells
    per wave in the main kernel), against the oracle, with the FP32 filter
    bitwise equal; a capacity of 24 vertices spills only the larger cells."""
    side = 20000 ** (1 / 3)
    x = W.uniform(20000, 3, side, 31)
    r = oracle.Oracle(x, [0] * 3, [side] * 3, [1, 1, 1]).cells(nthreads=oracle.num_threads())
    g = run(v, x, [0] * 3, [side] * 3, [1, 1, 1], capacity=3, cells_per_wave=2)
    assert np.all(g["status"] == v.VC_CELL_SPILLED) and g["diag"]["spilled"] == 20000
    assert_parity(g, r)
    f = run(v, x, [0] * 3, [side] * 3, [1, 1, 1], capacity=3, cells_per_wave=2, precision=v.VC_F32_FILTER)
    same_bits(g, f)
    h = run(v, x, [0] * 3, [side] * 3, [1, 1, 1], capacity=24, cells_per_wave=2)
    k = int(np.sum(h["status"] == v.VC_CELL_SPILLED))
    assert 0 < k < 20000 and h["diag"]["spilled"] == k
    assert_parity(h, r)


@pytest.mark.parametrize("form", [dict(), dict(slots=4), dict(cells_per_wave=2), dict(cells_per_wave=4)])
def test_forced_recheck_and_exact(v, form):
    """The slow stages of the side test taken on every decision: with
    VC_FORCE_RECHECK every FP32 filter test is re-done in FP64 (the recheck
    counter equals the test counter), with VC_FORCE_EXACT every FP64
    decision is in the exact predicate's band.  The one-cell forms take
    them exactly (the exact counter reaches the test counter) and give the
    cells of the default bands bit for bit; the grouped forms leave every
    cell with an in-band decision to the FP64 one-cell kernel of the spill
    pass, so forced, every cell goes there and comes out bit for bit as in
    the one-cell form.  All equal the oracle's, on a periodic and on a
    walled set."""
    grouped = form.get("cells_per_wave", 1) > 1
    for per, seed in (([1, 1, 1], 17), ([0, 0, 0], 18)):
        side = 4000 ** (1 / 3)
        x = W.uniform(4000, 3, side, seed)
        box = ([0] * 3, [side] * 3, per)
        base = run(v, x, *box, **form)
        assert_parity(base, oracle.Oracle(x, *box).cells(nthreads=oracle.num_threads()))
        f = run(v, x, *box, precision=v.VC_F32_FILTER, force=v.VC_FORCE_RECHECK, **form)
        same_bits(base, f)
        assert f["diag"]["recheck"] == f["diag"]["tests"] > 0
        e = run(v, x, *box, force=v.VC_FORCE_EXACT, **form)
        fe = run(v, x, *box, precision=v.VC_F32_FILTER, force=v.VC_FORCE_RECHECK | v.VC_FORCE_EXACT, **form)
        if grouped:
            one = run(v, x, *box)
            for g in (e, fe):
                assert g["diag"]["spilled"] == len(x) and np.all(g["status"] == v.VC_CELL_SPILLED)
                assert g["diag"]["exact"] >= g["diag"]["tests"] > 0
                g = dict(g, status=one["status"])
                same_bits(one, g)
        else:
            same_bits(base, e)
            assert e["diag"]["exact"] >= e["diag"]["tests"] > 0
            same_bits(base, fe)
            assert fe["diag"]["exact"] >= fe["diag"]["recheck"] == fe["diag"]["tests"]


def test_force_bits_checked(v):
    """Bits outside VC_FORCE_RECHECK | VC_FORCE_EXACT are refused."""
    x = W.uniform(100, 3, 1.0, 3)
    with pytest.raises(v.VcError) as e:
        run(v, x, [0] * 3, [1] * 3, [0] * 3, force=4)
    assert e.value.code == v.VC_E_ARG


@pytest.mark.parametrize("eps", [1e-8, 1e-13])
def test_ill_conditioned_vertices(v, eps):
    """A turned square lattice of 900 points in a slab of thickness eps:
    the cells are tall columns whose corners split into short edges, and
    those vertices solve 3x3 systems with |det| / (|n_a||n_b||n_c|) of order
    eps.  Every form against the oracle (itself pinned on such a set by the
    exact brute force), the FP32 filter bitwise within a form; on the coarse
    grid the grouped forms keep the columns apart from the cells with a
    side decision in the exact predicate's band (some at eps = 1e-8, all at
    1e-13), which they leave to the one-cell kernel, as they leave extended
    cells on the default grid."""
    x = W.thin_lattice(30, eps, spacing=0.025)
    box = ([0] * 3, [1] * 3, [0] * 3)
    r = oracle.Oracle(x, *box).cells()
    for grid in (None, [3, 3, 1]):
        kw = {} if grid is None else dict(grid=grid)
        for form in (dict(), dict(slots=4), dict(cells_per_wave=2), dict(cells_per_wave=4)):
            g = run(v, x, *box, **kw, **form)
            assert_parity(g, r)
            same_bits(g, run(v, x, *box, precision=v.VC_F32_FILTER, **kw, **form))
            if grid is not None and form.get("cells_per_wave", 1) > 1:
                assert g["diag"]["spilled"] == np.sum(g["status"] == v.VC_CELL_SPILLED)
                assert 0 < g["diag"]["spilled"] < len(x) if eps == 1e-8 else g["diag"]["spilled"] == len(x)
