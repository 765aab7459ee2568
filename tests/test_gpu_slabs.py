"""The chunked form (vc_tessellate_slabs): the cells of one set computed in
container-block chunks along z, each chunk's container holding its layers of
blocks and a halo, against the whole-set computation and the oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_2209_11606_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FIELDS = ("nv", "ne", "nf", "fo", "status")


@pytest.fixture(scope="module")
def v():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_11606_amd import vorohip
    return vorohip


def mask(v):
    return v.VC_VOLUME | v.VC_CENTROID | v.VC_COUNTS | v.VC_FACE_ORDERS | v.VC_NEIGHBOR_COUNT


def whole(v, x, lo, hi, per, **kw):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    return v.tessellate(xt, lo, hi, per, mask(v), **kw)


def slabs(v, x, lo, hi, per, nslab, halo, on_host=False, **kw):
    o = v.vc_options_init(3, lo, hi, per, **kw)
    xs = np.ascontiguousarray(x) if on_host else torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    r = v.vc_tessellate_slabs(xs, o, mask(v), nslab, halo)
    try:
        out = v.fetch(r, mask(v), len(x))
        out["diag"] = dict(zip(v.DIAG_NAMES, v.vc_result_copy(r, v.VC_F_DIAG)[:len(v.DIAG_NAMES)].tolist()))
        out["ms"] = v.vc_result_kernel_ms(r)
    finally:
        v.vc_result_destroy(r)
    return out


def same(a, b, bitwise_share=0.0):
    """Topology, face orders and status equal; volume and centroid to
    rounding, and at least `bitwise_share` of the volumes bit for bit."""
    for k in FIELDS:
        bad = np.nonzero(np.asarray(a[k]) != np.asarray(b[k]))[0]
        assert len(bad) == 0, (k, bad[:5])
    rel = np.abs(a["vol"] - b["vol"]) / b["vol"]
    assert rel.max() <= 1e-12, rel.max()
    scale = b["vol"] ** (1 / 3)
    assert (np.abs(a["cen"] - b["cen"]).max(1) / scale).max() <= 1e-12
    assert np.mean(a["vol"] == b["vol"]) >= bitwise_share


@pytest.mark.parametrize("nslab,halo", [(5, 3), (7, 1)])
def test_periodic_against_whole_set(v, nslab, halo):
    """A periodic uniform set (58^3 grid): every cell equal to the
    whole-set computation's.  With one layer of halo many cells' search
    radii reach past their chunk's range and are computed again."""
    n = 200_000
    side = n ** (1 / 3)
    x = W.uniform(n, 3, side, 41)
    box = ([0] * 3, [side] * 3, [1, 1, 1])
    ref = whole(v, x, *box, cells_per_wave=2)
    got = slabs(v, x, *box, nslab, halo, cells_per_wave=2)
    print("chunks", nslab, "halo", halo, "recomputed", got["diag"]["recomputed"], flush=True)
    same(got, ref, bitwise_share=0.99)
    if halo == 1:
        assert got["diag"]["recomputed"] > 0
    assert math.fsum(got["vol"]) == pytest.approx(side ** 3, rel=1e-12)


def test_walled_and_forms(v):
    """Walls along z (the end chunks have no halo beyond the walls), the
    one-cell and grouped forms and the FP32 filter, and positions on the
    host; sampled cells against the oracle."""
    n = 60_000
    x = W.uniform(n, 3, 1.0, 43)
    box = ([0] * 3, [1] * 3, [0, 0, 0])
    ref = whole(v, x, *box)
    for kw in (dict(), dict(cells_per_wave=2), dict(cells_per_wave=2, precision=v.VC_F32_FILTER)):
        got = slabs(v, x, *box, 4, 2, **kw)
        same(got, ref)
    got = slabs(v, x, *box, 3, 1, on_host=True, cells_per_wave=2)
    same(got, ref)
    idx = np.random.default_rng(5).choice(n, 400, replace=False)
    r = oracle.Oracle(x, *box).cells(idx, nthreads=oracle.num_threads())
    for k in ("nv", "ne", "nf"):
        assert np.array_equal(got[k][idx], r[k])
    assert np.array_equal(got["fo"][idx], r["fo"])
    assert np.max(np.abs(got["vol"][idx] - r["vol"]) / r["vol"]) <= 1e-12


def test_one_chunk_is_the_whole_set(v):
    """One chunk (its halo covers every layer: no certificate) gives the
    whole-set computation bit for bit; so does a halo wider than the set."""
    n = 30_000
    side = n ** (1 / 3)
    x = W.uniform(n, 3, side, 44)
    box = ([0] * 3, [side] * 3, [1, 0, 1])
    ref = whole(v, x, *box, cells_per_wave=2)
    for nslab, halo in ((1, 1), (3, 40)):
        got = slabs(v, x, *box, nslab, halo, cells_per_wave=2)
        same(got, ref, bitwise_share=1.0)
        assert got["diag"]["recomputed"] == 0


def test_clustered_and_empty_chunks(v):
    """Points crowding the plane z = 1/2 (extreme clustering) in a walled box,
    16 chunks: most chunks hold few particles or none, and the cells near the
    walls reach far; every cell equals the whole-set one."""
    w = W.clustered(40_000)
    box = (w["lo"], w["hi"], w["periodic"])
    ref = whole(v, w["xyz"], *box, grid=w["grid"])
    got = slabs(v, w["xyz"], *box, 16, 1, grid=w["grid"])
    print("clustered recomputed", got["diag"]["recomputed"], flush=True)
    same(got, ref)


def test_range_error(v):
    """A coordinate outside the box is VC_E_RANGE, as for a container."""
    x = W.uniform(1000, 3, 1.0, 45)
    x[17, 2] = 1.5
    o = v.vc_options_init(3, [0] * 3, [1] * 3, [0, 0, 0])
    with pytest.raises(v.VcError) as e:
        v.vc_tessellate_slabs(torch.from_numpy(x).to("cuda:0"), o, mask(v), 2, 1)
    assert e.value.code == v.VC_E_RANGE
