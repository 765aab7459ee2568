"""Clipped cells (section 3.1.3) and the imbalanced workloads of section 3.1
(localized and extreme clustering) on the GPU, through the C ABI, against
the FP64 oracle: identical topology (clip faces carry labels -7..-12),
volumes and centroids within 1e-12."""
import math

import numpy as np
import pytest

import oracle
from paper_2209_11606_amd import workloads as W
from test_gpu_2d import parity2
from test_gpu_parity import assert_parity, run, same_bits

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def v():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_11606_amd import vorohip
    return vorohip


@pytest.mark.parametrize("per", [[0, 0, 0], [1, 1, 1], [1, 0, 1]])
def test_clipped_3d_all_forms(v, per):
    """Every launch form on a set where about half the cells reach their
    clip cube; the FP32 filter stays bitwise identical within a form."""
    n = 3000
    x = W.uniform(n, 3, 1.0, 71)
    h = 1.9 * n ** (-1.0 / 3.0)
    r = oracle.Oracle(x, [0] * 3, [1] * 3, per, clip=h).cells(nthreads=8)
    clipped = sum(bool(np.any(l[:, 0] <= -7)) for l in r["nbr"])
    assert 0.1 * n < clipped < 0.9 * n
    for cpw in (1, 2, 4):
        g = run(v, x, [0] * 3, [1] * 3, per, clip=h, cells_per_wave=cpw)
        assert_parity(g, r)
        f = run(v, x, [0] * 3, [1] * 3, per, clip=h, cells_per_wave=cpw, precision=v.VC_F32_FILTER)
        same_bits(g, f)


def test_clipped_2d(v):
    x = W.uniform(5000, 2, 1.0, 72)
    h = 2.0 / math.sqrt(5000)
    for per in ([0, 0], [1, 1]):
        r = oracle.Oracle(x, [0, 0], [1, 1], per, clip=h).cells()
        assert any(bool(np.any(l[:, 0] <= -7)) for l in r["nbr"])
        xt = torch.from_numpy(x).to("cuda:0")
        g = v.tessellate(xt, [0, 0], [1, 1], per, v.VC_ALL | v.VC_PERIMETER, clip=h)
        g["nbr"] = v.neighbor_lists(g)
        parity2(g, r)


def test_clip_lattice_closed_form(v):
    """Simple-cubic lattice, clip side 0.8 < a: every cell is the clip cube."""
    x, hi = W.sc(6, 1.0)
    g = run(v, x, [0] * 3, hi, [1, 1, 1], clip=0.8)
    assert np.all(g["vol"] == 0.8 ** 3) and np.all(g["nf"] == 6)
    assert all(sorted(l[:, 0].tolist()) == [-12, -11, -10, -9, -8, -7] for l in g["nbr"])


@pytest.mark.parametrize("clip", [False, True])
def test_localized(v, clip):
    """The localized set (central cube of volume 0.1 of 2*10^5 uniform points,
    walled unit box, the paper's N_opt grid), with and without the paper's
    clip cube, every cell against the oracle."""
    w = W.localized(200_000)
    h = w["clip"] if clip else 0.0
    x = w["xyz"]
    r = oracle.Oracle(x, w["lo"], w["hi"], w["periodic"], grid=w["grid"], clip=h).cells(nthreads=8)
    for cpw in (1, 2):
        g = run(v, x, w["lo"], w["hi"], w["periodic"], grid=w["grid"], clip=h, cells_per_wave=cpw)
        assert_parity(g, r)
    if not clip:
        assert math.fsum(g["vol"]) == pytest.approx(1.0, rel=1e-12)


def test_extreme_clustering(v):
    """The extreme-clustering set (coordinates 1/2 + 4 (X - 1/2)^3, N_opt 0.5),
    every cell against the oracle, volumes tiling the box."""
    w = W.clustered(50_000)
    x = w["xyz"]
    r = oracle.Oracle(x, w["lo"], w["hi"], w["periodic"], grid=w["grid"]).cells(nthreads=8)
    for cpw in (1, 2):
        g = run(v, x, w["lo"], w["hi"], w["periodic"], grid=w["grid"], cells_per_wave=cpw)
        assert_parity(g, r)
    assert math.fsum(g["vol"]) == pytest.approx(1.0, rel=1e-12)


def test_clip_argument_errors(v):
    xt = torch.from_numpy(W.uniform(50, 3, 1.0, 3)).to("cuda:0")
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(v.VcError) as e:
            v.tessellate(xt, [0] * 3, [1] * 3, [0, 0, 0], clip=bad)
        assert e.value.code == v.VC_E_ARG


def test_subset_compute(v):
    """vc_compute_subset (the subset and ordered iterators of section 2.2.2):
    listed cells are bitwise the full computation's, in any order and from a
    host or device list; the others are VC_CELL_SKIPPED with empty neighbour
    lists; out-of-range indices are rejected before anything runs."""
    x = W.uniform(20_000, 3, 20_000 ** (1 / 3), 81)
    hi = [20_000 ** (1 / 3)] * 3
    xt = torch.from_numpy(x).to("cuda:0")
    full = v.tessellate(xt, [0] * 3, hi, [1, 1, 1], v.VC_ALL, cells_per_wave=2)
    ids = np.random.default_rng(3).permutation(20_000)[:2_500].astype(np.int64)
    o = v.vc_options_init(3, [0] * 3, hi, [1, 1, 1], cells_per_wave=2)
    c = v.vc_container_create(xt, o)
    r = v.vc_result_create(c, v.VC_ALL)
    try:
        for lst in (ids, torch.from_numpy(ids[::-1].copy()).to("cuda:0")):
            v.vc_compute_subset(c, r, lst)
            torch.cuda.synchronize()
            g = v.fetch(r, v.VC_ALL, 20_000)
            for k in ("vol", "cen", "nv", "ne", "nf", "fo", "status"):
                assert np.array_equal(g[k][ids], full[k][ids]), k
            skipped = np.ones(20_000, bool)
            skipped[ids] = False
            assert np.all(g["status"][skipped] == v.VC_CELL_SKIPPED)
            assert np.all(g["nf"][skipped] == 0)
            gl, fl = v.neighbor_lists(g), v.neighbor_lists(full)
            for i in ids[:200]:
                assert np.array_equal(gl[i], fl[i])
            assert all(len(gl[i]) == 0 for i in np.flatnonzero(skipped)[:200])
        v.vc_compute_subset(c, r, np.zeros(0, np.int64))
        assert np.all(v.fetch(r, v.VC_ALL, 20_000)["status"] == v.VC_CELL_SKIPPED)
        for bad in (np.array([5, 20_000]), torch.tensor([3, -1], dtype=torch.int64, device="cuda:0")):
            with pytest.raises(v.VcError) as e:
                v.vc_compute_subset(c, r, bad)
            assert e.value.code == v.VC_E_RANGE
        with pytest.raises(v.VcError) as e:
            v.vc_compute_subset(c, r, np.arange(20_001))
        assert e.value.code == v.VC_E_ARG
    finally:
        v.vc_result_destroy(r)
        v.vc_container_destroy(c)
