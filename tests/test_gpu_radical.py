"""Radical (power) tessellation of a polydisperse container (section 2.1.1)
on the GPU, through the C ABI (vc_container_set_radii), against the FP64
oracle and the exact brute force: identical topology and empty-cell set,
volumes and centroids within the bound derived below."""
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


def run(v, x, lo, hi, per, radii, **opt):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    mask = v.VC_ALL | (v.VC_PERIMETER if x.shape[1] == 2 else 0)
    out = v.tessellate(xt, lo, hi, per, mask, radii=radii, **opt)
    out["nbr"] = v.neighbor_lists(out)
    return out


def assert_radical(g, r, dim, v):
    """Empty cells: the same set, status VC_CELL_EMPTY, zero volume and no
    faces.  Other cells: identical topology and neighbours; volume within
    1e-12 relative plus 1e-14 s^d, centroid within 1e-12 of the cell's size
    plus 1e-12 s (s the mean spacing): radical cells can be slivers whose
    FP64 vertices are rounded relative to the coordinates, not to the
    sliver's thickness."""
    n = len(g["vol"])
    s = n ** (-1.0 / dim)
    empty = r["status"] == oracle.Oracle.EMPTY
    assert np.array_equal(g["status"] == v.VC_CELL_EMPTY, empty)
    assert np.all(g["status"][~empty] <= 1), np.unique(g["status"])
    assert np.all(g["vol"][empty] == 0) and np.all(g["nf"][empty] == 0) and np.all(g["nv"][empty] == 0)
    for key in ("nv", "ne", "nf"):
        bad = np.nonzero(g[key] != r[key])[0]
        assert len(bad) == 0, (key, bad[:5], g[key][bad[:5]], r[key][bad[:5]])
    if dim == 3:
        assert np.array_equal(g["fo"], r["fo"])
    for i in range(n):
        assert np.array_equal(g["nbr"][i], r["nbr"][i]), (i, g["nbr"][i].tolist(), r["nbr"][i].tolist())
    ok = ~empty
    dv = np.abs(g["vol"][ok] - r["vol"][ok])
    assert np.all(dv <= 1e-12 * r["vol"][ok] + 1e-14 * s ** dim), (dv / r["vol"][ok]).max()
    dc = np.abs(g["cen"][ok] - r["cen"][ok]).max(1)
    assert np.all(dc <= 1e-12 * r["vol"][ok] ** (1.0 / dim) + 1e-12 * s), dc.max()
    if dim == 2:
        assert np.all(np.abs(g["perim"][ok] - r["perim"][ok]) <= 1e-12 * r["perim"][ok])


@pytest.mark.parametrize("per", [[1, 1, 1], [0, 0, 0], [1, 0, 1]])
def test_radical_3d_all_forms(v, per):
    """Every launch form on 4000 points with radii up to one spacing (about
    8% empty cells); the FP32 filter stays bitwise identical within a form."""
    w = W.polydisperse(4000, 3, seed=81, rmax_frac=1.0, periodic=True)
    x, rad = w["xyz"], w["radii"]
    r = oracle.Oracle(x, [0] * 3, [1] * 3, per, radii=rad).cells(nthreads=8)
    assert 0.03 * 4000 < (r["status"] == 1).sum() < 0.2 * 4000
    assert math.fsum(r["vol"]) == pytest.approx(1.0, rel=1e-12)
    for cpw in (1, 2, 4):
        g = run(v, x, [0] * 3, [1] * 3, per, rad, cells_per_wave=cpw)
        assert_radical(g, r, 3, v)
        f = run(v, x, [0] * 3, [1] * 3, per, rad, cells_per_wave=cpw, precision=v.VC_F32_FILTER)
        for k in ("vol", "cen", "nv", "ne", "nf", "fo", "status", "nbr_off", "nbr_ids", "nbr_sh"):
            assert np.array_equal(g[k], f[k]), (cpw, k)


@pytest.mark.parametrize("per", [[1, 1], [0, 0], [0, 1]])
def test_radical_2d(v, per):
    w = W.polydisperse(6000, 2, seed=82, rmax_frac=0.8)
    x, rad = w["xyz"], w["radii"]
    r = oracle.Oracle(x, [0, 0], [1, 1], per, radii=rad).cells()
    assert (r["status"] == 1).sum() > 0
    for prec in (v.VC_FP64, v.VC_F32_FILTER):
        g = run(v, x, [0, 0], [1, 1], per, rad, precision=prec)
        assert_radical(g, r, 2, v)
    assert math.fsum(g["vol"]) == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("dim,per,seed", [(3, [1, 1, 1], 83), (3, [0, 0, 0], 84), (2, [1, 1], 85), (2, [0, 0], 86)])
def test_radical_tiny_brute_force(v, dim, per, seed):
    """Small sets against the exact rational brute force of the power
    diagram: the empty set and every face, directly."""
    n = 24 if dim == 3 else 40
    x = W.uniform(n, dim, 1.0, seed)
    rad = W.rng(seed + 50).random(n) * 1.2 * n ** (-1.0 / dim)
    g = run(v, x, [0] * dim, [1] * dim, per, rad)
    s = n ** (-1.0 / dim)
    empty = 0
    for i in range(n):
        b = brute.cell(x, i, [0] * dim, [1] * dim, per, radii=rad)
        assert (g["status"][i] == v.VC_CELL_EMPTY) == b["empty"], i
        empty += b["empty"]
        assert g["nv"][i] == b["nv"] and g["ne"][i] == b["ne"] and g["nf"][i] == b["nf"], i
        assert [tuple(t) for t in g["nbr"][i].tolist()] == [tuple(t) for t in b["nbr"]], i
        assert abs(g["vol"][i] - float(b["vol"])) <= 1e-13 * float(b["vol"]) + 1e-14 * s ** dim
    assert 0 < empty < n


def test_equal_radii_give_voronoi(v):
    """Equal radii: every radical plane is the bisector and the search bound
    2R (to 2^-40), so the cells are the Voronoi cells bit for bit; radii =
    None returns the container to Voronoi."""
    x = W.uniform(3000, 3, 1.0, 87)
    lo, hi, per = [0] * 3, [1] * 3, [1, 1, 1]
    xt = torch.from_numpy(x).to("cuda:0")
    for cpw in (1, 2):
        # the two kernels sum a cell's statistics in different orders
        base = v.tessellate(xt, lo, hi, per, v.VC_ALL, cells_per_wave=cpw)
        g = v.tessellate(xt, lo, hi, per, v.VC_ALL, radii=np.full(3000, 0.05), cells_per_wave=cpw)
        for k in ("vol", "nv", "ne", "nf", "fo", "nbr_off", "nbr_ids", "nbr_sh"):
            assert np.array_equal(g[k], base[k]), k
        assert np.abs(g["cen"] - base["cen"]).max() <= 1e-15
    o = v.vc_options_init(3, lo, hi, per, cells_per_wave=2)
    c = v.vc_container_create(xt, o)
    try:
        v.vc_container_set_radii(c, W.rng(1).random(3000) * 0.05)
        v.vc_container_set_radii(c, None)
        r = v.vc_result_create(c, v.VC_ALL)
        try:
            v.vc_compute(c, r)
            g = v.fetch(r, v.VC_ALL, 3000, 3)
        finally:
            v.vc_result_destroy(r)
    finally:
        v.vc_container_destroy(c)
    assert np.array_equal(g["vol"], base["vol"]) and np.array_equal(g["nbr_ids"], base["nbr_ids"])


def test_radii_follow_rebin_and_device_input(v):
    """Radii are kept by input index across vc_container_rebin; device radii
    are accepted; bad radii are rejected with VC_E_RANGE."""
    w = W.polydisperse(3000, 3, seed=88, rmax_frac=1.0)
    x, rad = w["xyz"], w["radii"]
    x2 = W.uniform(3000, 3, 1.0, 89)
    lo, hi, per = w["lo"], w["hi"], w["periodic"]
    o = v.vc_options_init(3, lo, hi, per, cells_per_wave=2)
    c = v.vc_container_create(torch.from_numpy(x).to("cuda:0"), o)
    try:
        v.vc_container_set_radii(c, torch.from_numpy(rad).to("cuda:0"))
        v.vc_container_rebin(c, torch.from_numpy(x2).to("cuda:0"))
        r = v.vc_result_create(c, v.VC_ALL)
        try:
            v.vc_compute(c, r)
            g = v.fetch(r, v.VC_ALL, 3000, 3)
        finally:
            v.vc_result_destroy(r)
        for bad in (-1.0, float("nan"), float("inf")):
            b = rad.copy()
            b[17] = bad
            with pytest.raises(v.VcError) as e:
                v.vc_container_set_radii(c, b)
            assert e.value.code == v.VC_E_RANGE
    finally:
        v.vc_container_destroy(c)
    g["nbr"] = v.neighbor_lists(g)
    ref = oracle.Oracle(x2, lo, hi, per, radii=rad).cells(nthreads=8)
    assert_radical(g, ref, 3, v)


def test_radical_batch(v):
    """A batch of polydisperse tessellations with one radius array over the
    whole batch: each member against the oracle."""
    members = [W.polydisperse(n, 3, seed=90 + t, rmax_frac=0.8, periodic=(t % 2 == 0)) for t, n in
               enumerate([500, 1200, 300, 2000])]
    xyz = np.concatenate([m["xyz"] for m in members])
    rad = np.concatenate([m["radii"] for m in members])
    offs = np.cumsum([0] + [len(m["xyz"]) for m in members]).astype(np.int64)
    opts = [v.vc_options_init(3, m["lo"], m["hi"], m["periodic"]) for m in members]
    st = torch.cuda.Stream()  # graph capture needs a stream of its own
    xt = torch.from_numpy(xyz).to("cuda:0")
    torch.cuda.synchronize()
    b = v.vc_batch_create(xt, offs, opts, st)
    try:
        v.vc_batch_set_radii(b, rad, st)
        r = v.vc_batch_result_create(b, v.VC_ALL)
        try:
            v.vc_batch_compute(b, r, True, st)
            v.vc_batch_compute(b, r, True, st)
            st.synchronize()
            g = v.fetch(r, v.VC_ALL, len(xyz), 3)
        finally:
            v.vc_result_destroy(r)
    finally:
        v.vc_batch_destroy(b)
    g["nbr"] = v.neighbor_lists(g)
    for t, m in enumerate(members):
        sl = slice(offs[t], offs[t + 1])
        sub = {k: g[k][sl] for k in ("vol", "cen", "nv", "ne", "nf", "fo", "status")}
        # neighbour labels of a batch are positions in the concatenation
        sub["nbr"] = [np.where(l[:, :1] >= 0, l - [offs[t], 0], l) for l in g["nbr"][sl]]
        ref = oracle.Oracle(m["xyz"], m["lo"], m["hi"], m["periodic"], radii=m["radii"]).cells()
        assert_radical(sub, ref, 3, v)
