"""The block bound of the search (section 2.1.3) on the GPU, through the C
ABI.  Every set here has cells that reach far beyond the precomputed list of
block offsets, so that the Chebyshev shell search decides them: a lattice
with a closed form, and localized sets on fine grids (Voronoi and radical,
3D and 2D) against the FP64 oracle.  The lattice also checks where the
search ends: its shell count is the one the block bound gives, computed
here from the geometry, below the radius bound's."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2209_11606_amd import workloads as W
from test_gpu_2d import parity2
from test_gpu_parity import assert_parity, run, same_bits
from test_gpu_radical import assert_radical, run as rrun

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OFF_R = 4           # Chebyshev radius of the block-offset list
SAFETY = 2.0 ** -8  # widening of the balls' squared radii


@pytest.fixture(scope="module")
def v():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_11606_amd import vorohip
    return vorohip


def lattice_shells(frac, bs, a, r0):
    """Chebyshev shells r0, r0 + 1, ... searched for a particle at fraction
    frac of its block (block side bs) whose cell is the cube of side a, once
    the cube is final: under the radius bound (until the shell's inner gap
    reaches 2R) and under the bounding box of the balls B(v, |v|), radii
    widened as the kernels widen them (until a shell has no block meeting
    the box; that shell is searched too)."""
    rho = math.sqrt(3.0 * (a / 2) ** 2 * (1.0 + SAFETY)) * (1.0 + 2.0 ** -40)
    ext = a / 2 + rho  # the box is [-ext, ext] on every axis
    mrg = min(min(frac), 1.0 - max(frac)) * bs
    two_r = 2.0 * math.sqrt(3.0) * a / 2
    radius = next(r for r in range(r0, 1000) if (r - 1) * bs + mrg >= two_r) - r0

    def meets(r):
        # some block of shell r meets [-ext, ext]^3: on one axis at offset
        # +r or -r, the other axes anywhere within the shell
        return any((r - f) * bs < ext or (-r + 1 - f) * bs > -ext for f in frac)

    bound = next(r for r in range(r0, 1000) if not meets(r)) - r0 + 1
    return radius, bound


@pytest.mark.parametrize("cpw", [1, 2, 4])
def test_sc_lattice_fine_grid(v, cpw):
    """Simple-cubic lattice, 6^3 sites of spacing 1 in the periodic box of
    side 6 on an 87^3 grid: the spacing is 14.5 block sides, so the offset
    list (Chebyshev radius 4) holds no neighbour and every cell is found by
    the shell search.  Every cell is the unit cube with its six face
    neighbours.  The neighbours lie in shells 14 and 15; once the cube is
    final the bounding box of the balls ends the search after shell 21 (17
    shells searched), where the radius bound would go on to shell 25 (21)."""
    m, g = 6, 87
    x, hi = W.sc(m, 1.0)
    out = run(v, x, [0] * 3, hi, [1, 1, 1], grid=[g] * 3, cells_per_wave=cpw)
    n = m ** 3
    # the grouped forms leave extended cells to the one-cell kernel of the
    # spill pass after their first gather of 64 / cpw blocks
    spilled = cpw > 1
    assert np.all(out["status"] == (v.VC_CELL_SPILLED if spilled else v.VC_CELL_OK))
    assert np.all(out["nf"] == 6) and np.all(out["nv"] == 8) and np.all(out["ne"] == 12)
    assert np.all(np.abs(out["vol"] - 1.0) <= 1e-12)
    assert np.all(np.abs(out["cen"]) <= 1e-12)  # relative to the particle
    ijk = np.rint(x - 0.5).astype(int)
    for i in range(n):
        want = sorted(int(np.ravel_multi_index(tuple((ijk[i] + s) % m), (m, m, m)))
                      for s in ([1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]))
        assert sorted(out["nbr"][i][:, 0].tolist()) == want, i
    bs = 6.0 / g
    assert {tuple(np.round((x[i] / bs) % 1.0, 6)) for i in range(n)} <= set(itertools.product([0.25, 0.75], repeat=3))
    counts = {lattice_shells(f, bs, 1.0, OFF_R + 1) for f in itertools.product([0.25, 0.75], repeat=3)}
    assert counts == {(21, 17)}
    d = out["diag"]
    assert d["fallback"] == n and d["shells"] == 17 * n
    assert d["spilled"] == (n if spilled else 0)
    # blocks loaded: in the offset list every block of the first chunk of 64
    # (the first cell is the whole box), then, as the one-cell kernel
    # applies the block bound to the list once the cell is extended, only
    # non-empty blocks that meet the balls (none), then, in the shells, the
    # non-empty blocks that meet the balls, among those of the 26 nearest
    # sites; a grouped form first gathers its 64 / cpw nearest blocks
    near = 64 + (64 // cpw if spilled else 0)
    assert n * (near + 6) <= d["blocks"] <= n * (near + 26)
    # particles loaded: the cell's own (twice in a grouped form), then
    # those of the blocks loaded
    own = 2 if spilled else 1
    assert n * (6 + own) <= d["loaded"] <= n * (26 + own)


@pytest.mark.parametrize("radical", [False, True])
def test_localized_fine_grid(v, radical):
    """The localized set of 60,000 uniform points (about 6,000 in the
    central cube of volume 0.1) in the walled unit box on a 40^3 grid: the
    cells on the cluster's surface reach the walls, 10 or more blocks away,
    and their search runs to shell 20 and beyond.  Every cell against the
    oracle, every launch form; the FP32 filter bitwise identical within a
    form.  Radical: radii uniform on [0, 0.8 s), s the cluster's spacing."""
    w = W.localized(60_000)
    x = w["xyz"]
    n = len(x)
    grid = [40] * 3
    if radical:
        s = (0.1 / n) ** (1.0 / 3.0)
        rad = W.rng(91).random(n) * 0.8 * s
        r = oracle.Oracle(x, w["lo"], w["hi"], w["periodic"], grid=grid, radii=rad).cells(nthreads=8)
        for cpw in (1, 2, 4):
            g = rrun(v, x, w["lo"], w["hi"], w["periodic"], rad, grid=grid, cells_per_wave=cpw)
            assert_radical(g, r, 3, v)
            assert g["diag"]["fallback"] > 0.1 * n
    else:
        r = oracle.Oracle(x, w["lo"], w["hi"], w["periodic"], grid=grid).cells(nthreads=8)
        for cpw in (1, 2, 4):
            g = run(v, x, w["lo"], w["hi"], w["periodic"], grid=grid, cells_per_wave=cpw)
            assert_parity(g, r)
            assert g["diag"]["fallback"] > 0.1 * n
            f = run(v, x, w["lo"], w["hi"], w["periodic"], grid=grid, cells_per_wave=cpw,
                    precision=v.VC_F32_FILTER)
            same_bits(g, f)
    assert math.fsum(g["vol"]) == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("radical", [False, True])
def test_localized_2d_fine_grid(v, radical):
    """The 2D localized set (central square of area 0.1 of 60,000 uniform
    points) in the walled unit square on a 100^2 grid, every cell against
    the oracle; the surface cells search rings out to the walls."""
    w = W.localized(60_000, dim=2)
    x = w["xyz"]
    n = len(x)
    grid = [100, 100]
    rad = W.rng(92).random(n) * 0.8 * math.sqrt(0.1 / n) if radical else None
    r = oracle.Oracle(x, w["lo"], w["hi"], w["periodic"], grid=grid, radii=rad).cells()
    for prec in (v.VC_FP64, v.VC_F32_FILTER):
        if radical:
            g = rrun(v, x, w["lo"], w["hi"], w["periodic"], rad, grid=grid, precision=prec)
            assert_radical(g, r, 2, v)
        else:
            xt = torch.from_numpy(x).to("cuda:0")
            g = v.tessellate(xt, w["lo"], w["hi"], w["periodic"], v.VC_ALL | v.VC_PERIMETER, grid=grid,
                             precision=prec)
            g["nbr"] = v.neighbor_lists(g)
            parity2(g, r)
        assert g["diag"]["fallback"] > 0.02 * n
    assert math.fsum(g["vol"]) == pytest.approx(1.0, rel=1e-12)
