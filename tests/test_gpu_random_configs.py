"""Random configurations against the FP64 oracle: dimension, periodicity per
axis, box position and shape, grids of 1 to 12 blocks per axis (so the
search wraps periodic images and runs the block bound's shell search), 5 to
3,000 points (eight sets of 5 to 39 points on grids of 1 to 3 blocks), with
and without a clip cube and radii.  Every cell, every
launch form (one, two and four 3D cells per wave)."""
import numpy as np
import pytest

import oracle
from paper_2209_11606_amd import workloads as W
from test_gpu_2d import parity2
from test_gpu_parity import assert_parity
from test_gpu_radical import assert_radical, run as rrun

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def v():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_11606_amd import vorohip
    return vorohip


def config(seed):
    rng = np.random.default_rng(7000 + seed)
    dim = 2 if seed % 3 == 0 else 3
    tiny = seed >= 24
    n = int(rng.integers(5, 40)) if tiny else int(rng.integers(5, 3000 if dim == 3 else 5000))
    per = [int(rng.random() < 0.5) for _ in range(dim)]
    lo = rng.uniform(-2.0, 2.0, dim)
    side = rng.uniform(0.5, 3.0, dim)
    hi = lo + side
    x = lo + W.rng(8000 + seed).random((n, dim)) * side
    x = np.minimum(x, np.nextafter(hi, lo))
    grid = [int(rng.integers(1, 4 if tiny else 13)) for _ in range(dim)]
    spacing = (np.prod(side) / n) ** (1.0 / dim)
    clip = float(rng.uniform(1.0, 4.0) * spacing) if rng.random() < 0.3 else 0.0
    radii = rng.random(n) * rng.uniform(0.3, 1.0) * spacing if rng.random() < 0.3 else None
    return dim, x, list(lo), list(hi), per, grid, clip, radii


@pytest.mark.parametrize("seed", range(32))
def test_random_config(v, seed):
    dim, x, lo, hi, per, grid, clip, radii = config(seed)
    r = oracle.Oracle(x, lo, hi, per, grid=grid, clip=clip, radii=radii).cells(nthreads=8)
    forms = (1, 2, 4) if dim == 3 else (1,)
    for cpw in forms:
        opt = dict(grid=grid, cells_per_wave=cpw)
        if clip:
            opt["clip"] = clip
        g = rrun(v, x, lo, hi, per, radii, **opt)
        print(f"seed {seed}: dim {dim} n {len(x)} per {per} grid {grid} clip {clip:.3g} "
              f"radii {radii is not None} cpw {cpw} fallback {g['diag']['fallback']}", flush=True)
        if radii is not None:
            assert_radical(g, r, dim, v)
        elif dim == 2:
            parity2(g, r)
        else:
            assert_parity(g, r)
