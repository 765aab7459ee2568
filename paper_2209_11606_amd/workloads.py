"""Seeded synthetic particle sets shaped like the paper's workloads.

This module only draws positions; it holds none of the Voronoi arithmetic and
imports nothing else from the package, so both the GPU library's callers and
the oracle-based tests can use it.

All draws come from numpy's Philox counter-based generator with an explicit
seed.  The paper's own inputs are ``rand()`` uniform draws (section 3.1 and
the example listing of section 2.2.3), which cannot be reproduced; these stand in.
"""
import math

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.Philox(key=int(seed)))


def uniform(n, dim, side=1.0, seed=0):
    """n i.i.d. uniform points in [0, side)^dim (homogeneous case of section 3.1)."""
    x = rng(seed).random((n, dim)) * side
    # a product can round up to side itself; keep the half-open box
    x[x >= side] = np.nextafter(side, 0.0)
    return x


def fcc(cells, a=1.0, sigma=0.0, seed=0):
    """Face-centred cubic lattice of cells[0] x cells[1] x cells[2] cubic unit
    cells of edge a (4 sites each), with isotropic Gaussian displacement of
    standard deviation sigma per coordinate, wrapped into the periodic box
    [0, cells*a).  Returns (xyz, box_hi)."""
    cx, cy, cz = cells
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]]) + 0.25
    g = np.stack(np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij"), -1).reshape(-1, 1, 3)
    x = ((g + basis[None]) * a).reshape(-1, 3)
    hi = np.array([cx, cy, cz], float) * a
    if sigma > 0:
        x = x + rng(seed).normal(0.0, sigma, x.shape)
        x = _wrap(x, hi)
    return x, hi


def bcc(m, a=1.0, sigma=0.0, seed=0, periodic=True):
    """Body-centred cubic lattice, m^3 cubic cells of edge a, sites at
    (i+1/4, j+1/4, k+1/4) a and (i+3/4, j+3/4, k+3/4) a, Gaussian displacement
    sigma per coordinate.  Periodic sets are wrapped into [0, m a); walled sets
    are clipped back inside.  Returns (xyz, box_hi)."""
    basis = np.array([[.25, .25, .25], [.75, .75, .75]])
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 1, 3)
    x = ((g + basis[None]) * a).reshape(-1, 3)
    hi = np.full(3, m * a)
    if sigma > 0:
        x = x + rng(seed).normal(0.0, sigma, x.shape)
        if periodic:
            x = _wrap(x, hi)
        else:
            x = np.clip(x, 0.0, np.nextafter(hi, 0.0))
    return x, hi


def sc(m, a=1.0):
    """Simple cubic lattice, sites at (i+1/2, j+1/2, k+1/2) a in [0, m a)^3."""
    g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    return (g + 0.5) * a, np.full(3, m * a)


def _wrap(x, hi):
    x = np.mod(x, hi)
    x[x >= hi] = 0.0
    return x


# ---------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------

def walled_1k(seed=1):
    """1,000 uniform points in the walled unit cube."""
    return dict(name="walled_uniform_1k", xyz=uniform(1000, 3, 1.0, seed), lo=[0.0] * 3, hi=[1.0] * 3,
                periodic=[0, 0, 0])


def periodic_1m(seed=2, n=1_000_000, side=100.0):
    """1,000,000 uniform points in the periodic cube of side 100 (density 1)."""
    return dict(name="periodic_uniform_1M", xyz=uniform(n, 3, side, seed), lo=[0.0] * 3, hi=[side] * 3,
                periodic=[1, 1, 1])


def fcc_10m(seed=3, cells=(125, 125, 160), sigma=1e-3):
    """Perturbed FCC, 125 x 125 x 160 cubic cells of edge 1 (exactly 10^7 sites),
    displacement N(0, (1e-3 a)^2) per coordinate, periodic."""
    x, hi = fcc(cells, 1.0, sigma, seed)
    return dict(name="fcc_perturbed_10M", xyz=x, lo=[0.0] * 3, hi=list(hi), periodic=[1, 1, 1])


def periodic_2d_10m(seed=4, n=10_000_000):
    """10,000,000 uniform points in the periodic unit square."""
    return dict(name="periodic_uniform_2d_10M", xyz=uniform(n, 2, 1.0, seed), lo=[0.0] * 2, hi=[1.0] * 2,
                periodic=[1, 1])


def periodic_102m(seed=5, n=102_400_000):
    """102,400,000 uniform points in the periodic unit cube."""
    return dict(name="periodic_uniform_102M", xyz=uniform(n, 3, 1.0, seed), lo=[0.0] * 3, hi=[1.0] * 3,
                periodic=[1, 1, 1])


def localized(n_prime=10_000_000, dim=3, seed=6):
    """Localized case of section 3.1: n_prime uniform points in the walled unit
    box, keeping those inside the central cube (square) of volume (area) 0.1,
    about n_prime / 10 points.  The grid follows the paper's table for this
    case (N_opt 49 in 3D, 30 in 2D; n = floor((n_prime / N_opt)^(1/dim)),
    126^3 and 1825^2 for n_prime = 10^8), and clip is the side of the cube
    the paper clips each cell with in 3D, h = 1.5 sqrt(3) d0 with
    d0 = n_prime^(-1/3) (section 3.1.3)."""
    x = uniform(n_prime, dim, 1.0, seed)
    half = 0.5 * 0.1 ** (1.0 / dim)
    x = x[np.all(np.abs(x - 0.5) <= half, axis=1)]
    n_opt = 49.0 if dim == 3 else 30.0
    g = int(math.floor((n_prime / n_opt) ** (1.0 / dim)))
    clip = 1.5 * math.sqrt(3.0) * n_prime ** (-1.0 / 3.0) if dim == 3 else 0.0
    return dict(name=f"localized_{dim}d_{n_prime}", xyz=np.ascontiguousarray(x), lo=[0.0] * dim, hi=[1.0] * dim,
                periodic=[0] * dim, grid=[g] * dim, n_opt=n_opt, clip=clip)


def clustered(n=1_000_000, dim=3, seed=7):
    """Extreme clustering of section 3.1: each coordinate is 1/2 + 4 (X - 1/2)^3
    with X uniform on [0, 1), in the walled unit box, so points crowd the
    planes x = 1/2 (and y, z = 1/2).  N_opt = 0.5 as in the paper's table:
    n = floor((n / 0.5)^(1/dim)) blocks per axis (584 in 3D for 10^8)."""
    X = rng(seed).random((n, dim))
    x = 0.5 + 4.0 * (X - 0.5) ** 3
    g = int(math.floor((n / 0.5) ** (1.0 / dim)))
    return dict(name=f"clustered_{dim}d_{n}", xyz=x, lo=[0.0] * dim, hi=[1.0] * dim, periodic=[0] * dim,
                grid=[g] * dim, n_opt=0.5, clip=0.0)


def polydisperse(n=1_000_000, dim=3, seed=8, rmax_frac=0.6, periodic=True):
    """Polydisperse container for the radical tessellation (section 2.1.1):
    n uniform points in the unit box with radii uniform on [0, rmax_frac s),
    s = n^(-1/dim) the mean spacing.  The points are random, not a packing,
    so wide radii leave some small particles with empty cells: about 0.6%
    in 3D and 3% in 2D at rmax_frac 0.6, 8% in 3D at 1.0."""
    x = uniform(n, dim, 1.0, seed)
    rad = rng(seed + 1).random(n) * (rmax_frac * n ** (-1.0 / dim))
    per = [1 if periodic else 0] * dim
    return dict(name=f"polydisperse_{dim}d_{n}", xyz=x, radii=rad, lo=[0.0] * dim, hi=[1.0] * dim, periodic=per)


def vorotop(n=1_000_000, seed=10):
    """The VoroTop systems of section 5: n uniform points in the periodic unit
    cube, every cell with its Weinberg code."""
    return dict(name=f"vorotop_{n}", xyz=uniform(n, 3, 1.0, seed), lo=[0.0] * 3, hi=[1.0] * 3, periodic=[1, 1, 1],
                weinberg=True)


def batch_sizes(count=4096, lo=100, hi=100_000, seed=1000):
    """Log-uniform tessellation sizes round(exp(U[ln lo, ln hi]))."""
    u = rng(seed).random(count)
    return np.rint(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))).astype(np.int64)


def batch_member(t, n_t):
    """Tessellation t of the batch: a 2 x 2 design over {periodic, walled} x
    {uniform, perturbed BCC (sigma = 0.05 a)}, density 1.  BCC sets hold
    2 m^3 sites with m = max(2, round((n_t/2)^(1/3)))."""
    periodic = (t % 2) == 0
    lattice = (t // 2) % 2 == 1
    seed = 1000 + t
    if lattice:
        m = max(2, int(round((n_t / 2) ** (1.0 / 3.0))))
        a = 2.0 ** (1.0 / 3.0)
        x, hi = bcc(m, a, 0.05 * a, seed, periodic)
        side = float(hi[0])
    else:
        side = float(n_t) ** (1.0 / 3.0)
        x = uniform(int(n_t), 3, side, seed)
    per = [1, 1, 1] if periodic else [0, 0, 0]
    return dict(xyz=x, lo=[0.0] * 3, hi=[side] * 3, periodic=per,
                kind=("periodic" if periodic else "walled") + ("_bcc" if lattice else "_uniform"))


def batch(count=4096, seed=1000, lo=100, hi=100_000):
    """The batched workload: count tessellations of log-uniform sizes."""
    sizes = batch_sizes(count, lo, hi, seed)
    return [batch_member(t, int(s)) for t, s in enumerate(sizes)]


def ring_face(k=40, rho=0.2, delta=0.05):
    """A crafted set in the walled unit cube whose two first cells have faces
    of k edges: particles at (1/2, 1/2, 1/2 -+ delta) and a ring of k
    particles at distance rho from the axis in the plane z = 1/2.  The face
    between the two axial particles lies in that plane and is bounded by one
    edge per ring particle (a k-gon of inradius (rho^2 - delta^2) / (2 rho));
    each axial cell also has a k-gon face on the wall beyond it."""
    t = 2.0 * math.pi * np.arange(k) / k
    ring = np.stack([0.5 + rho * np.cos(t), 0.5 + rho * np.sin(t), np.full(k, 0.5)], 1)
    axis = np.array([[0.5, 0.5, 0.5 - delta], [0.5, 0.5, 0.5 + delta]])
    return np.concatenate([axis, ring])


def thin_lattice(k=5, eps=1e-13, spacing=0.17, theta=0.3, seed=5):
    """A crafted set for ill-conditioned vertices, in the walled unit cube: a
    k x k square lattice (spacing `spacing`, turned by `theta` about the z
    axis, centred) in the plane z = 1/2, each point moved along z by up to
    eps/2.  Four lattice points around a square are cocircular in the plane,
    so the cells meet in tall columns whose corners split into short edges,
    and the three nearly vertical bisector planes of such a vertex have
    normals within about eps of one plane: the vertex's 3x3 system has
    |det| / (|n_a| |n_b| |n_c|) of order eps."""
    g = (np.arange(k) - (k - 1) / 2) * spacing
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = 0.5 + np.cos(theta) * X.ravel() - np.sin(theta) * Y.ravel()
    y = 0.5 + np.sin(theta) * X.ravel() + np.cos(theta) * Y.ravel()
    z = 0.5 + eps * (rng(seed).random(k * k) - 0.5)
    return np.ascontiguousarray(np.stack([x, y, z], 1))
