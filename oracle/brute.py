"""Exact brute-force Voronoi cells for tiny inputs -- TEST INFRASTRUCTURE ONLY.

The cell of particle i is the intersection of its initial box (section 2.1.2,
Eq. 1-2) with the kept half-spaces r.q <= q.q/2 (Eq. 3) of EVERY other
particle and every periodic image within two box lengths; no grid, no radius
bound, no block bound.  All arithmetic is exact (fractions.Fraction of the
FP64 inputs, with the relative vector q = fl(fl(x_j - x_i) + s L) as the data
of each plane).  A vertex is a point plus the set of planes it lies on; two
vertices are joined by an edge when they share two planes.

This is independent of the C oracle and of the GPU library (different
representation, different algorithm, exact arithmetic throughout) and is used
to pin both on inputs of at most ~50 particles.
"""
import math
from fractions import Fraction as Fr
from itertools import product

import numpy as np


def _shift_code(s):
    s = list(s) + [0] * (3 - len(s))
    return 25 * (s[2] + 2) + 5 * (s[1] + 2) + (s[0] + 2)


def _box_offset(p, lo, hi, periodic, d, side):
    """The domain's plane on one side of axis d, as a positive offset in the
    cell's frame (the FP64 value, as the inputs define it)."""
    if periodic[d]:
        return 0.5 * (float(hi[d]) - float(lo[d]))
    return float(hi[d]) - p[d] if side else -(float(lo[d]) - p[d])


def _planes(xyz, i, lo, hi, periodic, clip=0.0, radii=None):
    dim = xyz.shape[1]
    p = xyz[i]
    # radical planes: |x|^2 - ri^2 <= |x - q|^2 - rj^2, i.e. x.q <= (q.q + ri^2 - rj^2) / 2
    rr = None if radii is None else [Fr(float(r)) * Fr(float(r)) for r in radii]
    planes = []  # (normal tuple of Fr, offset Fr, label, image code, float |q|^2)
    # box planes: walls, or bisectors with own images at +-L e_d; with
    # clipping, a clip wall at h/2 on every side where it lies strictly inside
    for d in range(dim):
        for side in (0, 1):
            n = [Fr(0)] * dim
            if clip > 0 and 0.5 * clip < _box_offset(p, lo, hi, periodic, d, side):
                n[d] = Fr(1) if side else Fr(-1)
                planes.append((tuple(n), Fr(clip) / 2, -(7 + 2 * d + side), _shift_code([0] * dim), 0.0))
            elif periodic[d]:
                L = float(hi[d]) - float(lo[d])
                n[d] = Fr(L) if side else -Fr(L)
                h = Fr(L) * Fr(L) / 2
                sh = [0] * dim
                sh[d] = 1 if side else -1
                planes.append((tuple(n), h, i, _shift_code(sh), L * L))
            else:
                n[d] = Fr(1) if side else Fr(-1)
                h = Fr(float(hi[d]) - p[d]) if side else -Fr(float(lo[d]) - p[d])
                planes.append((tuple(n), h, -(2 * d + side + 1), _shift_code([0] * dim), 0.0))
    rng = [range(-2, 3) if periodic[d] else range(0, 1) for d in range(dim)]
    for j in range(len(xyz)):
        for s in product(*rng):
            if j == i and not any(s):
                continue
            if j == i and sum(abs(t) for t in s) == 1:
                continue  # the own images at +-L e_d are the box planes already
            q = []
            for d in range(dim):
                v = float(xyz[j, d]) - float(p[d])
                if s[d]:
                    v = v + s[d] * (float(hi[d]) - float(lo[d]))
                q.append(v)
            qf = [Fr(v) for v in q]
            h = sum(v * v for v in qf) / 2
            if rr is not None:
                h += (rr[i] - rr[j]) / 2
            planes.append((tuple(qf), h, j, _shift_code(s), float(sum(v * v for v in q))))
    return planes


def cell(xyz, i, lo, hi, periodic, clip=0.0, radii=None):
    """Exact cell of particle i (clipped by the cube of side `clip` centred
    on the particle when clip > 0; the radical cell when radii are given).
    Returns dict(vol, cen, nv, ne, nf, fo, nbr, empty, sizes, and in 2D perim,
    the sum of the edge lengths, each the square root of its exact square) with vol and cen as
    Fractions and nbr sorted (label, image) pairs."""
    xyz = np.asarray(xyz, dtype=np.float64)
    dim = xyz.shape[1]
    p = xyz[i]
    planes = _planes(xyz, i, lo, hi, periodic, clip, radii)
    # initial box: corners tight at one plane per axis (its offset along d)
    ext = []
    for d in range(dim):
        lo_pl, hi_pl = planes[2 * d], planes[2 * d + 1]
        ext.append((-lo_pl[1] / abs(lo_pl[0][d]), hi_pl[1] / abs(hi_pl[0][d])))
    verts = []
    for bits in product((0, 1), repeat=dim):
        pt = tuple(ext[d][bits[d]] for d in range(dim))
        verts.append((pt, frozenset(2 * d + bits[d] for d in range(dim))))
    order = sorted(range(2 * dim, len(planes)), key=lambda k: planes[k][4])
    need = dim - 1  # shared planes that make an edge (3D) / shared line (2D)
    for k in order:
        n, h = planes[k][0], planes[k][1]
        # float prefilter: skip planes that are clearly away from every vertex
        nf = [float(c) for c in n]
        hf = float(h)
        smax = -np.inf
        for pt, _ in verts:
            pf = [float(c) for c in pt]
            s = sum(a * b for a, b in zip(nf, pf)) - hf
            scale = sum(abs(a * b) for a, b in zip(nf, pf)) + abs(hf)
            smax = max(smax, s + 1e-9 * scale)
        if smax < 0:
            continue
        ss = [sum(a * b for a, b in zip(n, pt)) - h for pt, _ in verts]
        if max(ss) <= 0:
            verts = [(pt, tg | {k}) if s == 0 else (pt, tg) for (pt, tg), s in zip(verts, ss)]
            continue
        if min(ss) >= 0:
            # no vertex strictly inside: nothing with volume is left
            return dict(vol=Fr(0), cen=tuple(Fr(0) for _ in range(dim)), nv=0, ne=0, nf=0, fo=[0] * 32,
                        nbr=[], empty=True)
        new = []
        for (pt, tg), s in zip(verts, ss):
            if s < 0:
                new.append((pt, tg))
            elif s == 0:
                new.append((pt, tg | {k}))
        for a in range(len(verts)):
            if ss[a] >= 0:
                continue
            for b in range(len(verts)):
                if ss[b] <= 0:
                    continue
                common = verts[a][1] & verts[b][1]
                if len(common) < need:
                    continue
                t = ss[a] / (ss[a] - ss[b])
                pa, pb = verts[a][0], verts[b][0]
                pt = tuple(pa[d] + t * (pb[d] - pa[d]) for d in range(dim))
                new.append((pt, frozenset(common | {k})))
        verts = new
    return _stats(verts, planes, dim)


def _stats(verts, planes, dim):
    nv = len(verts)
    need = dim - 1
    edges = [(a, b) for a in range(nv) for b in range(a + 1, nv) if len(verts[a][1] & verts[b][1]) >= need]
    faces = {}
    for idx, (_, tg) in enumerate(verts):
        for k in tg:
            faces.setdefault(k, []).append(idx)
    if dim == 3:
        faces = {k: v for k, v in faces.items() if len(v) >= 3}
    else:
        faces = {k: v for k, v in faces.items() if len(v) >= 2}
    vol = Fr(0)
    cen = [Fr(0)] * dim
    fo = [0] * 32
    perim = []  # 2D: edge lengths, each the square root of an exact square
    for k, vs in faces.items():
        pts = [verts[v][0] for v in vs]
        # signed pieces (origin, face): the particle need not lie inside its
        # cell (radical cells), so each face is oriented by its outward normal
        n = planes[k][0]
        if dim == 3:
            ring = _ring(pts, n)
            if len(pts) < 32:
                fo[len(pts)] += 1
            a = ring[0]
            u = [ring[1][d] - a[d] for d in range(3)]
            w = [ring[2][d] - a[d] for d in range(3)]
            tn = (u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0])
            sgn = 1 if sum(tn[d] * n[d] for d in range(3)) > 0 else -1
            for t in range(1, len(ring) - 1):
                b, c = ring[t], ring[t + 1]
                det = (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0])
                       + a[2] * (b[0] * c[1] - b[1] * c[0]))
                tv = sgn * det / 6
                vol += tv
                for d in range(3):
                    cen[d] += tv * (a[d] + b[d] + c[d]) / 4
        else:
            a, b = pts
            # traverse the edge so that its outward normal is on the right
            if (b[1] - a[1]) * n[0] - (b[0] - a[0]) * n[1] < 0:
                a, b = b, a
            tri = (a[0] * b[1] - a[1] * b[0]) / 2
            vol += tri
            perim.append(math.sqrt((b[0] - a[0]) ** 2 + (b[1] - a[1]) ** 2))
            for d in range(2):
                cen[d] += tri * (a[d] + b[d]) / 3
    cen = [c / vol for c in cen]
    nbr = sorted((planes[k][2], planes[k][3]) for k in faces)
    ne = len(edges)
    sizes = sorted(len(vs) for vs in faces.values())
    out = dict(vol=vol, cen=cen, nv=nv, ne=ne if dim == 3 else nv, nf=len(faces), fo=fo, nbr=nbr, empty=False,
               sizes=sizes)
    if dim == 2:
        out["perim"] = math.fsum(perim)
    return out


def _ring(pts, normal):
    """Order the vertices of a convex planar polygon around its centroid
    (exact comparisons against the plane normal)."""
    m = len(pts)
    c = tuple(sum(p[d] for p in pts) / m for d in range(3))
    rel = [tuple(p[d] - c[d] for d in range(3)) for p in pts]
    ref = rel[0]

    def cross(u, v):
        return (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])

    def side(u):
        # 0: on the half-turn starting at ref (inclusive), 1: the other half
        s = sum(a * b for a, b in zip(cross(ref, u), normal))
        if s > 0:
            return 0
        if s < 0:
            return 1
        return 0 if sum(a * b for a, b in zip(ref, u)) > 0 else 1

    import functools

    def cmp(i, j):
        si, sj = side(rel[i]), side(rel[j])
        if si != sj:
            return si - sj
        s = sum(a * b for a, b in zip(cross(rel[i], rel[j]), normal))
        return -1 if s > 0 else (1 if s < 0 else 0)

    order = sorted(range(m), key=functools.cmp_to_key(cmp))
    return [pts[k] for k in order]
