"""The side predicate of the 3D cell kernels on the host, against exact
rationals.

The kernels decide the side of a candidate plane at a vertex (the
intersection of three planes) from the sign of
    s * D(a,b,c) = h_a D(b,c,p) - h_b D(a,c,p) + h_c D(a,b,p) - h_p D(a,b,c)
(Cramer's rule for the vertex of the bisectors of Eq. 3, or of the radical
planes of section 2.1.1, multiplied out).  The predicate's code in the
kernels' common header (the floating-point expansions, their compression and
the double-word stage in front of them) is compiled for the host here and
its signs are compared with the same expression in Python fractions on
near-degenerate and exactly degenerate configurations.  The double-word
stage must decide every configuration whose exact value is not zero, and
leave every exact zero to the expansions."""
import os
import random
import shutil
import subprocess
from fractions import Fraction as F

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "..", "paper_2209_11606_amd", "csrc", "cell_common.h")

HARNESS = r"""
#include <cstdio>
#include <cmath>
#define __device__
#define __noinline__
#define __forceinline__ inline
using std::fabs;
%s
static double ws[8192];
template <class P>
static void run(P *pl) {
    const P *r[4] = {&pl[0], &pl[1], &pl[2], &pl[3]};
    double nv[4][3];
    for (int i = 0; i < 4; i++) {
        nv[i][0] = plane_base(pl[i]).n0;
        nv[i][1] = plane_base(pl[i]).n1;
        nv[i][2] = plane_base(pl[i]).n2;
    }
    const int quick = dw_side3<P>(r, nv);
    const int full = exact_side3(pl[0], pl[1], pl[2], pl[3], ws);
    printf("%%d %%d\n", full, quick);
}
int main() {
    int rad;
    while (scanf("%%d", &rad) == 1) {
        PlaneD d[4];
        PlaneR q[4];
        double ri;
        for (int i = 0; i < 4; i++) {
            double n0, n1, n2, h, rj;
            int wall;
            if (scanf("%%la %%la %%la %%d %%la %%la", &n0, &n1, &n2, &wall, &h, &rj) != 6) return 1;
            d[i] = PlaneD{n0, n1, n2, h, wall};
            q[i].p = d[i];
            q[i].rj = rj;
        }
        if (scanf("%%la", &ri) != 1) return 1;
        for (int i = 0; i < 4; i++) q[i].ri = ri;
        if (rad) run(q); else run(d);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def predicate(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    src = open(HEADER).read()
    a = src.index("struct PlaneD {")
    b = src.index("// Exact sign of n_p.v - h_p at the 2D vertex")
    d = tmp_path_factory.mktemp("pred")
    cpp, exe = d / "pred.cpp", d / "pred"
    cpp.write_text(HARNESS % src[a:b])
    subprocess.run([gxx, "-O2", "-std=c++17", "-ffp-contract=off", "-o", str(exe), str(cpp)], check=True)

    def call(cases):
        lines = []
        for rad, planes, ri in cases:
            toks = [str(int(rad))]
            for (n, wall, h, rj) in planes:
                toks += [float(n[0]).hex(), float(n[1]).hex(), float(n[2]).hex(), str(int(wall)), float(h).hex(),
                         float(rj).hex()]
            toks.append(float(ri).hex())
            lines.append(" ".join(toks))
        out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
        return [tuple(map(int, l.split())) for l in out.stdout.split("\n") if l.strip()]
    return call


def det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def exact_sign(rad, planes, ri):
    """sign(s * D) * sign(D) in rationals: the side of plane p at the vertex
    of planes a, b, c (zero: on the plane, or no vertex)."""
    n = [[F(float(x)) for x in p[0]] for p in planes]
    h = []
    for (nv, wall, hw, rj), nf in zip(planes, n):
        if wall:
            h.append(F(float(hw)))
        else:
            v = sum(x * x for x in nf)
            if rad:
                v += F(float(ri)) ** 2 - F(float(rj)) ** 2
            h.append(v / 2)
    mi = [[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]]
    num = sum((-1) ** i * h[i] * det3([n[j] for j in mi[i]]) for i in range(4))
    den = det3(n[:3])
    return ((num > 0) - (num < 0)) * ((den > 0) - (den < 0))


def near_tie(rng, scale, rel):
    """Three random bisector normals and a fourth whose plane passes through
    their vertex up to rounding, optionally moved by a relative amount."""
    q = rng.normal(size=(3, 3)) * scale
    v = np.linalg.solve(q, 0.5 * (q * q).sum(1))
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    qp = (v + np.linalg.norm(v) * d) * (1.0 + rel)
    return [(row, 0, 0.0, 0.0) for row in np.vstack([q, qp])]


def test_voronoi_near_and_exact_ties(predicate):
    rng = np.random.default_rng(11)
    cases = []
    for t in range(1500):
        kind = t % 3
        if kind == 0:
            planes = near_tie(rng, 10.0 ** rng.uniform(-3, 3), 0.0)
        elif kind == 1:
            planes = near_tie(rng, 1.0, rng.choice([-1, 1]) * 10.0 ** rng.uniform(-15, -6))
        else:
            # lattice neighbours: small integer vectors, many exact ties
            while True:
                q = rng.integers(-2, 3, size=(4, 3)).astype(float)
                if all(np.any(row != 0) for row in q):
                    break
            planes = [(row, 0, 0.0, 0.0) for row in q]
        cases.append((False, planes, 0.0))
    got = predicate(cases)
    zeros = 0
    for (rad, planes, ri), (full, quick) in zip(cases, got):
        want = exact_sign(rad, planes, ri)
        assert full == want
        if want == 0:
            zeros += 1
            assert quick == 2
        else:
            assert quick == want
    assert zeros > 50


def test_walls_and_radical_planes(predicate):
    """Walls (axis normals, offsets as given) and radical planes
    (h = (q.q + ri^2 - rj^2) / 2) in the same expression."""
    rng = np.random.default_rng(12)
    cases = []
    for t in range(900):
        planes = near_tie(rng, 1.0, 0.0 if t % 2 else 10.0 ** rng.uniform(-14, -7))
        if t % 3 == 0:
            axis = int(rng.integers(3))
            nrm = np.zeros(3)
            nrm[axis] = rng.choice([-1.0, 1.0])
            k = int(rng.integers(4))
            planes[k] = (nrm, 1, float(rng.uniform(0.1, 2.0)), 0.0)
        rad = t % 3 == 1
        ri = float(rng.uniform(0.0, 0.3)) if rad else 0.0
        if rad:
            planes = [(n, w, h, 0.0 if w else float(rng.uniform(0.0, 0.3))) for (n, w, h, _) in planes]
        cases.append((rad, planes, ri))
    # exact zeros among radical planes: a lattice with equal radii
    for t in range(100):
        q = rng.integers(-2, 3, size=(4, 3)).astype(float)
        if not all(np.any(row != 0) for row in q):
            continue
        cases.append((True, [(row, 0, 0.0, 0.25) for row in q], 0.25))
    got = predicate(cases)
    for (rad, planes, ri), (full, quick) in zip(cases, got):
        want = exact_sign(rad, planes, ri)
        assert full == want
        assert quick == (2 if want == 0 else want)


def test_expansion_compression(predicate):
    """Long sums through the expansions (the double-word stage cannot decide
    an exact zero): lattice configurations scaled by powers of two far apart
    keep the exact zero, and one ulp moved off it gives the sign."""
    rng = random.Random(13)
    cases, wants = [], []
    for t in range(300):
        while True:
            q = np.array([[rng.randint(-3, 3) for _ in range(3)] for _ in range(4)], float)
            if all(np.any(row != 0) for row in q):
                break
        s = 2.0 ** rng.randint(-40, 40)
        q = q * s
        if t % 2:
            i, d = rng.randrange(4), rng.randrange(3)
            q[i][d] = np.nextafter(q[i][d], np.inf)
        planes = [(row, 0, 0.0, 0.0) for row in q]
        cases.append((False, planes, 0.0))
    got = predicate(cases)
    for (rad, planes, ri), (full, quick) in zip(cases, got):
        assert full == exact_sign(rad, planes, ri)
