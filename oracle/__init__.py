"""Oracle -- TEST INFRASTRUCTURE ONLY.

A plain serial FP64 CPU implementation of the per-particle Voronoi cell
construction of Voro++ (Lu, Lazar & Rycroft, section 2.1), written in C
(``voro_oracle.c``) and loaded here with ctypes, plus an exact rational brute
force (``brute.py``).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and imports nothing from it.

Per-cell results (section 2.1.2 and the topology discussion of section 4):
volume, centroid relative to the particle, vertex / edge / face counts, the
face-order vector fo[k] = number of faces with k edges, and one neighbour label
(j, image code) per face.  Labels -1..-6 are the walls x-, x+, y-, y+, z-, z+,
-7..-12 the faces of the clip cube when cells are clipped (section 3.1.3);
the image code of a periodic shift s is 25(s_z+2) + 5(s_y+2) + (s_x+2).

Weinberg codes (the cell-topology code of VoroTop, section 5, after Weinberg
1966): ``Oracle.weinberg`` walks every dart of the cell's edge graph from
every start and in both orientations and keeps the smallest code.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "voro_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
FO_LEN = 32
TAU = 2.0 ** -30  # FP64 band inside which the side test is decided exactly

COUNTER_NAMES = ["candidates", "radius_rejects", "vertex_tests", "cuts",
                 "new_vertices", "fan_triangles", "exact_decisions", "shells",
                 "audited", "audit_disagreements"]


def build(force=False):
    """Compile the oracle with gcc (plain C11, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp",
                           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.vo_create.restype = P
        lib.vo_create.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P, P]
        lib.vo_destroy.argtypes = [P]
        lib.vo_set_clip.argtypes = [P, ctypes.c_double]
        lib.vo_set_radii.restype = ctypes.c_int
        lib.vo_set_radii.argtypes = [P, P]
        lib.vo_cells.restype = ctypes.c_int
        lib.vo_cells.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                 P, P, P, P, P, P, P, P, ctypes.c_int, P, P, P]
        lib.vo_set_audit.argtypes = [ctypes.c_int]
        lib.vo_set_wb_rule.argtypes = [ctypes.c_int]
        lib.vo_exact_side.restype = ctypes.c_int
        lib.vo_exact_side.argtypes = [ctypes.c_int, P]
        lib.vo_num_threads.restype = ctypes.c_int
        lib.vo_cell_vertices.restype = ctypes.c_int
        lib.vo_cell_vertices.argtypes = [P, ctypes.c_int64, ctypes.c_double, P, ctypes.c_int]
        lib.vo_weinberg.restype = ctypes.c_int
        lib.vo_weinberg.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_double, P, ctypes.c_int, P, P, P]
        lib.vo_cell_edges.restype = ctypes.c_int
        lib.vo_cell_edges.argtypes = [P, ctypes.c_int64, ctypes.c_double, P, ctypes.c_int]
        lib.vo_cell_faces.restype = ctypes.c_int
        lib.vo_cell_faces.argtypes = [P, ctypes.c_int64, ctypes.c_double, P, P, P, P, ctypes.c_int, ctypes.c_int]
        _lib = lib
    return _lib


def grid_size(n, lo, hi, n_opt=5.0):
    """Block counts of section 2.1.4: lambda = (N / (N_opt Vol))^(1/d),
    n_d = ceil(lambda (b_d - a_d))."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    d = len(lo)
    vol = float(np.prod(hi - lo))
    lam = (n / (n_opt * vol)) ** (1.0 / d)
    return [max(1, int(math.ceil(lam * (hi[k] - lo[k])))) for k in range(d)]


def exact_side(rows, dim=3):
    """Exact sign of n_p.v - h_p at the vertex where planes rows[0..dim) meet;
    rows = 4 x (n0, n1, n2, h, wall) (row 2 unused in 2D, row 3 is p)."""
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.float64).reshape(4, 5))
    return _load().vo_exact_side(dim, r.ctypes.data)


class Oracle:
    """Serial FP64 cells of a container (box [lo, hi], per-axis periodicity).
    clip > 0 clips every cell by the cube of that side centred on its
    particle (section 3.1.3).  radii (n values) makes it the radical
    tessellation of the polydisperse container (section 2.1.1); a cell that
    comes out empty has status 1 (EMPTY) and zero volume, counts and faces.
    A complete cell with a face of 32 or more edges has the status flag 64
    (FO_OVER): its face-order vector does not count that face."""

    EMPTY = 1
    FO_OVER = 64  # status flag: a face has 32 or more edges, fo does not count it

    def __init__(self, xyz, lo, hi, periodic, grid=None, n_opt=5.0, clip=0.0, radii=None):
        lib = _load()
        self.xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64))
        self.n, self.dim = self.xyz.shape
        self.lo = np.asarray(lo, float)
        self.hi = np.asarray(hi, float)
        self.periodic = [int(bool(p)) for p in periodic]
        if grid is None:
            grid = grid_size(self.n, self.lo, self.hi, n_opt)
        self.grid = [int(g) for g in grid]
        lo3 = np.zeros(3)
        hi3 = np.ones(3)
        lo3[:self.dim] = self.lo
        hi3[:self.dim] = self.hi
        per = np.zeros(3, np.int32)
        per[:self.dim] = self.periodic
        g = np.ones(3, np.int32)
        g[:self.dim] = self.grid
        self._keep = (lo3, hi3, per, g)
        self._h = lib.vo_create(self.dim, self.xyz.ctypes.data, self.n, lo3.ctypes.data,
                                hi3.ctypes.data, per.ctypes.data, g.ctypes.data)
        if not self._h:
            raise ValueError("oracle: bad container arguments")
        self.clip = float(clip)
        lib.vo_set_clip(self._h, self.clip)
        self.radii = None
        if radii is not None:
            self.radii = np.ascontiguousarray(np.asarray(radii, dtype=np.float64))
            if self.radii.shape != (self.n,) or lib.vo_set_radii(self._h, self.radii.ctypes.data) != 0:
                raise ValueError("oracle: radii must be n finite values >= 0")

    def __del__(self):
        if getattr(self, "_h", None):
            _load().vo_destroy(self._h)
            self._h = None

    def cells(self, idx=None, nthreads=1, tau=TAU, maxnb=256, neighbors=True):
        """Cells of the particles idx (default: all).  Returns a dict of numpy
        arrays: vol, cen (m x dim), nv, ne, nf, fo (m x 32), perim, status,
        nbr (list of sorted (label, image) int64 arrays, one per cell),
        counters (dict)."""
        lib = _load()
        idx = np.arange(self.n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
        m = len(idx)
        vol = np.zeros(m)
        cen = np.zeros((m, 3))
        nv = np.zeros(m, np.int32)
        ne = np.zeros(m, np.int32)
        nf = np.zeros(m, np.int32)
        fo = np.zeros((m, FO_LEN), np.int32)
        perim = np.zeros(m)
        status = np.zeros(m, np.int32)
        cnt = np.zeros(len(COUNTER_NAMES), np.int64)
        if neighbors:
            nbr = np.zeros((m, maxnb), np.int32)
            nsh = np.zeros((m, maxnb), np.int32)
            pn, ps = nbr.ctypes.data, nsh.ctypes.data
        else:
            pn = ps = None
        rc = lib.vo_cells(self._h, idx.ctypes.data, m, nthreads, tau, vol.ctypes.data, cen.ctypes.data,
                          nv.ctypes.data, ne.ctypes.data, nf.ctypes.data, fo.ctypes.data, pn, ps, maxnb,
                          perim.ctypes.data, status.ctypes.data, cnt.ctypes.data)
        out = dict(vol=vol, cen=cen[:, :self.dim], nv=nv, ne=ne, nf=nf, fo=fo, perim=perim, status=status,
                   rc=rc, counters=dict(zip(COUNTER_NAMES, cnt.tolist())))
        if neighbors:
            lists = []
            for t in range(m):
                k = int(nf[t])
                lab = np.stack([nbr[t, :k].astype(np.int64), nsh[t, :k].astype(np.int64)], axis=1)
                order = np.lexsort((lab[:, 1], lab[:, 0]))
                lists.append(lab[order])
            out["nbr"] = lists
        if rc != 0:
            raise RuntimeError(f"oracle: cell computation failed with code {rc}")
        return out

    def weinberg(self, idx=None, nthreads=1, tau=TAU, maxlen=2048):
        """Weinberg codes of the 3D cells of the particles idx (default: all):
        the lexicographically smallest walk code over every starting dart and
        both orientations (Weinberg 1966; the topology code of VoroTop).
        Returns a dict: codes (list of uint8 arrays of length 2E; empty for an
        empty cell), sym (the number of (dart, orientation) pairs giving the
        code: the order of the graph's symmetry group), chiral (1 when only
        one orientation gives it)."""
        lib = _load()
        idx = np.arange(self.n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
        m = len(idx)
        codes = np.zeros((m, maxlen), np.uint8)
        ln = np.zeros(m, np.int32)
        sym = np.zeros(m, np.int32)
        ch = np.zeros(m, np.int32)
        rc = lib.vo_weinberg(self._h, idx.ctypes.data, m, nthreads, tau, codes.ctypes.data, maxlen, ln.ctypes.data,
                             sym.ctypes.data, ch.ctypes.data)
        if rc != 0:
            raise RuntimeError(f"oracle: Weinberg code failed with code {rc}")
        return dict(codes=[codes[t, :ln[t]].copy() for t in range(m)], len=ln, sym=sym, chiral=ch)

    def edges(self, i, tau=TAU):
        """Undirected edges (u, w), u < w, of the 3D cell of particle i."""
        buf = np.zeros((8192, 2), np.int32)
        k = _load().vo_cell_edges(self._h, int(i), tau, buf.ctypes.data, 8192)
        if k < 0:
            raise RuntimeError(f"oracle: cell computation failed with code {k}")
        return buf[:k].copy()

    def faces(self, i, tau=TAU):
        """Faces of the 3D cell of particle i: a list of (label, image code,
        vertex array relative to the particle), each face's vertices in one
        rotational sense."""
        lab = np.zeros(1024, np.int32)
        sh = np.zeros(1024, np.int32)
        ln = np.zeros(1024, np.int32)
        ring = np.zeros(16384, np.int32)
        k = _load().vo_cell_faces(self._h, int(i), tau, lab.ctypes.data, sh.ctypes.data, ln.ctypes.data,
                                  ring.ctypes.data, 1024, 16384)
        if k < 0:
            raise RuntimeError(f"oracle: cell computation failed with code {k}")
        v = self.vertices(i, tau)
        out, at = [], 0
        for f in range(k):
            out.append((int(lab[f]), int(sh[f]), v[ring[at:at + ln[f]]]))
            at += ln[f]
        return out

    def vertices(self, i, tau=TAU):
        """Vertices of the cell of particle i, relative to the particle."""
        buf = np.zeros((4096, 3))
        k = _load().vo_cell_vertices(self._h, int(i), tau, buf.ctypes.data, 4096)
        if k < 0:
            raise RuntimeError(f"oracle: cell computation failed with code {k}")
        return buf[:k, :self.dim].copy()


def set_weinberg_rule(rule):
    """Test-only: 0 restores Weinberg's walk rules; 1 plants the other
    rotational sense at revisited vertices, 2 drops the return along the
    arrival edge (for checks that the pins catch such mistakes)."""
    _load().vo_set_wb_rule(int(rule))


def num_threads():
    return _load().vo_num_threads()
