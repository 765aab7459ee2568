// cell3d.hip -- per-particle 3D Voronoi cell construction, one wavefront
// per cell (Voro++ method, section 2.1.2-2.1.3 of Lu, Lazar & Rycroft).
//
// Cell representation (dual / triangle form): the cell is a convex polytope
// given by its planes (box walls, own periodic images, and neighbour
// bisectors, Eq. 1-3) and by one triangle (a, b, c) of plane ids per vertex,
// listing the faces that meet there counter-clockwise seen from outside.
// Each lane owns S triangle slots in registers (vertex position in FP64).
// An LDS table etab[a][b] names the slot holding the directed edge a -> b,
// so the triangle across any edge is one LDS read.
//
// A cut by plane p (Eq. 3): every lane tests its vertices, s = q.v - q.q/2,
// a ballot gives the conflict set (vertices strictly outside).  Conflict
// triangles whose neighbour across an edge (a -> b) survives contribute the
// boundary edge (a, b); each becomes a new triangle (a, b, p), whose vertex is
// the intersection of planes a, b, p (Cramer's rule).  New triangles fill free
// slots in lane order.  No cyclic walk of the new face is needed.
//
// Side decisions: |s| <= tau * M (M >= sum |q_d v_d| + |h|) is decided
// exactly from the three planes of the vertex (s * det3 = det4 of the plane
// rows), with floating-point expansions.  A vertex exactly on the plane is
// kept.  With exact decisions the cell does not depend on the cut order.
//
// Candidates come block by block from a precomputed list of block offsets in
// nearest-first order; the particles of up to 64 blocks are loaded at once
// and taken in increasing distance.  A candidate at distance >= 2R (R the
// largest vertex distance) is skipped and the sweep stops when the next block
// is farther than 2R (the radius bound of section 2.1.3).  Past the list the
// search runs Chebyshev shells of blocks under the block bound of the same
// section: blocks and candidates outside the balls B(v, |v|) of the vertices
// are skipped, and the search ends at the first shell that misses their
// bounding box.
#include "cell_common.h"

namespace vc {

namespace {

template <int S, int MAXP, int K>
struct CellLDS {
    double pq[MAXP][4];       // plane normal q (or wall normal) and offset h
    double prj[MAXP];         // radius of each plane's neighbour (radical planes)
    int32_t plab[MAXP];       // neighbour id, or wall label
    uint8_t psh[MAXP];        // image code
    uint8_t pwall[MAXP];      // 1: wall plane (exact offset stored)
    uint8_t etab[MAXP][MAXP]; // slot of the triangle holding directed edge a -> b
    union alignas(16) {
        struct {              // statistics
            double pos[S * 64][3];
            uint32_t tpl[S * 64];
            int32_t lab[S * 64];
        } st;
        struct {              // candidate sweep: the current batch sorted by
            double cq[64][4];               // distance (q, |q|^2), and the
            double ch[64];                  // new vertices of a cut; plane
            double crj[64];                 // offsets and radii
            int32_t cid[64];
            uint8_t ccode[64];
            double npos[S * 64 + 8][3];
        } gc;
    } u;
    uint16_t bedge[S * 64 + 8];
    int32_t cpre[64];
    int32_t cbeg[64];
    uint8_t csh[64];
    int32_t forder[MAXP];
    int32_t fref[MAXP];
    int32_t fo[kFoLen];
};

template <int MAXP>
struct PlaneSet {
    static constexpr int W = (MAXP + 63) / 64;
    unsigned long long w[W];
    // bits of slots beyond MAXP in the last word (kept set: never free)
    static constexpr unsigned long long pad = (MAXP % 64) ? ~((1ull << (MAXP % 64)) - 1) : 0ull;
};

template <int S, int MAXP, int K>
__device__ __forceinline__ PlaneD plane_of(const CellLDS<S, MAXP, K> &sh, int k)
{
    PlaneD p;
    p.n0 = sh.pq[k][0];
    p.n1 = sh.pq[k][1];
    p.n2 = sh.pq[k][2];
    p.h = sh.pq[k][3];
    p.wall = sh.pwall[k];
    return p;
}

template <int S, int MAXP, int K>
__device__ __forceinline__ PlaneR plane_r(const CellLDS<S, MAXP, K> &sh, int k, double ri)
{
    return PlaneR{plane_of(sh, k), ri, sh.prj[k]};
}

// State of one cell held by a wave (registers are per lane; masks uniform).
template <int S, int MAXP, bool F32>
struct Cell {
    uint32_t tp[S];
    double vx[S], vy[S], vz[S];
    float fx[S], fy[S], fz[S];
    unsigned long long live[S];
    PlaneSet<MAXP> used;
    double R2;
    double R;
    double lim;   // squared search radius
    double ri;    // the particle's radius (radical tessellation), else 0
};

template <int S, int MAXP, bool F32>
__device__ __forceinline__ void update_radius(Cell<S, MAXP, F32> &c, int lane, const CellArgs &A)
{
    double m = 0.0;
#pragma unroll
    for (int s = 0; s < S; s++)
        if ((c.live[s] >> lane) & 1) m = fmax(m, c.vx[s] * c.vx[s] + c.vy[s] * c.vy[s] + c.vz[s] * c.vz[s]);
    c.R2 = wave_max(m);
    c.R = sqrt(c.R2);
    c.lim = search_lim(c.R2, c.R, A, c.ri);
}

template <int S, int MAXP, bool F32>
__device__ __forceinline__ bool radius_ok(const Cell<S, MAXP, F32> &c)
{
    return c.R2 < 1e300;  // false for NaN / Inf
}

// Collect the planes used by live triangles (when the plane slots run out).
template <int S, int MAXP, bool F32>
__device__ __forceinline__ void collect_planes(Cell<S, MAXP, F32> &c, int lane)
{
#pragma unroll
    for (int w = 0; w < PlaneSet<MAXP>::W; w++) {
        unsigned long long u = 0;
#pragma unroll
        for (int s = 0; s < S; s++) {
            if ((c.live[s] >> lane) & 1) {
#pragma unroll
                for (int k = 0; k < 3; k++) {
                    int pl = (c.tp[s] >> (8 * k)) & 0xff;
                    if ((pl >> 6) == w) u |= 1ull << (pl & 63);
                }
            }
        }
        c.used.w[w] = wave_or_u64(u);
    }
    c.used.w[PlaneSet<MAXP>::W - 1] |= PlaneSet<MAXP>::pad;
}

template <int S, int MAXP, bool F32>
__device__ __forceinline__ int free_plane(Cell<S, MAXP, F32> &c)
{
#pragma unroll
    for (int w = 0; w < PlaneSet<MAXP>::W; w++)
        if (~c.used.w[w]) return w * 64 + __builtin_ctzll(~c.used.w[w]);
    return -1;
}

// Test the cell against the bisector of candidate q (|q|^2 = d2) and cut it.
// Returns ST_OK or ST_CAP.
template <int S, int MAXP, bool F32, int K>
__device__ __forceinline__ int consider(const CellArgs &A, CellLDS<S, MAXP, K> &sh, Cell<S, MAXP, F32> &c, double q0, double q1,
                        double q2, double h, double rj, int32_t lab, int code, double *ws, unsigned long long *cnt,
                        int lane)
{
    const bool rad = A.rad != nullptr;
    const double Mub = (fabs(q0) + fabs(q1) + fabs(q2)) * c.R + fabs(h);
    const double band = A.tau * Mub;
    unsigned long long conf[S], inb[S];
    int ntest = 0;
    if (F32) {
        const float g0 = (float)q0, g1 = (float)q1, g2 = (float)q2, gh = (float)h;
        const float band32 = A.tau32 * ((fabsf(g0) + fabsf(g1) + fabsf(g2)) * ((float)c.R * 1.0000001f) + fabsf(gh));
        unsigned long long uns = 0;
        unsigned long long unsr[S];
#pragma unroll
        for (int s = 0; s < S; s++) {
            bool lv = (c.live[s] >> lane) & 1;
            float sv = fmaf(g0, c.fx[s], fmaf(g1, c.fy[s], fmaf(g2, c.fz[s], -gh)));
            conf[s] = __ballot(lv && sv > band32);
            unsr[s] = __ballot(lv && !(sv > band32) && !(sv < -band32));
            inb[s] = 0;
            uns |= unsr[s];
            ntest += __popcll(c.live[s]);
        }
        if (uns) {
#pragma unroll
            for (int s = 0; s < S; s++) {
                if (!unsr[s]) continue;
                bool u = (unsr[s] >> lane) & 1;
                double sv = fma(q0, c.vx[s], fma(q1, c.vy[s], fma(q2, c.vz[s], -h)));
                conf[s] |= __ballot(u && sv > band);
                inb[s] = __ballot(u && !(sv > band) && !(sv < -band));
                cnt[DC_RECHECK] += __popcll(unsr[s]);
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < S; s++) {
            bool lv = (c.live[s] >> lane) & 1;
            double sv = fma(q0, c.vx[s], fma(q1, c.vy[s], fma(q2, c.vz[s], -h)));
            conf[s] = __ballot(lv && sv > band);
            inb[s] = __ballot(lv && !(sv > band) && !(sv < -band));
            ntest += __popcll(c.live[s]);
        }
    }
    cnt[DC_TESTS] += ntest;
    // in-band vertices: exact decision, one lane at a time
    unsigned long long zero[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        unsigned long long m = inb[s];
        zero[s] = 0;
        while (m) {
            int l = __builtin_ctzll(m);
            m &= m - 1;
            int sg = 0;
            if (lane == l) {
                const PlaneD pp = {q0, q1, q2, h, 0};
                const uint32_t t3 = c.tp[s];
                if (rad)
                    sg = exact_side3(plane_r(sh, t3 & 0xff, c.ri), plane_r(sh, (t3 >> 8) & 0xff, c.ri),
                                     plane_r(sh, (t3 >> 16) & 0xff, c.ri), PlaneR{pp, c.ri, rj}, ws);
                else
                    sg = exact_side3(plane_of(sh, t3 & 0xff), plane_of(sh, (t3 >> 8) & 0xff),
                                     plane_of(sh, (t3 >> 16) & 0xff), pp, ws);
            }
            sg = __builtin_amdgcn_readlane(sg, l);
            if (sg > 0) conf[s] |= 1ull << l;
            if (sg == 0) zero[s] |= 1ull << l;
            cnt[DC_EXACT]++;
        }
    }
    unsigned long long anyc = 0;
#pragma unroll
    for (int s = 0; s < S; s++) anyc |= conf[s];
    if (!anyc) return ST_OK;
    if (rad) {
        // a radical plane can leave no vertex strictly inside: empty cell
        unsigned long long inside = 0;
#pragma unroll
        for (int s = 0; s < S; s++) inside |= c.live[s] & ~conf[s] & ~zero[s];
        if (!inside) {
#pragma unroll
            for (int s = 0; s < S; s++) c.live[s] = 0;
            return ST_EMPTY;
        }
    }

    // ---- cut ----
    int p = free_plane(c);
    if (p < 0) {
        collect_planes(c, lane);
        p = free_plane(c);
        if (p < 0) return ST_CAP;
    }
    // boundary edges of the conflict region
    uint32_t bfl = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        if ((conf[s] >> lane) & 1) {
            uint32_t t3 = c.tp[s];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
                int tw = sh.etab[b][a] & (S * 64 - 1);
                unsigned long long cw = 0;
#pragma unroll
                for (int r = 0; r < S; r++)
                    if ((tw >> 6) == r) cw = conf[r];
                if (!((cw >> (tw & 63)) & 1)) bfl |= 1u << (s * 3 + k);
            }
        }
    }
    int nb = __popc(bfl);
    int m;
    int o = ballot_excl_scan<(S == 2 ? 3 : 4)>(nb, m);
    int nfree = 0;
#pragma unroll
    for (int s = 0; s < S; s++) nfree += __popcll(~c.live[s] | conf[s]);
    if (m > nfree || m > S * 64 + 8) return ST_CAP;
    if (A.vcap > 0) {
        int keep = 0;
#pragma unroll
        for (int s = 0; s < S; s++) keep += __popcll(c.live[s] & ~conf[s]);
        if (keep + m > A.vcap) return ST_CAP;
    }
#pragma unroll
    for (int s = 0; s < S; s++) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            if ((bfl >> (s * 3 + k)) & 1) {
                uint32_t t3 = c.tp[s];
                int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
                sh.bedge[o++] = (uint16_t)(a | (b << 8));
            }
        }
    }
    if (lane == 0) {
        sh.pq[p][0] = q0;
        sh.pq[p][1] = q1;
        sh.pq[p][2] = q2;
        sh.pq[p][3] = h;
        if (A.rad) sh.prj[p] = rj;
        sh.plab[p] = lab;
        sh.psh[p] = (uint8_t)code;
        sh.pwall[p] = 0;
    }
    __syncthreads();
    // vertices of the new triangles (a, b, p), one per lane, staged in LDS
    for (int k = lane; k < m; k += 64) {
        uint16_t e = sh.bedge[k];
        double x, y, z;
        cramer(sh.pq[e & 0xff], sh.pq[e >> 8], sh.pq[p], x, y, z);
        sh.u.gc.npos[k][0] = x;
        sh.u.gc.npos[k][1] = y;
        sh.u.gc.npos[k][2] = z;
    }
    __syncthreads();
    // new triangles fill the free slots in slot order
    int before = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        unsigned long long fr = ~c.live[s] | conf[s];
        int rank = before + lane_rank(fr);
        bool take = ((fr >> lane) & 1) && rank < m;
        unsigned long long nw = __ballot(take);
        if (take) {
            uint16_t e = sh.bedge[rank];
            int a = e & 0xff, b = e >> 8;
            c.tp[s] = (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)p << 16);
            c.vx[s] = sh.u.gc.npos[rank][0];
            c.vy[s] = sh.u.gc.npos[rank][1];
            c.vz[s] = sh.u.gc.npos[rank][2];
            if (F32) {
                c.fx[s] = (float)c.vx[s];
                c.fy[s] = (float)c.vy[s];
                c.fz[s] = (float)c.vz[s];
            }
            uint8_t t = (uint8_t)(s * 64 + lane);
            sh.etab[a][b] = t;
            sh.etab[b][p] = t;
            sh.etab[p][a] = t;
        }
        c.live[s] = (c.live[s] & ~conf[s]) | nw;
        before += __popcll(fr);
    }
    c.used.w[p >> 6] |= 1ull << (p & 63);
    __syncthreads();
    update_radius(c, lane, A);
    cnt[DC_CUTS]++;
    cnt[DC_NEWV] += m;
    return radius_ok(c) ? ST_OK : ST_CAP;
}

// The cell's vertices as the ball list of the block bound, in the
// new-vertex buffer (unused outside cuts); returns their number.
template <int S, int MAXP, bool F32, int K>
__device__ __forceinline__ int bb_list(CellLDS<S, MAXP, K> &sh, const Cell<S, MAXP, F32> &c, int lane, double extra)
{
    static_assert(sizeof(sh.u.gc.npos) >= sizeof(float4) * S * 64, "ball list does not fit");
    float4 *list = reinterpret_cast<float4 *>(&sh.u.gc.npos[0][0]);
    int n = 0;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; s++) {
        const unsigned long long m = c.live[s];
        if ((m >> lane) & 1) bb_put(list, n + lane_rank(m), c.vx[s], c.vy[s], c.vz[s], extra);
        n += __popcll(m);
    }
    __syncthreads();
    return n;
}

// Load the particles of up to 64 blocks (one per lane: offset dx,dy,dz,
// valid) and feed them to the cell in increasing distance.
// Block bound (section 2.1.3) of one block per lane, at unfolded block
// coordinates t: false for a block outside a wall or one that misses the
// bounding box of the vertices' balls (met is set when some lane's block
// meets that box), then for an empty block, then for one that misses the
// balls themselves.
template <int S, int MAXP, bool F32, int K>
__device__ __forceinline__ bool bb_block(const CellArgs &A, CellLDS<S, MAXP, K> &sh, const Cell<S, MAXP, F32> &c,
                                         const Tess &T, const double *p, const int t[3], bool v, double extra,
                                         double pad, int lane, bool &met)
{
    const Grid &G = T.G;
    double ext[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < S; s++)
        if ((c.live[s] >> lane) & 1) bb_ext_add(ext, c.vx[s], c.vy[s], c.vz[s], extra);
#pragma unroll
    for (int k = 0; k < 6; k++) ext[k] = wave_max(ext[k]);
    double blo[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (!G.per[d] && (t[d] < 0 || t[d] >= G.g[d])) v = false;
        blo[d] = G.lo[d] + t[d] * G.bs[d] - p[d];
    }
    v = v && bb_in_ext(ext, blo, G.bs, pad, 3);
    if (!__ballot(v)) return false;
    met = true;
    v = v && bb_block_count<3>(A.start, T, t) > 0;
    if (!__ballot(v)) return false;
    const int nv = bb_list(sh, c, lane, extra);
    return v && bb_meets(reinterpret_cast<const float4 *>(&sh.u.gc.npos[0][0]), nv, blo, G.bs, pad, 3);
}

// A batch with at least bbmin candidates inside the radius bound is first
// tested against the balls of the block bound, one candidate per lane: a
// candidate outside every ball cannot cut (section 2.1.3), and this costs
// one pass over the vertex list instead of a side test of every vertex.
template <int S, int MAXP, bool F32, int K>
__device__ __forceinline__ int gather(const CellArgs &A, CellLDS<S, MAXP, K> &sh, Cell<S, MAXP, F32> &c, int si, const double *p,
                      const int *bc, int dx, int dy, int dz, bool valid, double *ws, unsigned long long *cnt, int lane,
                      int bbmin, double extra, double pad)
{
    const Tess &T = A.tess[A.part[si].tess];
    const Grid &G = T.G;
    int dd[3] = {dx, dy, dz};
    int bb[3], sv[3];
    bool ok = valid;
    double d2b = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int t = bc[d] + dd[d];
        if (G.per[d]) {
            int g = G.g[d];
            int w = ((t % g) + g) % g;
            sv[d] = (t - w) / g;
            bb[d] = w;
            if (sv[d] > 2 || sv[d] < -2) ok = false;
        } else {
            sv[d] = 0;
            bb[d] = t;
            if (t < 0 || t >= G.g[d]) ok = false;
        }
        double blo = G.lo[d] + t * G.bs[d];
        double e = fmax(0.0, fmax(blo - p[d], p[d] - (blo + G.bs[d])));
        d2b += e * e;
    }
    if (d2b >= c.lim) ok = false;
    int cntb = 0, beg = 0;
    if (ok) {
        int64_t blk = T.bbase + bb[0] + (int64_t)G.g[0] * (bb[1] + (int64_t)G.g[1] * bb[2]);
        beg = A.start[blk];
        cntb = A.start[blk + 1] - beg;
    }
    cnt[DC_BLOCKS] += __popcll(__ballot(ok));
    int incl = wave_incl_scan(cntb);
    int total = __builtin_amdgcn_readlane(incl, 63);
    cnt[DC_LOADED] += total;
    if (total == 0) return ST_OK;
    __syncthreads();
    sh.cpre[lane] = incl - cntb;
    sh.cbeg[lane] = beg;
    sh.csh[lane] = (uint8_t)(25 * (sv[2] + 2) + 5 * (sv[1] + 2) + (sv[0] + 2));
    __syncthreads();
    for (int c0 = 0; c0 < total; c0 += 64) {
        // load one candidate per lane
        int ci = c0 + lane;
        unsigned long long key = ~0ull;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, d2 = 0.0, h = 0.0, rj = 0.0;
        int32_t qid = 0;
        int code = kNoShift;
        if (ci < total) {
            // last block whose exclusive prefix is <= ci
            int lo = 0, hi = 63;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (sh.cpre[mid] <= ci) lo = mid; else hi = mid - 1;
            }
            int idx = sh.cbeg[lo] + (ci - sh.cpre[lo]);
            code = sh.csh[lo];
            int s0 = code % 5 - 2, s1 = (code / 5) % 5 - 2, s2 = code / 25 - 2;
            Particle q = A.part[idx];
            a0 = q.x - p[0];
            a1 = q.y - p[1];
            a2 = q.z - p[2];
            if (s0) a0 = a0 + s0 * G.L[0];
            if (s1) a1 = a1 + s1 * G.L[1];
            if (s2) a2 = a2 + s2 * G.L[2];
            d2 = a0 * a0 + a1 * a1 + a2 * a2;
            if (A.rad) {
                // radical plane (section 2.1.1): |x|^2 - ri^2 <= |x - q|^2 - rj^2
                rj = A.rad[idx];
                h = 0.5 * (d2 + radical_shift(c.ri, rj));
            } else {
                h = 0.5 * d2;
            }
            bool self = (idx == si) && code == kNoShift;
            if (!self && d2 < c.lim) key = __double_as_longlong(d2);
            qid = q.id;
        }
        if (__popcll(__ballot(key != ~0ull)) >= bbmin) {
            const int nv = bb_list(sh, c, lane, extra);
            const double q[3] = {a0, a1, a2}, zero[3] = {0.0, 0.0, 0.0};
            if (key != ~0ull && !bb_meets(reinterpret_cast<const float4 *>(&sh.u.gc.npos[0][0]), nv, q, zero, pad, 3))
                key = ~0ull;
        }
        // rank the batch by (distance, lane) and store it sorted
        unsigned long long vm = __ballot(key != ~0ull);
        int nval = __popcll(vm);
        if (nval == 0) continue;
        int rank = 0;
        for (unsigned long long m = vm; m; m &= m - 1) {
            int j = __builtin_ctzll(m);
            unsigned long long kj = readlane_u64(key, j);
            rank += (kj < key) || (kj == key && j < lane);
        }
        __syncthreads();
        if (key != ~0ull) {
            sh.u.gc.cq[rank][0] = a0;
            sh.u.gc.cq[rank][1] = a1;
            sh.u.gc.cq[rank][2] = a2;
            sh.u.gc.cq[rank][3] = d2;
            if (A.rad) {
                sh.u.gc.ch[rank] = h;
                sh.u.gc.crj[rank] = rj;
            }
            sh.u.gc.cid[rank] = qid;
            sh.u.gc.ccode[rank] = (uint8_t)code;
        }
        __syncthreads();
        // nearest first; stop at the first candidate beyond 2R
        for (int k = 0; k < nval; k++) {
            double md2 = sh.u.gc.cq[k][3];
            if (!(md2 < c.lim)) break;
            cnt[DC_CAND]++;
            if (md2 == 0.0) return ST_DUP;
            int st = consider<S, MAXP, F32, K>(A, sh, c, sh.u.gc.cq[k][0], sh.u.gc.cq[k][1], sh.u.gc.cq[k][2],
                                               A.rad ? sh.u.gc.ch[k] : 0.5 * md2, A.rad ? sh.u.gc.crj[k] : 0.0,
                                               sh.u.gc.cid[k], sh.u.gc.ccode[k], ws,
                                               cnt, lane);
            if (st != ST_OK) return st;
        }
    }
    return ST_OK;
}

template <int S, int MAXP, bool F32, int K>
__device__ __forceinline__ int cell_run(const CellArgs &A, CellLDS<S, MAXP, K> &sh, int si, double *ws, unsigned long long *cnt)
{
    const int lane = __lane_id();
    const Particle me = A.part[si];
    const Tess &T = A.tess[me.tess];
    const Grid &G = T.G;
    const double p[3] = {me.x, me.y, me.z};
    const int id = me.id;
    int bc[3], fl[3];
    double mrg[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        bc[d] = block_coord(G, p[d], d);
        double blo = G.lo[d] + bc[d] * G.bs[d];
        mrg[d] = fmin(p[d] - blo, blo + G.bs[d] - p[d]);
        fl[d] = offset_flip(G, p[d], bc[d], d);
    }
    Cell<S, MAXP, F32> c;
    c.ri = A.rad ? A.rad[si] : 0.0;
    const bool rad = A.rad != nullptr;
    // box planes (Eq. 1-2, clipped as in section 3.1.3); no register array
    // is indexed by d
    if (lane < 6) {
        const int d = lane >> 1, side = lane & 1;
        const double pd = d == 0 ? p[0] : (d == 1 ? p[1] : p[2]);
        const BoxSide b = box_side(T, pd, d, side, id);
        sh.pwall[lane] = (uint8_t)b.wall;
        sh.plab[lane] = b.lab;
        sh.psh[lane] = b.code;
        sh.pq[lane][0] = d == 0 ? b.nd : 0.0;
        sh.pq[lane][1] = d == 1 ? b.nd : 0.0;
        sh.pq[lane][2] = d == 2 ? b.nd : 0.0;
        sh.pq[lane][3] = b.h;
        sh.prj[lane] = c.ri;  // the own images carry the own radius
    }
    // corners: triangle (X, Y, Z) counter-clockwise when det(nX, nY, nZ) > 0
#pragma unroll
    for (int s = 0; s < S; s++) {
        c.tp[s] = 0;
        c.vx[s] = c.vy[s] = c.vz[s] = 0.0;
        c.fx[s] = c.fy[s] = c.fz[s] = 0.0f;
        c.live[s] = 0;
    }
    c.live[0] = 0xffull;
    if (lane < 8) {
        int bx = lane & 1, by = (lane >> 1) & 1, bz = (lane >> 2) & 1;
        int X = bx, Y = 2 + by, Z = 4 + bz;
        int neg = 3 - bx - by - bz;
        c.tp[0] = (neg & 1) ? (X | (Z << 8) | (Y << 16)) : (X | (Y << 8) | (Z << 16));
        double e[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const int b = (lane >> d) & 1;
            const double o = box_side(T, p[d], d, b, id).off;
            e[d] = b ? o : -o;
        }
        c.vx[0] = e[0];
        c.vy[0] = e[1];
        c.vz[0] = e[2];
        c.fx[0] = (float)e[0];
        c.fy[0] = (float)e[1];
        c.fz[0] = (float)e[2];
        uint32_t t3 = c.tp[0];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
            sh.etab[a][b] = (uint8_t)lane;
        }
    }
#pragma unroll
    for (int w = 0; w < PlaneSet<MAXP>::W; w++) c.used.w[w] = 0;
    c.used.w[0] = 0x3full;
    c.used.w[PlaneSet<MAXP>::W - 1] |= PlaneSet<MAXP>::pad;
    __syncthreads();
    update_radius(c, lane, A);

    // the balls of the block bound: radical widening and rounding allowance
    const double extra = rad ? fmax(*A.rmax * *A.rmax - c.ri * c.ri, 0.0) : 0.0;
    const double pad = bb_pad(G, p, 3);
    // nearest-first sweep over the precomputed block offsets; once the cell
    // is extended (2R beyond three block sides, past the first chunk), its
    // blocks go through the block bound too
    bool finished = false;
    for (int o0 = 0; o0 < A.noff; o0 += 64) {
        if (A.offs[o0].m * 0.25 * T.bsmin2 >= c.lim) {
            finished = true;
            break;
        }
        int o = o0 + lane;
        bool v = o < A.noff;
        Offset of = v ? A.offs[o] : Offset{0, 0, 0, 0};
        of.dx *= fl[0];
        of.dy *= fl[1];
        of.dz *= fl[2];
        if (o0 > 0 && c.lim > kBbExtended * T.bsmin2) {
            bool met = false;
            const int t[3] = {bc[0] + of.dx, bc[1] + of.dy, bc[2] + of.dz};
            v = bb_block(A, sh, c, T, p, t, v, extra, pad, lane, met);
            if (!__ballot(v)) continue;
        }
        int st = gather<S, MAXP, F32, K>(A, sh, c, si, p, bc, of.dx, of.dy, of.dz, v, ws, cnt, lane, kBbMinList, extra,
                                         pad);
        if (st != ST_OK) return st;
    }
    // beyond the list: whole Chebyshev shells, until the radius bound holds
    // or no block of a shell meets the bounding box of the block bound
    if (!finished) {
        cnt[DC_FALLBACK]++;
        for (int r = A.off_radius + 1;; r++) {
            if (r > kMaxShell || !radius_ok(c)) return ST_CAP;
            double lb = 1e300;
            bool exists = false;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                lb = fmin(lb, (r - 1) * G.bs[d] + mrg[d]);
                if (G.per[d] || bc[d] - r >= 0 || bc[d] + r < G.g[d]) exists = true;
            }
            if (!exists) break;
            if (lb > 0.0 && lb * lb >= c.lim) break;
            cnt[DC_SHELLS]++;
            const int tot = shell_size3(r);
            bool met = false;
            // four chunks of 64 blocks per step: the bounding box of the
            // balls once, then the four blocks' particle counts loaded
            // together, then the balls and the gather chunk by chunk
            constexpr int U = 4;
            for (int c0 = 0; c0 < tot; c0 += U * 64) {
                double ext[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < S; s++)
                    if ((c.live[s] >> lane) & 1) bb_ext_add(ext, c.vx[s], c.vy[s], c.vz[s], extra);
#pragma unroll
                for (int k = 0; k < 6; k++) ext[k] = wave_max(ext[k]);
                int qk[U], qn[U];
                bool any = false;
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int ix = c0 + u * 64 + lane;
                    int dx = 0, dy = 0, dz = 0;
                    bool v = ix < tot;
                    if (v) shell_block3(r, ix, dx, dy, dz);
                    const int t[3] = {bc[0] + dx, bc[1] + dy, bc[2] + dz};
                    double blo[3];
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        if (!G.per[d] && (t[d] < 0 || t[d] >= G.g[d])) v = false;
                        blo[d] = G.lo[d] + t[d] * G.bs[d] - p[d];
                    }
                    v = v && bb_in_ext(ext, blo, G.bs, pad, 3);
                    any = any || __ballot(v);
                    qk[u] = ix;
                    qn[u] = v ? 1 : 0;
                }
                if (!any) continue;
                met = true;
#pragma unroll
                for (int u = 0; u < U; u++) {
                    if (qn[u]) {
                        int dx, dy, dz;
                        shell_block3(r, qk[u], dx, dy, dz);
                        const int t[3] = {bc[0] + dx, bc[1] + dy, bc[2] + dz};
                        qn[u] = bb_block_count<3>(A.start, T, t);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    bool v = qn[u] > 0;
                    if (!__ballot(v)) continue;
                    int dx = 0, dy = 0, dz = 0;
                    if (qk[u] < tot) shell_block3(r, qk[u], dx, dy, dz);
                    const int nv = bb_list(sh, c, lane, extra);
                    const double blo[3] = {G.lo[0] + (bc[0] + dx) * G.bs[0] - p[0], G.lo[1] + (bc[1] + dy) * G.bs[1] - p[1],
                                           G.lo[2] + (bc[2] + dz) * G.bs[2] - p[2]};
                    v = v && bb_meets(reinterpret_cast<const float4 *>(&sh.u.gc.npos[0][0]), nv, blo, G.bs, pad, 3);
                    if (!__ballot(v)) continue;
                    int st = gather<S, MAXP, F32, K>(A, sh, c, si, p, bc, dx, dy, dz, v, ws, cnt, lane, 1, extra, pad);
                    if (st != ST_OK) return st;
                }
            }
            if (!met) break;
        }
    }

    // ---- statistics (a8) ----
    __syncthreads();
#pragma unroll
    for (int s = 0; s < S; s++) {
        int t = s * 64 + lane;
        bool lv = (c.live[s] >> lane) & 1;
        sh.u.st.tpl[t] = lv ? c.tp[s] : 0xffffffffu;
        sh.u.st.pos[t][0] = c.vx[s];
        sh.u.st.pos[t][1] = c.vy[s];
        sh.u.st.pos[t][2] = c.vz[s];
        sh.u.st.lab[t] = t;
    }
    for (int k = lane; k < MAXP; k += 64) {
        sh.forder[k] = 0;
        sh.fref[k] = 0x7fffffff;
    }
    if (lane < kFoLen) sh.fo[lane] = 0;
    __syncthreads();
    for (int t = lane; t < S * 64; t += 64) {
        uint32_t t3 = sh.u.st.tpl[t];
        if (t3 == 0xffffffffu) continue;
        for (int k = 0; k < 3; k++) atomicMin(&sh.fref[(t3 >> (8 * k)) & 0xff], t);
    }
    __syncthreads();
    // Zero-length edges (a degenerate vertex split over several triangles):
    // the edge (a, b) between slot t and its twin has zero length when the
    // vertex of t lies on the twin's third plane d.  Bit (s*3+k) of zb.
    uint32_t zb = 0, ib = 0;
    for (int j = 0; j < 3 * S; j++) {
        int t = (j / 3) * 64 + lane, k = j % 3;
        uint32_t t3 = sh.u.st.tpl[t];
        if (t3 == 0xffffffffu) continue;
        int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
        uint32_t w3 = sh.u.st.tpl[sh.etab[b][a] & (S * 64 - 1)];
        int d = (int)(w3 & 0xff) + (int)((w3 >> 8) & 0xff) + (int)((w3 >> 16) & 0xff) - a - b;
        d = min(max(d, 0), MAXP - 1);
        const double *nd = sh.pq[d];
        const double *v = sh.u.st.pos[t];
        double sd = nd[0] * v[0] + nd[1] * v[1] + nd[2] * v[2] - nd[3];
        double bd = A.tau * ((fabs(nd[0]) + fabs(nd[1]) + fabs(nd[2])) * c.R + fabs(nd[3]));
        if (!(sd < -bd)) ib |= 1u << j;
    }
    if (__ballot(ib != 0)) {
        for (int j = 0; j < 3 * S; j++) {
            unsigned long long m = __ballot((ib >> j) & 1);
            while (m) {
                int l = __builtin_ctzll(m);
                m &= m - 1;
                if (lane == l) {
                    int t = (j / 3) * 64 + lane, k = j % 3;
                    uint32_t t3 = sh.u.st.tpl[t];
                    int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
                    uint32_t w3 = sh.u.st.tpl[sh.etab[b][a] & (S * 64 - 1)];
                    int d = (int)(w3 & 0xff) + (int)((w3 >> 8) & 0xff) + (int)((w3 >> 16) & 0xff) - a - b;
                    d = min(max(d, 0), MAXP - 1);
                    int sg = rad ? exact_side3(plane_r(sh, t3 & 0xff, c.ri), plane_r(sh, (t3 >> 8) & 0xff, c.ri),
                                               plane_r(sh, (t3 >> 16) & 0xff, c.ri), plane_r(sh, d, c.ri), ws)
                                 : exact_side3(plane_of(sh, t3 & 0xff), plane_of(sh, (t3 >> 8) & 0xff),
                                               plane_of(sh, (t3 >> 16) & 0xff), plane_of(sh, d), ws);
                    if (sg == 0) zb |= 1u << j;
                }
                cnt[DC_EXACT]++;
            }
        }
    }
    // face orders and the fan over each face from its reference vertex:
    // tetrahedra (0, r_a, v_twin, v_t), the twin across a -> b being the
    // previous vertex of face a counter-clockwise
    // The apex is the particle when it lies strictly inside the cell (every
    // face offset h > 0, always so for a Voronoi cell), else one vertex.
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    if (rad) {
        bool in = true;
#pragma unroll
        for (int s = 0; s < S; s++)
            if ((c.live[s] >> lane) & 1)
#pragma unroll
                for (int k = 0; k < 3; k++) in = in && sh.pq[(c.tp[s] >> (8 * k)) & 0xff][3] > 0.0;
        if (__ballot(!in)) {
            int t0 = 0;
#pragma unroll
            for (int s = S - 1; s >= 0; s--)
                if (c.live[s]) t0 = s * 64 + __builtin_ctzll(c.live[s]);
            o0 = sh.u.st.pos[t0][0];
            o1 = sh.u.st.pos[t0][1];
            o2 = sh.u.st.pos[t0][2];
        }
    }
    double v6 = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int j = 0; j < 3 * S; j++) {
        int t = (j / 3) * 64 + lane, k = j % 3;
        uint32_t t3 = sh.u.st.tpl[t];
        if (t3 == 0xffffffffu) continue;
        int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
        if (!((zb >> j) & 1)) atomicAdd(&sh.forder[a], 1);
        const double *r0 = sh.u.st.pos[sh.fref[a]];
        const double *w0 = sh.u.st.pos[sh.etab[b][a] & (S * 64 - 1)];
        const double *v0 = sh.u.st.pos[t];
        const double r[3] = {r0[0] - o0, r0[1] - o1, r0[2] - o2};
        const double w[3] = {w0[0] - o0, w0[1] - o1, w0[2] - o2};
        const double v[3] = {v0[0] - o0, v0[1] - o1, v0[2] - o2};
        double det = r[0] * (w[1] * v[2] - w[2] * v[1]) - r[1] * (w[0] * v[2] - w[2] * v[0]) +
                     r[2] * (w[0] * v[1] - w[1] * v[0]);
        v6 += det;
        m0 += det * (r[0] + w[0] + v[0]);
        m1 += det * (r[1] + w[1] + v[1]);
        m2 += det * (r[2] + w[2] + v[2]);
    }
    // vertices: triangles joined by zero-length edges are one vertex
    int nvert = 0;
#pragma unroll
    for (int s = 0; s < S; s++) nvert += __popcll(c.live[s]);
    if (__ballot(zb != 0)) {
        for (int it = 0; it < 4 * S * 64; it++) {
            bool ch = false;
            for (int j = 0; j < 3 * S; j++) {
                if (!((zb >> j) & 1)) continue;
                int t = (j / 3) * 64 + lane, k = j % 3;
                uint32_t t3 = sh.u.st.tpl[t];
                int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
                int o = sh.u.st.lab[sh.etab[b][a] & (S * 64 - 1)];
                if (o < sh.u.st.lab[t]) {
                    sh.u.st.lab[t] = o;
                    ch = true;
                }
            }
            __syncthreads();
            if (!__ballot(ch)) break;
        }
        nvert = 0;
        for (int t0 = 0; t0 < S * 64; t0 += 64) {
            int t = t0 + lane;
            nvert += __popcll(__ballot(sh.u.st.tpl[t] != 0xffffffffu && sh.u.st.lab[t] == t));
        }
    }
    __syncthreads();
    // faces with at least three distinct vertices are the cell's faces
    int nface = 0, sumord = 0, rk = 0;
    bool capfail = false, foover = false;
    for (int k0 = 0; k0 < MAXP; k0 += 64) {
        int k = k0 + lane;
        int ord = k < MAXP ? sh.forder[k] : 0;
        bool real = ord >= 3;
        unsigned long long rb = __ballot(real);
        int rank = rk + lane_rank(rb);
        if (real) {
            if (ord < kFoLen) atomicAdd(&sh.fo[ord], 1);
            if ((A.mask & (16 | 32)) && A.nbr) {
                if (rank < kMaxNbr) {
                    A.nbr[(int64_t)id * kMaxNbr + rank] = sh.plab[k];
                    A.nsh[(int64_t)id * kMaxNbr + rank] = sh.psh[k];
                }
            }
        }
        rk += __popcll(rb);
        sumord += wave_isum(real ? ord : 0);
        foover = foover || __ballot(real && ord >= kFoLen) != 0;
    }
    nface = rk;
    if (nface > kMaxNbr) capfail = true;
    double vol6 = wave_sum(v6);
    double M0 = wave_sum(m0), M1 = wave_sum(m1), M2 = wave_sum(m2);
    __syncthreads();
    if (A.wbg && !capfail) {
        // the vertex positions are no longer needed: their LDS holds the
        // record's scratch (zero-length edge bits, vertex numbers, degrees)
        uint8_t *wsc = reinterpret_cast<uint8_t *>(&sh.u.st.pos[0][0]);
        const int wl = wb_record<64, S, MAXP>(A.wbg + (int64_t)id * kWbStride, sumord, sh.u.st.tpl, sh.u.st.lab,
                                              sh.etab, wsc, wsc + 64 * S, wsc + 128 * S, zb, lane, 0);
        if (lane == 0) A.wbl[id] = wl;
    }
    if (lane == 0) {
        double vol = vol6 / 6.0;
        if (A.vol) A.vol[id] = vol;
        if (A.cen) {
            A.cen[3 * (int64_t)id + 0] = o0 + M0 / (4.0 * vol6);
            A.cen[3 * (int64_t)id + 1] = o1 + M1 / (4.0 * vol6);
            A.cen[3 * (int64_t)id + 2] = o2 + M2 / (4.0 * vol6);
        }
        if (A.nv) A.nv[id] = nvert;
        if (A.ne) A.ne[id] = sumord / 2;
        if (A.nf) A.nf[id] = nface;
    }
    if (A.fo && lane < kFoLen) A.fo[(int64_t)id * kFoLen + lane] = (uint8_t)min(sh.fo[lane], 255);
    if (capfail) return ST_CAP;
    if (A.lim_out && lane == 0) A.lim_out[si] = c.lim;
    return foover ? ST_FO_OVER : ST_OK;
}

// Waves per SIMD (the register allocator is held to that budget): three for
// the two-slot main kernel (168 registers; its LDS allows three), two for
// the four-slot one (its LDS allows two), one for the spill kernel.  At
// three waves the two-slot kernel spills about 50 registers and still runs
// a fifth faster than at two.  spill_mode: 0 the
// main pass (a cell beyond the capacity goes to the spill list), 2 a first
// spill pass (its cells are marked SPILLED, and a cell beyond the capacity
// goes on to the next list), 1 the last pass (beyond its capacity a cell is
// VC_CELL_CAPACITY)
template <int S, int MAXP, bool F32, int K, bool RAD, bool WB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MAXP == 48 ? (S == 2 ? 3 : 2) : 1))) void k_cells(CellArgs Ain,
                                                                                                     int spill_mode)
{
    // the Voronoi instantiation carries no radical code, and one without
    // Weinberg records none of their code: those pointers are compile-time
    // nulls
    CellArgs A = Ain;
    if (!RAD) A.rad = nullptr;
    if (!WB) {
        A.wbg = nullptr;
        A.wbl = nullptr;
    }
    __shared__ CellLDS<S, MAXP, K> sh;
    const int lane = __lane_id();
    double *ws = A.xscratch + (size_t)blockIdx.x * A.xscratch_len;
    unsigned long long cnt[DC_N];
#pragma unroll
    for (int k = 0; k < DC_N; k++) cnt[k] = 0;
    const int ncell = A.ncell_dev ? __builtin_amdgcn_readfirstlane(*A.ncell_dev) : A.ncell;
    // claims are dynamic and the waves below this one take every cell, so a
    // wave with nothing left to claim leaves without touching the queue (a
    // short spill list then costs a few atomics instead of one per wave)
    if ((int64_t)blockIdx.x * A.chunk >= ncell) return;
    for (;;) {
        int base = 0;
        if (lane == 0) base = atomicAdd(A.queue, A.chunk);
        base = __builtin_amdgcn_readfirstlane(base);
        if (base >= ncell) break;
        int end = min(base + A.chunk, ncell);
        for (int ci = base; ci < end; ci++) {
            int si = A.cell_list ? A.cell_list[ci] : ci;
            int st = cell_run<S, MAXP, F32, K>(A, sh, si, ws, cnt);
            const int fov = st & ST_FO_OVER;
            st &= ~ST_FO_OVER;
            if (st != ST_OK && A.fo && lane < kFoLen) A.fo[(int64_t)A.part[si].id * kFoLen + lane] = 0;
            if (lane == 0) {
                int id = A.part[si].id;
                if (st != ST_OK) {
                    // no statistics for this cell (yet): empty outputs; an
                    // empty radical cell has zero volume
                    const double f = st == ST_EMPTY ? 0.0 : __builtin_nan("");
                    if (A.vol) A.vol[id] = f;
                    if (A.cen) A.cen[3 * (int64_t)id] = A.cen[3 * (int64_t)id + 1] = A.cen[3 * (int64_t)id + 2] = f;
                    if (A.nv) A.nv[id] = 0;
                    if (A.ne) A.ne[id] = 0;
                    if (A.nf) A.nf[id] = 0;
                    if (A.wbl) A.wbl[id] = 0;
                }
                if (st == ST_EMPTY) {
                    A.status[id] = (uint8_t)ST_EMPTY;
                } else if (st == ST_OK) {
                    A.status[id] = (uint8_t)((spill_mode ? 1 : 0) | fov);
                } else if (st == ST_DUP) {
                    A.status[id] = 3;
                } else if (spill_mode != 1) {
                    A.status[id] = 1;
                    int pos = atomicAdd(A.spill_count, 1);
                    A.spill_list[pos] = si;
                } else {
                    A.status[id] = 2;
                }
                if (st == ST_CAP && spill_mode == 0) cnt[DC_SPILL]++;
            }
            __syncthreads();
        }
    }
    if (lane < DC_N) {
        unsigned long long v = 0;
#pragma unroll
        for (int k = 0; k < DC_N; k++)
            if (k == lane) v = cnt[k];
        // counters are wave-uniform except the spill count (lane 0)
        if (lane == DC_SPILL) v = readlane_u64(cnt[DC_SPILL], 0);
        if (v) atomicAdd(&A.diag[lane], v);
    }
}

}  // namespace

hipError_t launch_cells(const CellArgs &a, int precision, int slots, int waves, hipStream_t s)
{
    const bool rad = a.rad != nullptr, wb = a.wbg != nullptr, f32 = precision == 1;
#define VC_CELLS(S)                                                                              \
    do {                                                                                         \
        if (rad) {                                                                               \
            if (wb) {                                                                            \
                if (f32) k_cells<S, 48, true, 1, true, true><<<waves, 64, 0, s>>>(a, 0);         \
                else k_cells<S, 48, false, 1, true, true><<<waves, 64, 0, s>>>(a, 0);            \
            } else {                                                                             \
                if (f32) k_cells<S, 48, true, 1, true, false><<<waves, 64, 0, s>>>(a, 0);        \
                else k_cells<S, 48, false, 1, true, false><<<waves, 64, 0, s>>>(a, 0);           \
            }                                                                                    \
        } else {                                                                                 \
            if (wb) {                                                                            \
                if (f32) k_cells<S, 48, true, 1, false, true><<<waves, 64, 0, s>>>(a, 0);        \
                else k_cells<S, 48, false, 1, false, true><<<waves, 64, 0, s>>>(a, 0);           \
            } else {                                                                             \
                if (f32) k_cells<S, 48, true, 1, false, false><<<waves, 64, 0, s>>>(a, 0);       \
                else k_cells<S, 48, false, 1, false, false><<<waves, 64, 0, s>>>(a, 0);          \
            }                                                                                    \
        }                                                                                        \
    } while (0)
    if (slots == 4) VC_CELLS(4);
    else VC_CELLS(2);
#undef VC_CELLS
    return hipGetLastError();
}

// The first spill pass: the one-cell kernel of the main pass (capacity
// 128), for the cells the grouped kernel left (extended or beyond its
// capacity); its own overflows go on to the large-capacity pass.
hipError_t launch_cells_handoff(const CellArgs &a, int waves, hipStream_t s)
{
    const bool rad = a.rad != nullptr, wb = a.wbg != nullptr;
    if (rad) {
        if (wb) k_cells<2, 48, false, 1, true, true><<<waves, 64, 0, s>>>(a, 2);
        else k_cells<2, 48, false, 1, true, false><<<waves, 64, 0, s>>>(a, 2);
    } else {
        if (wb) k_cells<2, 48, false, 1, false, true><<<waves, 64, 0, s>>>(a, 2);
        else k_cells<2, 48, false, 1, false, false><<<waves, 64, 0, s>>>(a, 2);
    }
    return hipGetLastError();
}

hipError_t launch_cells_spill(const CellArgs &a, int waves, hipStream_t s)
{
    const bool rad = a.rad != nullptr, wb = a.wbg != nullptr;
    if (rad) {
        if (wb) k_cells<4, 128, false, 1, true, true><<<waves, 64, 0, s>>>(a, 1);
        else k_cells<4, 128, false, 1, true, false><<<waves, 64, 0, s>>>(a, 1);
    } else {
        if (wb) k_cells<4, 128, false, 1, false, true><<<waves, 64, 0, s>>>(a, 1);
        else k_cells<4, 128, false, 1, false, false><<<waves, 64, 0, s>>>(a, 1);
    }
    return hipGetLastError();
}

}  // namespace vc
