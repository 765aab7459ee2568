// cell3d_group.hip -- the 3D cell kernel with several cells per wavefront.
//
// The algorithm is the one of cell3d.hip (dual triangle cells, ballot side
// tests with an exact fallback, cuts that re-triangulate the conflict region,
// nearest-first candidates with the radius bound, fan statistics); only the
// mapping differs: each cell is owned by a group of G lanes (G = 16 or 32,
// so 64/G cells per wave) and every cross-lane step stays inside the group:
// ballots are read through the group's bit field, reductions and scans use
// DPP row operations (plus one lane exchange across rows for G = 32), and
// the groups share the wave's instruction stream.  Per-cell work that is the
// same for every lane of a cell (candidate selection, plane bookkeeping,
// radius updates, statistics reductions) is thus issued once for 64/G cells.
//
// Groups take different control paths, so LDS hand-offs use a workgroup-scope
// fence (one wave per workgroup) instead of a barrier.
#include "cell_common.h"

namespace vc {

namespace {

template <int G>
struct Grp {
    static constexpr int CPW = 64 / G;
    static constexpr unsigned long long MASK = G == 64 ? ~0ull : ((1ull << G) - 1ull);
};

__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

template <int G>
__device__ __forceinline__ unsigned long long gballot(bool p, int gb)
{
    return (__ballot(p) >> gb) & Grp<G>::MASK;
}

__device__ __forceinline__ int grank(unsigned long long m, int gl)
{
    return __popcll(m & ((1ull << gl) - 1ull));
}

// reductions over the group; every lane of the group gets the result
template <int G>
__device__ __forceinline__ double gmax(double v)
{
    v = fmax(v, dpp_f64<DPP_QUAD_1032, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_QUAD_2301, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_ROW_HALF_MIRROR, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_ROW_MIRROR, 0xf>(v, v));
    if (G >= 32) v = fmax(v, __shfl_xor(v, 16));
    if (G >= 64) v = fmax(v, __shfl_xor(v, 32));
    return v;
}

template <int G>
__device__ __forceinline__ double gsum(double v)
{
    v = v + dpp_f64<DPP_QUAD_1032, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_QUAD_2301, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_ROW_HALF_MIRROR, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_ROW_MIRROR, 0xf>(0.0, v);
    if (G >= 32) v = v + __shfl_xor(v, 16);
    if (G >= 64) v = v + __shfl_xor(v, 32);
    return v;
}

template <int G>
__device__ __forceinline__ int gisum(int v)
{
    v = v + dpp_i32<DPP_QUAD_1032, 0xf>(0, v);
    v = v + dpp_i32<DPP_QUAD_2301, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_HALF_MIRROR, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_MIRROR, 0xf>(0, v);
    if (G >= 32) v = v + __shfl_xor(v, 16);
    if (G >= 64) v = v + __shfl_xor(v, 32);
    return v;
}

template <int G>
__device__ __forceinline__ unsigned long long gmin_u64(unsigned long long v)
{
    unsigned long long w;
    w = dpp_u64<DPP_QUAD_1032, 0xf>(v, v);
    v = w < v ? w : v;
    w = dpp_u64<DPP_QUAD_2301, 0xf>(v, v);
    v = w < v ? w : v;
    w = dpp_u64<DPP_ROW_HALF_MIRROR, 0xf>(v, v);
    v = w < v ? w : v;
    w = dpp_u64<DPP_ROW_MIRROR, 0xf>(v, v);
    v = w < v ? w : v;
    if (G >= 32) {
        w = __shfl_xor(v, 16);
        v = w < v ? w : v;
    }
    if (G >= 64) {
        w = __shfl_xor(v, 32);
        v = w < v ? w : v;
    }
    return v;
}

template <int G>
__device__ __forceinline__ unsigned long long gor_u64(unsigned long long v)
{
    v |= dpp_u64<DPP_QUAD_1032, 0xf>(0ull, v);
    v |= dpp_u64<DPP_QUAD_2301, 0xf>(0ull, v);
    v |= dpp_u64<DPP_ROW_HALF_MIRROR, 0xf>(0ull, v);
    v |= dpp_u64<DPP_ROW_MIRROR, 0xf>(0ull, v);
    if (G >= 32) v |= __shfl_xor(v, 16);
    if (G >= 64) v |= __shfl_xor(v, 32);
    return v;
}

// inclusive prefix sum inside the group
template <int G>
__device__ __forceinline__ int gscan_incl(int v)
{
    v = v + dpp_i32<DPP_ROW_SHR1, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_SHR2, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_SHR4, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_SHR8, 0xf>(0, v);
    if (G >= 32) v = v + dpp_i32<DPP_ROW_BCAST15, 0xa>(0, v);
    if (G >= 64) v = v + dpp_i32<DPP_ROW_BCAST31, 0xc>(0, v);
    return v;
}

// exclusive prefix of small counts (< 2^BITS) inside the group
template <int G, int BITS>
__device__ __forceinline__ int gballot_scan(int v, int gb, int gl, int &total)
{
    int r = 0, t = 0;
#pragma unroll
    for (int b = 0; b < BITS; b++) {
        unsigned long long m = gballot<G>((v >> b) & 1, gb);
        r += grank(m, gl) << b;
        t += __popcll(m) << b;
    }
    total = t;
    return r;
}

template <int G, int S, int MAXP>
struct GLDS {
    double pq[MAXP][4];
    int32_t plab[MAXP];
    uint8_t psh[MAXP];
    uint8_t pwall[MAXP];
    uint8_t etab[MAXP][MAXP];
    union {
        struct {
            double pos[G * S][3];
            uint32_t tpl[G * S];
            int32_t lab[G * S];
        } st;
        struct {
            double cq[G][4];
            int32_t cid[G];
            uint8_t ccode[G];
            double npos[G][3];
        } gc;
    } u;
    uint16_t bedge[G * S + 8];
    int32_t cpre[G];
    int32_t cbeg[G];
    uint8_t csh[G];
    int32_t forder[MAXP];
    int32_t fref[MAXP];
    int32_t fo[kFoLen];
};

template <int G, int S, int MAXP>
__device__ __forceinline__ PlaneD gplane(const GLDS<G, S, MAXP> &sh, int k)
{
    PlaneD p;
    p.n0 = sh.pq[k][0];
    p.n1 = sh.pq[k][1];
    p.n2 = sh.pq[k][2];
    p.h = sh.pq[k][3];
    p.wall = sh.pwall[k];
    return p;
}

// one cell, held by a group (all masks are the group's bit fields)
template <int S, bool F32>
struct GCell {
    uint32_t tp[S];
    double vx[S], vy[S], vz[S];
    float fx[S], fy[S], fz[S];
    unsigned long long live[S];
    unsigned long long used;  // plane slots in use (bit k)
    double R2, R;
};

template <int G, int S, bool F32>
__device__ __forceinline__ void g_update_radius(GCell<S, F32> &c, int gl)
{
    double m = 0.0;
#pragma unroll
    for (int s = 0; s < S; s++)
        if ((c.live[s] >> gl) & 1) m = fmax(m, c.vx[s] * c.vx[s] + c.vy[s] * c.vy[s] + c.vz[s] * c.vz[s]);
    c.R2 = gmax<G>(m);
    c.R = sqrt(c.R2);
}

template <int MAXP>
__device__ __forceinline__ int g_free_plane(unsigned long long used)
{
    constexpr unsigned long long valid = MAXP >= 64 ? ~0ull : ((1ull << MAXP) - 1ull);
    unsigned long long fr = ~used & valid;
    return fr ? __builtin_ctzll(fr) : -1;
}

template <int G, int S, int MAXP, bool F32>
__device__ __forceinline__ int g_consider(const CellArgs &A, GLDS<G, S, MAXP> &sh, GCell<S, F32> &c, double q0,
                                          double q1, double q2, double d2, int32_t lab, int code, double *ws,
                                          unsigned long long *cnt, int lane, int gl, int gb)
{
    const double h = 0.5 * d2;
    const double Mub = (fabs(q0) + fabs(q1) + fabs(q2)) * c.R + h;
    const double band = A.tau * Mub;
    unsigned long long conf[S], inb[S];
    int ntest = 0;
    if (F32) {
        const float g0 = (float)q0, g1 = (float)q1, g2 = (float)q2, gh = (float)h;
        const float band32 = 0x1p-21f * ((fabsf(g0) + fabsf(g1) + fabsf(g2)) * ((float)c.R * 1.0000001f) + gh);
        unsigned long long uns = 0, unsr[S];
#pragma unroll
        for (int s = 0; s < S; s++) {
            bool lv = (c.live[s] >> gl) & 1;
            float sv = fmaf(g0, c.fx[s], fmaf(g1, c.fy[s], fmaf(g2, c.fz[s], -gh)));
            conf[s] = gballot<G>(lv && sv > band32, gb);
            unsr[s] = gballot<G>(lv && !(sv > band32) && !(sv < -band32), gb);
            inb[s] = 0;
            uns |= unsr[s];
            ntest += __popcll(c.live[s]);
        }
        if (uns) {
#pragma unroll
            for (int s = 0; s < S; s++) {
                bool u = (unsr[s] >> gl) & 1;
                double sv = fma(q0, c.vx[s], fma(q1, c.vy[s], fma(q2, c.vz[s], -h)));
                conf[s] |= gballot<G>(u && sv > band, gb);
                inb[s] = gballot<G>(u && !(sv > band) && !(sv < -band), gb);
                cnt[DC_RECHECK] += __popcll(unsr[s]);
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < S; s++) {
            bool lv = (c.live[s] >> gl) & 1;
            double sv = fma(q0, c.vx[s], fma(q1, c.vy[s], fma(q2, c.vz[s], -h)));
            conf[s] = gballot<G>(lv && sv > band, gb);
            inb[s] = gballot<G>(lv && !(sv > band) && !(sv < -band), gb);
            ntest += __popcll(c.live[s]);
        }
    }
    cnt[DC_TESTS] += ntest;
    // in-band vertices: exact decision, one lane of the wave at a time
#pragma unroll
    for (int s = 0; s < S; s++) {
        unsigned long long wm = __ballot((inb[s] >> gl) & 1);
        while (wm) {
            int l = __builtin_ctzll(wm);
            wm &= wm - 1;
            int sg = 0;
            if (lane == l) {
                PlaneD pp = {q0, q1, q2, h, 0};
                sg = exact_side3(gplane(sh, c.tp[s] & 0xff), gplane(sh, (c.tp[s] >> 8) & 0xff),
                                 gplane(sh, (c.tp[s] >> 16) & 0xff), pp, ws);
            }
            sg = __builtin_amdgcn_readlane(sg, l);
            if ((l / G) == (lane / G)) {
                if (sg > 0) conf[s] |= 1ull << (l % G);
                cnt[DC_EXACT]++;
            }
        }
    }
    unsigned long long anyc = 0;
#pragma unroll
    for (int s = 0; s < S; s++) anyc |= conf[s];
    if (!anyc) return ST_OK;

    // ---- cut ----
    int p = g_free_plane<MAXP>(c.used);
    if (p < 0) {
        unsigned long long u = 0;
#pragma unroll
        for (int s = 0; s < S; s++)
            if ((c.live[s] >> gl) & 1)
#pragma unroll
                for (int k = 0; k < 3; k++) u |= 1ull << ((c.tp[s] >> (8 * k)) & 0xff);
        c.used = gor_u64<G>(u);
        p = g_free_plane<MAXP>(c.used);
        if (p < 0) return ST_CAP;
    }
    uint32_t bfl = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        if ((conf[s] >> gl) & 1) {
            uint32_t t3 = c.tp[s];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
                int tw = sh.etab[b][a] & (G * S - 1);
                unsigned long long cw = 0;
#pragma unroll
                for (int r = 0; r < S; r++)
                    if (tw / G == r) cw = conf[r];
                if (!((cw >> (tw % G)) & 1)) bfl |= 1u << (s * 3 + k);
            }
        }
    }
    int nb = __popc(bfl);
    int m;
    int o = gballot_scan<G, (S <= 2 ? 3 : 4)>(nb, gb, gl, m);
    int nfree = 0;
#pragma unroll
    for (int s = 0; s < S; s++) nfree += __popcll((~c.live[s] | conf[s]) & Grp<G>::MASK);
    if (m > nfree || m > G * S + 8) return ST_CAP;
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
    if (gl == 0) {
        sh.pq[p][0] = q0;
        sh.pq[p][1] = q1;
        sh.pq[p][2] = q2;
        sh.pq[p][3] = h;
        sh.plab[p] = lab;
        sh.psh[p] = (uint8_t)code;
        sh.pwall[p] = 0;
    }
    lds_sync();
    // free slots in slot order take the new triangles (a, b, p) by rank
    int rk[S];
    bool take[S];
    int before = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        unsigned long long fr = (~c.live[s] | conf[s]) & Grp<G>::MASK;
        rk[s] = before + grank(fr, gl);
        take[s] = ((fr >> gl) & 1) && rk[s] < m;
        before += __popcll(fr);
    }
    // new vertices, G at a time, staged in LDS
    for (int k0 = 0; k0 < m; k0 += G) {
        int k = k0 + gl;
        if (k < m) {
            uint16_t e = sh.bedge[k];
            double x, y, z;
            cramer(sh.pq[e & 0xff], sh.pq[e >> 8], sh.pq[p], x, y, z);
            sh.u.gc.npos[gl][0] = x;
            sh.u.gc.npos[gl][1] = y;
            sh.u.gc.npos[gl][2] = z;
        }
        lds_sync();
#pragma unroll
        for (int s = 0; s < S; s++) {
            if (take[s] && rk[s] >= k0 && rk[s] < k0 + G) {
                uint16_t e = sh.bedge[rk[s]];
                int a = e & 0xff, b = e >> 8;
                c.tp[s] = (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)p << 16);
                c.vx[s] = sh.u.gc.npos[rk[s] - k0][0];
                c.vy[s] = sh.u.gc.npos[rk[s] - k0][1];
                c.vz[s] = sh.u.gc.npos[rk[s] - k0][2];
                if (F32) {
                    c.fx[s] = (float)c.vx[s];
                    c.fy[s] = (float)c.vy[s];
                    c.fz[s] = (float)c.vz[s];
                }
                uint8_t t = (uint8_t)(s * G + gl);
                sh.etab[a][b] = t;
                sh.etab[b][p] = t;
                sh.etab[p][a] = t;
            }
        }
        lds_sync();
    }
#pragma unroll
    for (int s = 0; s < S; s++) c.live[s] = (c.live[s] & ~conf[s]) | gballot<G>(take[s], gb);
    c.used |= 1ull << p;
    lds_sync();
    g_update_radius<G, S, F32>(c, gl);
    cnt[DC_CUTS]++;
    cnt[DC_NEWV] += m;
    return c.R2 < 1e300 ? ST_OK : ST_CAP;
}

// particles of up to G blocks (one per lane), fed to the cell nearest first
template <int G, int S, int MAXP, bool F32>
__device__ __forceinline__ int g_gather(const CellArgs &A, GLDS<G, S, MAXP> &sh, GCell<S, F32> &c, const Tess &T,
                                        int si, const double *p, const int *bc, int dx, int dy, int dz, bool valid,
                                        double *ws, unsigned long long *cnt, int lane, int gl, int gb)
{
    const Grid &G3 = T.G;
    int dd[3] = {dx, dy, dz};
    int bb[3], sv[3];
    bool ok = valid;
    double d2b = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        int t = bc[d] + dd[d];
        if (G3.per[d]) {
            int g = G3.g[d];
            int w = ((t % g) + g) % g;
            sv[d] = (t - w) / g;
            bb[d] = w;
            if (sv[d] > 2 || sv[d] < -2) ok = false;
        } else {
            sv[d] = 0;
            bb[d] = t;
            if (t < 0 || t >= G3.g[d]) ok = false;
        }
        double blo = G3.lo[d] + t * G3.bs[d];
        double e = fmax(0.0, fmax(blo - p[d], p[d] - (blo + G3.bs[d])));
        d2b += e * e;
    }
    if (d2b >= 4.0 * c.R2 * kMargin) ok = false;
    int cntb = 0, beg = 0;
    if (ok) {
        int64_t blk = T.bbase + bb[0] + (int64_t)G3.g[0] * (bb[1] + (int64_t)G3.g[1] * bb[2]);
        beg = A.start[blk];
        cntb = A.start[blk + 1] - beg;
    }
    cnt[DC_BLOCKS] += __popcll(gballot<G>(ok, gb));
    int incl = gscan_incl<G>(cntb);
    int total = __shfl(incl, gb + G - 1);
    if (total == 0) return ST_OK;
    lds_sync();
    sh.cpre[gl] = incl - cntb;
    sh.cbeg[gl] = beg;
    sh.csh[gl] = (uint8_t)(25 * (sv[2] + 2) + 5 * (sv[1] + 2) + (sv[0] + 2));
    lds_sync();
    for (int c0 = 0; c0 < total; c0 += G) {
        int ci = c0 + gl;
        unsigned long long key = ~0ull;
        if (ci < total) {
            int lo = 0, hi = G - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (sh.cpre[mid] <= ci) lo = mid; else hi = mid - 1;
            }
            int idx = sh.cbeg[lo] + (ci - sh.cpre[lo]);
            int code = sh.csh[lo];
            int s0 = code % 5 - 2, s1 = (code / 5) % 5 - 2, s2 = code / 25 - 2;
            Particle q = A.part[idx];
            double a0 = q.x - p[0], a1 = q.y - p[1], a2 = q.z - p[2];
            if (s0) a0 = a0 + s0 * G3.L[0];
            if (s1) a1 = a1 + s1 * G3.L[1];
            if (s2) a2 = a2 + s2 * G3.L[2];
            double d2 = a0 * a0 + a1 * a1 + a2 * a2;
            bool self = (idx == si) && code == kNoShift;
            if (!self && d2 < 4.0 * c.R2 * kMargin) key = __double_as_longlong(d2);
            sh.u.gc.cq[gl][0] = a0;
            sh.u.gc.cq[gl][1] = a1;
            sh.u.gc.cq[gl][2] = a2;
            sh.u.gc.cq[gl][3] = d2;
            sh.u.gc.cid[gl] = q.id;
            sh.u.gc.ccode[gl] = (uint8_t)code;
        }
        lds_sync();
        for (;;) {
            unsigned long long mk = gmin_u64<G>(key);
            if (mk == ~0ull) break;
            double md2 = __longlong_as_double((long long)mk);
            if (!(md2 < 4.0 * c.R2 * kMargin)) break;
            int ol = __builtin_ctzll(gballot<G>(key == mk, gb));
            if (gl == ol) key = ~0ull;
            cnt[DC_CAND]++;
            if (md2 == 0.0) return ST_DUP;
            int st = g_consider<G, S, MAXP, F32>(A, sh, c, sh.u.gc.cq[ol][0], sh.u.gc.cq[ol][1], sh.u.gc.cq[ol][2],
                                                 md2, sh.u.gc.cid[ol], sh.u.gc.ccode[ol], ws, cnt, lane, gl, gb);
            if (st != ST_OK) return st;
        }
        lds_sync();
    }
    return ST_OK;
}

template <int G, int S, int MAXP, bool F32>
__device__ __forceinline__ int g_cell_run(const CellArgs &A, GLDS<G, S, MAXP> &sh, int si, double *ws,
                                          unsigned long long *cnt, int lane, int gl, int gb)
{
    const Particle me = A.part[si];
    const Tess &T = A.tess[me.tess];
    const Grid &G3 = T.G;
    const double p[3] = {me.x, me.y, me.z};
    const int id = me.id;
    int bc[3];
    double mrg[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        bc[d] = block_coord(G3, p[d], d);
        double blo = G3.lo[d] + bc[d] * G3.bs[d];
        mrg[d] = fmin(p[d] - blo, blo + G3.bs[d] - p[d]);
    }
    GCell<S, F32> c;
    if (gl < 6) {
        int d = gl >> 1, side = gl & 1;
        double sg = side ? 1.0 : -1.0;
        double n[3] = {0.0, 0.0, 0.0};
        double h;
        if (G3.per[d]) {
            double L = G3.L[d];
            n[d] = sg * L;
            h = 0.5 * (L * L);
            sh.pwall[gl] = 0;
            sh.plab[gl] = id;
            sh.psh[gl] = (uint8_t)(kNoShift + (side ? 1 : -1) * (d == 0 ? 1 : (d == 1 ? 5 : 25)));
        } else {
            n[d] = sg;
            h = side ? (G3.hi[d] - p[d]) : -(G3.lo[d] - p[d]);
            sh.pwall[gl] = 1;
            sh.plab[gl] = -(2 * d + side + 1);
            sh.psh[gl] = kNoShift;
        }
        sh.pq[gl][0] = n[0];
        sh.pq[gl][1] = n[1];
        sh.pq[gl][2] = n[2];
        sh.pq[gl][3] = h;
    }
#pragma unroll
    for (int s = 0; s < S; s++) {
        c.tp[s] = 0;
        c.vx[s] = c.vy[s] = c.vz[s] = 0.0;
        c.fx[s] = c.fy[s] = c.fz[s] = 0.0f;
        c.live[s] = 0;
    }
    c.live[0] = 0xffull;
    if (gl < 8) {
        int bx = gl & 1, by = (gl >> 1) & 1, bz = (gl >> 2) & 1;
        int X = bx, Y = 2 + by, Z = 4 + bz;
        int neg = 3 - bx - by - bz;
        c.tp[0] = (neg & 1) ? (X | (Z << 8) | (Y << 16)) : (X | (Y << 8) | (Z << 16));
        double e[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            int b = (gl >> d) & 1;
            if (G3.per[d]) e[d] = b ? 0.5 * G3.L[d] : -(0.5 * G3.L[d]);
            else e[d] = b ? (G3.hi[d] - p[d]) : (G3.lo[d] - p[d]);
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
            sh.etab[a][b] = (uint8_t)gl;
        }
    }
    c.used = 0x3full;
    lds_sync();
    g_update_radius<G, S, F32>(c, gl);

    bool finished = false;
    for (int o0 = 0; o0 < A.noff; o0 += G) {
        if (A.offs[o0].m * T.bsmin2 >= 4.0 * c.R2 * kMargin) {
            finished = true;
            break;
        }
        int o = o0 + gl;
        bool v = o < A.noff;
        Offset of = v ? A.offs[o] : Offset{0, 0, 0, 0};
        int st = g_gather<G, S, MAXP, F32>(A, sh, c, T, si, p, bc, of.dx, of.dy, of.dz, v, ws, cnt, lane, gl, gb);
        if (st != ST_OK) return st;
    }
    if (!finished) {
        cnt[DC_FALLBACK]++;
        for (int r = A.off_radius + 1;; r++) {
            if (r > kMaxShell || !(c.R2 < 1e300)) return ST_CAP;
            double lb = 1e300;
            bool exists = false;
#pragma unroll
            for (int d = 0; d < 3; d++) {
                lb = fmin(lb, (r - 1) * G3.bs[d] + mrg[d]);
                if (G3.per[d] || bc[d] - r >= 0 || bc[d] + r < G3.g[d]) exists = true;
            }
            if (!exists) break;
            if (lb > 0.0 && lb * lb >= 4.0 * c.R2 * kMargin) break;
            int side = 2 * r + 1;
            int tot = side * side * side;
            for (int c0 = 0; c0 < tot; c0 += G) {
                int ix = c0 + gl;
                int dx = ix % side - r, dy = (ix / side) % side - r, dz = ix / (side * side) - r;
                int ch = max(abs(dx), max(abs(dy), abs(dz)));
                bool v = ix < tot && ch == r;
                if (!gballot<G>(v, gb)) continue;
                int st = g_gather<G, S, MAXP, F32>(A, sh, c, T, si, p, bc, dx, dy, dz, v, ws, cnt, lane, gl, gb);
                if (st != ST_OK) return st;
            }
        }
    }

    // ---- statistics ----
    lds_sync();
#pragma unroll
    for (int s = 0; s < S; s++) {
        int t = s * G + gl;
        bool lv = (c.live[s] >> gl) & 1;
        sh.u.st.tpl[t] = lv ? c.tp[s] : 0xffffffffu;
        sh.u.st.pos[t][0] = c.vx[s];
        sh.u.st.pos[t][1] = c.vy[s];
        sh.u.st.pos[t][2] = c.vz[s];
        sh.u.st.lab[t] = t;
    }
    for (int k = gl; k < MAXP; k += G) {
        sh.forder[k] = 0;
        sh.fref[k] = 0x7fffffff;
    }
    for (int k = gl; k < kFoLen; k += G) sh.fo[k] = 0;
    lds_sync();
    for (int t = gl; t < S * G; t += G) {
        uint32_t t3 = sh.u.st.tpl[t];
        if (t3 == 0xffffffffu) continue;
        for (int k = 0; k < 3; k++) atomicMin(&sh.fref[(t3 >> (8 * k)) & 0xff], t);
    }
    lds_sync();
    uint32_t zb = 0, ib = 0;
    for (int j = 0; j < 3 * S; j++) {
        int t = (j / 3) * G + gl, k = j % 3;
        uint32_t t3 = sh.u.st.tpl[t];
        if (t3 == 0xffffffffu) continue;
        int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
        uint32_t w3 = sh.u.st.tpl[sh.etab[b][a] & (G * S - 1)];
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
            unsigned long long wm = __ballot((ib >> j) & 1);
            while (wm) {
                int l = __builtin_ctzll(wm);
                wm &= wm - 1;
                if (lane == l) {
                    int t = (j / 3) * G + gl, k = j % 3;
                    uint32_t t3 = sh.u.st.tpl[t];
                    int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
                    uint32_t w3 = sh.u.st.tpl[sh.etab[b][a] & (G * S - 1)];
                    int d = (int)(w3 & 0xff) + (int)((w3 >> 8) & 0xff) + (int)((w3 >> 16) & 0xff) - a - b;
                    d = min(max(d, 0), MAXP - 1);
                    int sg = exact_side3(gplane(sh, t3 & 0xff), gplane(sh, (t3 >> 8) & 0xff),
                                         gplane(sh, (t3 >> 16) & 0xff), gplane(sh, d), ws);
                    if (sg == 0) zb |= 1u << j;
                }
                if ((l / G) == (lane / G)) cnt[DC_EXACT]++;
            }
        }
    }
    double v6 = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int j = 0; j < 3 * S; j++) {
        int t = (j / 3) * G + gl, k = j % 3;
        uint32_t t3 = sh.u.st.tpl[t];
        if (t3 == 0xffffffffu) continue;
        int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
        if (!((zb >> j) & 1)) atomicAdd(&sh.forder[a], 1);
        const double *r = sh.u.st.pos[sh.fref[a]];
        const double *w = sh.u.st.pos[sh.etab[b][a] & (G * S - 1)];
        const double *v = sh.u.st.pos[t];
        double det = r[0] * (w[1] * v[2] - w[2] * v[1]) - r[1] * (w[0] * v[2] - w[2] * v[0]) +
                     r[2] * (w[0] * v[1] - w[1] * v[0]);
        v6 += det;
        m0 += det * (r[0] + w[0] + v[0]);
        m1 += det * (r[1] + w[1] + v[1]);
        m2 += det * (r[2] + w[2] + v[2]);
    }
    int nvert = 0;
#pragma unroll
    for (int s = 0; s < S; s++) nvert += __popcll(c.live[s]);
    if (gballot<G>(zb != 0, gb)) {
        for (int it = 0; it < 4 * S * G; it++) {
            bool ch = false;
            for (int j = 0; j < 3 * S; j++) {
                if (!((zb >> j) & 1)) continue;
                int t = (j / 3) * G + gl, k = j % 3;
                uint32_t t3 = sh.u.st.tpl[t];
                int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
                int o = sh.u.st.lab[sh.etab[b][a] & (G * S - 1)];
                if (o < sh.u.st.lab[t]) {
                    sh.u.st.lab[t] = o;
                    ch = true;
                }
            }
            lds_sync();
            if (!gballot<G>(ch, gb)) break;
        }
        nvert = 0;
        for (int t0 = 0; t0 < S * G; t0 += G) {
            int t = t0 + gl;
            nvert += __popcll(gballot<G>(sh.u.st.tpl[t] != 0xffffffffu && sh.u.st.lab[t] == t, gb));
        }
    }
    lds_sync();
    int rk = 0, sumord = 0;
    for (int k0 = 0; k0 < MAXP; k0 += G) {
        int k = k0 + gl;
        int ord = k < MAXP ? sh.forder[k] : 0;
        bool real = ord >= 3;
        unsigned long long rb = gballot<G>(real, gb);
        int rank = rk + grank(rb, gl);
        if (real) {
            if (ord < kFoLen) atomicAdd(&sh.fo[ord], 1);
            if ((A.mask & (16 | 32)) && A.nbr && rank < kMaxNbr) {
                A.nbr[(int64_t)id * kMaxNbr + rank] = sh.plab[k];
                A.nsh[(int64_t)id * kMaxNbr + rank] = sh.psh[k];
            }
        }
        rk += __popcll(rb);
        sumord += gisum<G>(real ? ord : 0);
    }
    int nface = rk;
    double vol6 = gsum<G>(v6);
    double M0 = gsum<G>(m0), M1 = gsum<G>(m1), M2 = gsum<G>(m2);
    lds_sync();
    if (gl == 0) {
        double vol = vol6 / 6.0;
        if (A.vol) A.vol[id] = vol;
        if (A.cen) {
            A.cen[3 * (int64_t)id + 0] = M0 / (4.0 * vol6);
            A.cen[3 * (int64_t)id + 1] = M1 / (4.0 * vol6);
            A.cen[3 * (int64_t)id + 2] = M2 / (4.0 * vol6);
        }
        if (A.nv) A.nv[id] = nvert;
        if (A.ne) A.ne[id] = sumord / 2;
        if (A.nf) A.nf[id] = nface;
    }
    if (A.fo)
        for (int k = gl; k < kFoLen; k += G) A.fo[(int64_t)id * kFoLen + k] = (uint8_t)min(sh.fo[k], 255);
    return nface > kMaxNbr ? ST_CAP : ST_OK;
}

// occupancy target of two waves per SIMD (the LDS of four cells allows about
// two): the register allocator is held to that budget
template <int G, int S, int MAXP, bool F32>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_cells_group(CellArgs A)
{
    static_assert(((G * S) & (G * S - 1)) == 0 && G * S <= 256, "slot count must be a power of two");
    __shared__ GLDS<G, S, MAXP> shv[Grp<G>::CPW];
    const int lane = __lane_id();
    const int gl = lane % G, gb = lane - gl;
    GLDS<G, S, MAXP> &sh = shv[lane / G];
    double *ws = A.xscratch + (size_t)blockIdx.x * A.xscratch_len;
    unsigned long long cnt[DC_N];
#pragma unroll
    for (int k = 0; k < DC_N; k++) cnt[k] = 0;
    const int ncell = A.ncell;
    for (;;) {
        int base = 0;
        if (gl == 0) base = atomicAdd(A.queue, A.chunk);
        base = __shfl(base, gb);
        if (base >= ncell) break;
        int end = min(base + A.chunk, ncell);
        for (int ci = base; ci < end; ci++) {
            int si = A.cell_list ? A.cell_list[ci] : ci;
            int st = g_cell_run<G, S, MAXP, F32>(A, sh, si, ws, cnt, lane, gl, gb);
            int id = A.part[si].id;
            if (st != ST_OK && A.fo)
                for (int k = gl; k < kFoLen; k += G) A.fo[(int64_t)id * kFoLen + k] = 0;
            if (gl == 0) {
                if (st != ST_OK) {
                    if (A.vol) A.vol[id] = __builtin_nan("");
                    if (A.cen) A.cen[3 * (int64_t)id] = A.cen[3 * (int64_t)id + 1] = A.cen[3 * (int64_t)id + 2] = __builtin_nan("");
                    if (A.nv) A.nv[id] = 0;
                    if (A.ne) A.ne[id] = 0;
                    if (A.nf) A.nf[id] = 0;
                }
                if (st == ST_OK) {
                    A.status[id] = 0;
                } else if (st == ST_DUP) {
                    A.status[id] = 3;
                } else {
                    A.status[id] = 1;
                    int pos = atomicAdd(A.spill_count, 1);
                    A.spill_list[pos] = si;
                    cnt[DC_SPILL]++;
                }
            }
            lds_sync();
        }
    }
    // counters: every group's leader adds its cell's totals
    if (gl == 0) {
#pragma unroll
        for (int k = 0; k < DC_N; k++)
            if (cnt[k]) atomicAdd(&A.diag[k], cnt[k]);
    }
}

}  // namespace

hipError_t launch_cells_group(const CellArgs &a, int precision, int cpw, int waves, hipStream_t s)
{
    if (cpw == 4) {
        if (precision == 1) k_cells_group<16, 4, 32, true><<<waves, 64, 0, s>>>(a);
        else k_cells_group<16, 4, 32, false><<<waves, 64, 0, s>>>(a);
    } else if (cpw == 2) {
        if (precision == 1) k_cells_group<32, 2, 40, true><<<waves, 64, 0, s>>>(a);
        else k_cells_group<32, 2, 40, false><<<waves, 64, 0, s>>>(a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vc
