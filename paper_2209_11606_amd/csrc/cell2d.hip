// cell2d.hip -- per-particle 2D Voronoi cells (the planar form of section
// 2.1: the cell starts as the box of Eq. 1-2 and is cut by the bisector
// half-planes of Eq. 3 in nearest-first order until the radius bound holds).
//
// A cell is a convex polygon held by a group of G lanes (64/G cells per
// wave).  Each polygon vertex is a pair of line ids (a, b): the edge that
// enters it lies on line a, the edge that leaves it on line b, counter-
// clockwise.  LDS maps byin[l] / byout[l] name the vertex whose entering /
// leaving edge lies on line l, so the neighbours of a vertex are one read
// away.  A cut by line p removes the contiguous run of outside vertices; its
// first vertex (a, .) and last vertex (., b) give the two new vertices
// (a, p) and (p, b).  Side decisions as in 3D: FP64 (or FP32 with an FP64
// recheck) outside a band, exact inside it.
#include "cell_common.h"

namespace vc {

namespace {

__device__ __forceinline__ void lds_sync2()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

template <int G>
__device__ __forceinline__ unsigned long long gb2(bool p, int gb)
{
    constexpr unsigned long long M = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    return (__ballot(p) >> gb) & M;
}

template <int G>
__device__ __forceinline__ double g2max(double v)
{
    if (G >= 2) v = fmax(v, dpp_f64<DPP_QUAD_1032, 0xf>(v, v));
    if (G >= 4) v = fmax(v, dpp_f64<DPP_QUAD_2301, 0xf>(v, v));
    if (G >= 8) v = fmax(v, dpp_f64<DPP_ROW_HALF_MIRROR, 0xf>(v, v));
    if (G >= 16) v = fmax(v, dpp_f64<DPP_ROW_MIRROR, 0xf>(v, v));
    if (G >= 32) v = fmax(v, __shfl_xor(v, 16));
    if (G >= 64) v = fmax(v, __shfl_xor(v, 32));
    return v;
}

template <int G>
__device__ __forceinline__ double g2sum(double v)
{
    if (G >= 2) v = v + dpp_f64<DPP_QUAD_1032, 0xf>(0.0, v);
    if (G >= 4) v = v + dpp_f64<DPP_QUAD_2301, 0xf>(0.0, v);
    if (G >= 8) v = v + dpp_f64<DPP_ROW_HALF_MIRROR, 0xf>(0.0, v);
    if (G >= 16) v = v + dpp_f64<DPP_ROW_MIRROR, 0xf>(0.0, v);
    if (G >= 32) v = v + __shfl_xor(v, 16);
    if (G >= 64) v = v + __shfl_xor(v, 32);
    return v;
}

template <int G>
__device__ __forceinline__ unsigned long long g2min_u64(unsigned long long v)
{
    unsigned long long w;
    if (G >= 2) { w = dpp_u64<DPP_QUAD_1032, 0xf>(v, v); v = w < v ? w : v; }
    if (G >= 4) { w = dpp_u64<DPP_QUAD_2301, 0xf>(v, v); v = w < v ? w : v; }
    if (G >= 8) { w = dpp_u64<DPP_ROW_HALF_MIRROR, 0xf>(v, v); v = w < v ? w : v; }
    if (G >= 16) { w = dpp_u64<DPP_ROW_MIRROR, 0xf>(v, v); v = w < v ? w : v; }
    if (G >= 32) { w = __shfl_xor(v, 16); v = w < v ? w : v; }
    if (G >= 64) { w = __shfl_xor(v, 32); v = w < v ? w : v; }
    return v;
}

template <int G>
__device__ __forceinline__ unsigned long long g2or_u64(unsigned long long v)
{
    if (G >= 2) v |= dpp_u64<DPP_QUAD_1032, 0xf>(0ull, v);
    if (G >= 4) v |= dpp_u64<DPP_QUAD_2301, 0xf>(0ull, v);
    if (G >= 8) v |= dpp_u64<DPP_ROW_HALF_MIRROR, 0xf>(0ull, v);
    if (G >= 16) v |= dpp_u64<DPP_ROW_MIRROR, 0xf>(0ull, v);
    if (G >= 32) v |= __shfl_xor(v, 16);
    if (G >= 64) v |= __shfl_xor(v, 32);
    return v;
}

// inclusive prefix sum inside a group of G lanes (G <= 16 stays in a row)
template <int G>
__device__ __forceinline__ int g2scan(int v, int gl)
{
    int w;
    w = dpp_i32<DPP_ROW_SHR1, 0xf>(0, v);
    if (G >= 2) v = v + ((gl % G) >= 1 ? w : 0);
    w = dpp_i32<DPP_ROW_SHR2, 0xf>(0, v);
    if (G >= 4) v = v + ((gl % G) >= 2 ? w : 0);
    w = dpp_i32<DPP_ROW_SHR4, 0xf>(0, v);
    if (G >= 8) v = v + ((gl % G) >= 4 ? w : 0);
    w = dpp_i32<DPP_ROW_SHR8, 0xf>(0, v);
    if (G >= 16) v = v + ((gl % G) >= 8 ? w : 0);
    if (G >= 32) v = v + dpp_i32<DPP_ROW_BCAST15, 0xa>(0, v);
    if (G >= 64) v = v + dpp_i32<DPP_ROW_BCAST31, 0xc>(0, v);
    return v;
}

template <int G, int S, int MAXL>
struct L2 {
    double lq[MAXL][3];   // line normal (n0, n1) and offset h
    double lrj[MAXL];     // radius of each line's neighbour (radical lines)
    int32_t llab[MAXL];
    uint8_t lsh[MAXL];
    uint8_t lwall[MAXL];
    uint8_t byin[MAXL];   // slot of the vertex whose entering edge lies on line l
    uint8_t byout[MAXL];  // slot of the vertex whose leaving edge lies on line l
    union alignas(16) {
        struct {
            double pos[G * S][2];
            uint32_t tpl[G * S];
        } st;
        struct {
            double cq[G][3];
            double ch[G];     // line offsets h
            double crj[G];    // neighbour radii
            int32_t cid[G];
            uint8_t ccode[G];
            double nv[2][2];
            uint32_t nt[2];
        } gc;
    } u;
    int32_t cpre[G];
    int32_t cbeg[G];
    uint8_t csh[G];
};

template <int G, int S, int MAXL>
__device__ __forceinline__ PlaneD line_of(const L2<G, S, MAXL> &sh, int k)
{
    PlaneD p;
    p.n0 = sh.lq[k][0];
    p.n1 = sh.lq[k][1];
    p.n2 = 0.0;
    p.h = sh.lq[k][2];
    p.wall = sh.lwall[k];
    return p;
}

template <int G, int S, int MAXL>
__device__ __forceinline__ PlaneR line_r(const L2<G, S, MAXL> &sh, int k, double ri)
{
    return PlaneR{line_of(sh, k), ri, sh.lrj[k]};
}

template <int S, bool F32>
struct Poly {
    uint32_t tp[S];  // a | b << 8
    double vx[S], vy[S];
    float fx[S], fy[S];
    unsigned long long live[S];
    unsigned long long used;
    double R2, R;
    double lim;   // squared search radius
    double ri;    // the particle's radius (radical tessellation), else 0
};

template <int G, int S, bool F32>
__device__ __forceinline__ void p_radius(Poly<S, F32> &c, int gl, const CellArgs &A)
{
    double m = 0.0;
#pragma unroll
    for (int s = 0; s < S; s++)
        if ((c.live[s] >> gl) & 1) m = fmax(m, c.vx[s] * c.vx[s] + c.vy[s] * c.vy[s]);
    c.R2 = g2max<G>(m);
    c.R = sqrt(c.R2);
    c.lim = search_lim(c.R2, c.R, A, c.ri);
}

template <int G, int S, int MAXL, bool F32>
__device__ __forceinline__ int p_consider(const CellArgs &A, L2<G, S, MAXL> &sh, Poly<S, F32> &c, double q0,
                                          double q1, double h, double rj, int32_t lab, int code, double *ws,
                                          unsigned long long *cnt, int lane, int gl, int gb)
{
    const bool rad = A.rad != nullptr;
    const double band = A.tau * ((fabs(q0) + fabs(q1)) * c.R + fabs(h));
    unsigned long long conf[S], inb[S];
    int ntest = 0;
    if (F32) {
        const float g0 = (float)q0, g1 = (float)q1, gh = (float)h;
        const float band32 = A.tau32 * ((fabsf(g0) + fabsf(g1)) * ((float)c.R * 1.0000001f) + fabsf(gh));
        unsigned long long uns = 0, unsr[S];
#pragma unroll
        for (int s = 0; s < S; s++) {
            bool lv = (c.live[s] >> gl) & 1;
            float sv = fmaf(g0, c.fx[s], fmaf(g1, c.fy[s], -gh));
            conf[s] = gb2<G>(lv && sv > band32, gb);
            unsr[s] = gb2<G>(lv && !(sv > band32) && !(sv < -band32), gb);
            inb[s] = 0;
            uns |= unsr[s];
            ntest += __popcll(c.live[s]);
        }
        if (uns) {
#pragma unroll
            for (int s = 0; s < S; s++) {
                bool u = (unsr[s] >> gl) & 1;
                double sv = fma(q0, c.vx[s], fma(q1, c.vy[s], -h));
                conf[s] |= gb2<G>(u && sv > band, gb);
                inb[s] = gb2<G>(u && !(sv > band) && !(sv < -band), gb);
                cnt[DC_RECHECK] += __popcll(unsr[s]);
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < S; s++) {
            bool lv = (c.live[s] >> gl) & 1;
            double sv = fma(q0, c.vx[s], fma(q1, c.vy[s], -h));
            conf[s] = gb2<G>(lv && sv > band, gb);
            inb[s] = gb2<G>(lv && !(sv > band) && !(sv < -band), gb);
            ntest += __popcll(c.live[s]);
        }
    }
    cnt[DC_TESTS] += ntest;
    unsigned long long zero[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        unsigned long long wm = __ballot((inb[s] >> gl) & 1);
        zero[s] = 0;
        while (wm) {
            int l = __builtin_ctzll(wm);
            wm &= wm - 1;
            int sg = 0;
            if (lane == l) {
                const PlaneD pp = {q0, q1, 0.0, h, 0};
                const int a = c.tp[s] & 0xff, b = (c.tp[s] >> 8) & 0xff;
                if (rad)
                    sg = exact_side2(line_r(sh, a, c.ri), line_r(sh, b, c.ri), PlaneR{pp, c.ri, rj}, ws);
                else
                    sg = exact_side2(line_of(sh, a), line_of(sh, b), pp, ws);
            }
            sg = __builtin_amdgcn_readlane(sg, l);
            if ((l / G) == (lane / G)) {
                if (sg > 0) conf[s] |= 1ull << (l % G);
                if (sg == 0) zero[s] |= 1ull << (l % G);
                cnt[DC_EXACT]++;
            }
        }
    }
    unsigned long long anyc = 0;
#pragma unroll
    for (int s = 0; s < S; s++) anyc |= conf[s];
    if (!anyc) return ST_OK;
    if (rad) {
        // a radical line can leave no vertex strictly inside: empty cell
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
    constexpr unsigned long long valid = MAXL >= 64 ? ~0ull : ((1ull << MAXL) - 1ull);
    unsigned long long fl = ~c.used & valid;
    if (!fl) {
        unsigned long long u = 0;
#pragma unroll
        for (int s = 0; s < S; s++)
            if ((c.live[s] >> gl) & 1) u |= (1ull << (c.tp[s] & 0xff)) | (1ull << ((c.tp[s] >> 8) & 0xff));
        c.used = g2or_u64<G>(u);
        fl = ~c.used & valid;
        if (!fl) return ST_CAP;
    }
    const int p = __builtin_ctzll(fl);
    // ends of the run of removed vertices
    bool first = false, last = false;
#pragma unroll
    for (int s = 0; s < S; s++) {
        if ((conf[s] >> gl) & 1) {
            int a = c.tp[s] & 0xff, b = (c.tp[s] >> 8) & 0xff;
            int pr = sh.byout[a] & (G * S - 1), su = sh.byin[b] & (G * S - 1);
            unsigned long long cp = 0, cs = 0;
#pragma unroll
            for (int r = 0; r < S; r++) {
                if (pr / G == r) cp = conf[r];
                if (su / G == r) cs = conf[r];
            }
            if (!((cp >> (pr % G)) & 1)) {
                first = true;
                double x, y;
                double Lp[3] = {q0, q1, h};
                cramer2(sh.lq[a], Lp, x, y);
                sh.u.gc.nv[0][0] = x;
                sh.u.gc.nv[0][1] = y;
                sh.u.gc.nt[0] = (uint32_t)a | ((uint32_t)p << 8);
            }
            if (!((cs >> (su % G)) & 1)) {
                last = true;
                double x, y;
                double Lp[3] = {q0, q1, h};
                cramer2(Lp, sh.lq[b], x, y);
                sh.u.gc.nv[1][0] = x;
                sh.u.gc.nv[1][1] = y;
                sh.u.gc.nt[1] = (uint32_t)p | ((uint32_t)b << 8);
            }
        }
    }
    // exactly one run: one first and one last vertex
    if (__popcll(gb2<G>(first, gb)) != 1 || __popcll(gb2<G>(last, gb)) != 1) return ST_CAP;
    int nfree = 0;
#pragma unroll
    for (int s = 0; s < S; s++) nfree += __popcll((~c.live[s] | conf[s]) & (G == 64 ? ~0ull : ((1ull << G) - 1ull)));
    if (nfree < 2) return ST_CAP;
    if (A.vcap > 0) {
        int keep = 0;
#pragma unroll
        for (int s = 0; s < S; s++) keep += __popcll(c.live[s] & ~conf[s]);
        if (keep + 2 > A.vcap) return ST_CAP;
    }
    if (gl == 0) {
        sh.lq[p][0] = q0;
        sh.lq[p][1] = q1;
        sh.lq[p][2] = h;
        if (A.rad) sh.lrj[p] = rj;
        sh.llab[p] = lab;
        sh.lsh[p] = (uint8_t)code;
        sh.lwall[p] = 0;
    }
    lds_sync2();
    int before = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        unsigned long long fr = (~c.live[s] | conf[s]) & (G == 64 ? ~0ull : ((1ull << G) - 1ull));
        int rk = before + __popcll(fr & ((1ull << gl) - 1ull));
        bool take = ((fr >> gl) & 1) && rk < 2;
        unsigned long long nw = gb2<G>(take, gb);
        if (take) {
            uint32_t t2 = sh.u.gc.nt[rk];
            c.tp[s] = t2;
            c.vx[s] = sh.u.gc.nv[rk][0];
            c.vy[s] = sh.u.gc.nv[rk][1];
            if (F32) {
                c.fx[s] = (float)c.vx[s];
                c.fy[s] = (float)c.vy[s];
            }
            uint8_t t = (uint8_t)(s * G + gl);
            sh.byin[t2 & 0xff] = t;
            sh.byout[(t2 >> 8) & 0xff] = t;
        }
        c.live[s] = (c.live[s] & ~conf[s]) | nw;
        before += __popcll(fr);
    }
    c.used |= 1ull << p;
    lds_sync2();
    p_radius<G, S, F32>(c, gl, A);
    cnt[DC_CUTS]++;
    cnt[DC_NEWV] += 2;
    return c.R2 < 1e300 ? ST_OK : ST_CAP;
}

template <int G, int S, int MAXL, bool F32>
__device__ __forceinline__ int p_gather(const CellArgs &A, L2<G, S, MAXL> &sh, Poly<S, F32> &c, const Tess &T, int si,
                                        const double *p, const int *bc, int dx, int dy, bool valid, double *ws,
                                        unsigned long long *cnt, int lane, int gl, int gb)
{
    const Grid &Gr = T.G;
    int dd[2] = {dx, dy};
    int bb[2], sv[2];
    bool ok = valid;
    double d2b = 0.0;
#pragma unroll
    for (int d = 0; d < 2; d++) {
        int t = bc[d] + dd[d];
        if (Gr.per[d]) {
            int g = Gr.g[d];
            int w = ((t % g) + g) % g;
            sv[d] = (t - w) / g;
            bb[d] = w;
            if (sv[d] > 2 || sv[d] < -2) ok = false;
        } else {
            sv[d] = 0;
            bb[d] = t;
            if (t < 0 || t >= Gr.g[d]) ok = false;
        }
        double blo = Gr.lo[d] + t * Gr.bs[d];
        double e = fmax(0.0, fmax(blo - p[d], p[d] - (blo + Gr.bs[d])));
        d2b += e * e;
    }
    if (d2b >= c.lim) ok = false;
    int cntb = 0, beg = 0;
    if (ok) {
        int64_t blk = T.bbase + bb[0] + (int64_t)Gr.g[0] * bb[1];
        beg = A.start[blk];
        cntb = A.start[blk + 1] - beg;
    }
    cnt[DC_BLOCKS] += __popcll(gb2<G>(ok, gb));
    int incl = g2scan<G>(cntb, gl);
    int total = __shfl(incl, gb + G - 1);
    cnt[DC_LOADED] += total;
    if (total == 0) return ST_OK;
    lds_sync2();
    sh.cpre[gl] = incl - cntb;
    sh.cbeg[gl] = beg;
    sh.csh[gl] = (uint8_t)(25 * 2 + 5 * (sv[1] + 2) + (sv[0] + 2));
    lds_sync2();
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
            int s0 = code % 5 - 2, s1 = (code / 5) % 5 - 2;
            Particle q = A.part[idx];
            double a0 = q.x - p[0], a1 = q.y - p[1];
            if (s0) a0 = a0 + s0 * Gr.L[0];
            if (s1) a1 = a1 + s1 * Gr.L[1];
            double d2 = a0 * a0 + a1 * a1;
            double h = 0.5 * d2, rj = 0.0;
            if (A.rad) {
                // radical line (section 2.1.1): |x|^2 - ri^2 <= |x - q|^2 - rj^2
                rj = A.rad[idx];
                h = 0.5 * (d2 + radical_shift(c.ri, rj));
            }
            bool self = (idx == si) && code == kNoShift;
            if (!self && d2 < c.lim) key = __double_as_longlong(d2);
            sh.u.gc.cq[gl][0] = a0;
            sh.u.gc.cq[gl][1] = a1;
            sh.u.gc.cq[gl][2] = d2;
            if (A.rad) {
                sh.u.gc.ch[gl] = h;
                sh.u.gc.crj[gl] = rj;
            }
            sh.u.gc.cid[gl] = q.id;
            sh.u.gc.ccode[gl] = (uint8_t)code;
        }
        lds_sync2();
        for (;;) {
            unsigned long long mk = g2min_u64<G>(key);
            if (mk == ~0ull) break;
            double md2 = __longlong_as_double((long long)mk);
            if (!(md2 < c.lim)) break;
            int ol = __builtin_ctzll(gb2<G>(key == mk, gb));
            if (gl == ol) key = ~0ull;
            cnt[DC_CAND]++;
            if (md2 == 0.0) return ST_DUP;
            int st = p_consider<G, S, MAXL, F32>(A, sh, c, sh.u.gc.cq[ol][0], sh.u.gc.cq[ol][1],
                                                 A.rad ? sh.u.gc.ch[ol] : 0.5 * md2, A.rad ? sh.u.gc.crj[ol] : 0.0,
                                                 sh.u.gc.cid[ol], sh.u.gc.ccode[ol], ws, cnt, lane, gl, gb);
            if (st != ST_OK) return st;
        }
        lds_sync2();
    }
    return ST_OK;
}

template <int G, int S, int MAXL, bool F32>
__device__ __forceinline__ int poly_run(const CellArgs &A, L2<G, S, MAXL> &sh, int si, double *ws,
                                        unsigned long long *cnt, int lane, int gl, int gb)
{
    const Particle me = A.part[si];
    const Tess &T = A.tess[me.tess];
    const Grid &Gr = T.G;
    const double p[2] = {me.x, me.y};
    const int id = me.id;
    int bc[2], fl[2];
    double mrg[2];
#pragma unroll
    for (int d = 0; d < 2; d++) {
        bc[d] = block_coord(Gr, p[d], d);
        double blo = Gr.lo[d] + bc[d] * Gr.bs[d];
        mrg[d] = fmin(p[d] - blo, blo + Gr.bs[d] - p[d]);
        fl[d] = offset_flip(Gr, p[d], bc[d], d);
    }
    Poly<S, F32> c;
    c.ri = A.rad ? A.rad[si] : 0.0;
    // box lines (Eq. 1-2, clipped as in section 3.1.3)
    if (gl < 4) {
        const int d = gl >> 1, side = gl & 1;
        const BoxSide b = box_side(T, d == 0 ? p[0] : p[1], d, side, id);
        sh.lwall[gl] = (uint8_t)b.wall;
        sh.llab[gl] = b.lab;
        sh.lsh[gl] = b.code;
        sh.lq[gl][0] = d == 0 ? b.nd : 0.0;
        sh.lq[gl][1] = d == 1 ? b.nd : 0.0;
        sh.lq[gl][2] = b.h;
        sh.lrj[gl] = c.ri;  // the own images carry the own radius
    }
#pragma unroll
    for (int s = 0; s < S; s++) {
        c.tp[s] = 0;
        c.vx[s] = c.vy[s] = 0.0;
        c.fx[s] = c.fy[s] = 0.0f;
        c.live[s] = 0;
    }
    c.live[0] = 0xfull;
    // corners counter-clockwise: (lo,lo) (hi,lo) (hi,hi) (lo,hi); vertex k
    // enters on line in[k] and leaves on line out[k]
    if (gl < 4) {
        const int cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
        const int lin[4] = {0, 2, 1, 3}, lout[4] = {2, 1, 3, 0};
        double ex[2], ey[2];
        ex[0] = -box_side(T, p[0], 0, 0, id).off;
        ex[1] = box_side(T, p[0], 0, 1, id).off;
        ey[0] = -box_side(T, p[1], 1, 0, id).off;
        ey[1] = box_side(T, p[1], 1, 1, id).off;
        c.tp[0] = (uint32_t)lin[gl] | ((uint32_t)lout[gl] << 8);
        c.vx[0] = ex[cx[gl]];
        c.vy[0] = ey[cy[gl]];
        c.fx[0] = (float)c.vx[0];
        c.fy[0] = (float)c.vy[0];
        sh.byin[lin[gl]] = (uint8_t)gl;
        sh.byout[lout[gl]] = (uint8_t)gl;
    }
    c.used = 0xfull;
    lds_sync2();
    p_radius<G, S, F32>(c, gl, A);

    bool finished = false;
    for (int o0 = 0; o0 < A.noff; o0 += G) {
        if (A.offs[o0].m * 0.25 * T.bsmin2 >= c.lim) {
            finished = true;
            break;
        }
        int o = o0 + gl;
        bool v = o < A.noff;
        Offset of = v ? A.offs[o] : Offset{0, 0, 0, 0};
        int st = p_gather<G, S, MAXL, F32>(A, sh, c, T, si, p, bc, of.dx * fl[0], of.dy * fl[1], v, ws, cnt, lane, gl, gb);
        if (st != ST_OK) return st;
    }
    // beyond the list: whole Chebyshev rings, until the radius bound holds or
    // no block of a ring meets the bounding box of the discs of the block
    // bound (section 2.1.3)
    if (!finished) {
        cnt[DC_FALLBACK]++;
        static_assert(sizeof(sh.u) >= sizeof(float4) * G * S, "ball list does not fit");
        float4 *bbl = reinterpret_cast<float4 *>(&sh.u);
        const double extra = A.rad ? fmax(*A.rmax * *A.rmax - c.ri * c.ri, 0.0) : 0.0;
        const double pad = bb_pad(Gr, p, 2);
        for (int r = A.off_radius + 1;; r++) {
            // a group of 8 lanes scans a ring 8 blocks at a time: a cell that
            // searches far goes to the spill pass, where 64 lanes scan it
            if (r > (G < 64 ? kRingSpill2 : kMaxShell) || !(c.R2 < 1e300)) return ST_CAP;
            double lb = 1e300;
            bool exists = false;
#pragma unroll
            for (int d = 0; d < 2; d++) {
                lb = fmin(lb, (r - 1) * Gr.bs[d] + mrg[d]);
                if (Gr.per[d] || bc[d] - r >= 0 || bc[d] + r < Gr.g[d]) exists = true;
            }
            if (!exists) break;
            if (lb > 0.0 && lb * lb >= c.lim) break;
            cnt[DC_SHELLS]++;
            const int tot = 8 * r;
            bool met = false;
            // the spill kernel's lanes take four blocks each per step, so the
            // particle counts of a far ring are loaded four at a time
            constexpr int U = G == 64 ? 4 : 1;
            for (int c0 = 0; c0 < tot; c0 += U * G) {
                // the bounding box of the discs, then the discs for the
                // non-empty blocks
                double ext[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < S; s++)
                    if ((c.live[s] >> gl) & 1) bb_ext_add(ext, c.vx[s], c.vy[s], 0.0, extra);
#pragma unroll
                for (int k = 0; k < 6; k++) ext[k] = g2max<G>(ext[k]);
                int qdx[U], qdy[U], qn[U];
                bool any = false;
#pragma unroll
                for (int u = 0; u < U; u++) {
                    const int ix = c0 + u * G + gl;
                    int dx = 0, dy = 0;
                    bool v = ix < tot;
                    if (v) ring_block2(r, ix, dx, dy);
                    const int t[3] = {bc[0] + dx, bc[1] + dy, 0};
                    double blo[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int d = 0; d < 2; d++) {
                        if (!Gr.per[d] && (t[d] < 0 || t[d] >= Gr.g[d])) v = false;
                        blo[d] = Gr.lo[d] + t[d] * Gr.bs[d] - p[d];
                    }
                    v = v && bb_in_ext(ext, blo, Gr.bs, pad, 2);
                    any = any || gb2<G>(v, gb);
                    qdx[u] = dx;
                    qdy[u] = dy;
                    qn[u] = v ? 1 : 0;
                }
                if (!any) continue;
                met = true;
#pragma unroll
                for (int u = 0; u < U; u++) {
                    if (qn[u]) {
                        const int t[3] = {bc[0] + qdx[u], bc[1] + qdy[u], 0};
                        qn[u] = bb_block_count<2>(A.start, T, t);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; u++) {
                    bool v = qn[u] > 0;
                    if (!gb2<G>(v, gb)) continue;
                    int nv = 0;
#pragma unroll
                    for (int s = 0; s < S; s++) {
                        const unsigned long long m = c.live[s];
                        if ((m >> gl) & 1)
                            bb_put(bbl, nv + __popcll(m & ((1ull << gl) - 1ull)), c.vx[s], c.vy[s], 0.0, extra);
                        nv += __popcll(m);
                    }
                    lds_sync2();
                    const double blo[3] = {Gr.lo[0] + (bc[0] + qdx[u]) * Gr.bs[0] - p[0],
                                           Gr.lo[1] + (bc[1] + qdy[u]) * Gr.bs[1] - p[1], 0.0};
                    v = v && bb_meets(bbl, nv, blo, Gr.bs, pad, 2);
                    if (!gb2<G>(v, gb)) continue;
                    int st = p_gather<G, S, MAXL, F32>(A, sh, c, T, si, p, bc, qdx[u], qdy[u], v, ws, cnt, lane, gl, gb);
                    if (st != ST_OK) return st;
                }
            }
            if (!met) break;
        }
    }

    // ---- statistics: area, centroid, perimeter, edges, neighbours ----
    lds_sync2();
#pragma unroll
    for (int s = 0; s < S; s++) {
        int t = s * G + gl;
        bool lv = (c.live[s] >> gl) & 1;
        sh.u.st.tpl[t] = lv ? c.tp[s] : 0xffffffffu;
        sh.u.st.pos[t][0] = c.vx[s];
        sh.u.st.pos[t][1] = c.vy[s];
    }
    lds_sync2();
    // edge on line b from vertex (a, b) to its successor (b, c): zero length
    // when the vertex lies on line c
    uint32_t ib = 0, zb = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        if (!((c.live[s] >> gl) & 1)) continue;
        int b = (c.tp[s] >> 8) & 0xff;
        uint32_t w2 = sh.u.st.tpl[sh.byin[b] & (G * S - 1)];
        int cc = min((int)((w2 >> 8) & 0xff), MAXL - 1);
        const double *nd = sh.lq[cc];
        double sd = nd[0] * c.vx[s] + nd[1] * c.vy[s] - nd[2];
        double bd = A.tau * ((fabs(nd[0]) + fabs(nd[1])) * c.R + fabs(nd[2]));
        if (!(sd < -bd)) ib |= 1u << s;
    }
    if (__ballot(ib != 0)) {
#pragma unroll
        for (int s = 0; s < S; s++) {
            unsigned long long wm = __ballot((ib >> s) & 1);
            while (wm) {
                int l = __builtin_ctzll(wm);
                wm &= wm - 1;
                if (lane == l) {
                    int a = c.tp[s] & 0xff, b = (c.tp[s] >> 8) & 0xff;
                    uint32_t w2 = sh.u.st.tpl[sh.byin[b] & (G * S - 1)];
                    int cc = min((int)((w2 >> 8) & 0xff), MAXL - 1);
                    const int sg = A.rad ? exact_side2(line_r(sh, a, c.ri), line_r(sh, b, c.ri), line_r(sh, cc, c.ri), ws)
                                         : exact_side2(line_of(sh, a), line_of(sh, b), line_of(sh, cc), ws);
                    if (sg == 0) zb |= 1u << s;
                }
                if ((l / G) == (lane / G)) cnt[DC_EXACT]++;
            }
        }
    }
    // triangles (apex, v, successor): the apex is the particle when it lies
    // strictly inside the cell (every edge line has h > 0, always so for a
    // Voronoi cell), else the cell's first live vertex, so that no term is
    // negative for a radical cell that misses its particle
    double o0 = 0.0, o1 = 0.0;
    {
        bool outside = false;
        int first = -1;
#pragma unroll
        for (int s = 0; s < S; s++) {
            bool lv = (c.live[s] >> gl) & 1;
            if (lv && !(sh.lq[(c.tp[s] >> 8) & 0xff][2] > 0.0)) outside = true;
            unsigned long long lm = gb2<G>(lv, gb);
            if (first < 0 && lm) first = s * G + __builtin_ctzll(lm);
        }
        if (gb2<G>(outside, gb) && first >= 0) {
            o0 = sh.u.st.pos[first][0];
            o1 = sh.u.st.pos[first][1];
        }
    }
    double ar = 0.0, m0 = 0.0, m1 = 0.0, per = 0.0;
    int ne = 0;
    unsigned long long posmask[S];
#pragma unroll
    for (int s = 0; s < S; s++) {
        bool lv = (c.live[s] >> gl) & 1;
        bool pos = lv && !((zb >> s) & 1);
        posmask[s] = gb2<G>(pos, gb);
        ne += __popcll(posmask[s]);
        if (lv) {
            int b = (c.tp[s] >> 8) & 0xff;
            const double *w0 = sh.u.st.pos[sh.byin[b] & (G * S - 1)];
            const double w[2] = {w0[0] - o0, w0[1] - o1};
            double x = c.vx[s] - o0, y = c.vy[s] - o1;
            double cr = x * w[1] - y * w[0];
            ar += cr;
            m0 += cr * (x + w[0]);
            m1 += cr * (y + w[1]);
            double dx = w0[0] - c.vx[s], dy = w0[1] - c.vy[s];
            per += sqrt(dx * dx + dy * dy);
        }
    }
    // neighbours: the lines of the positive-length edges, in slot order
    if ((A.mask & (16 | 32)) && A.nbr) {
        int before = 0;
#pragma unroll
        for (int s = 0; s < S; s++) {
            int rank = before + __popcll(posmask[s] & ((1ull << gl) - 1ull));
            if (((posmask[s] >> gl) & 1) && rank < kMaxNbr) {
                int b = (c.tp[s] >> 8) & 0xff;
                A.nbr[(int64_t)id * kMaxNbr + rank] = sh.llab[b];
                A.nsh[(int64_t)id * kMaxNbr + rank] = sh.lsh[b];
            }
            before += __popcll(posmask[s]);
        }
    }
    double area2 = g2sum<G>(ar);
    double M0 = g2sum<G>(m0), M1 = g2sum<G>(m1), P = g2sum<G>(per);
    lds_sync2();
    if (gl == 0) {
        if (A.vol) A.vol[id] = 0.5 * area2;
        if (A.cen) {
            A.cen[3 * (int64_t)id + 0] = o0 + M0 / (3.0 * area2);
            A.cen[3 * (int64_t)id + 1] = o1 + M1 / (3.0 * area2);
            A.cen[3 * (int64_t)id + 2] = 0.0;
        }
        if (A.nv) A.nv[id] = ne;
        if (A.ne) A.ne[id] = ne;
        if (A.nf) A.nf[id] = ne;
        if (A.perim) A.perim[id] = P;
    }
    if (A.fo)
        for (int k = gl; k < kFoLen; k += G) A.fo[(int64_t)id * kFoLen + k] = 0;
    return ne > kMaxNbr ? ST_CAP : ST_OK;
}

// two waves per SIMD (the register allocator is held to that budget): the
// spill kernel's far ring searches need the waves more than the registers
template <int G, int S, int MAXL, bool F32, bool RAD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_cells2d(CellArgs Ain, int spill_mode)
{
    // the Voronoi instantiation carries no radical code: its rad pointer is
    // a compile-time null
    CellArgs A = Ain;
    if (!RAD) A.rad = nullptr;
    static_assert(((G * S) & (G * S - 1)) == 0 && G * S <= 256, "slot count must be a power of two");
    __shared__ L2<G, S, MAXL> shv[64 / G];
    const int lane = __lane_id();
    const int gl = lane % G, gb = lane - gl;
    L2<G, S, MAXL> &sh = shv[lane / G];
    double *ws = A.xscratch + (size_t)blockIdx.x * A.xscratch_len;
    unsigned long long cnt[DC_N];
#pragma unroll
    for (int k = 0; k < DC_N; k++) cnt[k] = 0;
    const int ncell = A.ncell_dev ? *A.ncell_dev : A.ncell;
    for (;;) {
        int base = 0;
        if (gl == 0) base = atomicAdd(A.queue, A.chunk);
        base = __shfl(base, gb);
        if (base >= ncell) break;
        int end = min(base + A.chunk, ncell);
        for (int ci = base; ci < end; ci++) {
            int si = A.cell_list ? A.cell_list[ci] : ci;
            int st = poly_run<G, S, MAXL, F32>(A, sh, si, ws, cnt, lane, gl, gb);
            if (st != ST_OK && A.fo)
                for (int k = gl; k < kFoLen; k += G) A.fo[(int64_t)A.part[si].id * kFoLen + k] = 0;
            if (gl == 0) {
                int id = A.part[si].id;
                if (st != ST_OK) {
                    // an empty radical cell has zero area and perimeter
                    const double f = st == ST_EMPTY ? 0.0 : __builtin_nan("");
                    if (A.vol) A.vol[id] = f;
                    if (A.cen) A.cen[3 * (int64_t)id] = A.cen[3 * (int64_t)id + 1] = f;
                    if (A.nv) A.nv[id] = 0;
                    if (A.ne) A.ne[id] = 0;
                    if (A.nf) A.nf[id] = 0;
                    if (A.perim) A.perim[id] = f;
                }
                if (st == ST_EMPTY) {
                    A.status[id] = (uint8_t)ST_EMPTY;
                } else if (st == ST_OK) {
                    A.status[id] = spill_mode ? 1 : 0;
                } else if (st == ST_DUP) {
                    A.status[id] = 3;
                } else if (!spill_mode) {
                    A.status[id] = 1;
                    int pos = atomicAdd(A.spill_count, 1);
                    A.spill_list[pos] = si;
                    cnt[DC_SPILL]++;
                } else {
                    A.status[id] = 2;
                }
            }
            lds_sync2();
        }
    }
    if (gl == 0) {
#pragma unroll
        for (int k = 0; k < DC_N; k++)
            if (cnt[k]) atomicAdd(&A.diag[k], cnt[k]);
    }
}

}  // namespace

hipError_t launch_cells2d(const CellArgs &a, int precision, int waves, hipStream_t s)
{
    if (a.rad) {
        if (precision == 1) k_cells2d<8, 2, 32, true, true><<<waves, 64, 0, s>>>(a, 0);
        else k_cells2d<8, 2, 32, false, true><<<waves, 64, 0, s>>>(a, 0);
    } else {
        if (precision == 1) k_cells2d<8, 2, 32, true, false><<<waves, 64, 0, s>>>(a, 0);
        else k_cells2d<8, 2, 32, false, false><<<waves, 64, 0, s>>>(a, 0);
    }
    return hipGetLastError();
}

hipError_t launch_cells2d_spill(const CellArgs &a, int waves, hipStream_t s)
{
    if (a.rad) k_cells2d<64, 4, 64, false, true><<<waves, 64, 0, s>>>(a, 1);
    else k_cells2d<64, 4, 64, false, false><<<waves, 64, 0, s>>>(a, 1);
    return hipGetLastError();
}

}  // namespace vc
