// cell_common.h -- device pieces shared by the cell kernels: the exact side
// predicate (floating-point expansions), DPP wave helpers, the vertex of
// three planes, and status / counter codes.
#pragma once
#include "vc_internal.h"

namespace vc {
namespace {

constexpr double kMargin = 1.0 + 0x1p-30;  // radius-bound safety factor on squared distances
constexpr int kBbMinList = 16;             // candidates of a batch that turn on the ball test in the offset list
constexpr double kBbExtended = 9.0;        // (2R / smallest block side)^2 above which the offset list's blocks are tested
constexpr int kMaxShell = 1024;            // largest Chebyshev shell searched; beyond it the cell fails
constexpr int kRingSpill2 = 32;            // 2D: rings searched by a narrow group before the cell is spilled

struct PlaneD {
    double n0, n1, n2, h;
    int wall;
};

// A plane of a radical cell: h = (q.q + ri^2 - rj^2) / 2 with ri the radius
// of the cell's particle and rj that of the neighbour (a wall keeps its h).
struct PlaneR {
    PlaneD p;
    double ri, rj;
};

template <class P>
constexpr bool kRadicalPlane = sizeof(P) > sizeof(PlaneD);

__device__ __forceinline__ const PlaneD &plane_base(const PlaneD &p) { return p; }
__device__ __forceinline__ const PlaneD &plane_base(const PlaneR &p) { return p.p; }

// ---------------------------------------------------------------------------
// Exact sign with floating-point expansions (Shewchuk 1997): a list of
// doubles, nonoverlapping and increasing in magnitude, whose exact sum is the
// value; Grow-Expansion adds one double exactly.  Runs on one lane at a time
// with the wave's workspace in global memory.
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)

__device__ inline void xs_two_sum(double a, double b, double &x, double &y)
{
    double s = a + b;
    double bv = s - a;
    double av = s - bv;
    x = s;
    y = (a - av) + (b - bv);
}

__device__ inline void xs_two_prod(double a, double b, double &x, double &y)
{
    double p = a * b;
    x = p;
    y = __builtin_fma(a, b, -p);
}

// e <- e + b (in place: output component k is written at index <= its input)
__device__ inline int xs_grow(double *e, int n, double b)
{
    double q = b;
    int k = 0;
    for (int i = 0; i < n; i++) {
        double x, y;
        xs_two_sum(q, e[i], x, y);
        if (y != 0.0) e[k++] = y;
        q = x;
    }
    if (q != 0.0 || k == 0) e[k++] = q;
    return k;
}

// Compress (Shewchuk 1997): the same exact sum in fewer components, still
// nonoverlapping and increasing in magnitude, in place.  A downward pass of
// Two-Sum from the largest component keeps only the parts that did not fit,
// an upward pass renormalises them.
__device__ inline int xs_compress(double *e, int m)
{
    double Q = e[m - 1];
    int bottom = m - 1;
    for (int i = m - 2; i >= 0; i--) {
        double x, y;
        xs_two_sum(Q, e[i], x, y);
        if (y != 0.0) {
            e[bottom--] = x;
            Q = y;
        } else {
            Q = x;
        }
    }
    e[bottom] = Q;
    int top = 0;
    for (int i = bottom + 1; i < m; i++) {
        double x, y;
        xs_two_sum(e[i], Q, x, y);
        Q = x;
        if (y != 0.0) e[top++] = y;
    }
    e[top++] = Q;
    return top;
}

// the accumulator is compressed whenever it grows past this many components
// (every Grow-Expansion step walks the whole list, in the global workspace)
constexpr int kXsCompressAt = 16;

__device__ inline int xs_add_prod(double *e, int n, double a, double b)
{
    double x, y;
    xs_two_prod(a, b, x, y);
    if (y != 0.0) n = xs_grow(e, n, y);
    n = xs_grow(e, n, x);
    return n > kXsCompressAt ? xs_compress(e, n) : n;
}

__device__ inline int xs_sign(const double *e, int n)
{
    double t = e[n - 1];
    return (t > 0.0) - (t < 0.0);
}

// The exact offset of a plane as a short list of doubles summing to it:
// q.q/2 for a bisector (three exact squares, halved), (q.q + ri^2 - rj^2)/2
// for a radical plane (five exact squares, halved), h for a wall.
__device__ inline int xs_radical_terms(const PlaneR &p, double *out, int k)
{
    if (p.p.wall) return k;
    double x, y;
    xs_two_prod(p.ri, p.ri, x, y);
    out[k++] = 0.5 * x;
    out[k++] = 0.5 * y;
    xs_two_prod(p.rj, p.rj, x, y);
    out[k++] = -0.5 * x;
    out[k++] = -0.5 * y;
    return k;
}

__device__ inline int xs_offset(const PlaneD &p, double *out)
{
    if (p.wall) {
        out[0] = p.h;
        return 1;
    }
    double v[3] = {p.n0, p.n1, p.n2};
    int k = 0;
    for (int d = 0; d < 3; d++) {
        double x, y;
        xs_two_prod(v[d], v[d], x, y);
        out[k++] = 0.5 * x;
        out[k++] = 0.5 * y;
    }
    return k;
}

__device__ inline int xs_offset(const PlaneR &p, double *out)
{
    return xs_radical_terms(p, out, xs_offset(p.p, out));
}

// acc += sgn * h_list * det3(u, v, w) over the six permutation products.
__device__ int xs_acc_hdet(double *acc, int n, const double *hl, int nh, double sgn, const double *u,
                           const double *v, const double *w)
{
    const int pm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}, {2, 1, 0}};
    for (int k = 0; k < 6; k++) {
        double sg = k < 3 ? sgn : -sgn;
        double x, y;
        xs_two_prod(sg * u[pm[k][0]], v[pm[k][1]], x, y);
        // (x + y) * w exactly = four doubles
        double t[4];
        xs_two_prod(x, w[pm[k][2]], t[0], t[1]);
        xs_two_prod(y, w[pm[k][2]], t[2], t[3]);
        for (int a = 0; a < 4; a++) {
            if (t[a] == 0.0) continue;
            for (int b = 0; b < nh; b++) {
                if (hl[b] == 0.0) continue;
                n = xs_add_prod(acc, n, t[a], hl[b]);
            }
        }
    }
    return n;
}

// ---------------------------------------------------------------------------
// Double-word stage.  The expression of the exact sign below is first
// evaluated with pairs hi + lo of doubles (about 106 bits) together with a
// bound on the error; when the value lies outside its bound the sign is
// certain, and only values within it (exact ties, as on lattices) go on to
// the expansions, whose many dependent steps through the workspace cost
// about a millisecond per call.  The pair operations are the accurate
// double-word algorithms of Joldes, Muller and Popescu (2017), with relative
// errors of at most 3u^2 (sum), 2u^2 (product by a double) and 4u^2
// (product), u = 2^-53.
// ---------------------------------------------------------------------------
struct Dw {
    double hi, lo;
};

// Fast-Two-Sum: exact when |a| >= |b| (or a = 0)
__device__ inline Dw dw_fast(double a, double b)
{
    double s = a + b;
    return Dw{s, b - (s - a)};
}

__device__ inline Dw dw_add(Dw a, Dw b)
{
    double sh, sl, th, tl;
    xs_two_sum(a.hi, b.hi, sh, sl);
    xs_two_sum(a.lo, b.lo, th, tl);
    Dw v = dw_fast(sh, sl + th);
    return dw_fast(v.hi, v.lo + tl);
}

__device__ inline Dw dw_mul_d(Dw a, double b)
{
    double ch, cl;
    xs_two_prod(a.hi, b, ch, cl);
    return dw_fast(ch, __builtin_fma(a.lo, b, cl));
}

__device__ inline Dw dw_mul(Dw a, Dw b)
{
    double ch, cl;
    xs_two_prod(a.hi, b.hi, ch, cl);
    double t = a.lo * b.lo;
    t = __builtin_fma(a.hi, b.lo, t);
    t = __builtin_fma(a.lo, b.hi, t);
    return dw_fast(ch, cl + t);
}

// det of the rows u, v, w as a pair; mag = sum of the six |products|.  Each
// product is an exact pair (Two-Product) times a double; the error is at
// most 2u^2 mag for the products and 3u^2 mag for each of the five sums.
__device__ inline Dw dw_det3(const double *u, const double *v, const double *w, double &mag)
{
    Dw acc{0.0, 0.0};
    mag = 0.0;
    const double x[6] = {u[0], u[1], u[2], -u[0], -u[1], -u[2]};
    const double y[6] = {v[1], v[2], v[0], v[2], v[0], v[1]};
    const double z[6] = {w[2], w[0], w[1], w[1], w[2], w[0]};
#pragma unroll
    for (int k = 0; k < 6; k++) {
        double ph, pl;
        xs_two_prod(x[k], y[k], ph, pl);
        acc = dw_add(acc, dw_mul_d(Dw{ph, pl}, z[k]));
        mag += fabs(ph) * fabs(z[k]);
    }
    return acc;
}

// The sign of exact_side3's expression, or 2 when the double-word stage
// cannot certify it.  Error of the numerator N = sum_i +-h_i D_i, with H_i
// the sum of |terms| of h_i and P_i the mag of D_i: at most 27u^2 H_i for h_i
// (nine sums), 17u^2 P_i for D_i, 48u^2 H_i P_i for the product with both
// propagated, and 9u^2 sum H_i P_i for the three sums: below 2^-100 M with
// M = sum H_i P_i.  The bound taken is 2^-96 M (and 2^-96 P for the
// denominator), so |N.hi| above it fixes the sign of N.  Outside
// [2^-900, 2^900] the expansions decide (underflow and overflow).
template <class P>
__device__ inline int dw_side3(const P *const *r, const double (*nv)[3])
{
    const int mi[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    Dw num{0.0, 0.0};
    double bound = 0.0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        double hl[kRadicalPlane<P> ? 10 : 6];
        const int nh = xs_offset(*r[i], hl);
        Dw h{0.0, 0.0};
        double hm = 0.0;
        for (int k = 0; k < nh; k++) {
            h = dw_add(h, Dw{hl[k], 0.0});
            hm += fabs(hl[k]);
        }
        double pm;
        Dw d = dw_det3(nv[mi[i][0]], nv[mi[i][1]], nv[mi[i][2]], pm);
        Dw t = dw_mul(h, d);
        if (i & 1) t = Dw{-t.hi, -t.lo};
        num = dw_add(num, t);
        bound += hm * pm;
    }
    double pd;
    const Dw den = dw_det3(nv[0], nv[1], nv[2], pd);
    if (!(bound > 0x1p-900 && bound < 0x1p900 && pd > 0x1p-900 && pd < 0x1p900)) return 2;
    if (!(fabs(num.hi) > bound * 0x1p-96) || !(fabs(den.hi) > pd * 0x1p-96)) return 2;
    return ((num.hi > 0.0) == (den.hi > 0.0)) ? 1 : -1;
}

// Exact sign of n_p.v - h_p at v = planes a, b, c:
//   s * D(a,b,c) = h_a D(b,c,p) - h_b D(a,c,p) + h_c D(a,b,p) - h_p D(a,b,c).
// P is PlaneD (Voronoi) or PlaneR (radical).
template <class P>
__device__ __noinline__ int exact_side3(P a, P b, P c, P p, double *ws)
{
    const P *r[4] = {&a, &b, &c, &p};
    double nv[4][3];
    for (int i = 0; i < 4; i++) {
        nv[i][0] = plane_base(*r[i]).n0;
        nv[i][1] = plane_base(*r[i]).n1;
        nv[i][2] = plane_base(*r[i]).n2;
    }
    const int mi[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    const int quick = dw_side3<P>(r, nv);
    if (quick != 2) return quick;
    double hl[kRadicalPlane<P> ? 10 : 6];  // the plane offset's exact terms
    int n = 0;
    for (int i = 0; i < 4; i++) {
        int nh = xs_offset(*r[i], hl);
        n = xs_acc_hdet(ws, n, hl, nh, (i & 1) ? -1.0 : 1.0, nv[mi[i][0]], nv[mi[i][1]], nv[mi[i][2]]);
    }
    int s4 = n ? xs_sign(ws, n) : 0;
    double one = 1.0;
    int m = xs_acc_hdet(ws, 0, &one, 1, 1.0, nv[0], nv[1], nv[2]);
    int s3 = m ? xs_sign(ws, m) : 0;
    return s4 * s3;
}

// Exact sign of n_p.v - h_p at the 2D vertex v = lines a, b:
//   s * D(a,b) = -h_a D(b,p) + h_b D(a,p) - h_p D(a,b),  D = 2x2 determinant.
__device__ int xs_acc_hdet2(double *acc, int n, const double *hl, int nh, double sgn, const double *u,
                            const double *v)
{
    double t[4];
    xs_two_prod(sgn * u[0], v[1], t[0], t[1]);
    xs_two_prod(-sgn * u[1], v[0], t[2], t[3]);
    for (int a = 0; a < 4; a++) {
        if (t[a] == 0.0) continue;
        for (int b = 0; b < nh; b++) {
            if (hl[b] == 0.0) continue;
            n = xs_add_prod(acc, n, t[a], hl[b]);
        }
    }
    return n;
}

__device__ inline int xs_offset2(const PlaneD &p, double *out)
{
    if (p.wall) {
        out[0] = p.h;
        return 1;
    }
    double v[2] = {p.n0, p.n1};
    int k = 0;
    for (int d = 0; d < 2; d++) {
        double x, y;
        xs_two_prod(v[d], v[d], x, y);
        out[k++] = 0.5 * x;
        out[k++] = 0.5 * y;
    }
    return k;
}

__device__ inline int xs_offset2(const PlaneR &p, double *out)
{
    return xs_radical_terms(p, out, xs_offset2(p.p, out));
}

template <class P>
__device__ __noinline__ int exact_side2(P a, P b, P p, double *ws)
{
    const P *r[3] = {&a, &b, &p};
    double nv[3][2];
    for (int i = 0; i < 3; i++) {
        nv[i][0] = plane_base(*r[i]).n0;
        nv[i][1] = plane_base(*r[i]).n1;
    }
    const int mi[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    const double sg[3] = {-1.0, 1.0, -1.0};
    double hl[kRadicalPlane<P> ? 8 : 4];
    int n = 0;
    for (int i = 0; i < 3; i++) {
        int nh = xs_offset2(*r[i], hl);
        n = xs_acc_hdet2(ws, n, hl, nh, sg[i], nv[mi[i][0]], nv[mi[i][1]]);
    }
    int s3 = n ? xs_sign(ws, n) : 0;
    double one = 1.0;
    int m = xs_acc_hdet2(ws, 0, &one, 1, 1.0, nv[0], nv[1]);
    int s2 = m ? xs_sign(ws, m) : 0;
    return s3 * s2;
}

// r_i^2 - r_j^2 of a radical plane (section 2.1.1) with each square rounded
// on its own (no fused multiply-add): equal radii give exactly 0, and the
// plane is then the bisector bit for bit
__device__ __forceinline__ double radical_shift(double ri, double rj)
{
    return ri * ri - rj * rj;
}

#pragma clang fp contract(fast)

// ---------------------------------------------------------------------------
// Wave helpers.  Reductions and scans use DPP lane movement (quad
// permutations, row mirrors, row shifts and the row broadcasts of the
// 64-wide wave) and end with a readlane, so the result is wave-uniform and
// no LDS round trip is taken.
// ---------------------------------------------------------------------------
enum {
    DPP_QUAD_1032 = 0xB1,     // quad_perm [1,0,3,2]
    DPP_QUAD_2301 = 0x4E,     // quad_perm [2,3,0,1]
    DPP_ROW_SHR1 = 0x111,
    DPP_ROW_SHR2 = 0x112,
    DPP_ROW_SHR4 = 0x114,
    DPP_ROW_SHR8 = 0x118,
    DPP_ROW_MIRROR = 0x140,
    DPP_ROW_HALF_MIRROR = 0x141,
    DPP_ROW_BCAST15 = 0x142,  // lane 15 of each row to the next row
    DPP_ROW_BCAST31 = 0x143   // lane 31 to rows 2 and 3
};

template <int CTRL, int RM>
__device__ __forceinline__ int dpp_i32(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, RM, 0xf, false);
}

template <int CTRL, int RM>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long old, unsigned long long v)
{
    int lo = __builtin_amdgcn_update_dpp((int)(unsigned)old, (int)(unsigned)v, CTRL, RM, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(old >> 32), (int)(unsigned)(v >> 32), CTRL, RM, 0xf, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

template <int CTRL, int RM>
__device__ __forceinline__ double dpp_f64(double old, double v)
{
    return __builtin_bit_cast(double, dpp_u64<CTRL, RM>(__builtin_bit_cast(unsigned long long, old),
                                                         __builtin_bit_cast(unsigned long long, v)));
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int l)
{
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    return __builtin_bit_cast(double, readlane_u64(__builtin_bit_cast(unsigned long long, v), l));
}

__device__ __forceinline__ int lane_rank(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_f64<DPP_QUAD_1032, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_QUAD_2301, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_ROW_HALF_MIRROR, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_ROW_MIRROR, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_ROW_BCAST15, 0xa>(v, v));
    v = fmax(v, dpp_f64<DPP_ROW_BCAST31, 0xc>(v, v));
    return readlane_f64(v, 63);
}

// fixed combination order: the sum is the same on every run
__device__ __forceinline__ double wave_sum(double v)
{
    v = v + dpp_f64<DPP_QUAD_1032, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_QUAD_2301, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_ROW_HALF_MIRROR, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_ROW_MIRROR, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_ROW_BCAST15, 0xa>(0.0, v);
    v = v + dpp_f64<DPP_ROW_BCAST31, 0xc>(0.0, v);
    return readlane_f64(v, 63);
}

__device__ __forceinline__ int wave_isum(int v)
{
    v = v + dpp_i32<DPP_QUAD_1032, 0xf>(0, v);
    v = v + dpp_i32<DPP_QUAD_2301, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_HALF_MIRROR, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_MIRROR, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_BCAST15, 0xa>(0, v);
    v = v + dpp_i32<DPP_ROW_BCAST31, 0xc>(0, v);
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long v)
{
    v |= dpp_u64<DPP_QUAD_1032, 0xf>(0ull, v);
    v |= dpp_u64<DPP_QUAD_2301, 0xf>(0ull, v);
    v |= dpp_u64<DPP_ROW_HALF_MIRROR, 0xf>(0ull, v);
    v |= dpp_u64<DPP_ROW_MIRROR, 0xf>(0ull, v);
    v |= dpp_u64<DPP_ROW_BCAST15, 0xa>(0ull, v);
    v |= dpp_u64<DPP_ROW_BCAST31, 0xc>(0ull, v);
    return readlane_u64(v, 63);
}

// inclusive prefix sum over the wave (row shifts, then row broadcasts)
__device__ __forceinline__ int wave_incl_scan(int v)
{
    v = v + dpp_i32<DPP_ROW_SHR1, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_SHR2, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_SHR4, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_SHR8, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_BCAST15, 0xa>(0, v);
    v = v + dpp_i32<DPP_ROW_BCAST31, 0xc>(0, v);
    return v;
}

// exclusive prefix of small non-negative counts (< 2^BITS) by bit ballots
template <int BITS>
__device__ __forceinline__ int ballot_excl_scan(int v, int &total)
{
    int r = 0, t = 0;
#pragma unroll
    for (int b = 0; b < BITS; b++) {
        unsigned long long m = __ballot((v >> b) & 1);
        r += lane_rank(m) << b;
        t += __popcll(m) << b;
    }
    total = t;
    return r;
}

// vertex of planes A, B, C by Cramer's rule
// vertex of lines A, B (n.r = h, rows n0 n1 h) by Cramer's rule
__device__ __forceinline__ void cramer2(const double *A, const double *B, double &x, double &y)
{
    double det = A[0] * B[1] - A[1] * B[0];
    double inv = 1.0 / det;
    x = (A[2] * B[1] - A[1] * B[2]) * inv;
    y = (A[0] * B[2] - A[2] * B[0]) * inv;
}

__device__ __forceinline__ void cramer(const double *A, const double *B, const double *C, double &x, double &y, double &z)
{
    double bc0 = B[1] * C[2] - B[2] * C[1], bc1 = B[2] * C[0] - B[0] * C[2], bc2 = B[0] * C[1] - B[1] * C[0];
    double ca0 = C[1] * A[2] - C[2] * A[1], ca1 = C[2] * A[0] - C[0] * A[2], ca2 = C[0] * A[1] - C[1] * A[0];
    double ab0 = A[1] * B[2] - A[2] * B[1], ab1 = A[2] * B[0] - A[0] * B[2], ab2 = A[0] * B[1] - A[1] * B[0];
    double det = A[0] * bc0 + A[1] * bc1 + A[2] * bc2;
    double inv = 1.0 / det;
    x = (A[3] * bc0 + B[3] * ca0 + C[3] * ab0) * inv;
    y = (A[3] * bc1 + B[3] * ca1 + C[3] * ab1) * inv;
    z = (A[3] * bc2 + B[3] * ca2 + C[3] * ab2) * inv;
}

// The initial plane on one side of axis d (Eq. 1-2): the wall, or on a
// periodic axis the bisector with the particle's own image at +-L; with
// clipping (section 3.1.3) the clip wall at half the cube's side, where that
// lies strictly inside.  `off` is the corner coordinate's magnitude.
struct BoxSide {
    double nd, h, off;  // normal along d, offset, corner offset
    int wall;
    int32_t lab;
    uint8_t code;
};

__device__ __forceinline__ BoxSide box_side(const Tess &T, double pd, int d, int side, int32_t self)
{
    const Grid &G = T.G;
    const double sg = side ? 1.0 : -1.0;
    const double off = G.per[d] ? 0.5 * G.L[d] : (side ? (G.hi[d] - pd) : -(G.lo[d] - pd));
    BoxSide b;
    if (T.clip_half > 0.0 && T.clip_half < off) {
        b.nd = sg;
        b.h = T.clip_half;
        b.off = T.clip_half;
        b.wall = 1;
        b.lab = -(7 + 2 * d + side);
        b.code = kNoShift;
    } else if (G.per[d]) {
        const double L = G.L[d];
        b.nd = sg * L;
        b.h = 0.5 * (L * L);
        b.off = off;
        b.wall = 0;
        b.lab = self;
        b.code = (uint8_t)(kNoShift + (side ? 1 : -1) * (d == 0 ? 1 : (d == 1 ? 5 : 25)));
    } else {
        b.nd = sg;
        b.h = off;
        b.off = off;
        b.wall = 1;
        b.lab = -(2 * d + side + 1);
        b.code = kNoShift;
    }
    return b;
}

// Squared search radius from the radius bound R (an upper bound of the
// vertex norms; R2 >= R^2 ... both upper bounds): a candidate at distance d
// can cut only if d^2 - 2 R d + ri^2 - rj^2 < 0 for some vertex, i.e.
// d < R + sqrt(R^2 + rmax^2 - ri^2); without radii that is 2R.  The result
// carries the radius bound's safety factor.
__device__ __forceinline__ double search_lim(double R2, double R, const CellArgs &A, double ri)
{
    if (!A.rad) return 4.0 * R2 * kMargin;
    const double rm = *A.rmax;
    const double t = fmax(R2 + (rm * rm - ri * ri), 0.0);
    const double l = R + sqrt(t) * (1.0 + 0x1p-40);
    return l * l * kMargin;
}

// Reflection of the nearest-first block offsets along axis d: -1 when the
// particle lies in the upper half of its block k, so that the list's near
// side (negative offsets come first within a gap class) is the particle's
// near side.  The gap classes are symmetric, so the order stays nearest
// first in the guaranteed gap.
__device__ __forceinline__ int offset_flip(const Grid &G, double x, int k, int d)
{
    const double blo = G.lo[d] + k * G.bs[d];
    return (x - blo) * 2.0 > G.bs[d] ? -1 : 1;
}

enum { ST_OK = 0, ST_CAP = 1, ST_DUP = 3, ST_EMPTY = 5 };
// status flag of a complete cell with a face of kFoLen or more edges: the
// face-order vector does not count that face
constexpr int ST_FO_OVER = 64;


// ---------------------------------------------------------------------------
// Block bound (section 2.1.3).  A particle at q (relative to the cell's
// particle) cuts the cell only if some vertex v lies strictly beyond its
// plane, v.q > |q|^2 / 2, that is |q - v| < |v|: q lies in the union U of the
// balls B(v, |v|).  A block whose box meets none of them holds no particle
// that can cut.  U only shrinks as the cell is cut.
//
// The shell search tests every block of a Chebyshev shell against the
// axis-aligned bounding box of U (six numbers, cheap per block); once no
// block of a shell meets that box, the box lies inside the shell and every
// block farther out misses it, so the search is complete.  A non-empty
// block that meets the box is then tested against the balls themselves
// before its particles are loaded.
// ---------------------------------------------------------------------------

// One vertex's part of the bounding box of U: ext[d] >= v_d + rho and
// ext[3 + d] >= rho - v_d, rho the ball radius widened as in the ball list.
__device__ __forceinline__ void bb_ext_add(double ext[6], double x, double y, double z, double extra)
{
    const double rho = sqrt((x * x + y * y + z * z + extra) * (1.0 + 0x1p-8)) * (1.0 + 0x1p-40);
    ext[0] = fmax(ext[0], x + rho);
    ext[1] = fmax(ext[1], y + rho);
    ext[2] = fmax(ext[2], z + rho);
    ext[3] = fmax(ext[3], rho - x);
    ext[4] = fmax(ext[4], rho - y);
    ext[5] = fmax(ext[5], rho - z);
}

// Does the box [lo - pad, lo + bs + pad] meet the bounding box of U?
__device__ __forceinline__ bool bb_in_ext(const double ext[6], const double lo[3], const double bs[3], double pad,
                                          int dim)
{
    bool in = true;
#pragma unroll
    for (int d = 0; d < 3; d++)
        if (d < dim) in = in && lo[d] - pad < ext[d] && lo[d] + bs[d] + pad > -ext[3 + d];
    return in;
}

// Chebyshev shell r >= 1 of blocks, enumerated directly (24 r^2 + 2 blocks
// in 3D, 8 r in 2D): block k of the shell at offset (dx, dy, dz).  3D: the
// faces z = -r and z = r whole, then y = -r and y = r without their z
// edges, then x = -r and x = r inside both.
__device__ __forceinline__ int shell_size3(int r) { return 24 * r * r + 2; }

__device__ __forceinline__ void shell_block3(int r, int k, int &dx, int &dy, int &dz)
{
    const int a = 2 * r + 1, b = 2 * r - 1;
    if (k < 2 * a * a) {
        const int f = k / (a * a), m = k - f * a * a;
        dz = f ? r : -r;
        dx = m % a - r;
        dy = m / a - r;
        return;
    }
    k -= 2 * a * a;
    if (k < 2 * a * b) {
        const int f = k / (a * b), m = k - f * a * b;
        dy = f ? r : -r;
        dx = m % a - r;
        dz = m / a - (r - 1);
        return;
    }
    k -= 2 * a * b;
    const int f = k / (b * b), m = k - f * b * b;
    dx = f ? r : -r;
    dy = m % b - (r - 1);
    dz = m / b - (r - 1);
}

// 2D ring: the four sides in turn, 2 r blocks each, counter-clockwise from
// the corner (-r, -r).
__device__ __forceinline__ void ring_block2(int r, int k, int &dx, int &dy)
{
    const int side = k / (2 * r), m = k - side * 2 * r;
    if (side == 0) {
        dx = -r + m;
        dy = -r;
    } else if (side == 1) {
        dx = r;
        dy = -r + m;
    } else if (side == 2) {
        dx = r - m;
        dy = r;
    } else {
        dx = -r;
        dy = r - m;
    }
}

// Particle count of the block at unfolded block coordinates t (t[2] = 0 in
// 2D); 0 for a block outside a wall or more than two periods away, which the
// gathers skip as well.
template <int DIM>
__device__ __forceinline__ int bb_block_count(const int32_t *start, const Tess &T, const int t[3])
{
    const Grid &G = T.G;
    int bb[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; d++) {
        const int g = G.g[d];
        if (G.per[d]) {
            const int w = ((t[d] % g) + g) % g;
            const int sv = (t[d] - w) / g;
            if (sv > 2 || sv < -2) return 0;
            bb[d] = w;
        } else {
            if (t[d] < 0 || t[d] >= g) return 0;
            bb[d] = t[d];
        }
    }
    const int64_t blk = T.bbase + bb[0] + (int64_t)G.g[0] * (bb[1] + (DIM == 3 ? (int64_t)G.g[1] * bb[2] : 0));
    return start[blk + 1] - start[blk];
}

// For a radical cell the plane of a particle of radius rj is
// v.q > (|q|^2 + ri^2 - rj^2) / 2, so the ball grows to the squared radius
// |v|^2 + rmax^2 - ri^2 (extra = max(rmax^2 - ri^2, 0): the balls still
// hold the particle, and U stays star-shaped about it).
//
// The list of a cell's vertices for the test: x, y, z and the squared ball
// radius as floats, the latter widened by 2^-8 so that the float rounding
// of the coordinates can only keep a block, never drop one that the FP64
// cell would need.
// Rounding allowance of the block boxes: far above the error of a block
// bound or of a relative particle position (a few units in the last place of
// the container's coordinates), far below a block side.
__device__ __forceinline__ double bb_pad(const Grid &G, const double *p, int dim)
{
    double m = 0.0;
    for (int d = 0; d < dim; d++) m = fmax(m, fabs(p[d]) + fabs(G.lo[d]) + 3.0 * G.L[d]);
    return m * 0x1p-40;
}

__device__ __forceinline__ void bb_put(float4 *list, int j, double x, double y, double z, double extra)
{
    list[j] = make_float4((float)x, (float)y, (float)z,
                          (float)(x * x + y * y + z * z + extra) * (1.0f + 0x1p-8f));
}

// Does the box [lo, lo + bs] (relative coordinates, z ignored in 2D) meet a
// ball of the list?  The box is widened by pad, which covers the rounding of
// block bounds and particle positions relative to the cell's particle, and
// its corners are rounded outward to float.
__device__ __forceinline__ bool bb_meets(const float4 *list, int nv, const double lo[3], const double bs[3], double pad,
                                         int dim)
{
    float l[3], h[3];
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const double lo_d = d < dim ? lo[d] - pad : 0.0, hi_d = d < dim ? lo[d] + bs[d] + pad : 0.0;
        l[d] = __double2float_rd(lo_d);
        h[d] = __double2float_ru(hi_d);
    }
    for (int j = 0; j < nv; j++) {
        const float4 v = list[j];
        const float e0 = fmaxf(0.0f, fmaxf(l[0] - v.x, v.x - h[0]));
        const float e1 = fmaxf(0.0f, fmaxf(l[1] - v.y, v.y - h[1]));
        const float e2 = fmaxf(0.0f, fmaxf(l[2] - v.z, v.z - h[2]));
        if (e0 * e0 + e1 * e1 + e2 * e2 < v.w) return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Edge-graph records for the Weinberg codes (the cell-topology code of
// VoroTop; section 5).  A cell's vertex is a class of triangles joined by
// zero-length edges; around it, its edges come in the order of the
// triangles' planes (a, b, c), so every vertex sees its edges in one common
// rotational sense.  The record lists the vertices in slot order of their
// first triangle.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wb_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

template <int GW>
__device__ __forceinline__ unsigned long long grp_ballot(bool p, int gb)
{
    const unsigned long long m = __builtin_amdgcn_ballot_w64(p);
    return GW == 64 ? m : (m >> gb) & ((1ull << GW) - 1ull);
}

template <int GW>
__device__ __forceinline__ int grp_isum(int v)
{
#pragma unroll
    for (int m = 1; m < GW; m <<= 1) v += __shfl_xor(v, m, GW);
    return v;
}

// slot of the triangle across edge k (planes k, k+1) of slot s
template <int NT, int MAXP>
__device__ __forceinline__ int wb_twin(const uint32_t *tpl, const uint8_t (*etab)[MAXP], int s, int k)
{
    const uint32_t t3 = tpl[s];
    const int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * (k == 2 ? 0 : k + 1))) & 0xff;
    return etab[b][a] & (NT - 1);
}

// Once around the vertex that slot r belongs to, starting at r's first
// edge of positive length.  A zero-length edge is stepped through into the
// next triangle of the same vertex, continuing after the shared edge.  The
// positive edges give the neighbours w_0 .. w_{m-1} in rotation order (as
// vertex numbers); a face that degenerated to a segment between two real
// faces (a plane that only touches the cell along an edge) makes the same
// neighbour appear twice in a row, so each run of equal neighbours counts
// once: emit(j, w_i) for every i with w_i != w_{i+1} (cyclically).  An edge
// back into the vertex itself is not an edge of the cell.  Returns the
// degree, or -1 for an inconsistent graph (or no positive edge at r).
template <int NT, int MAXP, class F>
__device__ __forceinline__ int wb_walk(const uint32_t *tpl, const uint8_t (*etab)[MAXP], const uint8_t *zbt,
                                       const uint8_t *vid, int r, F emit)
{
    int k0 = 0;
    while (k0 < 3 && ((zbt[r] >> k0) & 1)) k0++;
    if (k0 == 3) return -1;
    const int self = vid[r];
    int s = r, k = k0, n = 0, nraw = 0, first = -1, pend = -1;
    do {
        const int w = vid[wb_twin<NT, MAXP>(tpl, etab, s, k)];
        if (w != self) {
            if (nraw == 0) {
                first = w;
            } else if (w != pend) {
                emit(n, pend);
                n++;
            }
            pend = w;
            if (++nraw > 255) return -1;
        }
        k = k == 2 ? 0 : k + 1;
        int guard = 0;
        while ((zbt[s] >> k) & 1) {
            const int b = (tpl[s] >> (8 * (k == 2 ? 0 : k + 1))) & 0xff;
            const int s2 = wb_twin<NT, MAXP>(tpl, etab, s, k);
            const uint32_t u3 = tpl[s2];
            int k2 = 0;
            while (k2 < 3 && (int)((u3 >> (8 * k2)) & 0xff) != b) k2++;
            if (k2 == 3 || ++guard > NT) return -1;
            s = s2;
            k = k2 == 2 ? 0 : k2 + 1;
        }
    } while (s != r || k != k0);
    if (nraw > 0 && pend != first) {
        emit(n, pend);
        n++;
    }
    return n;
}

// Write the record of a finished cell: [V][D low][D high], the degree of
// each vertex, each vertex's neighbours in rotation order.  GW lanes hold
// the cell, slot t = s * GW + gl; bit 3s + k of zb: edge k of the lane's
// slot s has zero length; lab[t]: first slot of t's vertex.  zbt, vid and
// degs are LDS scratch of GW * S bytes.  Returns (in every lane) the code
// length D = 2E, or 0 when the record does not fit or the graph is found
// inconsistent: no code for the cell.
template <int GW, int S, int MAXP>
__device__ __noinline__ int wb_record(uint8_t *rec, int D, const uint32_t *tpl, const int32_t *lab, const uint8_t (*etab)[MAXP],
                         uint8_t *zbt, uint8_t *vid, uint8_t *degs, uint32_t zb, int gl, int gb)
{
    constexpr int NT = GW * S;
    int V = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        const int t = s * GW + gl;
        zbt[t] = (uint8_t)((zb >> (3 * s)) & 7);
        const bool rep = tpl[t] != 0xffffffffu && lab[t] == t;
        const unsigned long long m = grp_ballot<GW>(rep, gb);
        if (rep) vid[t] = (uint8_t)min(V + __popcll(m & ((1ull << gl) - 1ull)), 255);
        V += __popcll(m);
    }
    if (V > kWbMaxV || D > kWbMaxD || 3 + V + D > kWbStride) return 0;
    wb_fence();
#pragma unroll
    for (int s = 0; s < S; s++) {
        const int t = s * GW + gl;
        if (tpl[t] != 0xffffffffu && lab[t] != t) vid[t] = vid[lab[t] & (NT - 1)];
    }
    wb_fence();
    // a vertex's walk starts at its first triangle with a positive edge
    int start[S];
    int sum = 0;
    bool bad = false;
#pragma unroll
    for (int s = 0; s < S; s++) {
        const int t = s * GW + gl;
        start[s] = -1;
        if (tpl[t] == 0xffffffffu || lab[t] != t) continue;
        int r = t;
        if (zbt[t] == 7)
            for (int u = 0; u < NT; u++)
                if (tpl[u] != 0xffffffffu && lab[u] == t && zbt[u] != 7) {
                    r = u;
                    break;
                }
        const int dg = wb_walk<NT, MAXP>(tpl, etab, zbt, vid, r, [](int, int) {});
        if (dg < 3) {
            bad = true;
            continue;
        }
        start[s] = r;
        degs[vid[t]] = (uint8_t)dg;
        sum += dg;
    }
    sum = grp_isum<GW>(sum);
    if (grp_ballot<GW>(bad, gb) || sum != D) return 0;
    wb_fence();
#pragma unroll
    for (int s = 0; s < S; s++) {
        if (start[s] < 0) continue;
        const int v = vid[s * GW + gl];
        int off = 0;
        for (int u = 0; u < v; u++) off += degs[u];
        rec[3 + v] = degs[v];
        uint8_t *out = rec + 3 + V + off;
        wb_walk<NT, MAXP>(tpl, etab, zbt, vid, start[s], [&](int j, int w) { out[j] = (uint8_t)w; });
    }
    if (gl == 0) {
        rec[0] = (uint8_t)V;
        rec[1] = (uint8_t)(D & 0xff);
        rec[2] = (uint8_t)(D >> 8);
    }
    return D;
}
enum { DC_CAND, DC_TESTS, DC_CUTS, DC_NEWV, DC_EXACT, DC_RECHECK, DC_SPILL, DC_BLOCKS, DC_FALLBACK, DC_SHELLS, DC_LOADED, DC_N };

}  // namespace
}  // namespace vc
