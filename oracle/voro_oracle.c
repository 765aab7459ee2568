/*
 * voro_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, double-precision CPU implementation of the per-particle
 * Voronoi cell construction of Voro++ (Lu, Lazar & Rycroft, "An extension to
 * Voro++ for multithreaded computation of Voronoi cells", section 2.1).  It is
 * the oracle that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code with the GPU library.
 *
 * What is computed (section 2.1.2): the cell of particle P, in coordinates
 * centred on P, starts as the container box (Eq. 1-2: [a-p, b-p] on a walled
 * axis, [-L/2, L/2] on a periodic axis, the latter being the bisectors with
 * P's own images at +-L) and is cut by the half-space of Eq. 3,
 * { r : r.q > q.q/2 } removed, for every other particle (and periodic image)
 * at relative position q.  Neighbours are taken shell by shell from a uniform
 * grid of blocks (section 2.1.3) and a neighbour farther than 2R is skipped,
 * R being the largest vertex distance (the radius bound of section 2.1.3);
 * when a whole shell of blocks is farther than 2R the cell is complete.
 *
 * Representation: a convex polyhedron as a list of faces, each face a cyclic
 * list of vertex ids, counter-clockwise seen from outside.  A cut classifies
 * every vertex, clips each face (Sutherland-Hodgman), and closes the hole
 * with a new face chained from the cut segments of the clipped faces.  Each
 * new vertex is placed at the intersection of its three defining planes.
 *
 * Side decisions: s = n.v - h in FP64; if |s| <= tau*M (M = sum|n_d v_d|+|h|)
 * the sign is taken exactly from the symbolic definition of the vertex (the
 * three planes it lies on): s * det3(n_a,n_b,n_c) = det4([n_i, -h_i]), which
 * is evaluated exactly with dyadic big-integer arithmetic (every double is an
 * integer times a power of two).
 * A vertex exactly on the plane is kept and creates no new vertex.  With exact
 * decisions the resulting polytope is unique, whatever the cut order.
 *
 * The 2D form (section 2.1: "identical in both 2D and 3D") clips a polygon.
 *
 * Weinberg codes (section 5, the topology code that VoroTop computes for each
 * cell; after Weinberg 1966): the cell's edges as darts, one walk over every
 * dart per starting dart and orientation under Weinberg's three turning
 * rules, and the smallest resulting code.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define VO_MAXP 512   /* planes per cell */
#define VO_MAXV 1024  /* live vertices per cell */
#define VO_MAXF 256   /* faces per cell */
#define VO_MAXFV 128  /* vertices per face */
#define VO_FO 32      /* length of the face-order vector */

enum { VO_OK = 0, VO_EMPTY = 1, VO_ERR_CAP = -1, VO_ERR_TOPO = -2, VO_ERR_ARG = -3, VO_ERR_MEM = -4 };

/* counters (per call, summed over cells) */
enum { C_CAND = 0, C_RREJ, C_TESTS, C_CUTS, C_NEWV, C_TRIS, C_EXACT, C_SHELLS, C_AUDIT, C_AUDIT_BAD, C_NCOUNT };

/* ------------------------------------------------------------------------ */
/* Exact arithmetic: dyadic rationals m * 2^e with a sign-magnitude big      */
/* integer m (32-bit limbs).  Every double is such a number, and sums and    */
/* products of them are computed without rounding.                          */
/* ------------------------------------------------------------------------ */

#define XL 400 /* limbs: 12800 bits, enough for products of five doubles */

typedef struct {
    int sign;  /* -1, 0, +1 */
    int len;   /* used limbs */
    int exp;   /* value = sign * mag * 2^exp */
    uint32_t mag[XL];
} xnum;

static void x_norm(xnum *a)
{
    while (a->len > 0 && a->mag[a->len - 1] == 0) a->len--;
    if (a->len == 0) { a->sign = 0; a->exp = 0; }
}

static void x_from_double(xnum *a, double v)
{
    memset(a, 0, sizeof(*a) - sizeof(a->mag));
    if (v == 0.0) { a->sign = 0; a->len = 0; a->exp = 0; return; }
    int e;
    double f = frexp(fabs(v), &e);        /* |v| = f 2^e, f in [0.5, 1) */
    uint64_t m = (uint64_t)ldexp(f, 53);  /* exact: 53-bit integer */
    a->sign = v < 0 ? -1 : 1;
    a->exp = e - 53;
    a->mag[0] = (uint32_t)m;
    a->mag[1] = (uint32_t)(m >> 32);
    a->len = 2;
    x_norm(a);
}

/* mag <<= k bits */
static void x_shl(xnum *a, int k)
{
    if (a->sign == 0 || k == 0) return;
    int w = k / 32, b = k % 32;
    if (a->len + w + 1 > XL) abort();
    for (int i = a->len - 1 + w + 1; i >= 0; i--) {
        uint64_t hi = (i - w >= 0 && i - w < a->len) ? a->mag[i - w] : 0;
        uint64_t lo = (i - w - 1 >= 0 && i - w - 1 < a->len) ? a->mag[i - w - 1] : 0;
        uint64_t v = b ? ((hi << b) | (lo >> (32 - b))) : hi;
        a->mag[i] = (uint32_t)v;
    }
    a->len = a->len + w + 1;
    a->exp -= k;
    x_norm(a);
}

static int x_cmpmag(const xnum *a, const xnum *b)
{
    if (a->len != b->len) return a->len < b->len ? -1 : 1;
    for (int i = a->len - 1; i >= 0; i--)
        if (a->mag[i] != b->mag[i]) return a->mag[i] < b->mag[i] ? -1 : 1;
    return 0;
}

/* r = a + b (r may not alias) */
static void x_add(const xnum *a0, const xnum *b0, xnum *r)
{
    static _Thread_local xnum A, B;
    if (a0->sign == 0) { *r = *b0; return; }
    if (b0->sign == 0) { *r = *a0; return; }
    A = *a0;
    B = *b0;
    /* align to the smaller exponent */
    if (A.exp > B.exp) x_shl(&A, A.exp - B.exp);
    else if (B.exp > A.exp) x_shl(&B, B.exp - A.exp);
    memset(r, 0, sizeof(*r) - sizeof(r->mag));
    r->exp = A.exp;
    int n = A.len > B.len ? A.len : B.len;
    if (n + 1 > XL) abort();
    if (A.sign == B.sign) {
        uint64_t carry = 0;
        for (int i = 0; i < n; i++) {
            uint64_t s = carry + (i < A.len ? A.mag[i] : 0) + (i < B.len ? B.mag[i] : 0);
            r->mag[i] = (uint32_t)s;
            carry = s >> 32;
        }
        r->mag[n] = (uint32_t)carry;
        r->len = n + 1;
        r->sign = A.sign;
    } else {
        const xnum *big = &A, *sml = &B;
        int c = x_cmpmag(&A, &B);
        if (c == 0) { r->sign = 0; r->len = 0; r->exp = 0; return; }
        if (c < 0) { big = &B; sml = &A; }
        int64_t borrow = 0;
        for (int i = 0; i < n; i++) {
            int64_t d = (int64_t)(i < big->len ? big->mag[i] : 0) - (i < sml->len ? sml->mag[i] : 0) - borrow;
            borrow = d < 0;
            if (d < 0) d += ((int64_t)1 << 32);
            r->mag[i] = (uint32_t)d;
        }
        r->len = n;
        r->sign = big->sign;
    }
    x_norm(r);
}

/* r = a * b (r may not alias) */
static void x_mul(const xnum *a, const xnum *b, xnum *r)
{
    memset(r, 0, sizeof(*r) - sizeof(r->mag));
    if (a->sign == 0 || b->sign == 0) { r->sign = 0; r->len = 0; r->exp = 0; return; }
    int n = a->len + b->len;
    if (n > XL) abort();
    memset(r->mag, 0, (size_t)n * sizeof(uint32_t));
    for (int i = 0; i < a->len; i++) {
        uint64_t carry = 0;
        for (int j = 0; j < b->len; j++) {
            uint64_t t = (uint64_t)a->mag[i] * b->mag[j] + r->mag[i + j] + carry;
            r->mag[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        int k = i + b->len;
        while (carry) {
            uint64_t t = (uint64_t)r->mag[k] + carry;
            r->mag[k++] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    r->len = n;
    r->sign = a->sign * b->sign;
    r->exp = a->exp + b->exp;
    x_norm(r);
}

static void x_neg(xnum *a) { a->sign = -a->sign; }

/* r = det of the 3x3 matrix with rows u, v, w (exact) */
static void x_det3(const double *u, const double *v, const double *w, xnum *r)
{
    static const int perm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}, {2, 1, 0}};
    static _Thread_local xnum a, b, c, ab, abc, acc, t;
    memset(&acc, 0, sizeof(acc) - sizeof(acc.mag));
    for (int k = 0; k < 6; k++) {
        x_from_double(&a, u[perm[k][0]]);
        x_from_double(&b, v[perm[k][1]]);
        x_from_double(&c, w[perm[k][2]]);
        x_mul(&a, &b, &ab);
        x_mul(&ab, &c, &abc);
        if (k >= 3) x_neg(&abc);
        x_add(&acc, &abc, &t);
        acc = t;
    }
    *r = acc;
}

/* r = det of the 2x2 matrix with rows u, v (exact) */
static void x_det2(const double *u, const double *v, xnum *r)
{
    static _Thread_local xnum a, b, p1, p2;
    x_from_double(&a, u[0]);
    x_from_double(&b, v[1]);
    x_mul(&a, &b, &p1);
    x_from_double(&a, u[1]);
    x_from_double(&b, v[0]);
    x_mul(&a, &b, &p2);
    x_neg(&p2);
    x_add(&p1, &p2, r);
}

/* ------------------------------------------------------------------------ */
/* Planes                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double n[3];  /* normal; for a bisector n = q */
    double h;     /* kept side n.r <= h; FP64 value of q.q/2 for a bisector */
    int wall;     /* 1: axis-aligned wall with exact (n, h) */
    int32_t label;  /* neighbour id j, or -1..-6 for the walls x-,x+,y-,y+,z-,z+ */
    int radical;    /* radical plane: h = (q.q + ri^2 - rj^2) / 2 */
    double ri, rj;  /* radii of the cell's particle and of the neighbour */
    int32_t shift;  /* periodic image code 25(sz+2)+5(sy+2)+(sx+2) */
} oplane;

/* exact offset h of a plane: q.q/2 for a bisector, (q.q + ri^2 - rj^2)/2 for
 * a radical plane, the stored value for a wall */
static void x_plane_h(const oplane *p, int dim, xnum *r)
{
    static _Thread_local xnum a, sq, acc, t;
    if (p->wall) { x_from_double(r, p->h); return; }
    memset(&acc, 0, sizeof(acc) - sizeof(acc.mag));
    for (int d = 0; d < dim; d++) {
        x_from_double(&a, p->n[d]);
        x_mul(&a, &a, &sq);
        x_add(&acc, &sq, &t);
        acc = t;
    }
    if (p->radical) {
        x_from_double(&a, p->ri);
        x_mul(&a, &a, &sq);
        x_add(&acc, &sq, &t);
        acc = t;
        x_from_double(&a, p->rj);
        x_mul(&a, &a, &sq);
        sq.sign = -sq.sign;
        x_add(&acc, &sq, &t);
        acc = t;
    }
    if (acc.sign != 0) acc.exp -= 1; /* halve */
    *r = acc;
}

/* Exact sign of s = n_p.v - h_p for the vertex v where planes a, b, c (3D) or
 * a, b (2D) meet.  Uses s * det(N) = det([n_i, -h_i]) (Cramer's rule for the
 * homogeneous coordinate), expanded along the offset column: in 3D
 *   det4 = h_a D(b,c,p) - h_b D(a,c,p) + h_c D(a,b,p) - h_p D(a,b,c),
 * in 2D
 *   det3 = -h_a D(b,p) + h_b D(a,p) - h_p D(a,b). */
static int exact_side(const oplane *pa, const oplane *pb, const oplane *pc, const oplane *pp, int dim)
{
    static _Thread_local xnum hx, dd, prod, acc, t, dn;
    memset(&acc, 0, sizeof(acc) - sizeof(acc.mag));
    if (dim == 3) {
        const oplane *rows[4] = {pa, pb, pc, pp};
        static const int minor[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
        static const int sg[4] = {1, -1, 1, -1};
        for (int i = 0; i < 4; i++) {
            x_plane_h(rows[i], 3, &hx);
            if (sg[i] < 0) x_neg(&hx);
            x_det3(rows[minor[i][0]]->n, rows[minor[i][1]]->n, rows[minor[i][2]]->n, &dd);
            x_mul(&hx, &dd, &prod);
            x_add(&acc, &prod, &t);
            acc = t;
        }
        x_det3(pa->n, pb->n, pc->n, &dn);
    } else {
        const oplane *rows[3] = {pa, pb, pp};
        static const int minor[3][2] = {{1, 2}, {0, 2}, {0, 1}};
        static const int sg[3] = {-1, 1, -1};
        for (int i = 0; i < 3; i++) {
            x_plane_h(rows[i], 2, &hx);
            if (sg[i] < 0) x_neg(&hx);
            x_det2(rows[minor[i][0]]->n, rows[minor[i][1]]->n, &dd);
            x_mul(&hx, &dd, &prod);
            x_add(&acc, &prod, &t);
            acc = t;
        }
        x_det2(pa->n, pb->n, &dn);
    }
    return acc.sign * dn.sign;
}

/* ------------------------------------------------------------------------ */
/* Cell workspace                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int dim;
    double tau;
    int audit;            /* re-decide every test outside the band exactly */
    int np;
    oplane pl[VO_MAXP];
    int nv;
    double v[VO_MAXV][3];
    int vp[VO_MAXV][3];   /* defining planes of each vertex */
    /* faces (3D) */
    int nf;
    int fplane[VO_MAXF];
    int fn[VO_MAXF];
    int fv[VO_MAXF][VO_MAXFV];
    /* 2D polygon: vertex order and the line leaving each vertex */
    int pn;
    int pv[VO_MAXV];
    int pe[VO_MAXV];
    /* scratch */
    double tv[VO_MAXV][3];
    int tvp[VO_MAXV][3];
    double s[VO_MAXV];
    signed char sg[VO_MAXV];
    int64_t cnt[C_NCOUNT];
} ocell;

/* side decision of vertex v against plane p: -1 inside, 0 on, +1 outside */
static int decide(ocell *c, int v, const oplane *p)
{
    double s, m;
    if (c->dim == 3) {
        double t0 = p->n[0] * c->v[v][0], t1 = p->n[1] * c->v[v][1], t2 = p->n[2] * c->v[v][2];
        s = ((t0 + t1) + t2) - p->h;
        m = fabs(t0) + fabs(t1) + fabs(t2) + fabs(p->h);
    } else {
        double t0 = p->n[0] * c->v[v][0], t1 = p->n[1] * c->v[v][1];
        s = (t0 + t1) - p->h;
        m = fabs(t0) + fabs(t1) + fabs(p->h);
    }
    c->s[v] = s;
    const int *d = c->vp[v];
    if (s > c->tau * m || s < -c->tau * m) {
        int sg = s > 0.0 ? 1 : -1;
        if (c->audit) {
            /* the decision outside the band must be the exact sign */
            c->cnt[C_AUDIT]++;
            if (exact_side(&c->pl[d[0]], &c->pl[d[1]], c->dim == 3 ? &c->pl[d[2]] : NULL, p, c->dim) != sg)
                c->cnt[C_AUDIT_BAD]++;
        }
        return sg;
    }
    c->cnt[C_EXACT]++;
    return exact_side(&c->pl[d[0]], &c->pl[d[1]], c->dim == 3 ? &c->pl[d[2]] : NULL, p, c->dim);
}

static double max_r2(const ocell *c)
{
    double r2 = 0.0;
    for (int i = 0; i < c->nv; i++) {
        double a = c->v[i][0] * c->v[i][0] + c->v[i][1] * c->v[i][1] + c->v[i][2] * c->v[i][2];
        if (a > r2) r2 = a;
    }
    return r2;
}

static int shift_code(const int s[3]) { return 25 * (s[2] + 2) + 5 * (s[1] + 2) + (s[0] + 2); }

/* Offset of the domain's bounding plane on one side of axis d, in the
 * cell's frame (positive): half the period on a periodic axis (the bisector
 * with the particle's own image), else the distance to the wall. */
static double domain_offset(const double *p, const double *lo, const double *hi, const int *per, int d, int side)
{
    if (per[d]) return 0.5 * (hi[d] - lo[d]);
    return side ? (hi[d] - p[d]) : -(lo[d] - p[d]);
}

/* the two bounding planes of axis d: index 2d (low side), 2d+1 (high side).
 * With clipping (section 3.1.3: the cell starts from a cube of side h
 * centred on the particle), a side whose half-side h/2 is strictly inside
 * the domain's plane becomes an axis-aligned clip wall, labelled -7..-12
 * (x-, x+, y-, y+, z-, z+); ext receives the corner offsets. */
static void box_planes(ocell *c, const double *p, const double *lo, const double *hi, const int *per, int self,
                       double clip, double ext[3][2])
{
    c->np = 0;
    for (int d = 0; d < c->dim; d++) {
        for (int side = 0; side < 2; side++) {
            oplane *q = &c->pl[c->np++];
            memset(q, 0, sizeof(*q));
            double sgn = side ? 1.0 : -1.0;
            double off = domain_offset(p, lo, hi, per, d, side);
            double half = 0.5 * clip;
            if (clip > 0.0 && half < off) {
                q->wall = 1;
                q->n[d] = sgn;
                q->h = half;
                q->label = -(7 + 2 * d + side);
                q->shift = shift_code((int[3]){0, 0, 0});
                ext[d][side] = side ? half : -half;
            } else if (per[d]) {
                /* bisector with own image at sgn*L: n = sgn*L e_d, h = L^2/2 */
                double L = hi[d] - lo[d];
                q->wall = 0;
                q->n[d] = sgn * L;
                q->h = 0.5 * (L * L);
                q->label = self;
                int sh[3] = {0, 0, 0};
                sh[d] = side ? 1 : -1;
                q->shift = shift_code(sh);
                ext[d][side] = side ? off : -off;
            } else {
                /* wall: r_d >= a_d - p_d  or  r_d <= b_d - p_d */
                q->wall = 1;
                q->n[d] = sgn;
                q->h = off;
                q->label = -(2 * d + side + 1);
                q->shift = shift_code((int[3]){0, 0, 0});
                ext[d][side] = side ? (hi[d] - p[d]) : (lo[d] - p[d]);
            }
        }
    }
}

/* Initial cell = box (Eq. 1-2), or the clip cube inside it. */
static void cell_init(ocell *c, const double *p, const double *lo, const double *hi, const int *per, int self,
                      double clip)
{
    double ext[3][2];
    box_planes(c, p, lo, hi, per, self, clip, ext);
    if (c->dim == 3) {
        c->nv = 8;
        for (int k = 0; k < 8; k++) {
            for (int d = 0; d < 3; d++) {
                int b = (k >> d) & 1;
                c->v[k][d] = ext[d][b];
                c->vp[k][d] = 2 * d + b;
            }
        }
        c->nf = 6;
        for (int d = 0; d < 3; d++) {
            int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
            for (int side = 0; side < 2; side++) {
                int f = 2 * d + side;
                c->fplane[f] = f;
                c->fn[f] = 4;
                /* (e1,e2) = (+,+), (-,+), (-,-), (+,-) is counter-clockwise seen
                 * from +e_d; reversed for the low side */
                static const int pat[4][2] = {{1, 1}, {0, 1}, {0, 0}, {1, 0}};
                for (int k = 0; k < 4; k++) {
                    int kk = side ? k : 3 - k;
                    c->fv[f][k] = (side << d) | (pat[kk][0] << e1) | (pat[kk][1] << e2);
                }
            }
        }
    } else {
        /* polygon corners CCW: (lo,lo) (hi,lo) (hi,hi) (lo,hi); edge k lies on
         * line y-, x+, y+, x- respectively */
        static const int cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
        static const int edge[4] = {2, 1, 3, 0};
        c->nv = 4;
        c->pn = 4;
        for (int k = 0; k < 4; k++) {
            c->v[k][0] = ext[0][cx[k]];
            c->v[k][1] = ext[1][cy[k]];
            c->v[k][2] = 0.0;
            c->vp[k][0] = cx[k];
            c->vp[k][1] = 2 + cy[k];
            c->vp[k][2] = -1;
            c->pv[k] = k;
            c->pe[k] = edge[k];
        }
    }
}

/* new vertex on the segment from an inside vertex a (s<0) to an outside b */
static void interp(const ocell *c, int a, int b, double *out)
{
    double sa = c->s[a], sb = c->s[b];
    double t = sa / (sa - sb);
    if (!(t >= 0.0)) t = 0.0;
    if (t > 1.0) t = 1.0;
    for (int d = 0; d < 3; d++) out[d] = c->v[a][d] + t * (c->v[b][d] - c->v[a][d]);
}

/* The point where three planes meet (Cramer's rule on n.r = h).  A new
 * vertex is placed here from its defining planes rather than interpolated
 * along the cut edge, so its rounding does not grow with the distance to
 * earlier (possibly far-away) vertices. */
static int solve3(const oplane *a, const oplane *b, const oplane *c, double *out)
{
    double bc[3] = {b->n[1] * c->n[2] - b->n[2] * c->n[1], b->n[2] * c->n[0] - b->n[0] * c->n[2],
                    b->n[0] * c->n[1] - b->n[1] * c->n[0]};
    double ca[3] = {c->n[1] * a->n[2] - c->n[2] * a->n[1], c->n[2] * a->n[0] - c->n[0] * a->n[2],
                    c->n[0] * a->n[1] - c->n[1] * a->n[0]};
    double ab[3] = {a->n[1] * b->n[2] - a->n[2] * b->n[1], a->n[2] * b->n[0] - a->n[0] * b->n[2],
                    a->n[0] * b->n[1] - a->n[1] * b->n[0]};
    double det = a->n[0] * bc[0] + a->n[1] * bc[1] + a->n[2] * bc[2];
    if (det == 0.0) return 0;
    for (int d = 0; d < 3; d++) out[d] = (a->h * bc[d] + b->h * ca[d] + c->h * ab[d]) / det;
    return 1;
}

/* the point where two lines meet (2D) */
static int solve2(const oplane *a, const oplane *b, double *out)
{
    double det = a->n[0] * b->n[1] - a->n[1] * b->n[0];
    if (det == 0.0) return 0;
    out[0] = (a->h * b->n[1] - a->n[1] * b->h) / det;
    out[1] = (a->n[0] * b->h - a->h * b->n[0]) / det;
    out[2] = 0.0;
    return 1;
}

/* Cut the 3D cell by plane *P.  Returns 1 if it cut, 0 if not, <0 on error. */
static int cut3(ocell *c, const oplane *P)
{
    int any = 0, inside = 0;
    for (int i = 0; i < c->nv; i++) {
        c->sg[i] = (signed char)decide(c, i, P);
        if (c->sg[i] > 0) any = 1;
        if (c->sg[i] < 0) inside = 1;
    }
    c->cnt[C_TESTS] += c->nv;
    if (!any) return 0;
    if (!inside) {
        /* no vertex strictly inside: what is left has no volume (radical
         * planes can remove a whole cell) */
        c->nv = 0;
        c->nf = 0;
        return 2;
    }
    if (c->np >= VO_MAXP) return VO_ERR_CAP;
    int pid = c->np++;
    c->pl[pid] = *P;
    c->cnt[C_CUTS]++;

    int nv0 = c->nv;
    /* new vertices on crossing edges, keyed by the (unordered) vertex pair */
    int ek[VO_MAXV][2], nek = 0;
    int segn[VO_MAXV]; /* successor of an on-plane vertex along the new face */
    int nseg = 0;
    for (int i = 0; i < VO_MAXV; i++) segn[i] = -1;
    int seg_start = -1;

    int out[VO_MAXFV * 2];
    for (int f = 0; f < c->nf; f++) {
        int n = c->fn[f], m = 0;
        for (int k = 0; k < n; k++) {
            int u = c->fv[f][k], w = c->fv[f][(k + 1) % n];
            if (c->sg[u] <= 0) out[m++] = u;
            if ((c->sg[u] < 0 && c->sg[w] > 0) || (c->sg[u] > 0 && c->sg[w] < 0)) {
                int lo = u < w ? u : w, hi = u < w ? w : u, x = -1;
                for (int e = 0; e < nek; e++)
                    if (ek[e][0] == lo && ek[e][1] == hi) { x = nv0 + e; break; }
                if (x < 0) {
                    if (c->nv >= VO_MAXV) return VO_ERR_CAP;
                    x = c->nv++;
                    ek[nek][0] = lo;
                    ek[nek][1] = hi;
                    nek++;
                    if (c->sg[u] < 0) interp(c, u, w, c->v[x]); else interp(c, w, u, c->v[x]);
                    c->vp[x][0] = c->fplane[f];
                    c->vp[x][1] = -1;
                    c->vp[x][2] = pid;
                    c->sg[x] = 0;
                    c->cnt[C_NEWV]++;
                } else {
                    c->vp[x][1] = c->fplane[f];
                }
                out[m++] = x;
            }
        }
        if (m >= VO_MAXFV) return VO_ERR_CAP;
        if (m < 3) { c->fn[f] = 0; continue; }
        c->fn[f] = m;
        memcpy(c->fv[f], out, (size_t)m * sizeof(int));
        /* the edge of this face that lies on the cut plane: consecutive on-plane
         * vertices a -> b; the new face runs b -> a */
        for (int k = 0; k < m; k++) {
            int a = out[k], b = out[(k + 1) % m];
            if (c->sg[a] == 0 && c->sg[b] == 0) {
                if (segn[b] >= 0) return VO_ERR_TOPO;
                segn[b] = a;
                seg_start = b;
                nseg++;
            }
        }
    }
    if (nseg < 3) return VO_ERR_TOPO;
    /* new vertices from their three defining planes (the interpolated point
     * is kept only if the planes were found singular) */
    for (int x = nv0; x < c->nv; x++) {
        if (c->vp[x][1] < 0) return VO_ERR_TOPO;
        double w[3];
        if (solve3(&c->pl[c->vp[x][0]], &c->pl[c->vp[x][1]], &c->pl[c->vp[x][2]], w))
            memcpy(c->v[x], w, sizeof(w));
    }
    /* drop emptied faces */
    int nf = 0;
    for (int f = 0; f < c->nf; f++) {
        if (c->fn[f] == 0) continue;
        if (nf != f) {
            c->fplane[nf] = c->fplane[f];
            c->fn[nf] = c->fn[f];
            memcpy(c->fv[nf], c->fv[f], (size_t)c->fn[f] * sizeof(int));
        }
        nf++;
    }
    /* chain the new face */
    if (nf >= VO_MAXF || nseg >= VO_MAXFV) return VO_ERR_CAP;
    int cur = seg_start, k = 0;
    do {
        c->fv[nf][k++] = cur;
        cur = segn[cur];
        if (cur < 0 || k > nseg) return VO_ERR_TOPO;
    } while (cur != seg_start);
    if (k != nseg) return VO_ERR_TOPO;
    c->fplane[nf] = pid;
    c->fn[nf] = nseg;
    c->nf = nf + 1;

    /* renumber the live vertices densely (through scratch copies) */
    int map[VO_MAXV];
    for (int i = 0; i < c->nv; i++) map[i] = -1;
    int nv = 0;
    for (int f = 0; f < c->nf; f++)
        for (int q = 0; q < c->fn[f]; q++) {
            int v = c->fv[f][q];
            if (map[v] < 0) {
                map[v] = nv;
                memcpy(c->tv[nv], c->v[v], sizeof(c->v[0]));
                memcpy(c->tvp[nv], c->vp[v], sizeof(c->vp[0]));
                nv++;
            }
            c->fv[f][q] = map[v];
        }
    memcpy(c->v, c->tv, (size_t)nv * sizeof(c->v[0]));
    memcpy(c->vp, c->tvp, (size_t)nv * sizeof(c->vp[0]));
    c->nv = nv;
    return 1;
}

/* Cut the 2D polygon by line *P. */
static int cut2(ocell *c, const oplane *P)
{
    int any = 0, inside = 0;
    for (int k = 0; k < c->pn; k++) {
        int v = c->pv[k];
        c->sg[v] = (signed char)decide(c, v, P);
        if (c->sg[v] > 0) any = 1;
        if (c->sg[v] < 0) inside = 1;
    }
    c->cnt[C_TESTS] += c->pn;
    if (!any) return 0;
    if (!inside) {
        c->nv = 0;
        c->pn = 0;
        return 2;
    }
    if (c->np >= VO_MAXP) return VO_ERR_CAP;
    int pid = c->np++;
    c->pl[pid] = *P;
    c->cnt[C_CUTS]++;
    int nv_[VO_MAXV], ne_[VO_MAXV], m = 0;
    int n = c->pn;
    for (int k = 0; k < n; k++) {
        int u = c->pv[k], w = c->pv[(k + 1) % n];
        int line = c->pe[k];
        int su = c->sg[u], sw = c->sg[w];
        if (su <= 0) {
            nv_[m] = u;
            /* the edge leaving u: along its own line unless u is on the cut
             * line and the next vertex is cut away */
            ne_[m] = (su == 0 && sw > 0) ? pid : line;
            m++;
        }
        if ((su < 0 && sw > 0) || (su > 0 && sw < 0)) {
            if (c->nv >= VO_MAXV) return VO_ERR_CAP;
            int x = c->nv++;
            if (su < 0) interp(c, u, w, c->v[x]); else interp(c, w, u, c->v[x]);
            c->vp[x][0] = line;
            c->vp[x][1] = pid;
            c->vp[x][2] = -1;
            {
                double pt[3];
                if (solve2(&c->pl[line], &c->pl[pid], pt)) memcpy(c->v[x], pt, sizeof(pt));
            }
            c->cnt[C_NEWV]++;
            nv_[m] = x;
            ne_[m] = (su < 0) ? pid : line;
            m++;
        }
    }
    if (m < 3) return VO_ERR_TOPO;
    /* compact (through scratch copies) */
    for (int k = 0; k < m; k++) {
        memcpy(c->tv[k], c->v[nv_[k]], sizeof(c->v[0]));
        memcpy(c->tvp[k], c->vp[nv_[k]], sizeof(c->vp[0]));
    }
    memcpy(c->v, c->tv, (size_t)m * sizeof(c->v[0]));
    memcpy(c->vp, c->tvp, (size_t)m * sizeof(c->vp[0]));
    for (int k = 0; k < m; k++) { c->pv[k] = k; c->pe[k] = ne_[k]; }
    c->pn = m;
    c->nv = m;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Container: a plain uniform grid with a stable counting sort               */
/* ------------------------------------------------------------------------ */

typedef struct vo_handle {
    int dim;
    int64_t n;
    double lo[3], hi[3], L[3], bs[3];
    int per[3];
    int g[3];
    int64_t nb;
    int64_t *start;  /* nb+1 */
    int64_t *ids;    /* particle ids sorted by block */
    double *xyz;     /* n x 3 (z = 0 in 2D) */
    int *blk;        /* block index per particle */
    double clip;     /* side of the clip cube, 0: none */
    double *rad;     /* radii (radical tessellation), NULL: Voronoi */
    double rmax;     /* largest radius */
} vo_handle;

static int block_coord(const vo_handle *H, double x, int d)
{
    int k = (int)floor((x - H->lo[d]) / H->bs[d]);
    if (k < 0) k = 0;
    if (k >= H->g[d]) k = H->g[d] - 1;
    return k;
}

vo_handle *vo_create(int dim, const double *xyz, int64_t n, const double *lo, const double *hi,
                     const int *periodic, const int *grid)
{
    if ((dim != 2 && dim != 3) || n < 1) return NULL;
    vo_handle *H = (vo_handle *)calloc(1, sizeof(vo_handle));
    if (!H) return NULL;
    H->dim = dim;
    H->n = n;
    H->nb = 1;
    for (int d = 0; d < 3; d++) {
        if (d < dim) {
            H->lo[d] = lo[d];
            H->hi[d] = hi[d];
            H->per[d] = periodic[d] ? 1 : 0;
            H->g[d] = grid[d] > 0 ? grid[d] : 1;
        } else {
            H->lo[d] = 0.0;
            H->hi[d] = 1.0;
            H->per[d] = 0;
            H->g[d] = 1;
        }
        H->L[d] = H->hi[d] - H->lo[d];
        H->bs[d] = H->L[d] / H->g[d];
        H->nb *= H->g[d];
    }
    H->xyz = (double *)malloc((size_t)n * 3 * sizeof(double));
    H->blk = (int *)malloc((size_t)n * sizeof(int));
    H->start = (int64_t *)calloc((size_t)H->nb + 1, sizeof(int64_t));
    H->ids = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!H->xyz || !H->blk || !H->start || !H->ids) return NULL;
    for (int64_t i = 0; i < n; i++) {
        for (int d = 0; d < 3; d++) H->xyz[3 * i + d] = d < dim ? xyz[dim * i + d] : 0.0;
        int k0 = block_coord(H, H->xyz[3 * i], 0);
        int k1 = block_coord(H, H->xyz[3 * i + 1], 1);
        int k2 = block_coord(H, H->xyz[3 * i + 2], 2);
        H->blk[i] = k0 + H->g[0] * (k1 + H->g[1] * k2);
        H->start[H->blk[i] + 1]++;
    }
    for (int64_t b = 0; b < H->nb; b++) H->start[b + 1] += H->start[b];
    int64_t *fill = (int64_t *)malloc((size_t)H->nb * sizeof(int64_t));
    memcpy(fill, H->start, (size_t)H->nb * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) H->ids[fill[H->blk[i]]++] = i;
    free(fill);
    return H;
}

/* Clip every cell by the cube of side h centred on its particle (0: none). */
void vo_set_clip(vo_handle *H, double h)
{
    if (H) H->clip = h > 0.0 ? h : 0.0;
}

/* Radical (power) tessellation: the cell of i is the set of points x with
 * |x - p_i|^2 - r_i^2 <= |x - p_j|^2 - r_j^2 for every j (the radical Voronoi
 * tessellation that the paper's polydisperse container computes, section
 * 2.1.1).  r: n radii, or NULL for the plain Voronoi tessellation. */
int vo_set_radii(vo_handle *H, const double *r)
{
    if (!H) return VO_ERR_ARG;
    free(H->rad);
    H->rad = NULL;
    H->rmax = 0.0;
    if (!r) return VO_OK;
    H->rad = (double *)malloc((size_t)H->n * sizeof(double));
    if (!H->rad) return VO_ERR_MEM;
    for (int64_t i = 0; i < H->n; i++) {
        if (!(r[i] >= 0.0) || !isfinite(r[i])) return VO_ERR_ARG;
        H->rad[i] = r[i];
        if (r[i] > H->rmax) H->rmax = r[i];
    }
    return VO_OK;
}

void vo_destroy(vo_handle *H)
{
    if (!H) return;
    free(H->rad);
    free(H->xyz);
    free(H->blk);
    free(H->start);
    free(H->ids);
    free(H);
}

typedef struct { double d2; int64_t j; int shift; double q[3]; } ocand;

static int cand_cmp(const void *a, const void *b)
{
    const ocand *x = (const ocand *)a, *y = (const ocand *)b;
    if (x->d2 != y->d2) return x->d2 < y->d2 ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return (x->shift > y->shift) - (x->shift < y->shift);
}

/* Compute the cell of particle i.  Returns VO_OK or an error code. */
/* Squared search radius: a candidate at distance d can cut only if some
 * vertex v (|v| <= R) has v.q > h, i.e. d^2 - 2Rd + ri^2 - rj^2 < 0, so d < R +
 * sqrt(R^2 + rmax^2 - ri^2); without radii that is 2R. */
static double search_r2(const vo_handle *H, double r2, double ri)
{
    if (!H->rad) return 4.0 * r2;
    double t = r2 + H->rmax * H->rmax - ri * ri;
    double l = sqrt(r2) + sqrt(t > 0.0 ? t : 0.0);
    return l * l * (1.0 + 0x1p-40);
}

static int compute_cell(const vo_handle *H, int64_t i, ocell *c, ocand **cbuf, int64_t *ccap)
{
    const int dim = H->dim;
    const double *p = &H->xyz[3 * i];
    const double ri = H->rad ? H->rad[i] : 0.0;
    c->dim = dim;
    cell_init(c, p, H->lo, H->hi, H->per, (int32_t)i, H->clip);
    double r2 = max_r2(c);
    int b[3], own = H->blk[i];
    b[0] = own % H->g[0];
    b[1] = (own / H->g[0]) % H->g[1];
    b[2] = own / (H->g[0] * H->g[1]);
    /* distance from p to the faces of its own block, per axis */
    double mrg[3];
    for (int d = 0; d < 3; d++) {
        double blo = H->lo[d] + b[d] * H->bs[d];
        double a = p[d] - blo, e = blo + H->bs[d] - p[d];
        mrg[d] = a < e ? a : e;
    }
    for (int r = 0;; r++) {
        /* lower bound on the distance to any block of Chebyshev shell r */
        if (r > 0) {
            double lb = INFINITY;
            int exists = 0;
            for (int d = 0; d < dim; d++) {
                double g = (r - 1) * H->bs[d] + mrg[d];
                if (g < lb) lb = g;
                if (H->per[d] || b[d] - r >= 0 || b[d] + r < H->g[d]) exists = 1;
            }
            if (!exists) break;
            if (lb > 0 && lb * lb >= search_r2(H, r2, ri)) break;
        }
        c->cnt[C_SHELLS]++;
        int rz = dim == 3 ? r : 0;
        int64_t nc = 0;
        for (int dz = -rz; dz <= rz; dz++)
            for (int dy = -r; dy <= r; dy++)
                for (int dx = -r; dx <= r; dx++) {
                    int ax = abs(dx), ay = abs(dy), az = abs(dz);
                    int cheb = ax > ay ? ax : ay;
                    if (az > cheb) cheb = az;
                    if (cheb != r) continue;
                    int off[3] = {dx, dy, dz}, bb[3], sh[3] = {0, 0, 0};
                    int ok = 1;
                    for (int d = 0; d < 3; d++) {
                        int t = b[d] + off[d];
                        if (H->per[d]) {
                            int gd = H->g[d];
                            int w = ((t % gd) + gd) % gd;
                            sh[d] = (t - w) / gd;
                            bb[d] = w;
                        } else {
                            if (t < 0 || t >= H->g[d]) ok = 0;
                            bb[d] = t;
                        }
                    }
                    if (!ok) continue;
                    int64_t blk = bb[0] + (int64_t)H->g[0] * (bb[1] + (int64_t)H->g[1] * bb[2]);
                    for (int64_t t = H->start[blk]; t < H->start[blk + 1]; t++) {
                        int64_t j = H->ids[t];
                        if (j == i && sh[0] == 0 && sh[1] == 0 && sh[2] == 0) continue;
                        if (nc >= *ccap) {
                            *ccap = *ccap * 2 + 64;
                            *cbuf = (ocand *)realloc(*cbuf, (size_t)*ccap * sizeof(ocand));
                            if (!*cbuf) return VO_ERR_MEM;
                        }
                        ocand *o = &(*cbuf)[nc++];
                        o->j = j;
                        o->shift = shift_code(sh);
                        /* relative vector: fl(fl(x_j - x_i) + s L) per axis */
                        for (int d = 0; d < 3; d++) {
                            double q = H->xyz[3 * j + d] - p[d];
                            if (sh[d] != 0) q = q + sh[d] * H->L[d];
                            o->q[d] = q;
                        }
                        o->d2 = o->q[0] * o->q[0] + o->q[1] * o->q[1] + o->q[2] * o->q[2];
                        if (sh[0] > 2 || sh[0] < -2 || sh[1] > 2 || sh[1] < -2 || sh[2] > 2 || sh[2] < -2)
                            o->d2 = INFINITY; /* farther than any cell can reach */
                    }
                }
        qsort(*cbuf, (size_t)nc, sizeof(ocand), cand_cmp);
        for (int64_t t = 0; t < nc; t++) {
            ocand *o = &(*cbuf)[t];
            c->cnt[C_CAND]++;
            if (o->d2 == 0.0) return VO_ERR_ARG; /* coincident particles */
            if (o->d2 >= search_r2(H, r2, ri)) { c->cnt[C_RREJ]++; continue; }
            oplane P;
            memset(&P, 0, sizeof(P));
            P.wall = 0;
            P.n[0] = o->q[0];
            P.n[1] = o->q[1];
            P.n[2] = o->q[2];
            if (H->rad) {
                /* radical plane: |x|^2 - ri^2 <= |x - q|^2 - rj^2 */
                const double rj = H->rad[o->j];
                P.radical = 1;
                P.ri = ri;
                P.rj = rj;
                P.h = 0.5 * (o->d2 + (ri * ri - rj * rj));
            } else {
                P.h = 0.5 * o->d2;
            }
            P.label = (int32_t)o->j;
            P.shift = o->shift;
            int rc = dim == 3 ? cut3(c, &P) : cut2(c, &P);
            if (rc < 0) return rc;
            if (rc == 2) return VO_EMPTY;
            if (rc > 0) r2 = max_r2(c);
        }
    }
    return VO_OK;
}

typedef struct {
    double vol, cen[3], perim;
    int nv, ne, nf;
    int fo[VO_FO];
    int fo_over; /* a face has VO_FO or more edges: fo does not count it */
} ostats;

/* status flag of a complete cell with a face of VO_FO or more edges (its
 * face-order vector then sums to less than F) */
#define VO_FO_OVER 64

/* statistics of a finished 3D cell: volume and centroid from the tetrahedra
 * (origin, f0, fk, fk+1) of a fan over each face; V, E, F; face orders */
static void stats3(ocell *c, ostats *st, int32_t *nbr, int32_t *nsh, int maxnb)
{
    double vol = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    int e2 = 0;
    memset(st->fo, 0, sizeof(st->fo));
    st->fo_over = 0;
    /* tetrahedra (o, f0, fk, fk+1) from the particle (o = 0) when it lies
     * strictly inside the cell (every face offset h > 0: always so for a
     * Voronoi cell), else from one vertex of the cell, so that every term is
     * >= 0 also for a radical cell that misses its particle */
    static const double zero[3] = {0.0, 0.0, 0.0};
    int inside = 1;
    for (int f = 0; f < c->nf; f++)
        if (!(c->pl[c->fplane[f]].h > 0.0)) inside = 0;
    const double *o = inside ? zero : c->v[c->fv[0][0]];
    for (int f = 0; f < c->nf; f++) {
        int n = c->fn[f];
        const double *a0 = c->v[c->fv[f][0]];
        const double a[3] = {a0[0] - o[0], a0[1] - o[1], a0[2] - o[2]};
        for (int k = 1; k + 1 < n; k++) {
            const double *b0 = c->v[c->fv[f][k]], *d0 = c->v[c->fv[f][k + 1]];
            const double b[3] = {b0[0] - o[0], b0[1] - o[1], b0[2] - o[2]};
            const double d[3] = {d0[0] - o[0], d0[1] - o[1], d0[2] - o[2]};
            double det = a[0] * (b[1] * d[2] - b[2] * d[1]) - a[1] * (b[0] * d[2] - b[2] * d[0]) +
                         a[2] * (b[0] * d[1] - b[1] * d[0]);
            double tv = det / 6.0;
            vol += tv;
            cx += tv * (a[0] + b[0] + d[0]) / 4.0;
            cy += tv * (a[1] + b[1] + d[1]) / 4.0;
            cz += tv * (a[2] + b[2] + d[2]) / 4.0;
            c->cnt[C_TRIS]++;
        }
        e2 += n;
        if (n < VO_FO) st->fo[n]++;
        else st->fo_over = 1;
        if (nbr && f < maxnb) {
            nbr[f] = c->pl[c->fplane[f]].label;
            nsh[f] = c->pl[c->fplane[f]].shift;
        }
    }
    st->vol = vol;
    st->cen[0] = o[0] + cx / vol;
    st->cen[1] = o[1] + cy / vol;
    st->cen[2] = o[2] + cz / vol;
    st->nv = c->nv;
    st->ne = e2 / 2;
    st->nf = c->nf;
    st->perim = 0.0;
}

/* 2D statistics: area by the shoelace sum, centroid, perimeter, edge count */
static void stats2(ocell *c, ostats *st, int32_t *nbr, int32_t *nsh, int maxnb)
{
    double area = 0.0, cx = 0.0, cy = 0.0, per = 0.0;
    int n = c->pn;
    /* triangles (o, v_k, v_k+1) from the particle when it lies strictly
     * inside the cell, else from the first vertex (a radical cell that misses
     * its particle) */
    static const double zero[3] = {0.0, 0.0, 0.0};
    int inside = 1;
    for (int k = 0; k < n; k++)
        if (!(c->pl[c->pe[k]].h > 0.0)) inside = 0;
    const double *o = inside ? zero : c->v[c->pv[0]];
    for (int k = 0; k < n; k++) {
        const double *a0 = c->v[c->pv[k]], *b0 = c->v[c->pv[(k + 1) % n]];
        const double a[2] = {a0[0] - o[0], a0[1] - o[1]}, b[2] = {b0[0] - o[0], b0[1] - o[1]};
        double cr = a[0] * b[1] - a[1] * b[0];
        area += cr / 2.0;
        cx += cr * (a[0] + b[0]) / 6.0;
        cy += cr * (a[1] + b[1]) / 6.0;
        double dx = b0[0] - a0[0], dy = b0[1] - a0[1];
        per += sqrt(dx * dx + dy * dy);
        if (nbr && k < maxnb) {
            nbr[k] = c->pl[c->pe[k]].label;
            nsh[k] = c->pl[c->pe[k]].shift;
        }
        c->cnt[C_TRIS]++;
    }
    memset(st->fo, 0, sizeof(st->fo));
    st->vol = area;
    st->cen[0] = o[0] + cx / area;
    st->cen[1] = o[1] + cy / area;
    st->cen[2] = 0.0;
    st->perim = per;
    st->nv = n;
    st->ne = n;
    st->nf = n;
}

/* Exactness audit switch: while set, every side decision taken outside the
 * band is also decided exactly, and disagreements are counted (test
 * infrastructure; set it before vo_cells, not during). */
static int g_audit = 0;

void vo_set_audit(int on)
{
    g_audit = on ? 1 : 0;
}

/* Compute the cells of the m particles idx[0..m).  Outputs (each may be
 * NULL): vol[m], cen[3m], nv/ne/nf[m], fo[32m], nbr/nsh[maxnb*m] (one label
 * per face, unsorted), perim[m], status[m], counters[C_NCOUNT] (summed).
 * nthreads > 1 runs the cells under an OpenMP dynamic schedule, each cell
 * still serial.  Returns 0, or the first per-cell error code. */
int vo_cells(const vo_handle *H, const int64_t *idx, int64_t m, int nthreads, double tau, double *vol,
             double *cen, int32_t *nv, int32_t *ne, int32_t *nf, int32_t *fo, int32_t *nbr, int32_t *nsh,
             int maxnb, double *perim, int32_t *status, int64_t *counters)
{
    if (!H || (m > 0 && !idx)) return VO_ERR_ARG;
    int err = 0;
    int64_t tot[C_NCOUNT];
    memset(tot, 0, sizeof(tot));
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
    {
        ocell *c = (ocell *)malloc(sizeof(ocell));
        int64_t ccap = 256;
        ocand *cbuf = (ocand *)malloc((size_t)ccap * sizeof(ocand));
        if (c) memset(c->cnt, 0, sizeof(c->cnt));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (int64_t t = 0; t < m; t++) {
            if (!c || !cbuf) { err = VO_ERR_MEM; continue; }
            c->tau = tau;
            c->audit = g_audit;
            int64_t i = idx[t];
            int rc = (i < 0 || i >= H->n) ? VO_ERR_ARG : compute_cell(H, i, c, &cbuf, &ccap);
            if (status) status[t] = rc;
            if (rc == VO_EMPTY) {
                /* an empty radical cell: zero volume, no faces */
                if (vol) vol[t] = 0.0;
                if (cen) cen[3 * t] = cen[3 * t + 1] = cen[3 * t + 2] = 0.0;
                if (nv) nv[t] = 0;
                if (ne) ne[t] = 0;
                if (nf) nf[t] = 0;
                if (fo) memset(fo + (size_t)t * VO_FO, 0, VO_FO * sizeof(int32_t));
                if (perim) perim[t] = 0.0;
                continue;
            }
            if (rc != VO_OK) {
#ifdef _OPENMP
#pragma omp critical
#endif
                if (!err) err = rc;
                continue;
            }
            ostats st;
            int32_t *nb = nbr ? nbr + (size_t)t * maxnb : NULL;
            int32_t *ns = nsh ? nsh + (size_t)t * maxnb : NULL;
            st.fo_over = 0;
            if (H->dim == 3) stats3(c, &st, nb, ns, maxnb); else stats2(c, &st, nb, ns, maxnb);
            if (status && st.fo_over) status[t] |= VO_FO_OVER;
            if (vol) vol[t] = st.vol;
            if (cen) for (int d = 0; d < 3; d++) cen[3 * t + d] = st.cen[d];
            if (nv) nv[t] = st.nv;
            if (ne) ne[t] = st.ne;
            if (nf) nf[t] = st.nf;
            if (fo) memcpy(fo + (size_t)t * VO_FO, st.fo, sizeof(st.fo));
            if (perim) perim[t] = st.perim;
        }
        if (c) {
#ifdef _OPENMP
#pragma omp critical
#endif
            for (int k = 0; k < C_NCOUNT; k++) tot[k] += c->cnt[k];
        }
        free(c);
        free(cbuf);
    }
    if (counters) memcpy(counters, tot, sizeof(tot));
    return err;
}

/* The exact side predicate alone, for tests: planes given as (n, h, wall)
 * rows a, b, c (c ignored in 2D) and p.  Returns -1, 0 or +1. */
int vo_exact_side(int dim, const double *rows /* 4 x 5: n0 n1 n2 h wall */)
{
    oplane pl[4];
    for (int k = 0; k < 4; k++) {
        memset(&pl[k], 0, sizeof(oplane));
        for (int d = 0; d < 3; d++) pl[k].n[d] = rows[5 * k + d];
        pl[k].h = rows[5 * k + 3];
        pl[k].wall = rows[5 * k + 4] != 0.0;
    }
    if (dim == 3) return exact_side(&pl[0], &pl[1], &pl[2], &pl[3], 3);
    return exact_side(&pl[0], &pl[1], NULL, &pl[3], 2);
}

int vo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Vertices of the cell of particle i (relative to the particle), for the
 * empty-sphere certificate in tests.  Writes up to maxv vertices (3 doubles
 * each, z = 0 in 2D) and returns their number, or a negative error code. */
int vo_cell_vertices(const vo_handle *H, int64_t i, double tau, double *out, int maxv)
{
    if (!H || i < 0 || i >= H->n) return VO_ERR_ARG;
    ocell *c = (ocell *)calloc(1, sizeof(ocell));
    int64_t ccap = 256;
    ocand *cbuf = (ocand *)malloc((size_t)ccap * sizeof(ocand));
    if (!c || !cbuf) { free(c); free(cbuf); return VO_ERR_MEM; }
    c->tau = tau;
    c->audit = 0;
    int rc = compute_cell(H, i, c, &cbuf, &ccap);
    if (rc == VO_EMPTY) rc = 0; /* no vertices */
    else if (rc == VO_OK) {
        int n = H->dim == 3 ? c->nv : c->pn;
        for (int k = 0; k < n && k < maxv; k++) {
            int v = H->dim == 3 ? k : c->pv[k];
            for (int d = 0; d < 3; d++) out[3 * k + d] = c->v[v][d];
        }
        rc = n;
    }
    free(c);
    free(cbuf);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Weinberg codes (the topology code of VoroTop, section 5; Weinberg 1966)   */
/* ------------------------------------------------------------------------ */

/* The edge graph of a finished 3D cell as darts (directed edges).  Each face
 * lists its vertices in one consistent rotational sense, so the dart u -> w
 * taken along face f has f on one fixed side; every edge gives two darts,
 * one in each of its two faces.  nxt: the next dart along the same face;
 * prv: the previous one; rev: the opposite dart. */
typedef struct {
    int nd, nv;
    int tail[2 * VO_MAXV], head[2 * VO_MAXV];
    int nxt[2 * VO_MAXV], prv[2 * VO_MAXV], rev[2 * VO_MAXV];
} odarts;

static int cell_darts(const ocell *c, odarts *g)
{
    int nd = 0;
    for (int f = 0; f < c->nf; f++) {
        int n = c->fn[f];
        if (nd + n > 2 * VO_MAXV) return VO_ERR_CAP;
        for (int k = 0; k < n; k++) {
            g->tail[nd + k] = c->fv[f][k];
            g->head[nd + k] = c->fv[f][(k + 1) % n];
            g->nxt[nd + k] = nd + (k + 1) % n;
            g->prv[nd + k] = nd + (k + n - 1) % n;
        }
        nd += n;
    }
    g->nd = nd;
    g->nv = c->nv;
    for (int d = 0; d < nd; d++) {
        g->rev[d] = -1;
        for (int e = 0; e < nd; e++)
            if (g->tail[e] == g->head[d] && g->head[e] == g->tail[d]) { g->rev[d] = e; break; }
        if (g->rev[d] < 0) return VO_ERR_TOPO;
    }
    return VO_OK;
}

/* The outgoing dart after dart d (which leaves vertex v) in the rotation
 * around v: orientation 0 turns one way, orientation 1 the other.  With f
 * the face of d, the dart that enters v along f is prv(d), and the next
 * dart around v is the one leaving v along the other face of that edge. */
static int rot(const odarts *g, int d, int o)
{
    return o == 0 ? g->nxt[g->rev[d]] : g->rev[g->prv[d]];
}

/* One Weinberg walk from dart d0 in orientation o: every dart once.  The
 * walk's vertices are numbered 1, 2, ... in the order they are first
 * reached, and the code is the number of the vertex each dart leaves, in
 * the order the darts are taken (2E numbers).  The rules: on reaching a
 * vertex for the first time, leave by the next dart in the rotation after
 * the one just arrived on (reversed); on reaching a vertex seen before,
 * go back along the same edge unless that was already done; otherwise
 * leave by the first unused dart in the rotation after the reversed
 * arrival dart. */
/* Test-only planted mistakes (vo_set_wb_rule): 0 = Weinberg's rules; 1 =
 * the other rotational sense at a vertex seen before; 2 = no return along the
 * arrival edge; 3 = the code lists the vertex each dart enters instead of the
 * one it leaves.  The pins of the hand-derived codes must fail under each. */
static int g_wb_rule = 0;

void vo_set_wb_rule(int rule)
{
    g_wb_rule = rule;
}

static int weinberg_walk(const odarts *g, int d0, int o, uint8_t *code, int *lab, unsigned char *used)
{
    for (int v = 0; v < g->nv; v++) lab[v] = 0;
    for (int d = 0; d < g->nd; d++) used[d] = 0;
    int nl = 1, d = d0;
    lab[g->tail[d0]] = 1;
    for (int k = 0; k < g->nd; k++) {
        used[d] = 1;
        const int v = g->head[d], r = g->rev[d], first = lab[v] == 0;
        if (first) lab[v] = ++nl;
        code[k] = (uint8_t)(g_wb_rule == 3 ? lab[v] : lab[g->tail[d]]);
        if (k == g->nd - 1) break;
        if (first) {
            d = rot(g, r, o);
        } else if (!used[r] && g_wb_rule != 2) {
            d = r;
        } else {
            const int so = g_wb_rule == 1 ? 1 - o : o;
            int e = rot(g, r, so), guard = 0;
            while (used[e]) {
                e = rot(g, e, so);
                if (++guard > g->nd) return VO_ERR_TOPO;
            }
            d = e;
        }
    }
    return VO_OK;
}

/* The cell's Weinberg code: the lexicographically smallest walk code over
 * every starting dart and both orientations.  sym = the number of (dart,
 * orientation) pairs that give it (the order of the graph's symmetry
 * group); chiral = 1 when only one orientation gives it.  Returns the code
 * length 2E, or a negative error. */
static int weinberg3(const ocell *c, uint8_t *best, int maxlen, int32_t *sym, int32_t *chiral)
{
    odarts *g = (odarts *)malloc(sizeof(odarts));
    uint8_t *code = (uint8_t *)malloc(2 * VO_MAXV);
    int *lab = (int *)malloc(VO_MAXV * sizeof(int));
    unsigned char *used = (unsigned char *)malloc(2 * VO_MAXV);
    int rc = (g && code && lab && used) ? cell_darts(c, g) : VO_ERR_MEM;
    if (rc == VO_OK && (g->nd > maxlen || c->nv > 255)) rc = VO_ERR_CAP;
    int count = 0, omask = 0;
    for (int o = 0; o < 2 && rc == VO_OK; o++)
        for (int d0 = 0; d0 < g->nd && rc == VO_OK; d0++) {
            rc = weinberg_walk(g, d0, o, code, lab, used);
            if (rc != VO_OK) break;
            int cmp = count == 0 ? -1 : memcmp(code, best, (size_t)g->nd);
            if (cmp < 0) {
                memcpy(best, code, (size_t)g->nd);
                count = 1;
                omask = 1 << o;
            } else if (cmp == 0) {
                count++;
                omask |= 1 << o;
            }
        }
    if (rc == VO_OK) {
        *sym = count;
        *chiral = omask != 3;
        rc = g->nd;
    }
    free(g);
    free(code);
    free(lab);
    free(used);
    return rc;
}

/* Weinberg codes of the 3D cells of the particles idx[0..m): code t in
 * codes[t * maxlen ...], its length 2E in len[t] (0 for an empty cell),
 * sym[t], chiral[t].  Returns 0 or the first per-cell error code. */
int vo_weinberg(const vo_handle *H, const int64_t *idx, int64_t m, int nthreads, double tau, uint8_t *codes,
                int maxlen, int32_t *len, int32_t *sym, int32_t *chiral)
{
    if (!H || H->dim != 3 || (m > 0 && (!idx || !codes || !len || !sym || !chiral))) return VO_ERR_ARG;
    int err = 0;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel num_threads(nthreads)
#endif
    {
        ocell *c = (ocell *)malloc(sizeof(ocell));
        int64_t ccap = 256;
        ocand *cbuf = (ocand *)malloc((size_t)ccap * sizeof(ocand));
        if (c) memset(c->cnt, 0, sizeof(c->cnt));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t t = 0; t < m; t++) {
            len[t] = sym[t] = chiral[t] = 0;
            if (!c || !cbuf) { err = VO_ERR_MEM; continue; }
            c->tau = tau;
            c->audit = 0;
            int64_t i = idx[t];
            int rc = (i < 0 || i >= H->n) ? VO_ERR_ARG : compute_cell(H, i, c, &cbuf, &ccap);
            if (rc == VO_EMPTY) continue;
            if (rc == VO_OK) rc = weinberg3(c, codes + (size_t)t * maxlen, maxlen, &sym[t], &chiral[t]);
            if (rc < 0) {
#ifdef _OPENMP
#pragma omp critical
#endif
                if (!err) err = rc;
                continue;
            }
            len[t] = rc;
        }
        free(c);
        free(cbuf);
    }
    return err;
}

/* Faces of the 3D cell of particle i, for geometry checks in tests: for
 * face f, its plane's label and image code and its vertex count, and its
 * vertex ids (indices into vo_cell_vertices' list) in one rotational sense,
 * packed one face after another in `ring`.  Returns the face count (up to
 * maxf faces and maxring ids written), or a negative error. */
int vo_cell_faces(const vo_handle *H, int64_t i, double tau, int32_t *lab, int32_t *shift, int32_t *len,
                  int32_t *ring, int maxf, int maxring)
{
    if (!H || H->dim != 3 || i < 0 || i >= H->n) return VO_ERR_ARG;
    ocell *c = (ocell *)calloc(1, sizeof(ocell));
    int64_t ccap = 256;
    ocand *cbuf = (ocand *)malloc((size_t)ccap * sizeof(ocand));
    if (!c || !cbuf) { free(c); free(cbuf); return VO_ERR_MEM; }
    c->tau = tau;
    int rc = compute_cell(H, i, c, &cbuf, &ccap);
    if (rc == VO_EMPTY) rc = 0;
    else if (rc == VO_OK) {
        int at = 0;
        for (int f = 0; f < c->nf; f++) {
            if (f < maxf) {
                const oplane *pl = &c->pl[c->fplane[f]];
                lab[f] = pl->label;
                shift[f] = pl->shift;
                len[f] = c->fn[f];
            }
            for (int k = 0; k < c->fn[f]; k++, at++)
                if (f < maxf && at < maxring) ring[at] = c->fv[f][k];
        }
        rc = c->nf;
    }
    free(c);
    free(cbuf);
    return rc;
}

/* Undirected edges of the 3D cell of particle i as vertex pairs (u < w),
 * for graph checks in tests.  Returns the edge count (up to maxe written),
 * or a negative error. */
int vo_cell_edges(const vo_handle *H, int64_t i, double tau, int32_t *out, int maxe)
{
    if (!H || H->dim != 3 || i < 0 || i >= H->n) return VO_ERR_ARG;
    ocell *c = (ocell *)calloc(1, sizeof(ocell));
    int64_t ccap = 256;
    ocand *cbuf = (ocand *)malloc((size_t)ccap * sizeof(ocand));
    if (!c || !cbuf) { free(c); free(cbuf); return VO_ERR_MEM; }
    c->tau = tau;
    int rc = compute_cell(H, i, c, &cbuf, &ccap);
    if (rc == VO_EMPTY) rc = 0;
    else if (rc == VO_OK) {
        int ne = 0;
        for (int f = 0; f < c->nf; f++)
            for (int k = 0; k < c->fn[f]; k++) {
                int u = c->fv[f][k], w = c->fv[f][(k + 1) % c->fn[f]];
                if (u < w) {
                    if (ne < maxe) {
                        out[2 * ne] = u;
                        out[2 * ne + 1] = w;
                    }
                    ne++;
                }
            }
        rc = ne;
    }
    free(c);
    free(cbuf);
    return rc;
}
