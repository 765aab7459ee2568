// cell3d_group.hip -- the 3D cell kernel with several cells per wavefront and
// synchronised cuts.
//
// The method is the one of cell3d.hip: a cell is a set of dual triangles
// (one per vertex, three plane ids each) with an edge table in LDS; a
// candidate plane (the bisector of Eq. 3) is tested against every vertex
// with a ballot, and a cut replaces the conflict region by a fan of new
// triangles around the new plane.  The candidates come from the grid blocks
// in nearest-first order (section 2.1.3) and the search ends by the radius
// bound (section 2.1.3).  Two kinds of cell are left to the spill pass, the
// one-cell kernel of cell3d.hip: a cell whose search radius still reaches
// four block sides after its nearest blocks, or whose search would run past
// the precomputed block offsets (an extended cell, section 3.1), whose 64
// lanes run the block bound's shell search there; and a cell with a side
// decision (a vertex test or an edge's degeneracy test) in the band of the
// exact predicate, which decides it there.  The exact expansions stay out
// of this kernel: they would hold registers that the cell state needs, for
// about one side test in 10^8 on random input.
//
// Mapping.  A cell is owned by a group of G lanes (G = 16 or 32, so 64/G
// cells share a wavefront).  Each group runs a small state machine:
//
//   NEW -> GATHER -> BATCH -> TEST -> (CUT -> TEST)* -> ... -> STATS -> NEW
//
// GATHER reads the particle counts of up to G blocks, BATCH loads up to G
// particles, keeps those inside the radius bound and sorts them by distance
// (a rank count over the group's keys), TEST takes the sorted candidates one
// at a time, and a conflict parks the group in CUT.  The cut itself (the
// costliest step) runs only once no group of the wave can advance without
// one, so that the cuts of the wave's cells run in the same instructions
// instead of one after another.  STATS (volume, centroid, counts, face
// orders, neighbours) is deferred in the same way.
//
// All masks are the group's bit fields (32 bits), reductions are DPP row
// operations plus one swizzle across the two rows of a 32-lane group.  Each
// group is one workgroup's slice of LDS; LDS hand-offs use a workgroup-scope
// fence (one wave per workgroup).
#include "cell_common.h"

namespace vc {

namespace {

template <int G>
struct Gw {
    static constexpr int CPW = 64 / G;
    static constexpr uint32_t FULL = G >= 32 ? 0xffffffffu : ((1u << G) - 1u);
};

enum { PH_NEW, PH_GATHER, PH_BATCH, PH_TEST, PH_CUT, PH_STATS, PH_DONE };

__device__ __forceinline__ void lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// the group's bits of a wave ballot
template <int G>
__device__ __forceinline__ uint32_t gbal(bool p, int gb)
{
    unsigned long long b = __builtin_amdgcn_ballot_w64(p);
    if (G == 32) return gb ? (uint32_t)(b >> 32) : (uint32_t)b;
    return (uint32_t)(b >> gb) & Gw<G>::FULL;
}

// lane i of a 32-lane group exchanges with lane i ^ 16
__device__ __forceinline__ int swz16(int v)
{
    return __builtin_amdgcn_ds_swizzle(v, 0x401f);
}

template <int G>
__device__ __forceinline__ uint32_t gmax_u32(uint32_t v)
{
    int x = (int)v;
    x = (int)max((uint32_t)x, (uint32_t)dpp_i32<DPP_QUAD_1032, 0xf>(x, x));
    x = (int)max((uint32_t)x, (uint32_t)dpp_i32<DPP_QUAD_2301, 0xf>(x, x));
    x = (int)max((uint32_t)x, (uint32_t)dpp_i32<DPP_ROW_HALF_MIRROR, 0xf>(x, x));
    x = (int)max((uint32_t)x, (uint32_t)dpp_i32<DPP_ROW_MIRROR, 0xf>(x, x));
    if (G >= 32) x = (int)max((uint32_t)x, (uint32_t)swz16(x));
    return (uint32_t)x;
}

template <int G>
__device__ __forceinline__ double gmax_f64(double v)
{
    v = fmax(v, dpp_f64<DPP_QUAD_1032, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_QUAD_2301, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_ROW_HALF_MIRROR, 0xf>(v, v));
    v = fmax(v, dpp_f64<DPP_ROW_MIRROR, 0xf>(v, v));
    if (G >= 32) {
        unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        unsigned lo = (unsigned)swz16((int)(unsigned)u), hi = (unsigned)swz16((int)(unsigned)(u >> 32));
        v = fmax(v, __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo));
    }
    return v;
}

template <int G>
__device__ __forceinline__ int gisum(int v)
{
    v = v + dpp_i32<DPP_QUAD_1032, 0xf>(0, v);
    v = v + dpp_i32<DPP_QUAD_2301, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_HALF_MIRROR, 0xf>(0, v);
    v = v + dpp_i32<DPP_ROW_MIRROR, 0xf>(0, v);
    if (G >= 32) v = v + swz16(v);
    return v;
}

// fixed combination order: the same sum on every run
template <int G>
__device__ __forceinline__ double gsum(double v)
{
    v = v + dpp_f64<DPP_QUAD_1032, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_QUAD_2301, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_ROW_HALF_MIRROR, 0xf>(0.0, v);
    v = v + dpp_f64<DPP_ROW_MIRROR, 0xf>(0.0, v);
    if (G >= 32) {
        unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        unsigned lo = (unsigned)swz16((int)(unsigned)u), hi = (unsigned)swz16((int)(unsigned)(u >> 32));
        double w = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
        // both rows add the same two partial sums in the same order
        v = (threadIdx.x & 16) ? w + v : v + w;
    }
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
    return v;
}

// exclusive prefix of small counts (< 2^BITS) inside the group, by ballots
template <int G, int BITS>
__device__ __forceinline__ int gballot_scan(int v, int gb, uint32_t below, int &total)
{
    int r = 0, t = 0;
#pragma unroll
    for (int b = 0; b < BITS; b++) {
        uint32_t m = gbal<G>((v >> b) & 1, gb);
        r += __popc(m & below) << b;
        t += __popc(m) << b;
    }
    total = t;
    return r;
}

// search state of a group that only the phase steps read (kept in LDS to
// leave registers for the side tests and cuts)
struct GState {
    double p[3];            // the particle
    int bc[3];              // its block
    int fl[3];              // reflection of the block offsets per axis (+1 or -1)
    int si, id;             // sorted index, input index
    double ri;              // the particle's radius (radical tessellation), else 0
    int cur;                // next offset index
    int gtot, gc0;          // candidates of the gather, next batch start
    int cell, cend;         // claimed range of the work queue
    int tcur;               // the tessellation whose record is in the group's Tess
    uint32_t cnt[DC_N];     // counters other than candidates and tests
};

// The group's LDS.  The radical instantiation has the same layout: its
// plane offsets already hold the radii, and the radii themselves fed only
// the exact predicate, which this kernel leaves to the one-cell kernel.
template <int G, int S, int MAXP, bool RAD>
struct SL {
    GState gs;
    Tess T;                 // the cell's tessellation
    double pq[MAXP][4];     // planes n.r = h (n = q for a bisector, h = |q|^2 / 2)
    int32_t plab[MAXP];
    uint8_t psh[MAXP];
    uint8_t pwall[MAXP];
    uint8_t etab[MAXP][MAXP];  // slot of the triangle holding directed edge a->b
    union alignas(16) {
        struct {               // the search
            double cq[G][6];   // the batch's candidates, nearest first: q, |q|^2, plane
                               // offset h, FP64 side-test band
            int32_t cid[G];
            int32_t cpre[G];   // the gather's blocks: candidates before, first particle, image code
            int32_t cbeg[G];
            uint16_t csh[G];   // the gather's blocks: image code | shifts + 2 in 3-bit fields << 7
            uint8_t ccode[G];
            uint16_t bedge[G * S + 8];
            union {
                uint32_t key[G];            // ranking keys (BATCH only)
                float cfb[G];               // then: the FP32 side-test bands (FP32 filter)
            } x;
        } w;
        struct {               // the statistics of the finished cell
            double pos[G * S][3];
            uint32_t tpl[G * S];
            int32_t lab[G * S];
            int32_t forder[MAXP];
            int32_t fref[MAXP];
            int32_t fo[kFoLen];
        } st;
    } u;
};

// one cell and its search state, held by a group (values are the same on
// every lane of the group, apart from the per-lane slots)
template <int S, bool F32>
struct SCell {
    uint32_t tp[S];              // plane ids a | b << 8 | c << 16
    double vx[S], vy[S], vz[S];  // vertex, relative to the particle
    float fx[S], fy[S], fz[S];
    uint32_t live[S];            // live slots (group bit fields)
    uint32_t conf[S];            // conflict slots of the pending cut
    uint32_t used;               // plane slots in use (at most 32)
    double lim, R;               // squared search radius, radius bound (upper bounds)
    int nlive;                   // live slots (vertices) of the cell
    int phase;
    int bn, bk;                  // candidates of the batch, next one
};

template <int MAXP>
__device__ __forceinline__ int free_plane(uint32_t used)
{
    static_assert(MAXP <= 32, "plane slots");
    constexpr uint32_t valid = MAXP >= 32 ? ~0u : ((1u << MAXP) - 1u);
    const uint32_t fr = ~used & valid;
    return fr ? __builtin_ctz(fr) : -1;
}

// Radius bound: the largest squared vertex norm, rounded up to 20 mantissa
// bits (the high word of the double plus one unit), so the group maximum is
// a 32-bit DPP reduction.  R2, R and the search radius are upper bounds, which is all the
// radius test and the error bands need.
template <int G, int S, bool F32>
__device__ __forceinline__ void update_radius(SCell<S, F32> &c, int gl, const CellArgs &A, double ri)
{
    uint32_t m = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        double x = c.vx[s] * c.vx[s] + c.vy[s] * c.vy[s] + c.vz[s] * c.vz[s];
        uint32_t hw = (uint32_t)(__builtin_bit_cast(unsigned long long, x) >> 32) + 1u;
        if ((c.live[s] >> gl) & 1) m = max(m, hw);
    }
    m = gmax_u32<G>(m);
    const double R2 = __builtin_bit_cast(double, (unsigned long long)m << 32);
    if (R2 > 1e-30 && R2 < 1e30)
        c.R = (double)__builtin_amdgcn_sqrtf((float)R2) * (1.0 + 0x1p-18);
    else
        c.R = sqrt(R2) * (1.0 + 0x1p-40);
    c.lim = search_lim(R2, c.R, A, ri);
}

template <int G, int S, int MAXP, bool F32, bool RAD>
__device__ __forceinline__ void cell_fail(const CellArgs &A, SL<G, S, MAXP, RAD> &sh, SCell<S, F32> &c, int st, int gl)
{
    const int id = sh.gs.id;
    if (A.fo)
        for (int k = gl; k < kFoLen; k += G) A.fo[(int64_t)id * kFoLen + k] = 0;
    if (gl == 0) {
        if (A.vol) A.vol[id] = __builtin_nan("");
        if (A.cen) A.cen[3 * (int64_t)id] = A.cen[3 * (int64_t)id + 1] = A.cen[3 * (int64_t)id + 2] = __builtin_nan("");
        if (A.nv) A.nv[id] = 0;
        if (A.ne) A.ne[id] = 0;
        if (A.nf) A.nf[id] = 0;
        if (A.wbl) A.wbl[id] = 0;
        if (st == ST_DUP) {
            A.status[id] = 3;
        } else {
            A.status[id] = 1;
            int pos = atomicAdd(A.spill_count, 1);
            A.spill_list[pos] = sh.gs.si;
        }
    }
    if (st != ST_DUP) sh.gs.cnt[DC_SPILL]++;
    c.phase = PH_NEW;
}

// ---- NEW: claim the next cell and set up the box (Eq. 1-2) ----
template <int G, int S, int MAXP, bool F32, bool RAD>
__device__ __forceinline__ void ph_new(const CellArgs &A, SL<G, S, MAXP, RAD> &sh, SCell<S, F32> &c, int ncell, int gl,
                                       int gb)
{
    if (sh.gs.cell >= sh.gs.cend) {
        int base = 0;
        if (gl == 0) base = atomicAdd(A.queue, A.chunk);
        base = __shfl(base, gb);
        sh.gs.cell = base;
        sh.gs.cend = min(base + A.chunk, ncell);
    }
    if (sh.gs.cell >= sh.gs.cend) {
        c.phase = PH_DONE;
        return;
    }
    const int si = A.cell_list ? A.cell_list[sh.gs.cell] : sh.gs.cell;
    sh.gs.cell++;
    const Particle me = A.part[si];
    sh.gs.si = si;
    sh.gs.id = me.id;
    sh.gs.ri = A.rad ? A.rad[si] : 0.0;
    sh.gs.p[0] = me.x;
    sh.gs.p[1] = me.y;
    sh.gs.p[2] = me.z;
    if (me.tess != sh.gs.tcur) {
        // cells come in block order, so the record changes once per
        // tessellation of a batch
        const int32_t *src = (const int32_t *)&A.tess[me.tess];
        int32_t *dst = (int32_t *)&sh.T;
        for (int k = gl; k < (int)(sizeof(Tess) / 4); k += G) dst[k] = src[k];
        lds_fence();
        sh.gs.tcur = me.tess;
    }
    lds_fence();
    const Grid &G3 = sh.T.G;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int k = block_coord(G3, sh.gs.p[d], d);
        sh.gs.bc[d] = k;
        sh.gs.fl[d] = offset_flip(G3, sh.gs.p[d], k, d);
    }
    if (gl < 6) {
        // face 2d + side of the box (Eq. 1-2, clipped as in section 3.1.3)
        const int d = gl >> 1, side = gl & 1;
        const double pd = d == 0 ? sh.gs.p[0] : (d == 1 ? sh.gs.p[1] : sh.gs.p[2]);
        const BoxSide b = box_side(sh.T, pd, d, side, sh.gs.id);
        sh.pwall[gl] = (uint8_t)b.wall;
        sh.plab[gl] = b.lab;
        sh.psh[gl] = b.code;
        sh.pq[gl][0] = d == 0 ? b.nd : 0.0;
        sh.pq[gl][1] = d == 1 ? b.nd : 0.0;
        sh.pq[gl][2] = d == 2 ? b.nd : 0.0;
        sh.pq[gl][3] = b.h;
    }
#pragma unroll
    for (int s = 0; s < S; s++) {
        c.tp[s] = 0;
        c.vx[s] = c.vy[s] = c.vz[s] = 0.0;
        c.fx[s] = c.fy[s] = c.fz[s] = 0.0f;
        c.live[s] = 0;
        c.conf[s] = 0;
    }
    c.live[0] = 0xffu;
    if (gl < 8) {
        int bx = gl & 1, by = (gl >> 1) & 1, bz = (gl >> 2) & 1;
        int X = bx, Y = 2 + by, Z = 4 + bz;
        int neg = 3 - bx - by - bz;
        c.tp[0] = (neg & 1) ? (X | (Z << 8) | (Y << 16)) : (X | (Y << 8) | (Z << 16));
        double e[3];
#pragma unroll
        for (int d = 0; d < 3; d++) {
            const int b = (gl >> d) & 1;
            const double o = box_side(sh.T, sh.gs.p[d], d, b, sh.gs.id).off;
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
            sh.etab[a][b] = (uint8_t)gl;
        }
    }
    c.used = 0x3fu;
    c.nlive = 8;
    lds_fence();
    update_radius<G, S, F32>(c, gl, A, sh.gs.ri);
    sh.gs.cur = 0;
    c.phase = PH_GATHER;
}

// ---- GATHER: particle counts of the next (up to) G blocks ----
template <int G, int S, int MAXP, bool F32, bool RAD>
__device__ __forceinline__ void ph_gather(const CellArgs &A, SL<G, S, MAXP, RAD> &sh, SCell<S, F32> &c, int gl, int gb,
                                          uint32_t *cnt)
{
    const Tess &T = sh.T;
    const Grid &G3 = T.G;
    const double lim = c.lim;
    int dd[3] = {0, 0, 0};
    bool v = false;
    if (sh.gs.cur >= A.noff) {
        // past the offset list: the shell search of the block bound is the
        // one-cell kernel's (the spill pass), as for the extended cells below
        c.phase = -ST_CAP;
        return;
    } else if (A.offs[sh.gs.cur].m * 0.25 * T.bsmin2 >= lim) {
        c.phase = PH_STATS;  // no block left in the offset list can hold a cutting particle
        return;
    } else if (sh.gs.cur >= G && lim > 16.0 * T.bsmin2) {
        // after the nearest blocks the search radius still reaches four
        // block sides, past most of the offset list: an extended cell
        // (section 3.1), left to the one-cell kernel of the spill pass,
        // which tests the list's blocks against the balls and takes 64
        // blocks of a shell per step
        c.phase = -ST_CAP;
        return;
    } else {
        int o = sh.gs.cur + gl;
        v = o < A.noff;
        Offset of = v ? A.offs[o] : Offset{0, 0, 0, 0};
        dd[0] = of.dx * sh.gs.fl[0];
        dd[1] = of.dy * sh.gs.fl[1];
        dd[2] = of.dz * sh.gs.fl[2];
        sh.gs.cur += G;
    }
    // the blocks: periodic wrap by whole periods (at most two each way), walls
    int bb[3], sv[3];
    bool ok = v;
    double d2b = 0.0;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        const int g = G3.g[d];
        int t = sh.gs.bc[d] + dd[d];
        int w = t, s = 0;
        if (G3.per[d]) {
            while (w < 0 && s > -3) {
                w += g;
                s--;
            }
            while (w >= g && s < 3) {
                w -= g;
                s++;
            }
            if (s > 2 || s < -2) ok = false;
        } else if (t < 0 || t >= g) {
            ok = false;
        }
        bb[d] = w;
        sv[d] = s;
        double blo = G3.lo[d] + t * G3.bs[d];
        double e = fmax(0.0, fmax(blo - sh.gs.p[d], sh.gs.p[d] - (blo + G3.bs[d])));
        d2b += e * e;
    }
    if (d2b >= lim) ok = false;
    int cntb = 0, beg = 0;
    if (ok) {
        int blk = T.bbase + bb[0] + G3.g[0] * (bb[1] + G3.g[1] * bb[2]);
        beg = A.start[blk];
        cntb = A.start[blk + 1] - beg;
    }
    sh.gs.cnt[DC_BLOCKS] += __popc(gbal<G>(ok, gb));
    int incl = gscan_incl<G>(cntb);
    int total = __shfl(incl, gb + G - 1);
    sh.gs.cnt[DC_LOADED] += total;
    if (total == 0) return;  // stay in GATHER: next blocks
    sh.u.w.cpre[gl] = incl - cntb;
    sh.u.w.cbeg[gl] = beg;
    sh.u.w.csh[gl] = (uint16_t)((25 * (sv[2] + 2) + 5 * (sv[1] + 2) + (sv[0] + 2)) |
                                (((sv[0] + 2) | ((sv[1] + 2) << 3) | ((sv[2] + 2) << 6)) << 7));
    lds_fence();
    sh.gs.gtot = total;
    sh.gs.gc0 = 0;
    c.phase = PH_BATCH;
}

// ---- BATCH: the next G particles of the gather, sorted by distance ----
template <int G, int S, int MAXP, bool F32, bool RAD>
__device__ __forceinline__ void ph_batch(const CellArgs &A, SL<G, S, MAXP, RAD> &sh, SCell<S, F32> &c, int gl, int gb,
                                         uint32_t below)
{
    if (sh.gs.gc0 >= sh.gs.gtot) {
        c.phase = PH_GATHER;
        return;
    }
    const Grid &G3 = sh.T.G;
    const int ci = sh.gs.gc0 + gl;
    uint32_t key = ~0u;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, d2 = 0.0, h = 0.0, rj = 0.0;
    int pid = 0, code = 0;
    if (ci < sh.gs.gtot) {
        int lo = 0, hi = G - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (sh.u.w.cpre[mid] <= ci) lo = mid;
            else hi = mid - 1;
        }
        int idx = sh.u.w.cbeg[lo] + (ci - sh.u.w.cpre[lo]);
        const int cs = sh.u.w.csh[lo];
        code = cs & 0x7f;
        const int s0 = ((cs >> 7) & 7) - 2, s1 = ((cs >> 10) & 7) - 2, s2 = ((cs >> 13) & 7) - 2;
        Particle q = A.part[idx];
        a0 = q.x - sh.gs.p[0];
        a1 = q.y - sh.gs.p[1];
        a2 = q.z - sh.gs.p[2];
        if (s0) a0 = a0 + s0 * G3.L[0];
        if (s1) a1 = a1 + s1 * G3.L[1];
        if (s2) a2 = a2 + s2 * G3.L[2];
        d2 = a0 * a0 + a1 * a1 + a2 * a2;
        pid = q.id;
        if (A.rad) {
            // radical plane (section 2.1.1): |x|^2 - ri^2 <= |x - q|^2 - rj^2
            const double ri = sh.gs.ri;
            rj = A.rad[idx];
            h = 0.5 * (d2 + radical_shift(ri, rj));
        } else {
            h = 0.5 * d2;
        }
        bool self = (idx == sh.gs.si) && code == kNoShift;
        // unique 32-bit keys: the high word of the distance (its exponent and
        // 20 mantissa bits) with the low five bits replaced by the lane, so
        // candidates closer than 2^-15 relative may swap; TEST ends a batch
        // only past that resolution
        if (!self && d2 < c.lim)
            key = ((uint32_t)(__builtin_bit_cast(unsigned long long, d2) >> 32) & ~31u) | (uint32_t)gl;
    }
    // the valid keys, compacted; each counts the smaller ones
    const bool valid = key != ~0u;
    const uint32_t gv = gbal<G>(valid, gb);
    const int bn = __popc(gv);
    if (valid) sh.u.w.x.key[__popc(gv & below)] = key;
    lds_fence();
    int rank = 0;
    if (valid && bn > 1)
        for (int j = 0; j < bn; j++) rank += sh.u.w.x.key[j] < key;
    if (valid) {
        // side-test bands with the radius bound of now: R only shrinks, so
        // a band taken now stays wide enough for every later test
        const double band = A.tau * ((fabs(a0) + fabs(a1) + fabs(a2)) * c.R + fabs(h));
        sh.u.w.cq[rank][0] = a0;
        sh.u.w.cq[rank][1] = a1;
        sh.u.w.cq[rank][2] = a2;
        sh.u.w.cq[rank][3] = d2;
        sh.u.w.cq[rank][4] = h;
        sh.u.w.cq[rank][5] = band;
        if (F32) {
            const float g0 = (float)a0, g1 = (float)a1, g2 = (float)a2, gh = (float)h;
            sh.u.w.x.cfb[rank] =
                A.tau32 * ((fabsf(g0) + fabsf(g1) + fabsf(g2)) * ((float)c.R * 1.0000001f) + fabsf(gh));
        }
        sh.u.w.cid[rank] = pid;
        sh.u.w.ccode[rank] = (uint8_t)code;
    }
    lds_fence();
    sh.gs.gc0 += G;
    c.bn = bn;
    c.bk = 0;
    // a candidate at distance zero (a coincident particle) sorts first
    if (gbal<G>(valid && d2 == 0.0, gb)) c.phase = -ST_DUP;
    else if (bn) c.phase = PH_TEST;
}

// ---- TEST: side of every vertex against the next candidate ----
// Side masks are whole-wave compares (only the testing groups' lanes are
// active, and a dead slot's lane is masked by the live mask), so the
// per-slot work is three FMAs and two compares; a group's bits are taken
// out only when it has a conflict and parks in CUT.  The candidate's
// offset and bands were set by BATCH.
template <int G, int S, int MAXP, bool F32, bool RAD>
__device__ __forceinline__ void ph_test(const CellArgs &A, SL<G, S, MAXP, RAD> &sh, SCell<S, F32> &c, uint32_t *cnt,
                                        int gl, int gb)
{
    if (c.bk >= c.bn) {
        c.phase = PH_BATCH;
        return;
    }
    const int k = c.bk;
    const double q0 = sh.u.w.cq[k][0], q1 = sh.u.w.cq[k][1], q2 = sh.u.w.cq[k][2], d2 = sh.u.w.cq[k][3];
    const double h = sh.u.w.cq[k][4], band = sh.u.w.cq[k][5];
    // issue the candidate's three LDS reads together, ahead of the range test
    __asm__ volatile("" ::: "memory");
    if (d2 * (1.0 - 0x1p-14) >= c.lim) {
        // sorted to within 2^-15: the rest of the batch is beyond the
        // radius bound too (a candidate just beyond it is tested and cuts
        // nothing)
        c.phase = PH_BATCH;
        return;
    }
    cnt[0]++;
    unsigned long long wc[S], wi[S];
    int nre = 0;
    if (F32) {
        const float g0 = (float)q0, g1 = (float)q1, g2 = (float)q2, gh = (float)h, band32 = sh.u.w.x.cfb[k];
        unsigned long long wu[S], wun = 0;
#pragma unroll
        for (int s = 0; s < S; s++) {
            const unsigned long long lv = __builtin_amdgcn_ballot_w64((c.live[s] >> gl) & 1);
            wc[s] = wu[s] = wi[s] = 0;
            if (!lv) continue;
            const float sv = fmaf(g0, c.fx[s], fmaf(g1, c.fy[s], fmaf(g2, c.fz[s], -gh)));
            wc[s] = lv & __builtin_amdgcn_fcmpf(sv, band32, 2);             // sv > band
            wu[s] = lv & __builtin_amdgcn_fcmpf(fabsf(sv), band32, 13);     // |sv| <= band or NaN
            wun |= wu[s];
        }
        if (wun) {
#pragma unroll
            for (int s = 0; s < S; s++) {
                if (!wu[s]) continue;
                const double sv = fma(q0, c.vx[s], fma(q1, c.vy[s], fma(q2, c.vz[s], -h)));
                wc[s] |= wu[s] & __builtin_amdgcn_fcmp(sv, band, 2);
                wi[s] = wu[s] & __builtin_amdgcn_fcmp(fabs(sv), band, 13);
                nre += __popc((uint32_t)(wu[s] >> gb) & Gw<G>::FULL);
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < S; s++) {
            const unsigned long long lv = __builtin_amdgcn_ballot_w64((c.live[s] >> gl) & 1);
            wc[s] = wi[s] = 0;
            if (!lv) continue;
            const double sv = fma(q0, c.vx[s], fma(q1, c.vy[s], fma(q2, c.vz[s], -h)));
            wc[s] = lv & __builtin_amdgcn_fcmp(sv, band, 2);         // sv > band
            wi[s] = lv & __builtin_amdgcn_fcmp(fabs(sv), band, 13);  // |sv| <= band or NaN
        }
    }
    // an in-band vertex needs the exact predicate: the cell is left to the
    // one-cell kernel of the spill pass, which decides it exactly; the tests
    // and rechecks of this step are not counted (that kernel counts its own)
    unsigned long long wib = 0;
#pragma unroll
    for (int s = 0; s < S; s++) wib |= wi[s];
    if ((uint32_t)(wib >> gb) & Gw<G>::FULL) {
        c.phase = -ST_CAP;
        return;
    }
    cnt[1] += c.nlive;
    if (F32) sh.gs.cnt[DC_RECHECK] += nre;
    unsigned long long wany = 0;
#pragma unroll
    for (int s = 0; s < S; s++) wany |= wc[s];
    if ((uint32_t)(wany >> gb) & Gw<G>::FULL) {
#pragma unroll
        for (int s = 0; s < S; s++) c.conf[s] = (uint32_t)(wc[s] >> gb) & Gw<G>::FULL;
        if (A.rad) {
            // a radical plane can leave no vertex strictly inside: the cell
            // is empty (a Voronoi cell always keeps its particle inside)
            uint32_t inside = 0;
#pragma unroll
            for (int s = 0; s < S; s++) inside |= c.live[s] & ~c.conf[s];
            if (!inside) {
#pragma unroll
                for (int s = 0; s < S; s++) {
                    c.live[s] = 0;
                    c.conf[s] = 0;
                }
                c.nlive = 0;
                c.phase = PH_STATS;
                return;
            }
        }
        c.phase = PH_CUT;
    } else {
        c.bk++;
    }
}

// ---- CUT: remove the conflict region, fan new triangles around the plane ----
template <int G, int S, int MAXP, bool F32, bool RAD>
__device__ __forceinline__ void ph_cut(const CellArgs &A, SL<G, S, MAXP, RAD> &sh, SCell<S, F32> &c, uint32_t *cnt,
                                       int gl, int gb, uint32_t below)
{
    const int k = c.bk;
    int p = free_plane<MAXP>(c.used);
    if (p < 0) {
        uint32_t u = 0;
#pragma unroll
        for (int s = 0; s < S; s++)
            if ((c.live[s] >> gl) & 1)
#pragma unroll
                for (int j = 0; j < 3; j++) u |= 1u << ((c.tp[s] >> (8 * j)) & 0xff);
        // group OR of the plane masks
#pragma unroll
        for (int sh_ = 1; sh_ < G; sh_ <<= 1) u |= (uint32_t)__shfl_xor((int)u, sh_);
        c.used = u;
        p = free_plane<MAXP>(c.used);
        if (p < 0) {
            c.phase = -ST_CAP;
            return;
        }
    }
    // boundary edges of the conflict region: conflict triangle edges whose
    // twin triangle is kept
    uint32_t bfl = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        if ((c.conf[s] >> gl) & 1) {
            uint32_t t3 = c.tp[s];
#pragma unroll
            for (int j = 0; j < 3; j++) {
                int a = (t3 >> (8 * j)) & 0xff, b = (t3 >> (8 * ((j + 1) % 3))) & 0xff;
                int tw = sh.etab[b][a] & (G * S - 1);
                uint32_t cw = 0;
#pragma unroll
                for (int r = 0; r < S; r++)
                    if (tw / G == r) cw = c.conf[r];
                if (!((cw >> (tw % G)) & 1)) bfl |= 1u << (s * 3 + j);
            }
        }
    }
    int nb = __popc(bfl);
    int m;
    int o = gballot_scan<G, (S <= 2 ? 3 : 4)>(nb, gb, below, m);
    int nfree = 0;
#pragma unroll
    for (int s = 0; s < S; s++) nfree += __popc(~c.live[s] | c.conf[s]);
    if (G < 32) nfree -= S * (32 - G);
    if (m > nfree || m > G * S + 8) {
        c.phase = -ST_CAP;
        return;
    }
    if (A.vcap > 0) {
        int keep = 0;
#pragma unroll
        for (int s = 0; s < S; s++) keep += __popc(c.live[s] & ~c.conf[s]);
        if (keep + m > A.vcap) {
            c.phase = -ST_CAP;
            return;
        }
    }
#pragma unroll
    for (int s = 0; s < S; s++) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            if ((bfl >> (s * 3 + j)) & 1) {
                uint32_t t3 = c.tp[s];
                int a = (t3 >> (8 * j)) & 0xff, b = (t3 >> (8 * ((j + 1) % 3))) & 0xff;
                sh.u.w.bedge[o++] = (uint16_t)(a | (b << 8));
            }
        }
    }
    if (gl == 0) {
        sh.pq[p][0] = sh.u.w.cq[k][0];
        sh.pq[p][1] = sh.u.w.cq[k][1];
        sh.pq[p][2] = sh.u.w.cq[k][2];
        sh.pq[p][3] = sh.u.w.cq[k][4];
        sh.plab[p] = sh.u.w.cid[k];
        sh.psh[p] = sh.u.w.ccode[k];
        sh.pwall[p] = 0;
    }
    lds_fence();
    // free slots in slot order take the new triangles (a, b, p) by rank
    int rk[S];
    bool take[S];
    int before = 0;
#pragma unroll
    for (int s = 0; s < S; s++) {
        uint32_t fr = (~c.live[s] | c.conf[s]) & Gw<G>::FULL;
        rk[s] = before + __popc(fr & below);
        take[s] = ((fr >> gl) & 1) && rk[s] < m;
        before += __popc(fr);
    }
    // each lane that takes a new triangle (a, b, p) computes its vertex
#pragma unroll
    for (int s = 0; s < S; s++) {
        if (take[s]) {
            uint16_t e = sh.u.w.bedge[rk[s]];
            int a = e & 0xff, b = e >> 8;
            double x, y, z;
            cramer(sh.pq[a], sh.pq[b], sh.pq[p], x, y, z);
            c.tp[s] = (uint32_t)a | ((uint32_t)b << 8) | ((uint32_t)p << 16);
            c.vx[s] = x;
            c.vy[s] = y;
            c.vz[s] = z;
            if (F32) {
                c.fx[s] = (float)x;
                c.fy[s] = (float)y;
                c.fz[s] = (float)z;
            }
            uint8_t t = (uint8_t)(s * G + gl);
            sh.etab[a][b] = t;
            sh.etab[b][p] = t;
            sh.etab[p][a] = t;
        }
    }
    lds_fence();
#pragma unroll
    for (int s = 0; s < S; s++) {
        c.live[s] = (c.live[s] & ~c.conf[s]) | gbal<G>(take[s], gb);
        c.conf[s] = 0;
    }
    c.used |= 1u << p;
    int nl = 0;
#pragma unroll
    for (int s = 0; s < S; s++) nl += __popc(c.live[s]);
    c.nlive = nl;
    update_radius<G, S, F32>(c, gl, A, sh.gs.ri);
    sh.gs.cnt[DC_CUTS]++;
    sh.gs.cnt[DC_NEWV] += m;
    c.bk++;
    c.phase = c.lim < 1e300 ? PH_TEST : -ST_CAP;
}

// ---- STATS: volume, centroid, V/E/F, face orders, neighbours ----
template <int G, int S, int MAXP, bool F32, bool RAD>
__device__ __forceinline__ void ph_stats(const CellArgs &A, SL<G, S, MAXP, RAD> &sh, SCell<S, F32> &c, uint32_t *cnt,
                                         int gl, int gb, uint32_t below)
{
    const int id = sh.gs.id;
    if (c.nlive == 0) {
        // an empty radical cell: zero volume, no vertices or faces
        if (gl == 0) {
            if (A.vol) A.vol[id] = 0.0;
            if (A.cen) A.cen[3 * (int64_t)id] = A.cen[3 * (int64_t)id + 1] = A.cen[3 * (int64_t)id + 2] = 0.0;
            if (A.nv) A.nv[id] = 0;
            if (A.ne) A.ne[id] = 0;
            if (A.nf) A.nf[id] = 0;
            if (A.wbl) A.wbl[id] = 0;
            A.status[id] = (uint8_t)ST_EMPTY;
        }
        if (A.fo)
            for (int k = gl; k < kFoLen; k += G) A.fo[(int64_t)id * kFoLen + k] = 0;
        c.phase = PH_NEW;
        return;
    }
    lds_fence();
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
        sh.u.st.forder[k] = 0;
        sh.u.st.fref[k] = 0x7fffffff;
    }
    for (int k = gl; k < kFoLen; k += G) sh.u.st.fo[k] = 0;
    lds_fence();
    for (int t = gl; t < S * G; t += G) {
        uint32_t t3 = sh.u.st.tpl[t];
        if (t3 == 0xffffffffu) continue;
        for (int j = 0; j < 3; j++) atomicMin(&sh.u.st.fref[(t3 >> (8 * j)) & 0xff], t);
    }
    lds_fence();
    // fan apex: the particle when it lies strictly inside the cell (every
    // face offset h > 0, always so for a Voronoi cell), else one vertex
    double o0 = 0.0, o1 = 0.0, o2 = 0.0;
    if (A.rad) {
        bool in = true;
#pragma unroll
        for (int s = 0; s < S; s++)
            if ((c.live[s] >> gl) & 1)
#pragma unroll
                for (int j = 0; j < 3; j++) in = in && sh.pq[(c.tp[s] >> (8 * j)) & 0xff][3] > 0.0;
        if (gbal<G>(!in, gb)) {
            int t0 = 0;
#pragma unroll
            for (int s = S - 1; s >= 0; s--)
                if (c.live[s]) t0 = s * G + __builtin_ctz(c.live[s]);
            o0 = sh.u.st.pos[t0][0];
            o1 = sh.u.st.pos[t0][1];
            o2 = sh.u.st.pos[t0][2];
        }
    }
    // one pass over the edges (a, b) of every live triangle: the edge's
    // degeneracy test and the face orders and fan terms that use it.  A
    // vertex whose opposite vertex across an edge lies on the vertex's
    // fourth plane is degenerate: the edge has zero length; a side clearly
    // inside decides it here, an in-band one is left to the exact
    // predicate of the one-cell kernel.  A fan
    // tetrahedron's volume is zero when its edge has zero length, so the
    // volume and moment sums take every edge; the face-order count skips
    // zero-length edges.
    uint32_t ib = 0;
    double v6 = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int j = 0; j < 3 * S; j++) {
        int t = (j / 3) * G + gl, k = j % 3;
        uint32_t t3 = sh.u.st.tpl[t];
        if (t3 == 0xffffffffu) continue;
        int a = (t3 >> (8 * k)) & 0xff, b = (t3 >> (8 * ((k + 1) % 3))) & 0xff;
        const int tw = sh.etab[b][a] & (G * S - 1);
        uint32_t w3 = sh.u.st.tpl[tw];
        int d = (int)(w3 & 0xff) + (int)((w3 >> 8) & 0xff) + (int)((w3 >> 16) & 0xff) - a - b;
        d = min(max(d, 0), MAXP - 1);
        const double *nd = sh.pq[d];
        const double *v0 = sh.u.st.pos[t];
        double sd = nd[0] * v0[0] + nd[1] * v0[1] + nd[2] * v0[2] - nd[3];
        double bd = A.tau * ((fabs(nd[0]) + fabs(nd[1]) + fabs(nd[2])) * c.R + fabs(nd[3]));
        if (!(sd < -bd)) ib |= 1u << j;
        else atomicAdd(&sh.u.st.forder[a], 1);
        const double *r0 = sh.u.st.pos[sh.u.st.fref[a]];
        const double *w0 = sh.u.st.pos[tw];
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
    if (gbal<G>(ib != 0, gb)) {
        // an edge whose length is in band: the exact predicate decides it
        // in the one-cell kernel of the spill pass (nothing of the cell has
        // been written yet)
        lds_fence();
        c.phase = -ST_CAP;
        return;
    }
    // no edge has zero length: every triangle is a vertex of its own
    int nvert = 0;
#pragma unroll
    for (int s = 0; s < S; s++) nvert += __popc(c.live[s]);
    lds_fence();
    int rk = 0, sumord = 0;
    bool foover = false;
    for (int k0 = 0; k0 < MAXP; k0 += G) {
        int k = k0 + gl;
        int ord = k < MAXP ? sh.u.st.forder[k] : 0;
        bool real = ord >= 3;
        uint32_t rb = gbal<G>(real, gb);
        int rank = rk + __popc(rb & below);
        if (real) {
            if (ord < kFoLen) atomicAdd(&sh.u.st.fo[ord], 1);
            if ((A.mask & (16 | 32)) && A.nbr && rank < kMaxNbr) {
                A.nbr[(int64_t)id * kMaxNbr + rank] = sh.plab[k];
                A.nsh[(int64_t)id * kMaxNbr + rank] = sh.psh[k];
            }
        }
        rk += __popc(rb);
        sumord += gisum<G>(real ? ord : 0);
        foover = foover || gbal<G>(real && ord >= kFoLen, gb) != 0u;
    }
    const int nface = rk;
    const double vol6 = gsum<G>(v6);
    const double M0 = gsum<G>(m0), M1 = gsum<G>(m1), M2 = gsum<G>(m2);
    lds_fence();
    if (nface > kMaxNbr) {
        cell_fail<G, S, MAXP, F32, RAD>(A, sh, c, ST_CAP, gl);
        return;
    }
    int wl = 0;
    if (A.wbg) {
        // the vertex positions are no longer needed: their LDS holds the
        // record's scratch (zero-length edge bits, vertex numbers, degrees)
        uint8_t *wsc = reinterpret_cast<uint8_t *>(&sh.u.st.pos[0][0]);
        wl = wb_record<G, S, MAXP>(A.wbg + (int64_t)id * kWbStride, sumord, sh.u.st.tpl, sh.u.st.lab, sh.etab, wsc,
                                   wsc + G * S, wsc + 2 * G * S, 0u, gl, gb);
    }
    if (gl == 0) {
        if (A.wbl) A.wbl[id] = wl;
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
        A.status[id] = (uint8_t)(foover ? ST_FO_OVER : ST_OK);
        if (A.lim_out) A.lim_out[sh.gs.si] = c.lim;
    }
    if (A.fo)
        for (int k = gl; k < kFoLen; k += G) A.fo[(int64_t)id * kFoLen + k] = (uint8_t)min(sh.u.st.fo[k], 255);
    lds_fence();
    c.phase = PH_NEW;
}

// candidates and tests are counted in registers, the rest in the group's LDS
template <int G, int S, int MAXP, bool RAD>
__device__ __forceinline__ void flush_counters(const CellArgs &A, SL<G, S, MAXP, RAD> &sh, uint32_t &ncand,
                                               uint32_t &ntest, int gl)
{
    sh.gs.cnt[DC_CAND] += ncand;
    sh.gs.cnt[DC_TESTS] += ntest;
    ncand = ntest = 0;
    lds_fence();
    if (gl < DC_N) {
        uint32_t v = sh.gs.cnt[gl];
        if (v) atomicAdd(&A.diag[gl], (unsigned long long)v);
    }
    lds_fence();
    if (gl < DC_N) sh.gs.cnt[gl] = 0;
    lds_fence();
}

// Occupancy target in waves per SIMD, to which the register allocator is
// held.  The two-cells-per-wave form runs four waves: 128 registers and,
// with 32 plane slots per cell, 10,016 bytes of LDS per wave (of the 10,240
// that sixteen waves per compute unit leave); a cell that needs more plane
// slots goes to the spill pass.  (The instantiation that writes Weinberg
// records spills more registers at that budget, around the record's call,
// and is still faster than at three waves.)
template <int G>
struct SyncWaves {
    static constexpr int value = G == 32 ? 4 : 2;
};

template <int G, int S, int MAXP, bool F32, bool RAD, bool WB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(SyncWaves<G>::value))) void k_cells_sync(CellArgs Ain)
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
    static_assert(((G * S) & (G * S - 1)) == 0 && G * S <= 256, "slot count must be a power of two");
    static_assert(G == 16 || G == 32, "group width");
    __shared__ SL<G, S, MAXP, RAD> shv[Gw<G>::CPW];
    const int lane = __lane_id();
    const int gl = lane % G, gb = lane - gl;
    const uint32_t below = (1u << gl) - 1u;
    SL<G, S, MAXP, RAD> &sh = shv[lane / G];
    uint32_t cnt[2] = {0, 0};  // candidates, vertex tests
    const int ncell = A.ncell;
    SCell<S, F32> c;
    c.phase = PH_NEW;
    if (gl < DC_N) sh.gs.cnt[gl] = 0;
    sh.gs.cell = 0;
    sh.gs.cend = 0;
    sh.gs.tcur = -1;
    lds_fence();
#ifdef VC_PHASE_CLOCKS
    // wave-level shader-clock cycles and executions of each phase body
    unsigned long long pclk[kPhaseSlots] = {}, pcnt[kPhaseSlots] = {};
    unsigned long long t_prev = clock64();
#define VC_PHASE_MARK(k, ran)                    \
    do {                                         \
        const unsigned long long t_ = clock64(); \
        pclk[k] += t_ - t_prev;                  \
        pcnt[k] += (ran) ? 1 : 0;                \
        t_prev = t_;                             \
    } while (0)
#define VC_PHASE_RAN(ph) (__ballot(c.phase == (ph)) != 0)
#else
#define VC_PHASE_RAN(ph) false
#define VC_PHASE_MARK(k, ran) \
    do {                      \
        (void)(ran);          \
    } while (0)
#endif
    for (;;) {
        const bool r_new = VC_PHASE_RAN(PH_NEW);
        if (c.phase == PH_NEW) {
            if (cnt[1] > (1u << 30) || sh.gs.cnt[DC_NEWV] > (1u << 30) || sh.gs.cnt[DC_LOADED] > (1u << 30))
                flush_counters<G, S, MAXP, RAD>(A, sh, cnt[0], cnt[1], gl);
            ph_new<G, S, MAXP, F32, RAD>(A, sh, c, ncell, gl, gb);
        }
        VC_PHASE_MARK(0, r_new);
        if (!__ballot(c.phase != PH_DONE)) break;
        const bool r_gat = VC_PHASE_RAN(PH_GATHER);
        if (c.phase == PH_GATHER) ph_gather<G, S, MAXP, F32, RAD>(A, sh, c, gl, gb, cnt);
        VC_PHASE_MARK(1, r_gat);
        const bool r_bat = VC_PHASE_RAN(PH_BATCH);
        if (c.phase == PH_BATCH) ph_batch<G, S, MAXP, F32, RAD>(A, sh, c, gl, gb, below);
        VC_PHASE_MARK(2, r_bat);
#ifdef VC_PHASE_CLOCKS
        while (c.phase == PH_TEST) {
            ph_test<G, S, MAXP, F32, RAD>(A, sh, c, cnt, gl, gb);
            pcnt[6]++;
        }
#else
        while (c.phase == PH_TEST) ph_test<G, S, MAXP, F32, RAD>(A, sh, c, cnt, gl, gb);
#endif
        VC_PHASE_MARK(3, true);
        // cuts and statistics wait until no group can advance without one
        if (!__ballot(c.phase == PH_NEW || c.phase == PH_GATHER || c.phase == PH_BATCH || c.phase < 0)) {
            const bool r_cut = VC_PHASE_RAN(PH_CUT);
            if (c.phase == PH_CUT) ph_cut<G, S, MAXP, F32, RAD>(A, sh, c, cnt, gl, gb, below);
            VC_PHASE_MARK(4, r_cut);
            const bool r_st = VC_PHASE_RAN(PH_STATS);
            if (c.phase == PH_STATS) ph_stats<G, S, MAXP, F32, RAD>(A, sh, c, cnt, gl, gb, below);
            VC_PHASE_MARK(5, r_st);
        }
        if (c.phase < 0) cell_fail<G, S, MAXP, F32, RAD>(A, sh, c, -c.phase, gl);
        VC_PHASE_MARK(7, true);
    }
    flush_counters<G, S, MAXP, RAD>(A, sh, cnt[0], cnt[1], gl);
#ifdef VC_PHASE_CLOCKS
    if (lane == 0)
        for (int k = 0; k < kPhaseSlots; k++) {
            atomicAdd(&A.diag[kPhaseClk + k], pclk[k]);
            atomicAdd(&A.diag[kPhaseCnt + k], pcnt[k]);
        }
#endif
#undef VC_PHASE_MARK
#undef VC_PHASE_RAN
}

}  // namespace

hipError_t launch_cells_group(const CellArgs &a, int precision, int cpw, int waves, hipStream_t s)
{
    const bool rad = a.rad != nullptr, wb = a.wbg != nullptr, f32 = precision == 1;
#define VC_GROUP(G, S, P)                                                                        \
    do {                                                                                         \
        if (rad) {                                                                               \
            if (wb) {                                                                            \
                if (f32) k_cells_sync<G, S, P, true, true, true><<<waves, 64, 0, s>>>(a);        \
                else k_cells_sync<G, S, P, false, true, true><<<waves, 64, 0, s>>>(a);           \
            } else {                                                                             \
                if (f32) k_cells_sync<G, S, P, true, true, false><<<waves, 64, 0, s>>>(a);       \
                else k_cells_sync<G, S, P, false, true, false><<<waves, 64, 0, s>>>(a);          \
            }                                                                                    \
        } else {                                                                                 \
            if (wb) {                                                                            \
                if (f32) k_cells_sync<G, S, P, true, false, true><<<waves, 64, 0, s>>>(a);       \
                else k_cells_sync<G, S, P, false, false, true><<<waves, 64, 0, s>>>(a);          \
            } else {                                                                             \
                if (f32) k_cells_sync<G, S, P, true, false, false><<<waves, 64, 0, s>>>(a);      \
                else k_cells_sync<G, S, P, false, false, false><<<waves, 64, 0, s>>>(a);         \
            }                                                                                    \
        }                                                                                        \
    } while (0)
    if (cpw == 4) VC_GROUP(16, 4, 32);
    else if (cpw == 2) VC_GROUP(32, 2, 32);
    else return hipErrorInvalidValue;
#undef VC_GROUP
    return hipGetLastError();
}

}  // namespace vc
