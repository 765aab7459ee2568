// weinberg.hip -- Weinberg codes of finished 3D cells: the cell-topology
// code that VoroTop computes for every cell (section 5; Weinberg 1966).
//
// Input: the edge-graph record each cell kernel wrote for its cell (see
// wb_record): V vertices, their degrees, and each vertex's neighbours in one
// common rotational sense.  A walk takes every dart (directed edge) once:
// on reaching a vertex for the first time it leaves by the next dart in the
// rotation after the reversed arrival dart; on reaching a vertex seen before
// it goes back along the same edge unless that was done already, and else
// leaves by the first unused dart in the rotation after the reversed arrival
// dart.  Vertices are numbered 1, 2, ... as first reached; the walk's code is
// the number of the vertex each dart leaves, 2E numbers.  The cell's code is
// the smallest walk code over all 2E starting darts and both rotational
// senses; its symmetry count is the number of (dart, sense) pairs giving it.
//
// One wavefront per cell.  The 4E candidate walks run 64 at a time, one per
// lane, in lockstep: at each step the lanes still alive share the same code
// prefix, the smallest next number is kept and every lane with a larger one
// drops out; a round whose prefix exceeds the best code so far stops.  The
// first round runs all 2E steps; later rounds usually stop within a few.
//
// Two kernels: k_weinberg_small takes the cells of up to 64 vertices and 192
// darts (all but a few in practice) with each lane's walk state in
// registers (vertices seen: a 64-bit mask; darts taken: three) and every
// turn a table lookup, so a step costs one or two LDS round trips; the
// general kernel takes the rest.
#include "cell_common.h"

namespace vc {
namespace {

struct WbLDS {
    uint8_t head[kWbMaxD];               // vertex each dart enters
    uint8_t tailv[kWbMaxD];              // vertex each dart leaves
    uint16_t rev[kWbMaxD];               // the opposite dart
    uint16_t base[kWbMaxV + 1];          // first dart of each vertex
    uint8_t deg[kWbMaxV];
    uint8_t best[kWbMaxD];               // smallest code so far
    uint8_t cur[kWbMaxD];                // the current round's code
    uint8_t lbl[kWbMaxV][64];            // per lane: vertex numbers of its walk
    uint32_t used[(kWbMaxD + 31) / 32][64];  // per lane: darts taken
};

__device__ __forceinline__ int wave_imin(int v)
{
    constexpr int kBig = 0x7fffffff;
    v = min(v, dpp_i32<DPP_QUAD_1032, 0xf>(kBig, v));
    v = min(v, dpp_i32<DPP_QUAD_2301, 0xf>(kBig, v));
    v = min(v, dpp_i32<DPP_ROW_HALF_MIRROR, 0xf>(kBig, v));
    v = min(v, dpp_i32<DPP_ROW_MIRROR, 0xf>(kBig, v));
    v = min(v, dpp_i32<DPP_ROW_BCAST15, 0xa>(kBig, v));
    v = min(v, dpp_i32<DPP_ROW_BCAST31, 0xc>(kBig, v));
    return __builtin_amdgcn_readlane(v, 63);
}

// next dart leaving the tail of d in the rotation (o = 0) or against it
__device__ __forceinline__ int wb_rot(const WbLDS &sh, int d, int o)
{
    const int v = sh.tailv[d], b = sh.base[v], n = sh.deg[v];
    if (o == 0) return d + 1 == b + n ? b : d + 1;
    return d == b ? b + n - 1 : d - 1;
}

__device__ __forceinline__ bool wb_used(const WbLDS &sh, int d, int lane)
{
    return (sh.used[d >> 5][lane] >> (d & 31)) & 1u;
}

constexpr int kSmV = 64, kSmD = 192;  // the small-cell kernel's limits

struct WbSmall {
    uint8_t head[kSmD];      // vertex each dart enters
    uint8_t tailv[kSmD];     // vertex each dart leaves
    uint8_t rev[kSmD];       // the opposite dart
    uint8_t rot[2][kSmD];    // next dart leaving the same vertex, in sense 0 / 1
    uint8_t turn[2][kSmD];   // rot(rev(d)): the way on after arriving by d
    uint8_t deg[kSmV];
    uint8_t base[kSmV + 1];  // first dart of each vertex
    uint8_t best[kSmD];      // smallest code so far
    uint8_t cur[kSmD];       // the current round's code
    uint16_t cand[2 * kSmD]; // candidate starts: 2 x dart + sense
    uint8_t lbl[kSmV][64];   // per lane: each vertex's number, written on its first visit
};

// OR of a small value over the wave
__device__ __forceinline__ int grp_or64(int v)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v |= __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ bool bit3(uint64_t u0, uint64_t u1, uint64_t u2, int d)
{
    const uint64_t w = d < 64 ? u0 : (d < 128 ? u1 : u2);
    return (w >> (d & 63)) & 1ull;
}

__device__ __forceinline__ void set3(uint64_t &u0, uint64_t &u1, uint64_t &u2, int d)
{
    const uint64_t b = 1ull << (d & 63);
    u0 |= d < 64 ? b : 0ull;
    u1 |= (d >= 64 && d < 128) ? b : 0ull;
    u2 |= d >= 128 ? b : 0ull;
}

constexpr int kWbChunk = 8;  // cells per work-queue grab of the small kernel

// The cells whose record has at most kSmV vertices and kSmD darts (and the
// cells without a record: symmetry 0).  The others are listed in big (their
// count in queue[2]) for the general kernel.
__global__ __launch_bounds__(64) void k_weinberg_small(const uint8_t *__restrict__ wbg,
                                                       const int32_t *__restrict__ wbl,
                                                       const int64_t *__restrict__ off, int64_t n,
                                                       uint8_t *__restrict__ codes, int32_t *__restrict__ sym,
                                                       uint8_t *__restrict__ chiral, int32_t *__restrict__ queue,
                                                       int32_t *__restrict__ big)
{
    __shared__ WbSmall sh;
    const int lane = __lane_id();
    for (;;) {
        int first = 0;
        if (lane == 0) first = atomicAdd(queue, kWbChunk);
        first = __builtin_amdgcn_readfirstlane(first);
        if (first >= n) break;
        const int last = (int)min((int64_t)first + kWbChunk, n);
        for (int cell = first; cell < last; cell++) {
            const int64_t id = cell;
            const uint8_t *rec = wbg + id * kWbStride;
            const int D = __builtin_amdgcn_readfirstlane(wbl[id]);
            const int V = D > 0 ? __builtin_amdgcn_readfirstlane((int)rec[0]) : 0;
            const int Drec = D > 0 ? __builtin_amdgcn_readfirstlane((int)(rec[1] | (rec[2] << 8))) : 0;
            const bool mine = D <= 0 || (V <= kSmV && D <= kSmD);
            bool ok = mine && D > 0 && V >= 4 && Drec == D;
            int count = 0, senses = 0;
            if (ok) {
                // degrees, first darts (a wave scan), dart ends, opposites, turns
                const int dg = lane < V ? rec[3 + lane] : 0;
                int inc = dg;
    #pragma unroll
                for (int m = 1; m < 64; m <<= 1) {
                    const int y = __shfl_up(inc, m);
                    if (lane >= m) inc += y;
                }
                const int b0 = inc - dg;
                if (lane < V) {
                    sh.deg[lane] = (uint8_t)dg;
                    sh.base[lane] = (uint8_t)min(b0, 255);
                    for (int j = 0; j < dg && b0 + j < kSmD; j++) sh.tailv[b0 + j] = (uint8_t)lane;
                }
                const int total = __builtin_amdgcn_readlane(inc, 63);
                ok = total == D;
                for (int d = lane; d < D; d += 64) sh.head[d] = rec[3 + V + d];
                wb_fence();
                bool bad = false;
                if (ok) {
                    for (int d = lane; d < D; d += 64) {
                        const int v = sh.tailv[d], w = sh.head[d];
                        int r = -1;
                        if (w < V)
                            for (int e = sh.base[w]; e < sh.base[w] + sh.deg[w]; e++)
                                if (sh.head[e] == v) r = e;
                        bad |= r < 0;
                        sh.rev[d] = (uint8_t)max(r, 0);
                        const int b = sh.base[v], nv = sh.deg[v];
                        sh.rot[0][d] = (uint8_t)(d + 1 == b + nv ? b : d + 1);
                        sh.rot[1][d] = (uint8_t)(d == b ? b + nv - 1 : d - 1);
                    }
                    wb_fence();
                    for (int d = lane; d < D; d += 64) {
                        const int r = sh.rev[d];
                        sh.turn[0][d] = sh.rot[0][r];
                        sh.turn[1][d] = sh.rot[1][r];
                    }
                    wb_fence();
                }
                ok = ok && __builtin_amdgcn_ballot_w64(bad) == 0;
            }
            int nc = 0;
            if (ok) {
                // A walk's code starts 1, 2, ..., p, 1 where p is the size of the
                // face on its turning side (it turns that way at every new
                // vertex until it closes that face), so only the starts on a
                // smallest face can give the smallest code: the candidates.
                int fs[2 * ((kSmD + 63) / 64)];
                int pmin = 0x7fffffff;
    #pragma unroll
                for (int j = 0; j < (kSmD + 63) / 64; j++) {
                    const int d = lane + 64 * j;
    #pragma unroll
                    for (int o = 0; o < 2; o++) {
                        int len = 0x7fffffff;
                        if (d < D) {
                            int e = d;
                            len = 0;
                            do {
                                e = sh.turn[o][e];
                                len++;
                            } while (e != d && len < 64);
                        }
                        fs[2 * j + o] = len;
                        pmin = min(pmin, len);
                    }
                }
                pmin = wave_imin(pmin);
    #pragma unroll
                for (int j = 0; j < (kSmD + 63) / 64; j++)
    #pragma unroll
                    for (int o = 0; o < 2; o++) {
                        const bool is = fs[2 * j + o] == pmin;
                        const unsigned long long b = __builtin_amdgcn_ballot_w64(is);
                        if (is) sh.cand[nc + lane_rank(b)] = (uint16_t)(2 * (lane + 64 * j) + o);
                        nc += __popcll(b);
                    }
                wb_fence();
            }
            if (ok) {
                // the candidate walks, 64 per round, one per lane
                bool have = false;
                for (int c0 = 0; c0 < nc; c0 += 64) {
                    bool alive = c0 + lane < nc;
                    const int cd = alive ? sh.cand[c0 + lane] : 0;
                    const int o = cd & 1;
                    int dcur = cd >> 1;
                    uint64_t vis = 0, u0 = 0, u1 = 0, u2 = 0;
                    int nl = 1, lab = 1;
                    if (alive) {
                        const int t = sh.tailv[dcur];
                        vis = 1ull << t;
                        sh.lbl[t][lane] = 1;
                    }
                    bool eq = have, better = !have, done = false;
                    for (int k = 0; k < D; k++) {
                        const int m = wave_imin(alive ? lab : 0x7fffffff);
                        if (m == 0x7fffffff) break;
                        if (eq) {
                            const int bk = __builtin_amdgcn_readfirstlane((int)sh.best[k]);
                            if (m > bk) break;
                            if (m < bk) {
                                eq = false;
                                better = true;
                            }
                        }
                        alive = alive && lab == m;
                        if (lane == 0) sh.cur[k] = (uint8_t)m;
                        if (k == D - 1) {
                            done = true;
                            break;
                        }
                        if (alive) {
                            set3(u0, u1, u2, dcur);
                            const int v = sh.head[dcur];
                            if (!((vis >> v) & 1ull)) {
                                vis |= 1ull << v;
                                lab = ++nl;
                                sh.lbl[v][lane] = (uint8_t)nl;
                                dcur = sh.turn[o][dcur];
                            } else {
                                lab = sh.lbl[v][lane];
                                const int r = sh.rev[dcur];
                                if (!bit3(u0, u1, u2, r)) {
                                    dcur = r;
                                } else {
                                    int e = sh.turn[o][dcur];
                                    for (int g = 0; g < 64 && bit3(u0, u1, u2, e); g++) e = sh.rot[o][e];
                                    dcur = e;
                                }
                            }
                        }
                    }
                    wb_fence();
                    if (done) {
                        const unsigned long long am = __builtin_amdgcn_ballot_w64(alive);
                        int sm = 0;
                        if (alive) sm = 1 << o;
                        sm = grp_or64(sm);
                        if (better) {
                            for (int k = lane; k < D; k += 64) sh.best[k] = sh.cur[k];
                            count = __popcll(am);
                            senses = sm;
                            have = true;
                        } else if (eq) {
                            count += __popcll(am);
                            senses |= sm;
                        }
                    }
                    wb_fence();
                }
                uint8_t *out = codes + off[id];
                for (int k = lane; k < D; k += 64) out[k] = sh.best[k];
            } else if (mine && D > 0 && D <= kWbMaxD) {
                uint8_t *out = codes + off[id];
                for (int k = lane; k < D; k += 64) out[k] = 0;
            }
            if (lane == 0) {
                if (mine) {
                    sym[id] = ok ? count : 0;
                    chiral[id] = ok && senses != 3;
                } else {
                    // beyond this kernel's limits: listed for the general kernel
                    big[atomicAdd(queue + 2, 1)] = cell;
                }
            }
            wb_fence();
        }
    }
}

// The cells listed by the small kernel (their count in queue[2]).
__global__ __launch_bounds__(64) void k_weinberg(const uint8_t *__restrict__ wbg, const int32_t *__restrict__ wbl,
                                                 const int64_t *__restrict__ off, const int32_t *__restrict__ big,
                                                 uint8_t *__restrict__ codes, int32_t *__restrict__ sym,
                                                 uint8_t *__restrict__ chiral, int32_t *__restrict__ queue)
{
    __shared__ WbLDS sh;
    const int lane = __lane_id();
    const int nbig = __builtin_amdgcn_readfirstlane(queue[2]);
    // Every branch below is taken by the whole wave (its condition is made
    // wave-uniform), and the loop body has no early exit: the next cell is
    // claimed only once the wave has reconverged.
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(queue + 1, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= nbig) break;
        const int64_t id = __builtin_amdgcn_readfirstlane(big[item]);
        const uint8_t *rec = wbg + id * kWbStride;
        const int D = __builtin_amdgcn_readfirstlane(wbl[id]);
        const int V = D > 0 ? __builtin_amdgcn_readfirstlane((int)rec[0]) : 0;
        const int Drec = D > 0 ? __builtin_amdgcn_readfirstlane((int)(rec[1] | (rec[2] << 8))) : 0;
        const bool mine = D > 0;
        bool ok = mine && D <= kWbMaxD && V >= 4 && V <= kWbMaxV && Drec == D;
        int count = 0, senses = 0;
        if (ok) {
            // vertex degrees, first darts (a wave scan), dart ends and opposites
            for (int v = lane; v < V; v += 64) sh.deg[v] = rec[3 + v];
            const int a = lane < V ? rec[3 + lane] : 0;
            int inc = a;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
                const int y = __shfl_up(inc, m);
                if (lane >= m) inc += y;
            }
            if (lane < V) sh.base[lane] = (uint16_t)(inc - a);
            const int tot = __shfl(inc, 63);
            const int b = lane + 64 < V ? rec[3 + lane + 64] : 0;
            int inc2 = b;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
                const int y = __shfl_up(inc2, m);
                if (lane >= m) inc2 += y;
            }
            if (lane + 64 < V) sh.base[lane + 64] = (uint16_t)(tot + inc2 - b);
            if (lane == 0) sh.base[V] = (uint16_t)D;
            wb_fence();
            for (int d = lane; d < D; d += 64) {
                sh.head[d] = rec[3 + V + d];
                int lo = 0, hi = V - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sh.base[mid] <= d) lo = mid; else hi = mid - 1;
                }
                sh.tailv[d] = (uint8_t)lo;
            }
            wb_fence();
            bool bad = false;
            for (int d = lane; d < D; d += 64) {
                const int v = sh.tailv[d], w = sh.head[d];
                int r = -1;
                if (w < V)
                    for (int e = sh.base[w]; e < sh.base[w] + sh.deg[w]; e++)
                        if (sh.head[e] == v) r = e;
                bad |= r < 0;
                sh.rev[d] = (uint16_t)max(r, 0);
            }
            wb_fence();
            const int last = __builtin_amdgcn_readfirstlane((int)sh.base[V - 1] + (int)sh.deg[V - 1]);
            ok = __builtin_amdgcn_ballot_w64(bad) == 0 && last == D;
        }
        if (ok) {
            // the candidate walks, 64 per round: lane l of a round starting
            // at c0 walks from dart (c0 + l) / 2 in sense (c0 + l) % 2
            bool have = false;
            for (int c0 = 0; c0 < 2 * D; c0 += 64) {
                const int c = c0 + lane;
                bool alive = c < 2 * D;
                const int o = lane & 1;
                int dcur = alive ? c >> 1 : 0;
                for (int v = 0; v < V; v++) sh.lbl[v][lane] = 0;
                for (int w = 0; w < (D + 31) / 32; w++) sh.used[w][lane] = 0u;
                int nl = 1;
                if (alive) sh.lbl[sh.tailv[dcur]][lane] = 1;
                bool eq = have, better = !have, done = false;
                for (int k = 0; k < D; k++) {
                    const int sk = alive ? sh.lbl[sh.tailv[dcur]][lane] : 0x7fffffff;
                    const int m = wave_imin(sk);
                    if (m == 0x7fffffff) break;
                    if (eq) {
                        const int bk = __builtin_amdgcn_readfirstlane((int)sh.best[k]);
                        if (m > bk) break;
                        if (m < bk) {
                            eq = false;
                            better = true;
                        }
                    }
                    alive = alive && sk == m;
                    if (lane == 0) sh.cur[k] = (uint8_t)m;
                    if (k == D - 1) {
                        done = true;
                        break;
                    }
                    if (alive) {
                        sh.used[dcur >> 5][lane] |= 1u << (dcur & 31);
                        const int v = sh.head[dcur], r = sh.rev[dcur];
                        if (sh.lbl[v][lane] == 0) {
                            sh.lbl[v][lane] = (uint8_t)(++nl);
                            dcur = wb_rot(sh, r, o);
                        } else if (!wb_used(sh, r, lane)) {
                            dcur = r;
                        } else {
                            int e = wb_rot(sh, r, o);
                            for (int g = 0; g < 256 && wb_used(sh, e, lane); g++) e = wb_rot(sh, e, o);
                            dcur = e;
                        }
                    }
                }
                wb_fence();
                if (done) {
                    const unsigned long long am = __builtin_amdgcn_ballot_w64(alive);
                    const int sm = ((am & 0x5555555555555555ull) ? 1 : 0) | ((am & 0xaaaaaaaaaaaaaaaaull) ? 2 : 0);
                    if (better) {
                        for (int k = lane; k < D; k += 64) sh.best[k] = sh.cur[k];
                        count = __popcll(am);
                        senses = sm;
                        have = true;
                    } else if (eq) {
                        count += __popcll(am);
                        senses |= sm;
                    }
                }
                wb_fence();
            }
            uint8_t *out = codes + off[id];
            for (int k = lane; k < D; k += 64) out[k] = sh.best[k];
        } else if (mine && D <= kWbMaxD) {
            // an inconsistent record: its slot of the codes is zeroed
            uint8_t *out = codes + off[id];
            for (int k = lane; k < D; k += 64) out[k] = 0;
        }
        if (mine && lane == 0) {
            sym[id] = ok ? count : 0;
            chiral[id] = ok && senses != 3;
        }
        wb_fence();
    }
}

}  // namespace

hipError_t launch_weinberg(const uint8_t *wbg, const int32_t *wbl, const int64_t *off, int64_t n, uint8_t *codes,
                           int32_t *sym, uint8_t *chiral, int32_t *queue, int32_t *big, int waves, hipStream_t s)
{
    if (n > 0) {
        k_weinberg_small<<<waves, 64, 0, s>>>(wbg, wbl, off, n, codes, sym, chiral, queue, big);
        k_weinberg<<<std::max(1, waves / 16), 64, 0, s>>>(wbg, wbl, off, big, codes, sym, chiral, queue);
    }
    return hipGetLastError();
}

}  // namespace vc
