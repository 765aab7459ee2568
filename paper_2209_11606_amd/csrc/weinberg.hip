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

__global__ __launch_bounds__(64) void k_weinberg(const uint8_t *__restrict__ wbg, const int32_t *__restrict__ wbl,
                                                 const int64_t *__restrict__ off, int64_t n,
                                                 uint8_t *__restrict__ codes, int32_t *__restrict__ sym,
                                                 uint8_t *__restrict__ chiral, int32_t *__restrict__ queue)
{
    __shared__ WbLDS sh;
    const int lane = __lane_id();
    // Every branch below is taken by the whole wave (its condition is made
    // wave-uniform), and the loop body has no early exit: the next cell is
    // claimed only once the wave has reconverged.
    for (;;) {
        int cell = 0;
        if (lane == 0) cell = atomicAdd(queue, 1);
        cell = __builtin_amdgcn_readfirstlane(cell);
        if (cell >= n) break;
        const int64_t id = cell;
        const uint8_t *rec = wbg + id * kWbStride;
        const int D = __builtin_amdgcn_readfirstlane(wbl[id]);
        const int V = D > 0 ? __builtin_amdgcn_readfirstlane((int)rec[0]) : 0;
        const int Drec = D > 0 ? __builtin_amdgcn_readfirstlane((int)(rec[1] | (rec[2] << 8))) : 0;
        bool ok = D > 0 && D <= kWbMaxD && V >= 4 && V <= kWbMaxV && Drec == D;
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
        } else if (D > 0 && D <= kWbMaxD) {
            // an inconsistent record: its slot of the codes is zeroed
            uint8_t *out = codes + off[id];
            for (int k = lane; k < D; k += 64) out[k] = 0;
        }
        if (lane == 0) {
            sym[id] = ok ? count : 0;
            chiral[id] = ok && senses != 3;
        }
        wb_fence();
    }
}

}  // namespace

hipError_t launch_weinberg(const uint8_t *wbg, const int32_t *wbl, const int64_t *off, int64_t n, uint8_t *codes,
                           int32_t *sym, uint8_t *chiral, int32_t *queue, int waves, hipStream_t s)
{
    if (n > 0) k_weinberg<<<waves, 64, 0, s>>>(wbg, wbl, off, n, codes, sym, chiral, queue);
    return hipGetLastError();
}

}  // namespace vc
