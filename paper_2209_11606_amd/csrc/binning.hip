// binning.hip -- container construction on the GPU: block index per
// particle, per-block counts, exclusive scan, and a scatter into a
// block-sorted particle array in a deterministic in-block order (by input id).
//
// This replaces the serial put() and the atomic slot capture of the paper's
// parallel insertion (section 2.2.5): the atomic counter gives each particle
// a provisional slot, and an exact prefix sum over the counts sizes every
// block, so no overflow buffer is needed.  The final slot is the particle's
// rank by id inside its block, which removes the run-to-run order dependence
// that the paper notes for parallel insertion.
#include <algorithm>

#include "vc_internal.h"

namespace vc {

namespace {

constexpr int kTB = 256;          // threads per block of the streaming kernels
constexpr int kScanItems = 8;     // elements per thread in the scan
constexpr int kScanTile = kTB * kScanItems;

__global__ __launch_bounds__(kTB) void k_bin_count(const double *__restrict__ xyz, int64_t n, int dim,
                                                   const Tess *__restrict__ tess, const int32_t *__restrict__ ptess,
                                                   int32_t *__restrict__ blk, int32_t *__restrict__ rank,
                                                   int32_t *__restrict__ count, int32_t *__restrict__ err)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        const Tess &T = tess[ptess ? ptess[i] : 0];
        const Grid &G = T.G;
        int k[3] = {0, 0, 0};
        bool bad = false;
        for (int d = 0; d < dim; d++) {
            double x = xyz[i * dim + d];
            // walled: lo <= x <= hi; periodic: lo <= x < hi; NaN fails both
            bool ok = G.per[d] ? (x >= G.lo[d] && x < G.hi[d]) : (x >= G.lo[d] && x <= G.hi[d]);
            bad |= !ok;
            k[d] = ok ? block_coord(G, x, d) : 0;
        }
        if (bad) atomicOr(err, 1);
        int32_t b = T.bbase + k[0] + G.g[0] * (k[1] + G.g[1] * k[2]);
        blk[i] = b;
        rank[i] = atomicAdd(&count[b], 1);
    }
}

// exclusive scan, phase 1: per-tile totals
template <typename T>
__global__ __launch_bounds__(kTB) void k_scan_tiles(const int32_t *__restrict__ in, int64_t n, T *__restrict__ tiles)
{
    __shared__ T red[kTB];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
    for (int j = 0; j < kScanItems; j++) {
        int64_t i = base + (int64_t)j * kTB + threadIdx.x;
        if (i < n) s += (T)in[i];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kTB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) tiles[blockIdx.x] = red[0];
}

// phase 2: exclusive scan of the tile totals in one workgroup
template <typename T>
__global__ __launch_bounds__(kTB) void k_scan_top(T *__restrict__ tiles, int64_t ntiles, T *__restrict__ total)
{
    __shared__ T buf[kTB];
    T carry = 0;
    for (int64_t c = 0; c < ntiles; c += kTB) {
        int64_t i = c + threadIdx.x;
        T v = i < ntiles ? tiles[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kTB; o <<= 1) {
            T w = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += w;
            __syncthreads();
        }
        T incl = buf[threadIdx.x];
        if (i < ntiles) tiles[i] = carry + incl - v;
        T chunk_total = buf[kTB - 1];
        __syncthreads();
        carry += chunk_total;
    }
    if (threadIdx.x == 0) *total = carry;
}

// phase 3: scan inside each tile plus the tile offset
template <typename T>
__global__ __launch_bounds__(kTB) void k_scan_final(const int32_t *__restrict__ in, int64_t n,
                                                    const T *__restrict__ tiles, T *__restrict__ out)
{
    __shared__ T buf[kTB];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T loc[kScanItems];
    T s = 0;
    for (int j = 0; j < kScanItems; j++) {
        int64_t i = base + j;
        loc[j] = i < n ? (T)in[i] : 0;
        s += loc[j];
    }
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kTB; o <<= 1) {
        T w = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
        __syncthreads();
        buf[threadIdx.x] += w;
        __syncthreads();
    }
    T run = tiles[blockIdx.x] + buf[threadIdx.x] - s;
    for (int j = 0; j < kScanItems; j++) {
        int64_t i = base + j;
        if (i < n) out[i] = run;
        run += loc[j];
    }
}

template <typename T>
__global__ void k_store_total(const T *__restrict__ total, T *__restrict__ dst)
{
    *dst = *total;
}

// provisional slots: the input index of each particle at its atomic slot
__global__ __launch_bounds__(kTB) void k_scatter_ids(int64_t n, const int32_t *__restrict__ blk,
                                                     const int32_t *__restrict__ rank, const int32_t *__restrict__ start,
                                                     int32_t *__restrict__ sid)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        sid[start[blk[i]] + rank[i]] = (int32_t)i;
}

// final slots: one thread per provisional slot counts the smaller input
// indices of its block (the threads of a wave share a block and read the
// same ids), and writes the particle record there.  Linear in the block's
// size per particle, parallel over the block's particles.
__global__ __launch_bounds__(kTB) void k_rank_scatter(const double *__restrict__ xyz, int64_t n, int dim,
                                                      const int32_t *__restrict__ ptess, const int32_t *__restrict__ blk,
                                                      const int32_t *__restrict__ start, const int32_t *__restrict__ sid,
                                                      Particle *__restrict__ part, int32_t *__restrict__ inv)
{
    for (int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x; t < n; t += (int64_t)gridDim.x * kTB) {
        const int32_t i = sid[t];
        const int32_t b = blk[i];
        const int s = start[b], e = start[b + 1];
        int r0 = 0, r1 = 0, r2 = 0, r3 = 0;
        int u = s;
        for (; u + 3 < e; u += 4) {
            r0 += sid[u] < i;
            r1 += sid[u + 1] < i;
            r2 += sid[u + 2] < i;
            r3 += sid[u + 3] < i;
        }
        for (; u < e; u++) r0 += sid[u] < i;
        Particle p;
        p.x = xyz[(int64_t)i * dim];
        p.y = xyz[(int64_t)i * dim + 1];
        p.z = dim == 3 ? xyz[(int64_t)i * dim + 2] : 0.0;
        p.id = i;
        p.tess = ptess ? ptess[i] : 0;
        const int slot = s + r0 + r1 + r2 + r3;
        part[slot] = p;
        inv[i] = slot;
    }
}

// radii moved to sorted-slot order (radical tessellation)
__global__ __launch_bounds__(kTB) void k_radii(const double *__restrict__ rin, int64_t n,
                                               const int32_t *__restrict__ inv, double *__restrict__ rad)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        rad[inv[i]] = rin[i];
}

// check of the radii and their maximum, kept as the bit pattern of a
// non-negative double (whose order is that of the values): a workgroup
// reduction, then one atomic per workgroup.  A radius that is negative or
// not finite sets the error flag.
__global__ __launch_bounds__(kTB) void k_radii_check(const double *__restrict__ rin, int64_t n,
                                                     unsigned long long *__restrict__ rmax_bits,
                                                     int32_t *__restrict__ err)
{
    __shared__ unsigned long long wmax[kTB / 64];
    unsigned long long m = 0;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) {
        double r = rin[i];
        if (!(r >= 0.0 && r <= 1.7976931348623157e308)) bad = true;
        else if (r > 0.0) m = max(m, (unsigned long long)__double_as_longlong(r));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, o));
    if (__lane_id() == 0) wmax[threadIdx.x / 64] = m;
    if (bad) *err = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kTB / 64; w++) m = max(m, wmax[w]);
        if (m) atomicMax(rmax_bits, m);
    }
}

// sorted slots of a list of input indices (a subset of the cells); an index
// outside [0, n) sets the error flag
__global__ __launch_bounds__(kTB) void k_subset_list(const int64_t *__restrict__ ids, int64_t m, int64_t n,
                                                     const int32_t *__restrict__ inv, int32_t *__restrict__ out,
                                                     int32_t *__restrict__ err)
{
    for (int64_t k = (int64_t)blockIdx.x * kTB + threadIdx.x; k < m; k += (int64_t)gridDim.x * kTB) {
        const int64_t i = ids[k];
        if (i < 0 || i >= n) {
            atomicOr(err, 1);
            out[k] = 0;
        } else {
            out[k] = inv[i];
        }
    }
}

__global__ __launch_bounds__(kTB) void k_fill_u8(uint8_t *p, int64_t n, uint8_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) p[i] = v;
}

__global__ __launch_bounds__(kTB) void k_fill(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB) p[i] = v;
}

// neighbour lists: per cell, sort the labels (id, image) and copy them into
// the CSR arrays at the cell's offset.  A group of 16 lanes takes a cell:
// lane l loads labels l, l + 16, l + 32, l + 48 (coalesced), the keys go to
// the group's LDS row, and each label's place is the number of the cell's
// keys below it (ties, which do not occur, by position).  The groups of a
// wave only share the wave's in-order LDS stream, so no barrier spans them.
constexpr int kNbrLanes = 16;
constexpr int kNbrGroups = kTB / kNbrLanes;

__global__ __launch_bounds__(kTB) void k_nbr_compact(const int32_t *__restrict__ nf, int64_t n,
                                                     const int32_t *__restrict__ nbr, const uint8_t *__restrict__ nsh,
                                                     const int64_t *__restrict__ off, int32_t *__restrict__ ids,
                                                     uint8_t *__restrict__ shifts)
{
    static_assert(kMaxNbr == 4 * kNbrLanes, "four labels per lane");
    __shared__ long long keys[kNbrGroups][kMaxNbr];
    const int g = threadIdx.x / kNbrLanes, l = threadIdx.x % kNbrLanes;
    for (int64_t i = (int64_t)blockIdx.x * kNbrGroups + g; i < n; i += (int64_t)gridDim.x * kNbrGroups) {
        int k = nf[i];
        if (k > kMaxNbr) k = kMaxNbr;
        long long mine[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int t = l + s * kNbrLanes;
            mine[s] = 0;
            if (t < k) {
                mine[s] = ((long long)nbr[i * kMaxNbr + t] << 8) | (long long)nsh[i * kMaxNbr + t];
                keys[g][t] = mine[s];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const int64_t o = off[i];
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int t = l + s * kNbrLanes;
            if (t < k) {
                int r = 0;
                for (int j = 0; j < k; j++) {
                    const long long kj = keys[g][j];
                    r += kj < mine[s] || (kj == mine[s] && j < t);
                }
                ids[o + r] = (int32_t)(mine[s] >> 8);
                shifts[o + r] = (uint8_t)(mine[s] & 0xff);
            }
        }
        // the row is rewritten by the group's next cell
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

int grid_for(int64_t n)
{
    int64_t g = (n + kTB - 1) / kTB;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// ---------------------------------------------------------------------------
// The chunked form (container-block chunks along z).  A chunk is a range of
// layers of blocks along z; its container holds the particles of the range
// widened by a halo of layers on each side (wrapped on a periodic axis).
// Selection keeps the input order (per-tile counts, a scan, then each tile
// writes its picks in order), so the chunk's in-block order is the full
// set's.
// ---------------------------------------------------------------------------
constexpr int kPickTile = 1024;

// layer k lies in the range of `len` layers from `first` (on a periodic axis
// the range wraps around the g layers)
__device__ __forceinline__ bool in_layers(int k, int first, int len, int g, int per)
{
    if (per) return ((k - first) % g + g) % g < len;
    return k >= first && k < first + len;
}

struct SlabPick {
    const double *xyz;
    Grid G;
    int e0, elen;            // the widened range of layers
    int k0, klen;            // the chunk's own layers
    const uint8_t *want;     // NULL: every particle of the chunk; else those with (want[i] & wbit)
    uint8_t wbit;
    double *oxyz;            // selected positions, input order
    int32_t *orig;           // their input indices
    uint8_t *own;            // 1: a particle of the chunk whose cell is wanted
    __device__ int layer(int64_t i) const { return block_coord(G, xyz[3 * i + 2], 2); }
    __device__ bool pick(int64_t i) const { return in_layers(layer(i), e0, elen, G.g[2], G.per[2]); }
    __device__ void emit(int64_t i, int64_t pos) const
    {
        oxyz[3 * pos + 0] = xyz[3 * i + 0];
        oxyz[3 * pos + 1] = xyz[3 * i + 1];
        oxyz[3 * pos + 2] = xyz[3 * i + 2];
        orig[pos] = (int32_t)i;
        const bool mine = in_layers(layer(i), k0, klen, G.g[2], G.per[2]) && (!want || (want[i] & wbit));
        own[pos] = mine ? 1 : 0;
    }
};

// the particles of the chunk whose cells are wanted (counted only)
struct OwnPick {
    const double *xyz;
    Grid G;
    int k0, klen;
    const uint8_t *want;
    uint8_t wbit;
    __device__ bool pick(int64_t i) const
    {
        return in_layers(block_coord(G, xyz[3 * i + 2], 2), k0, klen, G.g[2], G.per[2]) && (!want || (want[i] & wbit));
    }
    __device__ void emit(int64_t, int64_t) const {}
};

// sorted slots whose particle is wanted, in slot order (part[s].id is the
// particle's index in the chunk: taken before the ids are remapped)
struct SlotPick {
    const Particle *part;
    const uint8_t *own;
    int32_t *list;
    __device__ bool pick(int64_t s) const { return own[part[s].id] != 0; }
    __device__ void emit(int64_t s, int64_t pos) const { list[pos] = (int32_t)s; }
};

template <class P>
__global__ __launch_bounds__(kTB) void k_pick_count(P p, int64_t n, int32_t *__restrict__ cnt)
{
    __shared__ int wsum[kTB / 64];
    const int64_t base = (int64_t)blockIdx.x * kPickTile;
    int c = 0;
    for (int j = 0; j < kPickTile / kTB; j++) {
        const int64_t i = base + (int64_t)j * kTB + threadIdx.x;
        if (i < n && p.pick(i)) c++;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kTB / 64; w++) t += wsum[w];
        cnt[blockIdx.x] = t;
    }
}

template <class P>
__global__ __launch_bounds__(kTB) void k_pick_scatter(P p, int64_t n, const int32_t *__restrict__ start)
{
    __shared__ int wsum[kTB / 64];
    const int64_t base = (int64_t)blockIdx.x * kPickTile;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t off = start[blockIdx.x];
    for (int j = 0; j < kPickTile / kTB; j++) {
        const int64_t i = base + (int64_t)j * kTB + threadIdx.x;
        const bool pk = i < n && p.pick(i);
        const unsigned long long b = __ballot(pk);
        if (lane == 0) wsum[w] = __popcll(b);
        __syncthreads();
        int before = 0, tot = 0;
        for (int k = 0; k < kTB / 64; k++) {
            if (k < w) before += wsum[k];
            tot += wsum[k];
        }
        if (pk) p.emit(i, off + before + __popcll(b & ((1ull << lane) - 1ull)));
        off += tot;
        __syncthreads();
    }
}

// the chunk container's particles carry the full set's input indices
__global__ __launch_bounds__(kTB) void k_remap_ids(Particle *__restrict__ part, int64_t m,
                                                   const int32_t *__restrict__ orig)
{
    for (int64_t s = (int64_t)blockIdx.x * kTB + threadIdx.x; s < m; s += (int64_t)gridDim.x * kTB)
        part[s].id = orig[part[s].id];
}

// the range check of the binning, over the whole set (walled: lo <= x <= hi,
// periodic: lo <= x < hi, NaN fails)
__global__ __launch_bounds__(kTB) void k_range_check(const double *__restrict__ xyz, int64_t n, Grid G,
                                                     int32_t *__restrict__ err)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        for (int d = 0; d < 3; d++) {
            const double x = xyz[3 * i + d];
            bad |= !(G.per[d] ? (x >= G.lo[d] && x < G.hi[d]) : (x >= G.lo[d] && x <= G.hi[d]));
        }
    if (bad) atomicOr(err, 1);
}

// The chunk certificate: a particle farther than a finished cell's search
// radius (sqrt(lim), section 2.1.3) cannot cut it, so the cell is final when
// every particle missing from the chunk's container -- those beyond either
// end [zlo, zhi) of the widened range along z -- is that far; otherwise the
// cell is flagged to be computed again.  Cells that failed are left as they
// are.
__global__ __launch_bounds__(kTB) void k_slab_cert(const Particle *__restrict__ part, const int32_t *__restrict__ list,
                                                   int64_t m, const double *__restrict__ lim, double zlo, double zhi,
                                                   double per, double eps, uint8_t bit, uint8_t *__restrict__ status)
{
    for (int64_t k = (int64_t)blockIdx.x * kTB + threadIdx.x; k < m; k += (int64_t)gridDim.x * kTB) {
        const int32_t si = list[k];
        const int32_t id = part[si].id;
        const uint8_t st = status[id];
        if ((st & 63) > 1) continue;
        const double pz = part[si].z;
        double dlo = pz - zlo, dhi = zhi - pz;
        if (dlo < 0.0) dlo += per;
        if (dhi < 0.0) dhi += per;
        const double d = fmin(dlo, dhi) - eps;
        if (!(d > 0.0 && lim[si] < d * d)) status[id] = st | bit;
    }
}

// cells whose status carries `bit`
__global__ __launch_bounds__(kTB) void k_count_bit(const uint8_t *__restrict__ st, int64_t n, uint8_t bit,
                                                   int32_t *__restrict__ out)
{
    int c = 0;
    for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kTB)
        c += (st[i] & bit) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

template <class P>
hipError_t pick_impl(const P &p, int64_t n, int32_t *cnt, int32_t *start, int32_t *tmp, bool scatter, hipStream_t s);

template <typename T>
hipError_t scan_impl(const int32_t *in, int64_t n, T *out, T *tmp, hipStream_t s)
{
    // out has n + 1 entries; tmp holds ceil(n / tile) + 1 entries
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles < 1) ntiles = 1;
    k_scan_tiles<T><<<(unsigned)ntiles, kTB, 0, s>>>(in, n, tmp);
    k_scan_top<T><<<1, kTB, 0, s>>>(tmp, ntiles, tmp + ntiles);
    k_scan_final<T><<<(unsigned)ntiles, kTB, 0, s>>>(in, n, tmp, out);
    k_store_total<T><<<1, 1, 0, s>>>(tmp + ntiles, out + n);
    return hipGetLastError();
}

// count (and with `scatter`, write) the picks of `p` over n items: cnt and
// start hold ceil(n / kPickTile) (+ 1) entries, start[last] the total
template <class P>
hipError_t pick_impl(const P &p, int64_t n, int32_t *cnt, int32_t *start, int32_t *tmp, bool scatter, hipStream_t s)
{
    const int64_t tiles = pick_tiles(n);
    if (!scatter) {
        k_pick_count<P><<<(unsigned)tiles, kTB, 0, s>>>(p, n, cnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return scan_impl<int32_t>(cnt, tiles, start, tmp, s);
    }
    k_pick_scatter<P><<<(unsigned)tiles, kTB, 0, s>>>(p, n, start);
    return hipGetLastError();
}

}  // namespace

int64_t pick_tiles(int64_t n) { return std::max<int64_t>(1, (n + kPickTile - 1) / kPickTile); }

hipError_t launch_slab_pick(const double *xyz, int64_t n, const Grid &G, int e0, int elen, int k0, int klen,
                            const uint8_t *want, uint8_t wbit, double *oxyz, int32_t *orig, uint8_t *own,
                            int32_t *cnt, int32_t *start, int32_t *tmp, bool scatter, hipStream_t s)
{
    const SlabPick p{xyz, G, e0, elen, k0, klen, want, wbit, oxyz, orig, own};
    return pick_impl(p, n, cnt, start, tmp, scatter, s);
}

hipError_t launch_own_count(const double *xyz, int64_t n, const Grid &G, int k0, int klen, const uint8_t *want,
                            uint8_t wbit, int32_t *cnt, int32_t *start, int32_t *tmp, hipStream_t s)
{
    const OwnPick p{xyz, G, k0, klen, want, wbit};
    return pick_impl(p, n, cnt, start, tmp, false, s);
}

hipError_t launch_slot_list(const Particle *part, const uint8_t *own, int64_t m, int32_t *list, int32_t *cnt,
                            int32_t *start, int32_t *tmp, hipStream_t s)
{
    const SlotPick p{part, own, list};
    hipError_t e = pick_impl(p, m, cnt, start, tmp, false, s);
    if (e != hipSuccess) return e;
    return pick_impl(p, m, cnt, start, tmp, true, s);
}

hipError_t launch_remap_ids(Particle *part, int64_t m, const int32_t *orig, hipStream_t s)
{
    if (m > 0) k_remap_ids<<<grid_for(m), kTB, 0, s>>>(part, m, orig);
    return hipGetLastError();
}

hipError_t launch_range_check(const double *xyz, int64_t n, const Grid &G, int32_t *err, hipStream_t s)
{
    if (n > 0) k_range_check<<<grid_for(n), kTB, 0, s>>>(xyz, n, G, err);
    return hipGetLastError();
}

hipError_t launch_slab_cert(const Particle *part, const int32_t *list, int64_t m, const double *lim, double zlo,
                            double zhi, double per, double eps, uint8_t bit, uint8_t *status, hipStream_t s)
{
    if (m > 0) k_slab_cert<<<grid_for(m), kTB, 0, s>>>(part, list, m, lim, zlo, zhi, per, eps, bit, status);
    return hipGetLastError();
}

hipError_t launch_count_bit(const uint8_t *st, int64_t n, uint8_t bit, int32_t *out, hipStream_t s)
{
    if (n > 0) k_count_bit<<<grid_for(n), kTB, 0, s>>>(st, n, bit, out);
    return hipGetLastError();
}

hipError_t launch_bin_count(const double *xyz, int64_t n, int dim, const Tess *tess, const int32_t *ptess,
                            int32_t *blk, int32_t *rank, int32_t *count, int32_t *err, hipStream_t s)
{
    k_bin_count<<<grid_for(n), kTB, 0, s>>>(xyz, n, dim, tess, ptess, blk, rank, count, err);
    return hipGetLastError();
}

hipError_t launch_scan(const int32_t *count, int32_t *start, int64_t nb, int32_t *tmp, hipStream_t s)
{
    return scan_impl<int32_t>(count, nb, start, tmp, s);
}

hipError_t launch_scatter(const double *xyz, int64_t n, int dim, const int32_t *ptess, const int32_t *blk,
                          const int32_t *rank, const int32_t *start, int32_t *sid, Particle *part, int32_t *inv,
                          hipStream_t s)
{
    k_scatter_ids<<<grid_for(n), kTB, 0, s>>>(n, blk, rank, start, sid);
    k_rank_scatter<<<grid_for(n), kTB, 0, s>>>(xyz, n, dim, ptess, blk, start, sid, part, inv);
    return hipGetLastError();
}

hipError_t launch_subset_list(const int64_t *ids, int64_t m, int64_t n, const int32_t *inv, int32_t *out,
                              int32_t *err, hipStream_t s)
{
    if (m > 0) k_subset_list<<<grid_for(m), kTB, 0, s>>>(ids, m, n, inv, out, err);
    return hipGetLastError();
}

hipError_t launch_radii(const double *rin, int64_t n, const int32_t *inv, double *rad, hipStream_t s)
{
    k_radii<<<grid_for(n), kTB, 0, s>>>(rin, n, inv, rad);
    return hipGetLastError();
}

hipError_t launch_radii_check(const double *rin, int64_t n, double *rmax, int32_t *err, hipStream_t s)
{
    k_fill<<<1, kTB, 0, s>>>(reinterpret_cast<int32_t *>(rmax), 2, 0);
    const int g = std::min(grid_for(n), 1024);
    k_radii_check<<<g, kTB, 0, s>>>(rin, n, reinterpret_cast<unsigned long long *>(rmax), err);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s)
{
    if (n > 0) k_fill_u8<<<grid_for(n), kTB, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    k_fill<<<grid_for(n), kTB, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_nbr_offsets(const int32_t *nf, int64_t n, int64_t *offsets, int32_t *tmp, hipStream_t s)
{
    return scan_impl<int64_t>(nf, n, offsets, reinterpret_cast<int64_t *>(tmp), s);
}

hipError_t launch_nbr_compact(const int32_t *nf, int64_t n, const int32_t *nbr, const uint8_t *nsh, int64_t *offsets,
                              int32_t *ids, uint8_t *shifts, int32_t *tmp, hipStream_t s)
{
    (void)tmp;
    const int64_t groups = (n + kNbrGroups - 1) / kNbrGroups;
    const int blocks = (int)std::min<int64_t>(std::max<int64_t>(groups, 1), 65536);
    k_nbr_compact<<<blocks, kTB, 0, s>>>(nf, n, nbr, nsh, offsets, ids, shifts);
    return hipGetLastError();
}

int device_cu_count()
{
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) return 256;
    return cu;
}

}  // namespace vc
