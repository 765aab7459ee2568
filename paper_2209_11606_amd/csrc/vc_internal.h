// vc_internal.h -- data shared by the host runtime and the HIP kernels of
// the Voronoi cell library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vc {

constexpr int kWave = 64;
constexpr int kFoLen = 32;      // face-order vector length
constexpr int kMaxNbr = 64;     // neighbour slots per cell in the fixed-stride scratch
constexpr int kOffRadius = 4;   // Chebyshev radius of the precomputed block-offset list
constexpr int kNoShift = 62;    // image code of the zero shift: 25*2 + 5*2 + 2
// Edge-graph record of one cell for the Weinberg codes: [V][D low][D high],
// the degree of each vertex, then each vertex's neighbours in rotation
// order (3 + V + D bytes, D = 2E).  A cell whose record does not fit has no
// code.  Every vertex has degree >= 3, so V <= (kWbStride - 3) / 4.
constexpr int kWbStride = 384;
constexpr int kWbMaxD = kWbStride - 3;
constexpr int kWbMaxV = (kWbStride - 3) / 4;
// Phase profile of the grouped cell kernel (built with -DVC_PHASE_CLOCKS
// only): diagnostic slots kPhaseClk + k hold the shader-clock cycles the
// waves spent in phase k (0 NEW, 1 GATHER, 2 BATCH, 3 TEST, 4 CUT, 5 STATS,
// 7 the failure path and loop control), kPhaseCnt + k the number of times
// the phase body ran on a wave (slot 6: TEST iterations).
// status flag of the chunked form (a cell to compute again with a wider
// halo); never left in a returned result
constexpr int kStatusSlab = 128;

constexpr int kPhaseSlots = 8;
constexpr int kPhaseClk = 16;
constexpr int kPhaseCnt = 24;

// One particle in the block-sorted array (32 bytes: one aligned pair of
// 16-byte loads per lane).
struct alignas(32) Particle {
    double x, y, z;
    int32_t id;   // input index (over all tessellations of a batch)
    int32_t tess; // tessellation the particle belongs to
};

// Geometry of a container's grid of blocks (section 2.1.1, 2.1.4).
struct Grid {
    int dim;
    int g[3];         // blocks per axis
    int per[3];       // periodic flags
    double lo[3], hi[3], L[3];
    double bs[3];     // block side L/g
    double inv_bs[3]; // g/L
    int64_t nb;       // total blocks
};

// Block index of a coordinate along one axis: floor((x - lo) g / L), clamped.
__host__ __device__ inline int block_coord(const Grid &G, double x, int d)
{
    double t = (x - G.lo[d]) * G.inv_bs[d];
    int k = (int)floor(t);
    if (k < 0) k = 0;
    if (k >= G.g[d]) k = G.g[d] - 1;
    return k;
}

// One tessellation of a container: its grid, and where its particles and
// blocks start in the shared arrays.
struct Tess {
    Grid G;
    int32_t pbase;   // first particle (input index and sorted index)
    int32_t pcount;
    int32_t bbase;   // first block in the shared block arrays
    int32_t pad;
    double bsmin2;   // squared smallest block side
    double clip_half; // half the side of the clip cube (section 3.1.3), 0: none
};

// Block offset relative to a particle's own block, for a particle in the
// lower half of its block along every axis (the kernels reflect the offsets
// per axis to make it so).  m / 4 * bsmin2 bounds from below the squared
// distance from the particle to this block and to every block after it in
// the list, and to every block outside the list (m is in quarters of a
// squared block side); the list is in nearest-first order of the expected
// gap.
struct Offset {
    int dx, dy, dz, m;
};

// Arguments of the cell kernels.
struct CellArgs {
    const Tess *tess;          // tessellations (one for a plain container)
    const Particle *part;      // block-sorted particles
    const int32_t *start;      // block start offsets (global particle index), nb_total + 1
    const Offset *offs;        // nearest-first block offsets
    int noff;
    int off_radius;            // Chebyshev radius covered by offs
    int ncell;                 // cells in this launch
    const int32_t *ncell_dev;  // if set: the cell count is read from device memory
    const int32_t *cell_list;  // sorted indices to compute (NULL: 0..ncell-1)
    int32_t *queue;            // work-queue head (zeroed before the launch)
    int chunk;                 // cells per queue grab
    int vcap;                  // > 0: a cell with more live vertices moves to the spill pass
    double tau;                // FP64 band, relative
    float tau32;               // FP32 band of the filter, relative
    const double *rad;         // radii by sorted index (radical tessellation), or NULL
    const double *rmax;        // largest radius (device scalar)
    uint32_t mask;             // statistics mask
    // outputs, by particle id
    double *vol;
    double *cen;
    double *perim;             // 2D
    int32_t *nv, *ne, *nf;
    uint8_t *fo;
    int32_t *nbr;              // id * kMaxNbr + k
    uint8_t *nsh;
    uint8_t *status;
    // spill queue for cells beyond the kernel's capacity
    int32_t *spill_list;
    int32_t *spill_count;
    unsigned long long *diag;  // VC_DIAG_LEN counters
    double *xscratch;          // per-wave workspace of the exact predicate
    int xscratch_len;          // doubles per wave
    uint8_t *wbg;              // Weinberg codes requested: edge-graph records, id * kWbStride
    int32_t *wbl;              // code length 2E of each record, 0: no code
    // the chunked form: each finished cell's squared search radius, by
    // sorted index (NULL: not kept)
    double *lim_out;
};

// Launchers (defined in the .hip translation unit).
hipError_t launch_bin_count(const double *xyz, int64_t n, int dim, const Tess *tess, const int32_t *ptess,
                            int32_t *blk, int32_t *rank, int32_t *count, int32_t *err, hipStream_t s);
hipError_t launch_scan(const int32_t *count, int32_t *start, int64_t nb, int32_t *tmp, hipStream_t s);
hipError_t launch_scatter(const double *xyz, int64_t n, int dim, const int32_t *ptess, const int32_t *blk,
                          const int32_t *rank, const int32_t *start, int32_t *sid, Particle *part, int32_t *inv,
                          hipStream_t s);
hipError_t launch_subset_list(const int64_t *ids, int64_t m, int64_t n, const int32_t *inv, int32_t *out,
                              int32_t *err, hipStream_t s);
hipError_t launch_radii(const double *rin, int64_t n, const int32_t *inv, double *rad, hipStream_t s);
hipError_t launch_radii_check(const double *rin, int64_t n, double *rmax, int32_t *err, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_cells(const CellArgs &a, int precision, int slots, int waves, hipStream_t s);
hipError_t launch_cells_handoff(const CellArgs &a, int waves, hipStream_t s);
hipError_t launch_cells_spill(const CellArgs &a, int waves, hipStream_t s);
hipError_t launch_cells_group(const CellArgs &a, int precision, int cells_per_wave, int waves, hipStream_t s);
hipError_t launch_cells2d(const CellArgs &a, int precision, int waves, hipStream_t s);
hipError_t launch_cells2d_spill(const CellArgs &a, int waves, hipStream_t s);
// queue: three zeroed counters; big: n ints of scratch (cells for the
// general kernel)
hipError_t launch_weinberg(const uint8_t *wbg, const int32_t *wbl, const int64_t *off, int64_t n, uint8_t *codes,
                           int32_t *sym, uint8_t *chiral, int32_t *queue, int32_t *big, int waves, hipStream_t s);
hipError_t launch_nbr_compact(const int32_t *nf, int64_t n, const int32_t *nbr, const uint8_t *nsh,
                              int64_t *offsets, int32_t *ids, uint8_t *shifts, int32_t *tmp, hipStream_t s);
hipError_t launch_nbr_offsets(const int32_t *nf, int64_t n, int64_t *offsets, int32_t *tmp, hipStream_t s);
int device_cu_count();
// the chunked form: tiles of the order-preserving selection (count and start
// arrays hold pick_tiles(n) and pick_tiles(n) + 1 entries; the scan's
// workspace as for launch_scan over pick_tiles(n) entries)
int64_t pick_tiles(int64_t n);
hipError_t launch_slab_pick(const double *xyz, int64_t n, const Grid &G, int e0, int elen, int k0, int klen,
                            const uint8_t *want, uint8_t wbit, double *oxyz, int32_t *orig, uint8_t *own,
                            int32_t *cnt, int32_t *start, int32_t *tmp, bool scatter, hipStream_t s);
hipError_t launch_own_count(const double *xyz, int64_t n, const Grid &G, int k0, int klen, const uint8_t *want,
                            uint8_t wbit, int32_t *cnt, int32_t *start, int32_t *tmp, hipStream_t s);
hipError_t launch_slot_list(const Particle *part, const uint8_t *own, int64_t m, int32_t *list, int32_t *cnt,
                            int32_t *start, int32_t *tmp, hipStream_t s);
hipError_t launch_remap_ids(Particle *part, int64_t m, const int32_t *orig, hipStream_t s);
hipError_t launch_range_check(const double *xyz, int64_t n, const Grid &G, int32_t *err, hipStream_t s);
hipError_t launch_slab_cert(const Particle *part, const int32_t *list, int64_t m, const double *lim, double zlo,
                            double zhi, double per, double eps, uint8_t bit, uint8_t *status, hipStream_t s);
hipError_t launch_count_bit(const uint8_t *st, int64_t n, uint8_t bit, int32_t *out, hipStream_t s);

}  // namespace vc
