/*
 * vorohip.h -- C ABI of the MI355X (gfx950) Voronoi cell library.
 *
 * The library computes, for every particle of a container, its Voronoi cell
 * by the cell-based method of Voro++ (Lu, Lazar & Rycroft, section 2.1): the
 * cell starts as the container box (Eq. 1-2), is cut by the bisector
 * half-space of each nearby particle (Eq. 3) taken from a grid of blocks in
 * nearest-first order (section 2.1.3), and stops once no remaining particle
 * can reach it (radius bound, section 2.1.3).  Statistics of each cell are
 * then written out.
 *
 * Conventions shared by every call:
 *  - Every function returns a vc_status: VC_OK (0) or a negative error code.
 *    The message of the last error on the calling thread is vc_last_error().
 *    Nothing throws across this boundary.
 *  - Pointers named "device" are HIP device memory; "host" pointers are host
 *    memory.  Positions may be either (the library detects which).
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    All GPU work of a call is enqueued on that stream; a call returns once
 *    its work is enqueued, except where stated.
 *  - Handles are owned by the library and freed by the matching destroy call.
 *    A container or result may be used by one host thread at a time.
 *  - Per-cell outputs are indexed by input order (particle id).
 */
#ifndef VOROHIP_H
#define VOROHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int vc_status;
enum {
    VC_OK = 0,
    VC_E_ARG = -1,       /* null pointer, n < 1, hi <= lo, dim not 2 or 3, bad option */
    VC_E_RANGE = -2,     /* a coordinate outside the box, or NaN / Inf */
    VC_E_DUPLICATE = -3, /* two particles (or a particle and an image) coincide */
    VC_E_NOMEM = -4,     /* device allocation failed */
    VC_E_HIP = -5,       /* a HIP runtime call failed */
    VC_E_CAPACITY = -6,  /* a cell exceeded the largest capacity the library has */
    VC_E_STATE = -7      /* call made on a handle in the wrong state */
};

/* arithmetic of the plane-side vertex test (a5) */
enum { VC_FP64 = 0, VC_F32_FILTER = 1 };

/* statistics mask for vc_compute */
enum {
    VC_VOLUME = 1,          /* volume (3D) or area (2D) */
    VC_CENTROID = 2,        /* centroid relative to the particle */
    VC_COUNTS = 4,          /* vertex, edge and face counts */
    VC_FACE_ORDERS = 8,     /* face-order vector (3D) */
    VC_NEIGHBORS = 16,      /* neighbour list, CSR (implies the counts' face count) */
    VC_NEIGHBOR_COUNT = 32, /* number of neighbours (faces) only */
    VC_DIAG = 64,           /* run counters (exact decisions, rechecks, spills, ...) */
    VC_ALL = 127,           /* every field above */
    VC_PERIMETER = 128,     /* 2D only: cell perimeter */
    VC_WEINBERG = 256       /* 3D only: Weinberg code of each cell (VoroTop's
                               topology code, section 5; Weinberg 1966), its
                               symmetry count and chirality */
};

/* result fields for vc_result_get / vc_result_copy */
enum {
    VC_F_VOLUME = 0,      /* double[n] */
    VC_F_CENTROID = 1,    /* double[n * dim], particle-major */
    VC_F_NV = 2,          /* int32[n] vertex count (counts fit 16 bits; 32-bit arrays
                             are what torch and numpy index with directly) */
    VC_F_NE = 3,          /* int32[n] edge count */
    VC_F_NF = 4,          /* int32[n] face (neighbour) count */
    VC_F_FACE_ORDERS = 5, /* uint8[n * VC_FO_LEN]: fo[k] = faces with k edges */
    VC_F_NBR_OFFSETS = 6, /* int64[n + 1] CSR offsets into the two arrays below */
    VC_F_NBR_IDS = 7,     /* int32[total]: neighbour particle id, or -1..-6 for the
                             walls x-, x+, y-, y+, z-, z+ (2D: -1..-4) */
    VC_F_NBR_SHIFTS = 8,  /* uint8[total]: periodic image code
                             25(s_z+2) + 5(s_y+2) + (s_x+2), 62 = no shift;
                             base 5, shifts -2..2: in a periodic box that holds
                             few particles a cell reaches images two periods
                             away */
    VC_F_STATUS = 9,      /* uint8[n]: VC_CELL_* */
    VC_F_DIAG = 10,       /* int64[VC_DIAG_LEN] */
    VC_F_PERIMETER = 11,  /* double[n], 2D */
    VC_F_WB_OFFSETS = 12, /* int64[n + 1] CSR offsets into the Weinberg codes */
    VC_F_WB_CODES = 13,   /* uint8[total]: each cell's code, 2E vertex numbers;
                             none (length 0) for an empty or failed cell and
                             for a cell whose edge graph exceeds the record
                             (3 + V + 2E > 384 bytes) */
    VC_F_WB_SYM = 14,     /* int32[n]: the number of (starting dart, sense)
                             pairs that give the code = the order of the edge
                             graph's symmetry group; 0: no code */
    VC_F_WB_CHIRAL = 15   /* uint8[n]: 1 when only one rotational sense gives
                             the code (the cell has no mirror symmetry) */
};
/* The Weinberg code (VC_WEINBERG).  The edges of a 3D cell, each taken as
 * two darts (directed edges), are walked once each: from a starting dart,
 * on reaching a vertex for the first time leave by the next dart in the
 * rotation around that vertex after the one just arrived on; on reaching a
 * vertex seen before, go back along the same edge unless that was done
 * already, and else leave by the first unused dart in the rotation after the
 * one just arrived on.  Vertices are numbered 1, 2, ... as first reached and
 * the walk's code is the number of the vertex each dart leaves (2E numbers,
 * starting with 1).  The cell's code is the lexicographically smallest walk
 * code over all 2E starting darts and both rotational senses: two cells have
 * the same code exactly when their edge graphs are isomorphic.  Vertices
 * where more than three faces meet (zero-length edges merged) are single
 * vertices of higher degree. */
#define VC_FO_LEN 32
#define VC_DIAG_LEN 32

/* per-cell status (VC_F_STATUS).  VC_CELL_SPILLED: complete, computed by a
   pass after the main one (the main kernel left it: beyond its vertex
   capacity, or, in the forms with several cells per wavefront, an extended
   cell whose search reaches past the nearest blocks or a cell with a side
   decision in the exact predicate's band, which only the one-cell kernel
   takes); VC_CELL_CAPACITY: not
   computed, beyond the last pass's capacity. */
enum { VC_CELL_OK = 0, VC_CELL_SPILLED = 1, VC_CELL_CAPACITY = 2, VC_CELL_DUPLICATE = 3,
       VC_CELL_SKIPPED = 4, /* not in the list of vc_compute_subset */
       VC_CELL_EMPTY = 5,   /* radical tessellation: the cell has no volume */
       VC_CELL_RANGE = 6,   /* vc_tessellate_noalloc only: a coordinate of the call
                               lies outside the box; no field of the call is valid */
       /* flag bit, OR-ed into VC_CELL_OK or VC_CELL_SPILLED: the cell is
          complete but one of its faces has VC_FO_LEN (32) or more edges, so
          the face-order vector does not count that face and sums to less
          than the face count (the other fields are exact) */
       VC_CELL_FO_OVERFLOW = 64 };

/* diagnostic counters (VC_F_DIAG) */
enum {
    VC_D_CANDIDATES = 0,  /* candidates taken in nearest-first order */
    VC_D_TESTS = 1,       /* plane-side tests (candidates x live vertices) */
    VC_D_CUTS = 2,        /* cuts that removed part of a cell */
    VC_D_NEWV = 3,        /* vertices created */
    VC_D_EXACT = 4,       /* side decisions taken exactly */
    VC_D_RECHECK = 5,     /* FP32 tests re-done in FP64 (VC_F32_FILTER) */
    VC_D_SPILLED = 6,     /* cells the main pass left to the later passes */
    VC_D_BLOCKS = 7,      /* blocks whose particles were loaded */
    VC_D_FALLBACK = 8,    /* cells that searched beyond the precomputed offsets */
    VC_D_SHELLS = 9,      /* Chebyshev shells of blocks searched beyond them
                             (section 2.1.3: the block bound ends the search) */
    VC_D_LOADED = 10,     /* particles loaded from the blocks (before the radius
                             and ball tests) */
    VC_D_RECOMPUTED = 11  /* vc_tessellate_slabs: cells computed again with a
                             wider halo */
    /* slots 16..31 are written only by a library built with the phase
       profile of the grouped cell kernel (VC_PHASE_CLOCKS): 16 + k holds the
       shader-clock cycles its waves spent in phase k (0 claim a cell and set
       up its box, 1 gather block counts, 2 load and sort a batch, 3 side
       tests, 4 cuts, 5 statistics, 7 failures and loop control) and 24 + k
       how many times the phase ran on a wave (30: side-test iterations) */
};

typedef struct {
    int dim;             /* 2 or 3 */
    double lo[3], hi[3]; /* box [lo, hi] per axis (first dim entries used) */
    int periodic[3];     /* nonzero: periodic axis */
    double n_opt;        /* target particles per block (section 2.1.4); <= 0: 5.0 */
    int grid[3];         /* explicit block counts; all 0: from n_opt */
    int precision;       /* VC_FP64 or VC_F32_FILTER */
    int slots;           /* triangles per lane in the main cell kernel (2 or 4); 0: auto */
    int waves;           /* resident cell waves launched; 0: auto */
    int chunk;           /* cells taken per work-queue grab; 0: auto */
    int cells_per_wave;  /* cells sharing one wavefront: 1, 2 or 4; 0: 1 */
    double clip;         /* > 0: every cell starts as the cube (square) of this side
                            centred on its particle, cut to the box (section 3.1.3:
                            clipped cells); faces of the clip cube are labelled
                            -7..-12 (x-, x+, y-, y+, z-, z+); 0: the whole box */
    int capacity;        /* vertex capacity of the main cell kernel: a cell that would
                            hold more vertices moves to the large-capacity spill pass
                            (the overflow policy of section 2.2.5 applied to cells);
                            0: the kernel's own capacity (slots x lanes); a value below
                            4 in 3D (3 in 2D), fewer than any cut cell has, sends every
                            cell that is cut at all to the pass */
    int force;           /* testing aid, VC_FORCE_* bits, 0 in normal use: take every
                            side decision through a slower stage that must give
                            the same result (the bands of section 2.2.2's filter
                            made wide enough to hold every test) */
} vc_options;

/* vc_options.force bits. VC_FORCE_RECHECK: every FP32 test of VC_F32_FILTER
   is taken as unsure and re-done in FP64; VC_FORCE_EXACT: every FP64 side test
   falls in the band and is decided by the exact predicate. Results are the
   same as without the bits; only the diagnostic counters and the time differ,
   except that with VC_FORCE_EXACT the forms with several cells per wavefront
   (which hold no exact predicate) leave every cell to the one-cell kernel:
   status VC_CELL_SPILLED, and volumes and centroids as that form computes
   them (equal to the default's up to rounding; topology identical). */
enum { VC_FORCE_RECHECK = 1, VC_FORCE_EXACT = 2 };

typedef struct vc_container vc_container;
typedef struct vc_result vc_result;
typedef struct vc_batch vc_batch;

/* Fill *opt with defaults for a box (dim, lo, hi, periodic). */
vc_status vc_options_init(vc_options *opt, int dim, const double *lo, const double *hi, const int *periodic);

/* Create a container and bin the particles into its grid of blocks
 * (section 2.1.1; the atomic slot capture of section 2.2.5 becomes a counting
 * sort).  xyz: n x dim doubles, particle-major, host or device.  A walled
 * axis requires lo <= x <= hi, a periodic axis lo <= x < hi; otherwise
 * VC_E_RANGE.  The library copies the positions; the caller keeps ownership
 * of xyz.  Block counts follow section 2.1.4 (lambda = (N/(N_opt V))^(1/d),
 * n_d = ceil(lambda L_d)) unless opt->grid is set.  Synchronises `stream`
 * once (to read the range check).  On success *out owns device memory. */
vc_status vc_container_create(const double *xyz, int64_t n, const vc_options *opt, void *stream,
                              vc_container **out);

/* Re-bin new positions of the same count into an existing container (the
 * container clearing and re-use of section 3.2): no allocation.  Same range rules and
 * errors as vc_container_create; synchronises `stream` once to read the
 * range check.  On VC_E_RANGE the container holds the rejected positions and
 * must be re-binned before the next vc_compute. */
vc_status vc_container_rebin(vc_container *c, const double *xyz, void *stream);

/* Make the container's tessellation the radical (power) Voronoi tessellation
 * of a polydisperse system (section 2.1.1): particle i, of radius r_i, owns
 * the points x with |x - p_i|^2 - r_i^2 <= |x - p_j|^2 - r_j^2 for every j.
 * Each bisector of Eq. 3 becomes the radical plane of the two particles,
 * n.x <= (|q|^2 + r_i^2 - r_j^2) / 2 with q the neighbour's position relative
 * to p_i, and the search radius of a cell whose farthest vertex lies at R
 * grows from 2R to R + sqrt(R^2 + r_max^2 - r_i^2).  A cell can come out
 * empty (a small particle inside the power range of larger neighbours): it
 * gets status VC_CELL_EMPTY, zero volume, centroid and counts, and no faces.
 * A cell that does not contain its particle has its centroid, as always,
 * relative to the particle.
 * radii: n doubles, finite and >= 0, by input index (host or device); the
 * library copies them and keeps them across vc_container_rebin.  radii = NULL
 * returns the container to the plain Voronoi tessellation.  Equal radii give
 * the Voronoi cells.  Errors: VC_E_ARG (null container), VC_E_RANGE (a
 * negative or non-finite radius; the container is then plain Voronoi),
 * VC_E_NOMEM.  Synchronises `stream` once (to read the range check). */
vc_status vc_container_set_radii(vc_container *c, const double *radii, void *stream);

/* Block counts the library uses for n particles in the box of *opt
 * (section 2.1.4: lambda = (N/(N_opt V))^(1/d), n_d = ceil(lambda L_d),
 * unless opt->grid is set).  Host only: touches no GPU.  grid_out[3]
 * receives the counts (1 on unused axes). */
vc_status vc_grid_size(const vc_options *opt, int64_t n, int *grid_out);

/* Copy the container's binning to host memory (synchronous): block_start
 * (nb + 1 int32, nb = product of the block counts, summed over tessellations
 * for a batch; pass NULL to skip) and the input ids in block-sorted order
 * (n int32; NULL to skip).  nb_out (may be NULL) receives nb. */
vc_status vc_container_blocks(const vc_container *c, int32_t *block_start, int32_t *sorted_ids, int64_t *nb_out);

/* Allocate a result for a container and a statistics mask (VC_* bits).  The
 * result owns device arrays sized for the container; it can be filled many
 * times. */
vc_status vc_result_create(const vc_container *c, uint32_t mask, vc_result **out);

/* Compute every cell of the container into r (section 2.1.2-2.1.3: box
 * start, nearest-first bisector cuts, radius-bound termination, statistics).
 * Asynchronous on `stream`. */
vc_status vc_compute(vc_container *c, vc_result *r, void *stream);

/* Compute the cells of a subset of the particles (the paper's subset and
 * ordered iterators, section 2.2.2): ids holds m input indices (0 <= m <= n,
 * each in [0, n); host or device int64 array, detected as for positions),
 * taken through the same work queue.  Only the listed cells' fields are
 * written; every other cell gets status VC_CELL_SKIPPED, face count 0 and an
 * empty neighbour list, and its other fields are left as they were.  A
 * listed cell is bitwise the cell vc_compute gives.  An index out of range
 * is VC_E_RANGE (checked before any cell is computed; a device list is
 * checked on the device, and the call then waits for that check).  A repeated
 * index computes its cell twice. */
vc_status vc_compute_subset(vc_container *c, vc_result *r, const int64_t *ids, int64_t m, void *stream);

/* The cells of one large 3D set computed in container-block chunks along z,
 * with scratch memory for one chunk at a time instead of the whole set (the
 * container's blocks of section 2.1.4 taken as the unit of work, as the
 * paper's parallel schedules take them, section 2.2.4).  The grid is the
 * set's own (vc_options as for vc_container_create).  Its layers of blocks
 * along z are cut into nslab chunks of about equal size; a chunk's container
 * holds the particles of its layers and of `halo` more layers on each side
 * (wrapped on a periodic z axis), binned on the set's grid, and computes the
 * cells of its own particles.  A particle beyond the widened range is
 * farther than a finished cell's search radius (section 2.1.3) unless the
 * cell's radius reaches past an end of the range; such cells are computed
 * again with the halo doubled until none is left.  So every cell equals the
 * one vc_compute gives on the whole set (topology and face orders exactly,
 * volume and centroid to rounding: candidates enter in the same order, but
 * a cell computed again may take them in a different one).
 *
 * xyz: n x 3 positions, device or host (host ones are copied to the device
 * first); nslab >= 1 (at most the number of layers), halo >= 1 layers.  mask:
 * VC_VOLUME, VC_CENTROID, VC_COUNTS, VC_FACE_ORDERS, VC_NEIGHBOR_COUNT and
 * VC_DIAG only (other bits are VC_E_ARG).  *out receives a new result of n cells by
 * input index, owned by the caller (vc_result_destroy); it belongs to no
 * container, and vc_result_kernel_ms gives the time of the whole chunked
 * computation.  Errors as for vc_container_create; the call returns when
 * the cells are computed. */
vc_status vc_tessellate_slabs(const double *xyz, int64_t n, const vc_options *opt, uint32_t mask, int nslab, int halo,
                              void *stream, vc_result **out);

/* Elapsed time in milliseconds of the main cell kernel of the last
 * vc_compute on r (HIP events recorded around that launch on its stream).
 * Waits for that kernel to finish. */
vc_status vc_result_kernel_ms(vc_result *r, float *ms);

/* Device pointer and element count of a result field (no copy): the per-cell
 * statistics the paper reads from each computed cell (section 2.1.2 and the
 * per-cell accessors of the example listing of section 2.2.3: volume,
 * centroid, counts, face orders, neighbours), here for all cells at once as
 * device arrays indexed by input order (this library's design; the paper
 * reads them from one cell object at a time).  The pointer stays valid
 * until vc_result_destroy.  For the neighbour id and shift arrays the count
 * is known only after the compute finished: this call synchronises the
 * stream of the last compute to read it.  Errors: VC_E_ARG (null pointer,
 * unknown field), VC_E_STATE (a field not in the statistics mask),
 * VC_E_HIP. */
vc_status vc_result_get(vc_result *r, int field, void **dev_ptr, int64_t *count);

/* Copy a result field to host memory (synchronous): the fields of
 * vc_result_get, for callers that want them on the host (the paper's
 * per-cell output loop of section 2.2.3, done once for every cell).
 * host_dst receives count elements of the field's type (the sizes listed
 * with VC_F_*); bytes must be >= that size, else VC_E_ARG; errors as for
 * vc_result_get. */
vc_status vc_result_copy(vc_result *r, int field, void *host_dst, int64_t bytes);

void vc_result_destroy(vc_result *r);
void vc_container_destroy(vc_container *c);

/* --- batches of independent tessellations (one persistent launch) --------- */

/* Create a batch of n_tess independent 3D containers sharing one set of
 * device arrays: many separate problems in one launch (the dynamic
 * scheduling of uneven work in section 2.2.4, applied across containers as
 * well as across cells; batching is this library's design, the paper
 * threads one container at a time).  xyz_concat holds all positions back to back (n_total x 3
 * doubles, host or device); offsets[n_tess + 1] (host) gives the first
 * particle of each tessellation (offsets[0] = 0, offsets[n_tess] = n_total,
 * every tessellation non-empty); opts[n_tess] (host) the box, periodicity and
 * grid of each.  precision, slots, waves and chunk are taken from opts[0].
 * Range rules and errors as for vc_container_create.  Results are indexed by
 * position in xyz_concat.  Synchronises `stream` once. */
vc_status vc_batch_create(const double *xyz_concat, const int64_t *offsets, int64_t n_tess,
                          const vc_options *opts, void *stream, vc_batch **out);

/* Re-bin new positions (same counts) into a batch; as vc_container_rebin. */
vc_status vc_batch_rebin(vc_batch *b, const double *xyz_concat, void *stream);

/* Radii of every particle of a batch (n_total doubles in xyz_concat order),
 * or NULL; as vc_container_set_radii, with r_max taken over the whole batch
 * (a looser but valid search bound). */
vc_status vc_batch_set_radii(vc_batch *b, const double *radii_concat, void *stream);

/* Allocate a result for a batch (fields as for a container, over all
 * particles of the batch). */
vc_status vc_batch_result_create(const vc_batch *b, uint32_t mask, vc_result **out);

/* Compute every cell of every tessellation in one persistent launch over a
 * device work queue (the dynamic schedule of section 2.2.4, on the GPU).  If
 * `graph` is nonzero the launch sequence is captured once into a hipGraph on
 * `stream` (which must not be the null stream) and replayed by later calls
 * with the same result and stream.  Asynchronous. */
vc_status vc_batch_compute(vc_batch *b, vc_result *r, int graph, void *stream);

/* Launch parameters chosen by vc_batch_tune. */
typedef struct {
    int slots;          /* triangles per lane: 2 or 4 (cell capacity 128 or 256 vertices) */
    int waves;          /* resident waves launched */
    int chunk;          /* cells per work-queue grab */
    int cells_per_wave; /* cells processed together by one wave */
    float ms;           /* kernel time of the winner on the tuning sample */
    int capacity;       /* vertex capacity before the spill pass (vc_options.capacity;
                           0: the form's own) */
} vc_tuning;

/* Autotuner (the launch choices the paper leaves to the OpenMP schedule,
 * section 2.2.4, made here by measurement): times each launch configuration
 * -- cells per wave and slots (the form), vertex capacity before the spill
 * pass (the form's own or three quarters of it), cells per work-queue grab,
 * resident waves -- on a sample of the batch's cells (32 contiguous runs in
 * block order, 1/16 of the cells and at least 262,144 of them, so that cells
 * share their blocks in the cache as in a full launch), each once untimed
 * and twice timed; then times the best configuration of each form on every
 * cell and keeps the fastest for later vc_batch_compute calls, returning it
 * in *best (may be NULL; best->ms is its time on every cell).  Overwrites
 * the contents of r.  Synchronous.  A later vc_batch_compute with graph
 * capture re-captures with the chosen parameters. */
vc_status vc_batch_tune(vc_batch *b, vc_result *r, void *stream, vc_tuning *best);

/* As vc_batch_tune, on a sample drawn only from the tessellations
 * members[0..m) (host int64 indices into the batch), the final check on all
 * of their cells: the launch form best for one class of input.  The choice is kept for the whole batch, like
 * vc_batch_tune's.  Errors: VC_E_ARG (null or empty list), VC_E_RANGE (an
 * index outside the batch), VC_E_STATE, VC_E_NOMEM, VC_E_HIP. */
vc_status vc_batch_tune_members(vc_batch *b, vc_result *r, const int64_t *members, int64_t m, void *stream,
                                vc_tuning *best);

void vc_batch_destroy(vc_batch *b);

/* Measured vector FMA rate of the current device: the compute roof of the
 * cell kernels, which are bound by FP64 vector arithmetic.  precision:
 * VC_FP64, or VC_F32_FILTER for FP32 lanes (unpacked: the library is built
 * without packed FP32 instructions).
 * Runs one untimed and `reps` timed launches of eight independent FMA
 * chains per lane on every compute unit, on `stream`, and returns the best
 * rate in *tflops (10^12 flops/s, an FMA counted as 2).  Allocates and frees
 * its own device buffer; synchronous.  VC_E_ARG for a null tflops, reps < 1
 * or another precision. */
vc_status vc_device_fma_rate(int precision, int reps, void *stream, double *tflops);

/* The allocation-free form of vc_container_create followed by vc_compute,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  It calls
 * no hipMalloc, hipFree or other allocating routine: the block-sorted
 * particles, the binning arrays, the work-queue counters, the spill list
 * and the exact predicate's workspace live in one file-scope device array of
 * about 16.0 MiB that each GPU the library runs on holds until the process
 * ends.  Inputs and outputs are the caller's device memory:
 *   xyz: n x dim doubles (particle-major), 1 <= n <= 65536, inside the box
 *   of *opt (a coordinate outside it marks every cell VC_CELL_RANGE, on the
 *   device: the call does not synchronise); the grid of *opt may hold at
 *   most 65536 blocks; no radii.  Launch fields of *opt are used as by
 *   vc_container_create (waves capped at 512).
 *   vol (n), cen (3n), nv, ne (n), fo (n x VC_FO_LEN): written when non-NULL;
 *   nf (n) and status (n) are required.  Fields are indexed by input order
 *   and equal those of vc_compute with the same options.
 * Errors (host side, before any work is enqueued): VC_E_ARG for a null
 * required pointer, n or the block count beyond its maximum, host memory,
 * or bad options.  Asynchronous on `stream`.  The first call on a device
 * sets the array up (it takes its address and copies the block-offset
 * lists into it, synchronously), so make that call outside graph capture.
 * Every call on a device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (other streams, other threads)
 * race and must be serialised by the caller. */
vc_status vc_tessellate_noalloc(const double *xyz, int64_t n, const vc_options *opt, double *vol, double *cen,
                                int32_t *nv, int32_t *ne, int32_t *nf, uint8_t *fo, uint8_t *status, void *stream);

/* Message of the last error on the calling thread ("" if none). */
const char *vc_last_error(void);

/* Library version string. */
const char *vc_version(void);

#ifdef __cplusplus
}
#endif
#endif
