// api.cpp -- host runtime behind the C ABI of vorohip.h: argument checks,
// grid sizing (section 2.1.4), device allocation, the binning sequence, the
// nearest-first block-offset list, cell-kernel launches with the spill pass,
// neighbour-list compaction, batches of tessellations with hipGraph replay,
// and the launch-parameter autotuner.
//
// A container holds one or more tessellations in shared device arrays: the
// particles of all of them sorted block by block, one block-start array over
// all blocks, and a Tess record per tessellation (its grid and the first
// particle and block).  A plain container is the one-tessellation case.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/vorohip.h"
#include "peak.h"
#include "vc_internal.h"

using namespace vc;

namespace {

thread_local std::string g_err;

vc_status fail(vc_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return fail(VC_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
vc_status dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(VC_E_NOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    return VC_OK;
}

bool is_device_ptr(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Block offsets up to Chebyshev radius kOffRadius in nearest-first order for
// a particle in the lower half of its block along every axis (the kernels
// reflect the offsets per axis so that a particle's own half is that lower
// half): by the expected squared gap to the block, then by centre distance,
// then lexicographically (so the order is fixed).  With the particle uniform
// on [0, 1/2) of a block side, the expected squared gap along one axis, in
// twelfths of a squared side, is 0 for d = 0, 12a^2 + 6a + 1 for d = -(a+1)
// (the near side) and 12d^2 - 6d + 1 for d > 0 (the far side).
//
// Each entry carries the stopping bound of the search (section 2.1.3): the
// smallest guaranteed squared gap, in quarters of a squared block side, over
// it and every later entry.  In the reflected frame the gap along an axis is
// at least (|d| - 1) sides on the near side and (d - 1/2) sides on the far
// side, so one axis contributes 4 (|d| - 1)^2 or (2d - 1)^2 quarters.  Blocks
// outside the list (Chebyshev radius kOffRadius + 1 and beyond) are at least
// kOffRadius sides away, so the bound is capped at 4 kOffRadius^2: stopping
// at an entry then also covers every block beyond the list, and a cell
// reaching farther searches the whole list and goes on shell by shell.
std::vector<Offset> build_offsets(int dim)
{
    struct E { int g, e, c, dx, dy, dz; };
    auto eg = [](int d) {
        if (d == 0) return 0;
        if (d < 0) {
            const int a = -d - 1;
            return 12 * a * a + 6 * a + 1;
        }
        return 12 * d * d - 6 * d + 1;
    };
    auto gq = [](int d) {
        if (d == 0) return 0;
        if (d < 0) return 4 * (-d - 1) * (-d - 1);
        return (2 * d - 1) * (2 * d - 1);
    };
    std::vector<E> v;
    int rz = dim == 3 ? kOffRadius : 0;
    for (int dz = -rz; dz <= rz; dz++)
        for (int dy = -kOffRadius; dy <= kOffRadius; dy++)
            for (int dx = -kOffRadius; dx <= kOffRadius; dx++) {
                int d[3] = {dx, dy, dz};
                int g = 0, c = 0, e = 0;
                for (int k = 0; k < 3; k++) {
                    g += gq(d[k]);
                    c += d[k] * d[k];
                    e += eg(d[k]);
                }
                v.push_back({g, e, c, dx, dy, dz});
            }
    std::sort(v.begin(), v.end(), [](const E &a, const E &b) {
        if (a.e != b.e) return a.e < b.e;
        if (a.c != b.c) return a.c < b.c;
        if (a.dz != b.dz) return a.dz < b.dz;
        if (a.dy != b.dy) return a.dy < b.dy;
        return a.dx < b.dx;
    });
    std::vector<Offset> out(v.size());
    int rest = 4 * kOffRadius * kOffRadius;
    for (size_t i = v.size(); i-- > 0;) {
        rest = std::min(rest, v[i].g);
        out[i] = Offset{v[i].dx, v[i].dy, v[i].dz, rest};
    }
    return out;
}

vc_status check_options(const vc_options *o)
{
    if (!o) return fail(VC_E_ARG, "options: null pointer");
    if (o->dim != 2 && o->dim != 3) return fail(VC_E_ARG, "options: dim must be 2 or 3 (got %d)", o->dim);
    for (int d = 0; d < o->dim; d++) {
        if (!std::isfinite(o->lo[d]) || !std::isfinite(o->hi[d]) || !(o->hi[d] > o->lo[d]))
            return fail(VC_E_ARG, "options: box axis %d needs finite lo < hi", d);
        if (o->grid[d] < 0) return fail(VC_E_ARG, "options: negative grid size");
    }
    if (o->precision != VC_FP64 && o->precision != VC_F32_FILTER)
        return fail(VC_E_ARG, "options: precision must be VC_FP64 or VC_F32_FILTER");
    if (o->slots != 0 && o->slots != 2 && o->slots != 4) return fail(VC_E_ARG, "options: slots must be 0, 2 or 4");
    if (o->waves < 0 || o->chunk < 0) return fail(VC_E_ARG, "options: negative waves or chunk");
    if (o->cells_per_wave != 0 && o->cells_per_wave != 1 && o->cells_per_wave != 2 && o->cells_per_wave != 4)
        return fail(VC_E_ARG, "options: cells_per_wave must be 0, 1, 2 or 4");
    if (!std::isfinite(o->clip) || o->clip < 0.0) return fail(VC_E_ARG, "options: clip must be finite and >= 0");
    if (o->capacity < 0) return fail(VC_E_ARG, "options: capacity must be >= 0");
    if (o->force & ~(VC_FORCE_RECHECK | VC_FORCE_EXACT))
        return fail(VC_E_ARG, "options: force holds bits other than VC_FORCE_RECHECK | VC_FORCE_EXACT");
    return VC_OK;
}

// Section 2.1.4: lambda = (N / (N_opt V))^(1/d), n_d = ceil(lambda L_d).
Grid size_grid(const vc_options &o, int64_t n)
{
    Grid G;
    std::memset(&G, 0, sizeof G);
    G.dim = o.dim;
    double vol = 1.0;
    for (int d = 0; d < o.dim; d++) vol *= (o.hi[d] - o.lo[d]);
    double nopt = o.n_opt > 0 ? o.n_opt : 5.0;
    double lam = std::pow((double)n / (nopt * vol), 1.0 / o.dim);
    bool explicit_grid = o.grid[0] > 0;
    G.nb = 1;
    for (int d = 0; d < 3; d++) {
        if (d < o.dim) {
            G.lo[d] = o.lo[d];
            G.hi[d] = o.hi[d];
            G.per[d] = o.periodic[d] ? 1 : 0;
            long long g = explicit_grid ? o.grid[d] : (long long)std::ceil(lam * (o.hi[d] - o.lo[d]));
            G.g[d] = (int)std::max(1LL, std::min(g, 1LL << 20));
        } else {
            G.lo[d] = 0.0;
            G.hi[d] = 1.0;
            G.per[d] = 0;
            G.g[d] = 1;
        }
        G.L[d] = G.hi[d] - G.lo[d];
        G.bs[d] = G.L[d] / G.g[d];
        G.inv_bs[d] = G.g[d] / G.L[d];
        G.nb *= G.g[d];
    }
    return G;
}

// Side-test bands of the kernels: FP64 decisions within tau * M go to the
// exact predicate, FP32 filter decisions within tau32 * M to FP64. The
// VC_FORCE_* bits widen a band past every test.
void set_bands(CellArgs &A, int force)
{
    A.tau = (force & VC_FORCE_EXACT) ? 0x1p+600 : 0x1p-30;
    A.tau32 = (force & VC_FORCE_RECHECK) ? 0x1p+100f : 0x1p-21f;
}

struct Launch {
    int slots = 2, waves = 0, chunk = 4, cpw = 1;
    int vcap = 0;  // vertex capacity before the spill pass (0: the kernel's own)
};

}  // namespace

struct vc_container {
    int dim = 3;
    int64_t n = 0;
    int precision = VC_FP64;
    int force = 0;               // VC_FORCE_* bits
    std::vector<Tess> htess;
    Tess *tess = nullptr;
    int32_t *ptess = nullptr;    // tessellation of each input particle (batches only)
    int64_t nb = 0;              // blocks over all tessellations
    double *xyz = nullptr;       // device copy of the input positions (n x dim)
    Particle *part = nullptr;    // block-sorted particles
    int32_t *start = nullptr;    // nb + 1
    int32_t *count = nullptr;    // nb
    int32_t *blk = nullptr;      // n
    int32_t *rank = nullptr;     // n
    int32_t *sid = nullptr;      // n: input index at each provisional slot
    int32_t *inv = nullptr;      // n: sorted slot of each input index
    int32_t *subset = nullptr;   // n: sorted slots of a subset (vc_compute_subset), on first use
    int64_t *subset_ids = nullptr; // n: the subset's input indices copied from the host, on first use
    int32_t *err = nullptr;      // range-error flag
    int32_t *scan_tmp = nullptr;
    // radical tessellation (vc_container_set_radii): radii by input index,
    // by sorted slot (redone at every binning), and their maximum
    bool radical = false;
    double *rad_in = nullptr;
    double *rad = nullptr;
    double *rmax = nullptr;
    Offset *offs = nullptr;
    int noff = 0;
    int32_t *queue = nullptr;    // [0]: main queue head, [1]: spill queue head, [2]: spill count,
                                 // [3..5]: the Weinberg code kernels' heads and list count
    int32_t *spill_list = nullptr;
    int32_t *spill_list2 = nullptr;  // 3D: overflows of the first spill pass
    int32_t *sample_list = nullptr;  // tuning sample (batches)
    int nsample = 0;
    double *xscratch = nullptr;
    int xscratch_len = 3072;  // doubles: radical offsets make the expansions up to ~1.7x longer
    int max_waves = 0;
    Launch launch;
    // graph replay (batches)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const vc_result *graph_r = nullptr;
    hipStream_t graph_stream = nullptr;
};

struct vc_batch : vc_container {
};

struct vc_result {
    const vc_container *c = nullptr;
    uint32_t mask = 0;
    int64_t n = 0;
    int dim = 3;
    double *vol = nullptr, *cen = nullptr, *perim = nullptr;
    int32_t *nv = nullptr, *ne = nullptr, *nf = nullptr;
    uint8_t *fo = nullptr;
    int32_t *nbr = nullptr;  // fixed-stride scratch
    uint8_t *nsh = nullptr;
    int64_t *off = nullptr;  // CSR offsets (n + 1)
    int32_t *ids = nullptr;
    uint8_t *shifts = nullptr;
    int32_t *scan_tmp = nullptr;
    uint8_t *status = nullptr;
    // Weinberg codes: edge-graph records (n x kWbStride), code lengths, CSR
    // offsets and codes, symmetry counts, chirality
    uint8_t *wbg = nullptr;
    int32_t *wbl = nullptr;
    int64_t *wb_off = nullptr;
    uint8_t *wb_codes = nullptr;
    int32_t *wb_sym = nullptr;
    uint8_t *wb_chiral = nullptr;
    unsigned long long *diag = nullptr;
    hipStream_t last_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the main cell kernel
    hipEvent_t ev2 = nullptr;                 // after the spill passes
};

namespace {

void release_graph(vc_container *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_r = nullptr;
}

void free_container(vc_container *c)
{
    if (!c) return;
    release_graph(c);
    void *ps[] = {c->tess, c->ptess, c->xyz, c->part, c->start, c->count, c->blk, c->rank, c->sid, c->inv, c->subset, c->subset_ids, c->err, c->scan_tmp,
                  c->rad_in, c->rad, c->rmax, c->offs, c->queue, c->spill_list, c->spill_list2, c->sample_list,
                  c->xscratch};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    delete c;
}

void free_result(vc_result *r)
{
    if (!r) return;
    void *ps[] = {r->vol, r->cen, r->perim, r->nv, r->ne, r->nf, r->fo, r->nbr, r->nsh, r->off, r->ids, r->shifts,
                  r->scan_tmp, r->status, r->diag, r->wbg, r->wbl, r->wb_off, r->wb_codes, r->wb_sym, r->wb_chiral};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    if (r->ev0) (void)hipEventDestroy(r->ev0);
    if (r->ev1) (void)hipEventDestroy(r->ev1);
    if (r->ev2) (void)hipEventDestroy(r->ev2);
    delete r;
}

vc_status bin(vc_container *c, hipStream_t s)
{
    HIP_TRY(launch_fill_i32(c->count, c->nb, 0, s));
    HIP_TRY(launch_fill_i32(c->err, 1, 0, s));
    HIP_TRY(launch_bin_count(c->xyz, c->n, c->dim, c->tess, c->ptess, c->blk, c->rank, c->count, c->err, s));
    HIP_TRY(launch_scan(c->count, c->start, c->nb, c->scan_tmp, s));
    HIP_TRY(launch_scatter(c->xyz, c->n, c->dim, c->ptess, c->blk, c->rank, c->start, c->sid, c->part, c->inv, s));
    if (c->radical) HIP_TRY(launch_radii(c->rad_in, c->n, c->inv, c->rad, s));
    return VC_OK;
}

vc_status copy_in_and_bin(vc_container *c, const double *xyz, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(c->xyz, xyz, (size_t)c->n * c->dim * sizeof(double),
                           is_device_ptr(xyz) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    vc_status st = bin(c, s);
    if (st) return st;
    int32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (herr)
        return fail(VC_E_RANGE, "a coordinate lies outside the box (walled: lo <= x <= hi, periodic: lo <= x < hi) "
                                "or is not finite");
    return VC_OK;
}

// Build a container of one or more tessellations.  offsets: ntess + 1 particle
// offsets (host); opts: ntess options.
// Radii of the radical tessellation, or none (radii == NULL).
vc_status set_radii(vc_container *c, const double *radii, hipStream_t s)
{
    release_graph(c);  // a captured graph holds the previous cell arguments
    c->radical = false;
    if (!radii) return VC_OK;
    vc_status st;
    if (!c->rad_in && (st = dalloc(&c->rad_in, (size_t)c->n))) return st;
    if (!c->rad && (st = dalloc(&c->rad, (size_t)c->n))) return st;
    if (!c->rmax && (st = dalloc(&c->rmax, 1))) return st;
    HIP_TRY(hipMemcpyAsync(c->rad_in, radii, (size_t)c->n * sizeof(double),
                           is_device_ptr(radii) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fill_i32(c->err, 1, 0, s));
    HIP_TRY(launch_radii_check(c->rad_in, c->n, c->rmax, c->err, s));
    HIP_TRY(launch_radii(c->rad_in, c->n, c->inv, c->rad, s));
    int32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (herr) return fail(VC_E_RANGE, "a radius is negative or not finite");
    c->radical = true;
    return VC_OK;
}

vc_status create_common(vc_container *c, const double *xyz, const int64_t *offsets, int64_t ntess,
                        const vc_options *opts, hipStream_t s)
{
    const int dim = opts[0].dim;
    c->dim = dim;
    c->n = offsets[ntess];
    c->precision = opts[0].precision;
    c->force = opts[0].force;
    c->launch.slots = opts[0].slots > 0 ? opts[0].slots : 2;
    c->launch.chunk = opts[0].chunk > 0 ? opts[0].chunk : 4;
    c->launch.cpw = opts[0].cells_per_wave > 0 ? opts[0].cells_per_wave : 1;
    c->launch.vcap = opts[0].capacity;
    int cu = device_cu_count();
    c->launch.waves = opts[0].waves > 0 ? opts[0].waves : cu * 16;
    c->max_waves = std::max(c->launch.waves, cu * 32);
    c->htess.resize((size_t)ntess);
    int64_t nb = 0;
    for (int64_t t = 0; t < ntess; t++) {
        Tess &T = c->htess[(size_t)t];
        std::memset(&T, 0, sizeof T);
        int64_t cnt = offsets[t + 1] - offsets[t];
        T.G = size_grid(opts[t], cnt);
        T.pbase = (int32_t)offsets[t];
        T.pcount = (int32_t)cnt;
        T.bbase = (int32_t)nb;
        double bmin = T.G.bs[0];
        for (int d = 1; d < dim; d++) bmin = std::min(bmin, T.G.bs[d]);
        T.bsmin2 = bmin * bmin;
        T.clip_half = opts[t].clip > 0.0 ? 0.5 * opts[t].clip : 0.0;
        nb += T.G.nb;
        if (nb > (int64_t)INT32_MAX / 2) return fail(VC_E_ARG, "too many blocks (%lld)", (long long)nb);
    }
    c->nb = nb;
    std::vector<Offset> offs = build_offsets(dim);
    c->noff = (int)offs.size();
    int64_t ntiles = (nb + 2047) / 2048 + 2;
    vc_status st;
#define TRY(x)              \
    do {                    \
        st = (x);           \
        if (st) return st;  \
    } while (0)
    TRY(dalloc(&c->tess, (size_t)ntess));
    if (ntess > 1) TRY(dalloc(&c->ptess, (size_t)c->n));
    TRY(dalloc(&c->xyz, (size_t)c->n * dim));
    TRY(dalloc(&c->part, (size_t)c->n));
    TRY(dalloc(&c->start, (size_t)nb + 1));
    TRY(dalloc(&c->count, (size_t)nb));
    TRY(dalloc(&c->blk, (size_t)c->n));
    TRY(dalloc(&c->rank, (size_t)c->n));
    TRY(dalloc(&c->sid, (size_t)c->n));
    TRY(dalloc(&c->inv, (size_t)c->n));
    TRY(dalloc(&c->err, 1));
    TRY(dalloc(&c->scan_tmp, (size_t)ntiles * 2));
    TRY(dalloc(&c->offs, offs.size()));
    TRY(dalloc(&c->queue, 8));
    TRY(dalloc(&c->spill_list, (size_t)c->n));
    if (dim == 3) TRY(dalloc(&c->spill_list2, (size_t)c->n));
    TRY(dalloc(&c->xscratch, (size_t)c->max_waves * c->xscratch_len));
#undef TRY
    HIP_TRY(hipMemcpyAsync(c->tess, c->htess.data(), c->htess.size() * sizeof(Tess), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(c->offs, offs.data(), offs.size() * sizeof(Offset), hipMemcpyHostToDevice, s));
    if (ntess > 1) {
        std::vector<int32_t> pt((size_t)c->n);
        for (int64_t t = 0; t < ntess; t++)
            for (int64_t i = offsets[t]; i < offsets[t + 1]; i++) pt[(size_t)i] = (int32_t)t;
        HIP_TRY(hipMemcpyAsync(c->ptess, pt.data(), pt.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // pt goes out of scope
    }
    return copy_in_and_bin(c, xyz, s);
}

CellArgs cell_args(const vc_container *c, const vc_result *r)
{
    CellArgs A;
    std::memset(&A, 0, sizeof A);
    A.tess = c->tess;
    A.part = c->part;
    A.start = c->start;
    A.offs = c->offs;
    A.noff = c->noff;
    A.off_radius = kOffRadius;
    A.ncell = (int)c->n;
    A.cell_list = nullptr;
    A.ncell_dev = nullptr;
    A.queue = c->queue;
    A.chunk = c->launch.chunk;
    set_bands(A, c->force);
    A.mask = r->mask;
    A.vol = r->vol;
    A.cen = r->cen;
    A.perim = r->perim;
    A.nv = r->nv;
    A.ne = r->ne;
    A.nf = r->nf;
    A.fo = r->fo;
    A.nbr = r->nbr;
    A.nsh = r->nsh;
    A.status = r->status;
    A.spill_list = c->spill_list;
    A.spill_count = c->queue + 2;
    A.diag = r->diag;
    A.xscratch = c->xscratch;
    A.xscratch_len = c->xscratch_len;
    A.wbg = r->wbg;
    A.wbl = r->wbl;
    if (c->radical) {
        A.rad = c->rad;
        A.rmax = c->rmax;
    }
    return A;
}

// The passes after the main one, over the cells it left (their count is
// read on the device).  2D: the large-capacity pass.  3D after the grouped
// kernel: first the one-cell kernel (extended cells and cells beyond the
// grouped capacity), then the large-capacity pass over what overflows
// there; 3D after the one-cell kernel: the large-capacity pass.
hipError_t enqueue_spill(const vc_container *c, const CellArgs &A, int cpw, hipStream_t s)
{
    CellArgs B = A;
    B.cell_list = c->spill_list;
    B.queue = c->queue + 1;
    B.ncell_dev = c->queue + 2;
    B.ncell = (int)c->n;
    B.chunk = 1;
    B.vcap = 0;
    if (c->dim == 2) return launch_cells2d_spill(B, std::min(c->max_waves, 1024), s);
    if (cpw > 1) {
        CellArgs H = B;
        H.spill_list = c->spill_list2;
        H.spill_count = c->queue + 7;
        hipError_t e = launch_cells_handoff(H, std::min(c->max_waves, 4096), s);
        if (e != hipSuccess) return e;
        B.cell_list = c->spill_list2;
        B.queue = c->queue + 6;
        B.ncell_dev = c->queue + 7;
    }
    return launch_cells_spill(B, std::min(c->max_waves, 1024), s);
}

// The launch sequence of one compute (graph-capturable: fill kernels, no
// memset; events only when `events` is set).
vc_status enqueue_compute(vc_container *c, vc_result *r, hipStream_t s, bool events, const Launch &L,
                          const int32_t *cell_list = nullptr, int ncell = -1, bool compact_subset = false)
{
    CellArgs A = cell_args(c, r);
    A.chunk = L.chunk;
    A.vcap = L.vcap;
    if (cell_list) {
        A.cell_list = cell_list;
        A.ncell = ncell;
    }
    HIP_TRY(launch_fill_i32(c->queue, 8, 0, s));
    HIP_TRY(launch_fill_i32((int32_t *)r->diag, VC_DIAG_LEN * 2, 0, s));
    if (events) HIP_TRY(hipEventRecord(r->ev0, s));
    if (c->dim == 2) HIP_TRY(launch_cells2d(A, c->precision, std::min(L.waves, c->max_waves), s));
    else if (L.cpw > 1) HIP_TRY(launch_cells_group(A, c->precision, L.cpw, std::min(L.waves, c->max_waves), s));
    else HIP_TRY(launch_cells(A, c->precision, L.slots, std::min(L.waves, c->max_waves), s));
    if (events) HIP_TRY(hipEventRecord(r->ev1, s));
    HIP_TRY(enqueue_spill(c, A, L.cpw, s));
    if (events) HIP_TRY(hipEventRecord(r->ev2, s));
    if (r->mask & VC_WEINBERG) {
        // codes of every cell with a record, written at the scan of their lengths
        HIP_TRY(launch_nbr_offsets(r->wbl, r->n, r->wb_off, r->scan_tmp, s));
        // (the spill list is free again: its pass has run)
        HIP_TRY(launch_weinberg(r->wbg, r->wbl, r->wb_off, r->n, r->wb_codes, r->wb_sym, r->wb_chiral, c->queue + 3,
                                c->spill_list, (int)std::min<int64_t>(c->max_waves, r->n), s));
    }
    if ((r->mask & VC_NEIGHBORS) && (!cell_list || compact_subset)) {
        // CSR offsets by a scan of the face counts, then each cell's sorted
        // labels copied to its offset (capacity n * kMaxNbr always suffices)
        HIP_TRY(launch_nbr_offsets(r->nf, r->n, r->off, r->scan_tmp, s));
        HIP_TRY(launch_nbr_compact(r->nf, r->n, r->nbr, r->nsh, r->off, r->ids, r->shifts, nullptr, s));
    }
    r->last_stream = s;
    return VC_OK;
}

// Tuning sample: 32 contiguous runs of cells in block order, spread evenly
// over [lo, hi) and covering `want` cells, so that neighbouring cells share
// their blocks in the cache as in a full launch (a strided sample of single
// cells does not, and favours other launch forms).
void tuning_sample(int64_t lo, int64_t hi, int64_t want, std::vector<int32_t> &v)
{
    const int64_t n = hi - lo;
    if (n <= 0) return;
    const int64_t runs = std::min<int64_t>(32, n);
    const int64_t len = std::max<int64_t>(1, (std::min(want, n) + runs - 1) / runs);
    for (int64_t r = 0; r < runs; r++) {
        const int64_t a = lo + r * n / runs;
        for (int64_t i = a; i < std::min(a + len, hi); i++) v.push_back((int32_t)i);
    }
}

// Kernel time of one configuration on the cells of `list` (NULL: all): one
// untimed run, then the faster of `reps` timed runs.
vc_status time_launch(vc_container *b, vc_result *r, hipStream_t s, const Launch &L, const int32_t *list, int nlist,
                      int reps, float &out)
{
    out = 1e30f;
    for (int rep = 0; rep <= reps; rep++) {
        vc_status st = list ? enqueue_compute(b, r, s, true, L, list, nlist) : enqueue_compute(b, r, s, true, L);
        if (st) return st;
        if (rep == 0) continue;
        float ms = 0.f;
        HIP_TRY(hipEventSynchronize(r->ev2));
        HIP_TRY(hipEventElapsedTime(&ms, r->ev0, r->ev2));
        out = std::min(out, ms);
    }
    return VC_OK;
}

// Launch-configuration search.  Every configuration -- form (cells per
// wave, slots), the vertex capacity before the spill pass (the form's own or
// three quarters of it), cells per queue grab and resident waves -- is timed
// on the sample `list` (the faster of two runs after an untimed one); the
// best configuration of each form is then timed on the whole set `full`
// (NULL: every cell), and the fastest there wins.  A sample alone can rank
// the forms wrongly: on few cells a launch is dominated by its start and
// tail, where the one-cell form loses less than on a full launch.
vc_status tune(vc_container *b, vc_result *r, hipStream_t s, const int32_t *list, int nlist, const int32_t *full,
               int nfull, Launch &win, float &wms)
{
    const int cu = device_cu_count();
    const int form_c[][3] = {{1, 2, 128}, {1, 4, 256}, {2, 2, 64}, {4, 4, 64}};  // cpw, slots, capacity
    const int chunk_c[] = {1, 4, 16, 64};
    const int waves_c[] = {cu * 8, cu * 16, cu * 32};
    Launch best_of_form[4];
    float ms_of_form[4];
    for (int fi = 0; fi < 4; fi++) {
        const int *f = form_c[fi];
        ms_of_form[fi] = 1e30f;
        for (int cap4 : {4, 3})
            for (int ch : chunk_c)
                for (int wv : waves_c) {
                    Launch L;
                    L.cpw = f[0];
                    L.slots = f[1];
                    L.vcap = cap4 == 4 ? 0 : f[2] * cap4 / 4;
                    L.chunk = ch;
                    L.waves = wv;
                    float ms;
                    vc_status st = time_launch(b, r, s, L, list, nlist, 2, ms);
                    if (st) return st;
                    if (ms < ms_of_form[fi]) {
                        ms_of_form[fi] = ms;
                        best_of_form[fi] = L;
                    }
                }
    }
    wms = 1e30f;
    for (int fi = 0; fi < 4; fi++) {
        float ms;
        vc_status st = time_launch(b, r, s, best_of_form[fi], full, nfull, 1, ms);
        if (st) return st;
        if (ms < wms) {
            wms = ms;
            win = best_of_form[fi];
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    return VC_OK;
}

void report_tuning(const Launch &win, float wms, vc_tuning *best)
{
    if (!best) return;
    best->slots = win.slots;
    best->waves = win.waves;
    best->chunk = win.chunk;
    best->cells_per_wave = win.cpw;
    best->ms = wms;
    best->capacity = win.vcap;
}

// A result of n cells of dimension dim for the statistics mask, owned by
// container c (NULL: by none, as the chunked form's).
vc_status result_alloc(const vc_container *c, int64_t n, int dim, uint32_t mask, vc_result **out)
{
    if (mask & ~(uint32_t)(VC_ALL | VC_PERIMETER | VC_WEINBERG))
        return fail(VC_E_ARG, "result_create: unknown mask bits 0x%x", mask);
    if ((mask & VC_PERIMETER) && dim != 2) return fail(VC_E_ARG, "result_create: the perimeter is a 2D field");
    if ((mask & VC_WEINBERG) && dim != 3) return fail(VC_E_ARG, "result_create: Weinberg codes are a 3D field");
    vc_result *r = new (std::nothrow) vc_result();
    if (!r) return fail(VC_E_NOMEM, "host allocation failed");
    r->c = c;
    r->mask = mask;
    r->n = n;
    r->dim = dim;
    vc_status st = VC_OK;
#define TRY(x)               \
    do {                     \
        st = (x);            \
        if (st) {            \
            free_result(r);  \
            return st;       \
        }                    \
    } while (0)
    if (mask & VC_VOLUME) TRY(dalloc(&r->vol, n));
    if (mask & VC_CENTROID) TRY(dalloc(&r->cen, (size_t)n * 3));
    if (mask & VC_PERIMETER) TRY(dalloc(&r->perim, n));
    if (mask & VC_COUNTS) {
        TRY(dalloc(&r->nv, n));
        TRY(dalloc(&r->ne, n));
    }
    TRY(dalloc(&r->nf, n));
    if (mask & VC_FACE_ORDERS) TRY(dalloc(&r->fo, (size_t)n * kFoLen));
    if (mask & VC_NEIGHBORS) {
        TRY(dalloc(&r->nbr, (size_t)n * kMaxNbr));
        TRY(dalloc(&r->nsh, (size_t)n * kMaxNbr));
        TRY(dalloc(&r->off, (size_t)n + 1));
        TRY(dalloc(&r->ids, (size_t)n * kMaxNbr));
        TRY(dalloc(&r->shifts, (size_t)n * kMaxNbr));
    }
    if (mask & VC_WEINBERG) {
        TRY(dalloc(&r->wbg, (size_t)n * kWbStride));
        TRY(dalloc(&r->wbl, n));
        TRY(dalloc(&r->wb_off, (size_t)n + 1));
        TRY(dalloc(&r->wb_codes, (size_t)n * kWbMaxD));
        TRY(dalloc(&r->wb_sym, n));
        TRY(dalloc(&r->wb_chiral, n));
    }
    if (mask & (VC_NEIGHBORS | VC_WEINBERG)) TRY(dalloc(&r->scan_tmp, (size_t)((n + 2047) / 2048 + 2) * 2));
    TRY(dalloc(&r->status, n));
    TRY(dalloc(&r->diag, VC_DIAG_LEN));
#undef TRY
    if (hipEventCreate(&r->ev0) != hipSuccess || hipEventCreate(&r->ev1) != hipSuccess ||
        hipEventCreate(&r->ev2) != hipSuccess) {
        free_result(r);
        return fail(VC_E_HIP, "hipEventCreate failed");
    }
    *out = r;
    return VC_OK;
}

vc_status result_create(const vc_container *c, uint32_t mask, vc_result **out)
{
    if (!out) return fail(VC_E_ARG, "result_create: out is null");
    *out = nullptr;
    if (!c) return fail(VC_E_ARG, "result_create: container is null");
    return result_alloc(c, c->n, c->dim, mask, out);
}

// ---------------------------------------------------------------------------
// The allocation-free entry point (vc_tessellate_noalloc).  Every buffer the
// binning and the cell kernels need beyond the caller's positions and
// outputs lives in one file-scope device array, `scratch`, of a fixed size;
// each GPU holds its own copy until the process ends.  Host code never uses
// the array's name as an address: at the first call on a device its address
// is taken once with hipGetSymbolAddress and kept per device.

constexpr int64_t kNaMaxN = 1 << 16;       // particles per call
constexpr int64_t kNaMaxBlocks = 1 << 16;  // blocks of the grid
constexpr int kNaWaves = 512;              // resident cell waves (exact-predicate workspace)
constexpr int kNaXLen = 3072;              // workspace doubles per wave
constexpr int kNaMaxDevices = 64;

constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaOffs3 = 0;  // the 3D and 2D block-offset lists, written at set-up
constexpr size_t kNaOffs2 = kNaOffs3 + na_align(sizeof(Offset) * 729);
constexpr size_t kNaTess = kNaOffs2 + na_align(sizeof(Offset) * 81);
constexpr size_t kNaPart = kNaTess + na_align(sizeof(Tess));
constexpr size_t kNaBlk = kNaPart + na_align(sizeof(Particle) * kNaMaxN);
constexpr size_t kNaRank = kNaBlk + na_align(4 * kNaMaxN);
constexpr size_t kNaSid = kNaRank + na_align(4 * kNaMaxN);
constexpr size_t kNaInv = kNaSid + na_align(4 * kNaMaxN);
constexpr size_t kNaSpill = kNaInv + na_align(4 * kNaMaxN);
constexpr size_t kNaSpill2 = kNaSpill + na_align(4 * kNaMaxN);
constexpr size_t kNaStart = kNaSpill2 + na_align(4 * kNaMaxN);
constexpr size_t kNaCount = kNaStart + na_align(4 * (kNaMaxBlocks + 1));
constexpr size_t kNaScan = kNaCount + na_align(4 * kNaMaxBlocks);
constexpr size_t kNaErr = kNaScan + na_align(4 * 1024);
constexpr size_t kNaQueue = kNaErr + 256;
constexpr size_t kNaDiag = kNaQueue + 256;
constexpr size_t kNaX = kNaDiag + na_align(8 * VC_DIAG_LEN);
constexpr size_t kNaBytes = kNaX + (size_t)8 * kNaWaves * kNaXLen;  // about 16.0 MiB

static __device__ __align__(256) unsigned char scratch[kNaBytes];

__global__ void k_put_tess(Tess t, Tess *dst) { *dst = t; }

// a coordinate outside the box: every cell of the call gets VC_CELL_RANGE
__global__ void k_flag_range(const int32_t *err, uint8_t *status, int64_t n)
{
    if (!*err) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        status[i] = VC_CELL_RANGE;
}

std::mutex g_na_mutex;
unsigned char *g_na_ptr[kNaMaxDevices] = {};

// Set-up of the current device, once: the array's device address, and the
// block-offset lists copied into it.
vc_status na_scratch(unsigned char **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(VC_E_ARG, "vc_tessellate_noalloc: device %d not supported", dev);
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(VC_E_HIP, "vc_tessellate_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        unsigned char *b = static_cast<unsigned char *>(p);
        const std::vector<Offset> o3 = build_offsets(3), o2 = build_offsets(2);
        if (o3.size() != 729 || o2.size() != 81) return fail(VC_E_HIP, "vc_tessellate_noalloc: offset list sizes");
        HIP_TRY(hipMemcpy(b + kNaOffs3, o3.data(), o3.size() * sizeof(Offset), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(b + kNaOffs2, o2.data(), o2.size() * sizeof(Offset), hipMemcpyHostToDevice));
        g_na_ptr[dev] = b;
    }
    *out = g_na_ptr[dev];
    return VC_OK;
}

}  // namespace

extern "C" {

vc_status vc_options_init(vc_options *opt, int dim, const double *lo, const double *hi, const int *periodic)
{
    if (!opt || !lo || !hi || !periodic) return fail(VC_E_ARG, "vc_options_init: null pointer");
    if (dim != 2 && dim != 3) return fail(VC_E_ARG, "vc_options_init: dim must be 2 or 3");
    std::memset(opt, 0, sizeof(*opt));
    opt->dim = dim;
    for (int d = 0; d < dim; d++) {
        opt->lo[d] = lo[d];
        opt->hi[d] = hi[d];
        opt->periodic[d] = periodic[d] ? 1 : 0;
    }
    opt->n_opt = 5.0;
    opt->precision = VC_FP64;
    return VC_OK;
}

vc_status vc_container_create(const double *xyz, int64_t n, const vc_options *opt, void *stream, vc_container **out)
{
    if (!out) return fail(VC_E_ARG, "vc_container_create: out is null");
    *out = nullptr;
    if (!xyz) return fail(VC_E_ARG, "vc_container_create: xyz is null");
    if (n < 1) return fail(VC_E_ARG, "vc_container_create: n must be >= 1 (got %lld)", (long long)n);
    if (n > (int64_t)INT32_MAX / 2) return fail(VC_E_ARG, "vc_container_create: n too large");
    vc_status st = check_options(opt);
    if (st) return st;
    vc_container *c = new (std::nothrow) vc_container();
    if (!c) return fail(VC_E_NOMEM, "host allocation failed");
    int64_t offsets[2] = {0, n};
    st = create_common(c, xyz, offsets, 1, opt, (hipStream_t)stream);
    if (st) {
        free_container(c);
        return st;
    }
    *out = c;
    return VC_OK;
}

vc_status vc_container_rebin(vc_container *c, const double *xyz, void *stream)
{
    if (!c || !xyz) return fail(VC_E_ARG, "vc_container_rebin: null pointer");
    return copy_in_and_bin(c, xyz, (hipStream_t)stream);
}

vc_status vc_container_set_radii(vc_container *c, const double *radii, void *stream)
{
    if (!c) return fail(VC_E_ARG, "vc_container_set_radii: null container");
    return set_radii(c, radii, (hipStream_t)stream);
}

vc_status vc_result_create(const vc_container *c, uint32_t mask, vc_result **out)
{
    return result_create(c, mask, out);
}

vc_status vc_grid_size(const vc_options *opt, int64_t n, int *grid_out)
{
    if (!grid_out) return fail(VC_E_ARG, "vc_grid_size: null output");
    if (n < 1) return fail(VC_E_ARG, "vc_grid_size: n must be >= 1");
    vc_status st = check_options(opt);
    if (st) return st;
    Grid G = size_grid(*opt, n);
    for (int d = 0; d < 3; d++) grid_out[d] = G.g[d];
    return VC_OK;
}

vc_status vc_container_blocks(const vc_container *c, int32_t *block_start, int32_t *sorted_ids, int64_t *nb_out)
{
    if (!c) return fail(VC_E_ARG, "vc_container_blocks: null container");
    if (nb_out) *nb_out = c->nb;
    HIP_TRY(hipDeviceSynchronize());
    if (block_start)
        HIP_TRY(hipMemcpy(block_start, c->start, (size_t)(c->nb + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (sorted_ids) {
        std::vector<Particle> p((size_t)c->n);
        HIP_TRY(hipMemcpy(p.data(), c->part, p.size() * sizeof(Particle), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < p.size(); i++) sorted_ids[i] = p[i].id;
    }
    return VC_OK;
}

vc_status vc_compute(vc_container *c, vc_result *r, void *stream)
{
    if (!c || !r) return fail(VC_E_ARG, "vc_compute: null handle");
    if (r->c != c) return fail(VC_E_STATE, "vc_compute: result was created for another container");
    return enqueue_compute(c, r, (hipStream_t)stream, true, c->launch);
}

vc_status vc_compute_subset(vc_container *c, vc_result *r, const int64_t *ids, int64_t m, void *stream)
{
    if (!c || !r || (m > 0 && !ids)) return fail(VC_E_ARG, "vc_compute_subset: null argument");
    if (r->c != c) return fail(VC_E_STATE, "vc_compute_subset: result was created for another container");
    if (m < 0 || m > c->n) return fail(VC_E_ARG, "vc_compute_subset: need 0 <= m <= n (m = %lld)", (long long)m);
    hipStream_t s = (hipStream_t)stream;
    vc_status st;
#define TRY(x)              \
    do {                    \
        st = (x);           \
        if (st) return st;  \
    } while (0)
    if (!c->subset) TRY(dalloc(&c->subset, (size_t)c->n));
    const int64_t *dids = ids;
    if (m > 0 && !is_device_ptr(ids)) {
        for (int64_t k = 0; k < m; k++)
            if (ids[k] < 0 || ids[k] >= c->n)
                return fail(VC_E_RANGE, "vc_compute_subset: index %lld outside [0, n)", (long long)ids[k]);
        if (!c->subset_ids) TRY(dalloc(&c->subset_ids, (size_t)c->n));
        HIP_TRY(hipMemcpyAsync(c->subset_ids, ids, (size_t)m * sizeof(int64_t), hipMemcpyHostToDevice, s));
        dids = c->subset_ids;
    }
#undef TRY
    // the listed cells' sorted slots; a device list is range-checked here
    HIP_TRY(launch_fill_i32(c->err, 1, 0, s));
    HIP_TRY(launch_subset_list(dids, m, c->n, c->inv, c->subset, c->err, s));
    if (m > 0 && is_device_ptr(ids)) {
        int32_t herr = 0;
        HIP_TRY(hipMemcpyAsync(&herr, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (herr) return fail(VC_E_RANGE, "vc_compute_subset: an index lies outside [0, n)");
    }
    // cells not listed: status VC_CELL_SKIPPED, no faces (empty neighbour lists)
    HIP_TRY(launch_fill_u8(r->status, r->n, VC_CELL_SKIPPED, s));
    if (r->nf) HIP_TRY(launch_fill_i32(r->nf, r->n, 0, s));
    if (r->wbl) HIP_TRY(launch_fill_i32(r->wbl, r->n, 0, s));
    return enqueue_compute(c, r, s, true, c->launch, c->subset, (int)m, true);
}

// ---------------------------------------------------------------------------
// The chunked form (container-block chunks along z, for one large 3D set).
// Chunk j owns the layers [k0, k1) of the set's grid along z; its container
// holds the particles of [k0 - h, k1 + h) (wrapped on a periodic axis) on the
// full set's grid, so its blocks, in-block order and relative vectors are
// the full set's, and the cells of its own particles are computed there with
// the outputs written by input index.  A cell whose search radius reaches
// past the widened range is flagged (kStatusSlab) and computed again in a later
// pass with the halo doubled, until none is left; a range that covers every
// layer needs no certificate.  Scratch is the chunk's, not the set's.
// ---------------------------------------------------------------------------
namespace {

struct SlabBufs {
    int64_t cap = 0;
    double *xyz = nullptr;
    int32_t *orig = nullptr;
    uint8_t *own = nullptr;
    int32_t *list = nullptr;
    int64_t tcap = 0;  // pick tiles
    int32_t *cnt = nullptr, *start = nullptr, *tmp = nullptr;
    double *lim = nullptr;  // each computed cell's squared search radius, by sorted index
    ~SlabBufs()
    {
        void *ps[] = {xyz, orig, own, list, cnt, start, tmp, lim};
        for (void *p : ps)
            if (p) (void)hipFree(p);
    }
    vc_status reserve_tiles(int64_t items)
    {
        const int64_t t = pick_tiles(items);
        if (t <= tcap) return VC_OK;
        void *ps[] = {cnt, start, tmp};
        for (void *p : ps)
            if (p) (void)hipFree(p);
        cnt = start = tmp = nullptr;
        vc_status st;
        if ((st = dalloc(&cnt, (size_t)t)) || (st = dalloc(&start, (size_t)t + 1)) ||
            (st = dalloc(&tmp, (size_t)((t + 2047) / 2048 + 2) * 2)))
            return st;
        tcap = t;
        return VC_OK;
    }
    vc_status reserve(int64_t m)
    {
        if (m <= cap) return VC_OK;
        void *ps[] = {xyz, orig, own, list, lim};
        for (void *p : ps)
            if (p) (void)hipFree(p);
        xyz = nullptr;
        orig = nullptr;
        own = nullptr;
        list = nullptr;
        lim = nullptr;
        vc_status st;
        if ((st = dalloc(&xyz, (size_t)m * 3)) || (st = dalloc(&orig, (size_t)m)) || (st = dalloc(&own, (size_t)m)) ||
            (st = dalloc(&list, (size_t)m)) || (st = dalloc(&lim, (size_t)m)))
            return st;
        cap = m;
        return VC_OK;
    }
};

int32_t read_i32(const int32_t *d, hipStream_t s, hipError_t &e)
{
    int32_t v = 0;
    e = hipMemcpyAsync(&v, d, sizeof v, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return v;
}

// one chunk: select, bin on the full grid, compute the wanted cells of its
// own layers into r (by input index)
vc_status slab_pass(const double *dxyz, int64_t n, const vc_options &opt, const Grid &G, int k0, int k1, int h,
                    const uint8_t *want, vc_result *r, SlabBufs &B, hipStream_t s)
{
    const int nz = G.g[2];
    const int klen = k1 - k0;
    int e0 = k0 - h, elen = klen + 2 * h;
    bool cert = true;
    double zlo = -1e300, zhi = 1e300;
    if (G.per[2]) {
        if (elen >= nz) {
            e0 = 0;
            elen = nz;
            cert = false;
        } else {
            e0 = ((e0 % nz) + nz) % nz;
            zlo = G.lo[2] + e0 * G.bs[2];
            zhi = G.lo[2] + ((e0 + elen) % nz) * G.bs[2];
        }
    } else {
        const int e1 = std::min(nz, k1 + h);
        e0 = std::max(0, e0);
        elen = e1 - e0;
        if (e0 > 0) zlo = G.lo[2] + e0 * G.bs[2];
        if (e1 < nz) zhi = G.lo[2] + e1 * G.bs[2];
        cert = e0 > 0 || e1 < nz;
    }
    hipError_t he;
    vc_status st;
    // cells wanted in this chunk
    if ((st = B.reserve_tiles(n))) return st;
    HIP_TRY(launch_own_count(dxyz, n, G, k0, klen, want, kStatusSlab, B.cnt, B.start, B.tmp, s));
    const int32_t nown = read_i32(B.start + pick_tiles(n), s, he);
    HIP_TRY(he);
    if (nown == 0) return VC_OK;
    // the widened range's particles, in input order
    HIP_TRY(launch_slab_pick(dxyz, n, G, e0, elen, k0, klen, want, kStatusSlab, nullptr, nullptr, nullptr, B.cnt, B.start,
                             B.tmp, false, s));
    const int32_t m = read_i32(B.start + pick_tiles(n), s, he);
    HIP_TRY(he);
    if ((st = B.reserve(m))) return st;
    HIP_TRY(launch_slab_pick(dxyz, n, G, e0, elen, k0, klen, want, kStatusSlab, B.xyz, B.orig, B.own, B.cnt, B.start,
                             B.tmp, true, s));
    // the chunk's container on the full set's grid
    vc_options o = opt;
    for (int d = 0; d < 3; d++) o.grid[d] = G.g[d];
    vc_container *c = new (std::nothrow) vc_container();
    if (!c) return fail(VC_E_NOMEM, "host allocation failed");
    const int64_t offsets[2] = {0, m};
    st = create_common(c, B.xyz, offsets, 1, &o, s);
    if (!st) {
        st = [&]() -> vc_status {
            // the wanted cells' sorted slots, then the set's input indices
            if ((st = B.reserve_tiles(m))) return st;
            HIP_TRY(launch_slot_list(c->part, B.own, m, B.list, B.cnt, B.start, B.tmp, s));
            HIP_TRY(launch_remap_ids(c->part, m, B.orig, s));
            const int32_t nl = read_i32(B.start + pick_tiles(m), s, he);
            HIP_TRY(he);
            CellArgs A = cell_args(c, r);
            A.cell_list = B.list;
            A.ncell = nl;
            A.vcap = c->launch.vcap;
            if (cert) A.lim_out = B.lim;
            const Launch &L = c->launch;
            HIP_TRY(launch_fill_i32(c->queue, 8, 0, s));
            if (L.cpw > 1) HIP_TRY(launch_cells_group(A, c->precision, L.cpw, std::min(L.waves, c->max_waves), s));
            else HIP_TRY(launch_cells(A, c->precision, L.slots, std::min(L.waves, c->max_waves), s));
            HIP_TRY(enqueue_spill(c, A, L.cpw, s));
            if (cert)
                HIP_TRY(launch_slab_cert(c->part, B.list, nl, B.lim, zlo, zhi, G.per[2] ? G.L[2] : 0.0,
                                         0x1p-40 * (std::fabs(G.lo[2]) + std::fabs(G.hi[2]) + G.L[2]),
                                         (uint8_t)kStatusSlab, r->status, s));
            HIP_TRY(hipStreamSynchronize(s));
            return VC_OK;
        }();
    }
    if (st) (void)hipStreamSynchronize(s);  // nothing in flight may use the container
    free_container(c);
    return st;
}

}  // namespace

vc_status vc_tessellate_slabs(const double *xyz, int64_t n, const vc_options *opt, uint32_t mask, int nslab, int halo,
                              void *stream, vc_result **out)
{
    if (!out) return fail(VC_E_ARG, "vc_tessellate_slabs: out is null");
    *out = nullptr;
    if (!xyz) return fail(VC_E_ARG, "vc_tessellate_slabs: xyz is null");
    vc_status st = check_options(opt);
    if (st) return st;
    if (opt->dim != 3) return fail(VC_E_ARG, "vc_tessellate_slabs: the chunked form is 3D (dim = %d)", opt->dim);
    if (n < 1 || n > INT32_MAX / 2) return fail(VC_E_ARG, "vc_tessellate_slabs: n = %lld out of range", (long long)n);
    if (nslab < 1 || halo < 1) return fail(VC_E_ARG, "vc_tessellate_slabs: need nslab >= 1 and halo >= 1");
    if (mask & ~(uint32_t)(VC_VOLUME | VC_CENTROID | VC_COUNTS | VC_FACE_ORDERS | VC_NEIGHBOR_COUNT | VC_DIAG))
        return fail(VC_E_ARG, "vc_tessellate_slabs: mask 0x%x: the chunked form gives per-cell fields only "
                              "(no neighbour lists, perimeters or Weinberg codes)", mask);
    hipStream_t s = (hipStream_t)stream;
    const Grid G = size_grid(*opt, n);
    const int nz = G.g[2];
    nslab = std::min(nslab, nz);
    // the positions on the device (the caller's, or a copy of host ones)
    double *dcopy = nullptr;
    const double *dxyz = xyz;
    const bool on_host = !is_device_ptr(xyz);
    vc_result *r = nullptr;
    int32_t *flag = nullptr;
    SlabBufs B;  // chunk buffers, kept across chunks and passes
    st = result_alloc(nullptr, n, 3, mask, &r);
    if (!st) st = dalloc(&flag, 2);
    if (!st && on_host) st = dalloc(&dcopy, (size_t)n * 3);
    if (!st) {
        st = [&]() -> vc_status {
            hipError_t he;
            if (on_host) {
                HIP_TRY(hipMemcpyAsync(dcopy, xyz, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice, s));
                dxyz = dcopy;
            }
            HIP_TRY(launch_fill_i32(flag, 2, 0, s));
            HIP_TRY(launch_range_check(dxyz, n, G, flag, s));
            if (read_i32(flag, s, he)) {
                HIP_TRY(he);
                return fail(VC_E_RANGE, "a coordinate lies outside the box (walled: lo <= x <= hi, periodic: lo <= x "
                                        "< hi) or is not finite");
            }
            HIP_TRY(he);
            HIP_TRY(launch_fill_u8(r->status, n, 0, s));
            HIP_TRY(launch_fill_i32((int32_t *)r->diag, VC_DIAG_LEN * 2, 0, s));
            HIP_TRY(hipEventRecord(r->ev0, s));
            const uint8_t *want = nullptr;  // the first pass computes every cell
            unsigned long long again = 0;     // cells computed again
            for (int h = halo;; h *= 2) {
                for (int j = 0; j < nslab; j++) {
                    const int k0 = (int)((int64_t)j * nz / nslab), k1 = (int)((int64_t)(j + 1) * nz / nslab);
                    vc_status e = slab_pass(dxyz, n, *opt, G, k0, k1, h, want, r, B, s);
                    if (e) return e;
                }
                HIP_TRY(launch_fill_i32(flag + 1, 1, 0, s));
                HIP_TRY(launch_count_bit(r->status, n, kStatusSlab, flag + 1, s));
                const int32_t left = read_i32(flag + 1, s, he);
                HIP_TRY(he);
                if (left == 0) break;
                again += (unsigned long long)left;
                want = r->status;  // again, only the flagged cells
                if (h > 2 * nz) return fail(VC_E_STATE, "vc_tessellate_slabs: %d cells stayed unfinished", left);
            }
            HIP_TRY(hipEventRecord(r->ev1, s));
            HIP_TRY(hipMemcpyAsync(r->diag + VC_D_RECOMPUTED, &again, sizeof again, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            r->last_stream = s;
            return VC_OK;
        }();
    }
    if (st) (void)hipStreamSynchronize(s);  // nothing in flight may use what is freed
    if (flag) (void)hipFree(flag);
    if (dcopy) (void)hipFree(dcopy);
    if (st) {
        free_result(r);
        return st;
    }
    *out = r;
    return VC_OK;
}

vc_status vc_result_kernel_ms(vc_result *r, float *ms)
{
    if (!r || !ms) return fail(VC_E_ARG, "vc_result_kernel_ms: null pointer");
    HIP_TRY(hipEventSynchronize(r->ev1));
    HIP_TRY(hipEventElapsedTime(ms, r->ev0, r->ev1));
    return VC_OK;
}

vc_status vc_result_get(vc_result *r, int field, void **dev_ptr, int64_t *count)
{
    if (!r || !dev_ptr || !count) return fail(VC_E_ARG, "vc_result_get: null pointer");
    int64_t n = r->n;
    void *p = nullptr;
    int64_t k = 0;
    switch (field) {
    case VC_F_VOLUME: p = r->vol; k = n; break;
    case VC_F_CENTROID: p = r->cen; k = n * 3; break;
    case VC_F_NV: p = r->nv; k = n; break;
    case VC_F_NE: p = r->ne; k = n; break;
    case VC_F_NF: p = r->nf; k = n; break;
    case VC_F_FACE_ORDERS: p = r->fo; k = n * kFoLen; break;
    case VC_F_NBR_OFFSETS: p = r->off; k = n + 1; break;
    case VC_F_NBR_IDS:
    case VC_F_NBR_SHIFTS: {
        if (!(r->mask & VC_NEIGHBORS)) return fail(VC_E_STATE, "neighbour lists were not requested in the mask");
        HIP_TRY(hipStreamSynchronize(r->last_stream));
        HIP_TRY(hipMemcpy(&k, r->off + n, sizeof(int64_t), hipMemcpyDeviceToHost));
        p = field == VC_F_NBR_IDS ? (void *)r->ids : (void *)r->shifts;
        break;
    }
    case VC_F_STATUS: p = r->status; k = n; break;
    case VC_F_DIAG: p = r->diag; k = VC_DIAG_LEN; break;
    case VC_F_PERIMETER: p = r->perim; k = n; break;
    case VC_F_WB_OFFSETS: p = r->wb_off; k = n + 1; break;
    case VC_F_WB_CODES: {
        if (!(r->mask & VC_WEINBERG)) return fail(VC_E_STATE, "Weinberg codes were not requested in the mask");
        HIP_TRY(hipStreamSynchronize(r->last_stream));
        HIP_TRY(hipMemcpy(&k, r->wb_off + n, sizeof(int64_t), hipMemcpyDeviceToHost));
        p = r->wb_codes;
        break;
    }
    case VC_F_WB_SYM: p = r->wb_sym; k = n; break;
    case VC_F_WB_CHIRAL: p = r->wb_chiral; k = n; break;
    default: return fail(VC_E_ARG, "vc_result_get: unknown field %d", field);
    }
    if (!p) return fail(VC_E_STATE, "field %d was not requested in the statistics mask", field);
    *dev_ptr = p;
    *count = k;
    return VC_OK;
}

vc_status vc_result_copy(vc_result *r, int field, void *host_dst, int64_t bytes)
{
    if (!host_dst) return fail(VC_E_ARG, "vc_result_copy: null destination");
    void *p;
    int64_t k;
    vc_status st = vc_result_get(r, field, &p, &k);
    if (st) return st;
    static const int esz[] = {8, 8, 4, 4, 4, 1, 8, 4, 1, 1, 8, 8, 8, 1, 4, 1};
    int64_t need = k * esz[field];
    if (bytes < need) return fail(VC_E_ARG, "vc_result_copy: need %lld bytes, got %lld", (long long)need, (long long)bytes);
    HIP_TRY(hipStreamSynchronize(r->last_stream));
    HIP_TRY(hipMemcpy(host_dst, p, (size_t)need, hipMemcpyDeviceToHost));
    return VC_OK;
}

void vc_result_destroy(vc_result *r) { free_result(r); }

void vc_container_destroy(vc_container *c) { free_container(c); }

vc_status vc_batch_create(const double *xyz_concat, const int64_t *offsets, int64_t n_tess, const vc_options *opts,
                          void *stream, vc_batch **out)
{
    if (!out) return fail(VC_E_ARG, "vc_batch_create: out is null");
    *out = nullptr;
    if (!xyz_concat || !offsets || !opts) return fail(VC_E_ARG, "vc_batch_create: null pointer");
    if (n_tess < 1 || n_tess > (1 << 24)) return fail(VC_E_ARG, "vc_batch_create: bad tessellation count");
    if (offsets[0] != 0) return fail(VC_E_ARG, "vc_batch_create: offsets[0] must be 0");
    for (int64_t t = 0; t < n_tess; t++) {
        if (offsets[t + 1] <= offsets[t]) return fail(VC_E_ARG, "vc_batch_create: tessellation %lld is empty", (long long)t);
        vc_status st = check_options(&opts[t]);
        if (st) return st;
        if (opts[t].dim != 3) return fail(VC_E_ARG, "vc_batch_create: batches are 3D");
    }
    if (offsets[n_tess] > (int64_t)INT32_MAX / 2) return fail(VC_E_ARG, "vc_batch_create: too many particles");
    vc_batch *b = new (std::nothrow) vc_batch();
    if (!b) return fail(VC_E_NOMEM, "host allocation failed");
    hipStream_t s = (hipStream_t)stream;
    vc_status st = create_common(b, xyz_concat, offsets, n_tess, opts, s);
    if (!st) {
        // tuning sample: contiguous runs of cells in block order
        std::vector<int32_t> v;
        tuning_sample(0, b->n, std::max<int64_t>(b->n / 16, 1 << 18), v);
        b->nsample = (int)v.size();
        st = dalloc(&b->sample_list, v.size());
        if (!st) {
            hipError_t e = hipMemcpy(b->sample_list, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) st = fail(VC_E_HIP, "copy of the tuning sample failed");
        }
    }
    if (st) {
        free_container(b);
        return st;
    }
    *out = b;
    return VC_OK;
}

vc_status vc_batch_rebin(vc_batch *b, const double *xyz_concat, void *stream)
{
    if (!b || !xyz_concat) return fail(VC_E_ARG, "vc_batch_rebin: null pointer");
    return copy_in_and_bin(b, xyz_concat, (hipStream_t)stream);
}

vc_status vc_batch_set_radii(vc_batch *b, const double *radii_concat, void *stream)
{
    if (!b) return fail(VC_E_ARG, "vc_batch_set_radii: null batch");
    return set_radii(b, radii_concat, (hipStream_t)stream);
}

vc_status vc_batch_result_create(const vc_batch *b, uint32_t mask, vc_result **out)
{
    return result_create(b, mask, out);
}

vc_status vc_batch_compute(vc_batch *b, vc_result *r, int graph, void *stream)
{
    if (!b || !r) return fail(VC_E_ARG, "vc_batch_compute: null handle");
    if (r->c != b) return fail(VC_E_STATE, "vc_batch_compute: result was created for another batch");
    hipStream_t s = (hipStream_t)stream;
    if (!graph) return enqueue_compute(b, r, s, true, b->launch);
    if (!s) return fail(VC_E_ARG, "vc_batch_compute: graph capture needs a non-null stream");
    if (!b->gexec || b->graph_r != r || b->graph_stream != s) {
        release_graph(b);
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        vc_status st = enqueue_compute(b, r, s, false, b->launch);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(VC_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
        b->graph_r = r;
        b->graph_stream = s;
    }
    HIP_TRY(hipGraphLaunch(b->gexec, s));
    r->last_stream = s;
    return VC_OK;
}

vc_status vc_batch_tune(vc_batch *b, vc_result *r, void *stream, vc_tuning *best)
{
    if (!b || !r) return fail(VC_E_ARG, "vc_batch_tune: null handle");
    if (r->c != b) return fail(VC_E_STATE, "vc_batch_tune: result was created for another batch");
    Launch win = b->launch;
    float wms = 0.f;
    vc_status st = tune(b, r, (hipStream_t)stream, b->sample_list, b->nsample, nullptr, -1, win, wms);
    if (st) return st;
    b->launch = win;
    release_graph(b);
    report_tuning(win, wms, best);
    return VC_OK;
}

vc_status vc_batch_tune_members(vc_batch *b, vc_result *r, const int64_t *members, int64_t m, void *stream,
                                vc_tuning *best)
{
    if (!b || !r || !members || m < 1) return fail(VC_E_ARG, "vc_batch_tune_members: null or empty argument");
    if (r->c != b) return fail(VC_E_STATE, "vc_batch_tune_members: result was created for another batch");
    const int64_t nt = (int64_t)b->htess.size();
    std::vector<int32_t> all;
    for (int64_t k = 0; k < m; k++) {
        if (members[k] < 0 || members[k] >= nt)
            return fail(VC_E_RANGE, "vc_batch_tune_members: member %lld outside [0, %lld)", (long long)members[k],
                        (long long)nt);
        // a tessellation's cells are contiguous in block order
        const Tess &T = b->htess[(size_t)members[k]];
        for (int64_t i = T.pbase; i < (int64_t)T.pbase + T.pcount; i++) all.push_back((int32_t)i);
    }
    std::vector<int32_t> v;
    tuning_sample(0, (int64_t)all.size(), std::max<int64_t>((int64_t)all.size() / 16, 1 << 18), v);
    for (auto &x : v) x = all[(size_t)x];
    int32_t *list = nullptr, *full = nullptr;
    vc_status st = dalloc(&list, v.size());
    if (!st) st = dalloc(&full, all.size());
    Launch win = b->launch;
    float wms = 0.f;
    if (!st) {
        hipError_t e = hipMemcpy(list, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(full, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) st = fail(VC_E_HIP, "vc_batch_tune_members: copy of the sample failed");
        else st = tune(b, r, (hipStream_t)stream, list, (int)v.size(), full, (int)all.size(), win, wms);
    }
    if (list) (void)hipFree(list);
    if (full) (void)hipFree(full);
    if (st) return st;
    b->launch = win;
    release_graph(b);
    report_tuning(win, wms, best);
    return VC_OK;
}

void vc_batch_destroy(vc_batch *b) { free_container(b); }

vc_status vc_device_fma_rate(int precision, int reps, void *stream, double *tflops)
{
    if (!tflops || reps < 1 || (precision != VC_FP64 && precision != VC_F32_FILTER))
        return fail(VC_E_ARG, "vc_device_fma_rate: null tflops, reps < 1 or unknown precision");
    hipStream_t s = (hipStream_t)stream;
    const int blocks = device_cu_count() * 32, steps = 4096;
    double *out = nullptr;
    vc_status st = dalloc(&out, (size_t)blocks * 256);
    if (st) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    for (int r = 0; r <= reps && e == hipSuccess; r++) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch_fma_rate(out, precision == VC_FP64, blocks, steps, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && r > 0 && ms < best) best = ms;  // the first launch is untimed
    }
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(out);
    if (e != hipSuccess) return fail(VC_E_HIP, "vc_device_fma_rate: %s", hipGetErrorString(e));
    *tflops = (double)blocks * 256.0 * 8.0 * steps * 2.0 / (best * 1e-3) / 1e12;
    return VC_OK;
}

vc_status vc_tessellate_noalloc(const double *xyz, int64_t n, const vc_options *opt, double *vol, double *cen,
                                int32_t *nv, int32_t *ne, int32_t *nf, uint8_t *fo, uint8_t *status, void *stream)
{
    if (!xyz || !opt || !nf || !status) return fail(VC_E_ARG, "vc_tessellate_noalloc: null pointer");
    if (n < 1 || n > kNaMaxN)
        return fail(VC_E_ARG, "vc_tessellate_noalloc: n = %lld outside [1, %lld]", (long long)n, (long long)kNaMaxN);
    vc_status st = check_options(opt);
    if (st) return st;
    const void *ptrs[] = {xyz, vol, cen, nv, ne, nf, fo, status};
    for (const void *q : ptrs)
        if (q && !is_device_ptr(q))
            return fail(VC_E_ARG, "vc_tessellate_noalloc: positions and outputs must be device memory");
    Tess T;
    std::memset(&T, 0, sizeof T);
    T.G = size_grid(*opt, n);
    if (T.G.nb > kNaMaxBlocks)
        return fail(VC_E_ARG, "vc_tessellate_noalloc: %lld blocks, more than %lld", (long long)T.G.nb,
                    (long long)kNaMaxBlocks);
    T.pbase = 0;
    T.pcount = (int32_t)n;
    T.bbase = 0;
    double bmin = T.G.bs[0];
    for (int d = 1; d < opt->dim; d++) bmin = std::min(bmin, T.G.bs[d]);
    T.bsmin2 = bmin * bmin;
    T.clip_half = opt->clip > 0.0 ? 0.5 * opt->clip : 0.0;
    unsigned char *b = nullptr;
    if ((st = na_scratch(&b))) return st;
    hipStream_t s = (hipStream_t)stream;
    Tess *tess = reinterpret_cast<Tess *>(b + kNaTess);
    Particle *part = reinterpret_cast<Particle *>(b + kNaPart);
    int32_t *blk = reinterpret_cast<int32_t *>(b + kNaBlk), *rank = reinterpret_cast<int32_t *>(b + kNaRank);
    int32_t *sid = reinterpret_cast<int32_t *>(b + kNaSid), *inv = reinterpret_cast<int32_t *>(b + kNaInv);
    int32_t *spill = reinterpret_cast<int32_t *>(b + kNaSpill), *start = reinterpret_cast<int32_t *>(b + kNaStart);
    int32_t *count = reinterpret_cast<int32_t *>(b + kNaCount), *scan = reinterpret_cast<int32_t *>(b + kNaScan);
    int32_t *err = reinterpret_cast<int32_t *>(b + kNaErr), *queue = reinterpret_cast<int32_t *>(b + kNaQueue);
    unsigned long long *diag = reinterpret_cast<unsigned long long *>(b + kNaDiag);
    double *xs = reinterpret_cast<double *>(b + kNaX);
    // binning into the array (what must start at zero is cleared by kernels)
    k_put_tess<<<1, 1, 0, s>>>(T, tess);
    HIP_TRY(hipGetLastError());
    HIP_TRY(launch_fill_i32(count, T.G.nb, 0, s));
    HIP_TRY(launch_fill_i32(err, 1, 0, s));
    HIP_TRY(launch_bin_count(xyz, n, opt->dim, tess, nullptr, blk, rank, count, err, s));
    HIP_TRY(launch_scan(count, start, T.G.nb, scan, s));
    HIP_TRY(launch_scatter(xyz, n, opt->dim, nullptr, blk, rank, start, sid, part, inv, s));
    // cells: the launch sequence of vc_compute on the array's buffers
    HIP_TRY(launch_fill_i32(queue, 8, 0, s));
    HIP_TRY(launch_fill_i32(reinterpret_cast<int32_t *>(diag), VC_DIAG_LEN * 2, 0, s));
    CellArgs A;
    std::memset(&A, 0, sizeof A);
    A.tess = tess;
    A.part = part;
    A.start = start;
    A.offs = reinterpret_cast<const Offset *>(b + (opt->dim == 3 ? kNaOffs3 : kNaOffs2));
    A.noff = opt->dim == 3 ? 729 : 81;
    A.off_radius = kOffRadius;
    A.ncell = (int)n;
    A.queue = queue;
    A.chunk = opt->chunk > 0 ? opt->chunk : 4;
    A.vcap = opt->capacity;
    set_bands(A, opt->force);
    A.mask = (vol ? VC_VOLUME : 0) | (cen ? VC_CENTROID : 0) | (nv || ne ? VC_COUNTS : 0) | (fo ? VC_FACE_ORDERS : 0) |
             VC_NEIGHBOR_COUNT;
    A.vol = vol;
    A.cen = cen;
    A.nv = nv;
    A.ne = ne;
    A.nf = nf;
    A.fo = fo;
    A.status = status;
    A.spill_list = spill;
    A.spill_count = queue + 2;
    A.diag = diag;
    A.xscratch = xs;
    A.xscratch_len = kNaXLen;
    const int waves = std::min(opt->waves > 0 ? opt->waves : kNaWaves, kNaWaves);
    const int cpw = opt->cells_per_wave > 0 ? opt->cells_per_wave : 1;
    if (opt->dim == 2) HIP_TRY(launch_cells2d(A, opt->precision, waves, s));
    else if (cpw > 1) HIP_TRY(launch_cells_group(A, opt->precision, cpw, waves, s));
    else HIP_TRY(launch_cells(A, opt->precision, opt->slots > 0 ? opt->slots : 2, waves, s));
    // the passes after the main one, as for a container
    CellArgs B = A;
    B.cell_list = spill;
    B.queue = queue + 1;
    B.ncell_dev = queue + 2;
    B.chunk = 1;
    B.vcap = 0;
    if (opt->dim == 2) {
        HIP_TRY(launch_cells2d_spill(B, kNaWaves, s));
    } else {
        if (cpw > 1) {
            CellArgs H = B;
            H.spill_list = reinterpret_cast<int32_t *>(b + kNaSpill2);
            H.spill_count = queue + 7;
            HIP_TRY(launch_cells_handoff(H, kNaWaves, s));
            B.cell_list = H.spill_list;
            B.queue = queue + 6;
            B.ncell_dev = queue + 7;
        }
        HIP_TRY(launch_cells_spill(B, kNaWaves, s));
    }
    k_flag_range<<<(int)std::min<int64_t>((n + 255) / 256, 256), 256, 0, s>>>(err, status, n);
    HIP_TRY(hipGetLastError());
    return VC_OK;
}

const char *vc_last_error(void) { return g_err.c_str(); }

const char *vc_version(void) { return "vorohip 0.3 (gfx950)"; }

}  // extern "C"
