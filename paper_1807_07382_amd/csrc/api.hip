// api.hip -- the C ABI of libpentbatch (declared in include/pentbatch.h):
// argument checks, handle lifetime, schedule choice and kernel launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace pent;

namespace {

thread_local int g_status = PENT_OK;
thread_local int64_t g_pivot_row = -1;

inline int ret(int st)
{
    g_status = st;
    return st;
}

inline int hip_status(hipError_t e)
{
    if (e == hipSuccess) return PENT_OK;
    if (e == hipErrorOutOfMemory) return PENT_OUT_OF_MEMORY;
    return PENT_HIP_ERROR;
}

inline bool valid(pent_handle h) { return h != nullptr && h->magic == kMagic; }

// ---- stream-ordered scratch ----
// Scratch of the solves (status words, exchange areas, segment summaries)
// comes from a memory pool of the library's own on each device.  The
// device's default pool has a release threshold of zero: every
// synchronisation returns freed memory to the driver and the next
// allocation maps it again (about 0.3 ms of host time for the 70-170 MB of
// a large single pass).  This pool keeps up to kPoolKeepBytes reserved.
// Pools live until the process ends.
constexpr uint64_t kPoolKeepBytes = (uint64_t)4 << 30;
std::mutex g_pool_mu;
std::map<int, hipMemPool_t> g_pools;  // device -> pool

hipError_t device_pool(hipStream_t s, hipMemPool_t *out)
{
    int dev = 0;
    hipError_t e = hipStreamGetDevice(s, &dev);  // the stream's device, as hipMallocAsync
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pools.find(dev);
    if (it == g_pools.end()) {
        hipMemPoolProps props;
        std::memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        e = hipMemPoolCreate(&pool, &props);
        if (e != hipSuccess) return e;
        uint64_t keep = kPoolKeepBytes;
        e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
        if (e != hipSuccess) {
            (void)hipMemPoolDestroy(pool);
            return e;
        }
        it = g_pools.emplace(dev, pool).first;
    }
    *out = it->second;
    return hipSuccess;
}

// Stream-ordered scratch of `bytes` on s, on the stream's device (free it
// with hipFreeAsync on s).
hipError_t scratch_alloc(void **p, size_t bytes, hipStream_t s)
{
    hipMemPool_t pool = nullptr;
    const hipError_t e = device_pool(s, &pool);
    if (e != hipSuccess) return e;
    return hipMallocFromPoolAsync(p, bytes, pool, s);
}

void free_plan(pent_plan *p)
{
    if (!p) return;
    if (p->d_diag) (void)hipFree(p->d_diag);
    if (p->d_fac) (void)hipFree(p->d_fac);
    if (p->d_anorm) (void)hipFree(p->d_anorm);
    if (p->d_fwd) (void)hipFree(p->d_fwd);
    if (p->d_bwd) (void)hipFree(p->d_bwd);
    for (auto &c : p->seg)
        if (c.d_seg) (void)hipFree(c.d_seg);
    for (auto &c : p->grp)
        if (c.d_grp) (void)hipFree(c.d_grp);
    if (p->d_scan) (void)hipFree(p->d_scan);
    if (p->d_trec) (void)hipFree(p->d_trec);
    if (p->d_err) (void)hipFree(p->d_err);
    p->magic = 0;
    delete p;
}

// Allocate a plan whose diagonals (5n doubles, device) the caller fills.
pent_plan *new_plan(int64_t n, int *st)
{
    pent_plan *p = new (std::nothrow) pent_plan();
    if (!p) {
        *st = PENT_OUT_OF_MEMORY;
        return nullptr;
    }
    p->magic = 0;
    p->n = n;
    // past n, room for one more group of the many-matrix single pass (it
    // reads whole groups of 4 x kGroupSegRows records)
    p->npad = (n + 256 + kRecPad - 1) / kRecPad * kRecPad;
    p->d_diag = nullptr;
    p->d_fac = nullptr;
    p->d_anorm = nullptr;
    p->d_fwd = nullptr;
    p->d_bwd = nullptr;
    p->sched_kind = 0;
    p->sched_seg = 0;
    p->refine_tol = 0.0;
    p->d_scan = nullptr;
    p->d_trec = nullptr;
    p->scan_rows = 0;
    p->d_err = nullptr;
    p->onepass_cap[0] = p->onepass_cap[1] = 0;
    p->fix_cap = 0;
    p->t_cap = 0;
    p->tst_cap = 0;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc(&p->d_diag, sizeof(double) * 5 * n);
    if (e == hipSuccess) e = hipMalloc(&p->d_fac, sizeof(double) * 4 * n);
    if (e == hipSuccess) e = hipMalloc(&p->d_anorm, sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->d_fwd, sizeof(FwdRec) * p->npad);
    if (e == hipSuccess) e = hipMalloc(&p->d_bwd, sizeof(BwdRec) * p->npad);
    if (e == hipSuccess) e = hipMalloc(&p->d_err, sizeof(unsigned int));
    if (e == hipSuccess) e = hipMemset(p->d_err, 0, sizeof(unsigned int));
    if (e != hipSuccess) {
        free_plan(p);
        *st = hip_status(e);
        return nullptr;
    }
    *st = PENT_OK;
    return p;
}

// Co-resident single-pass units on the current device (queried once per plan).
void query_onepass_cap(pent_plan *p, int seg_rows)
{
    int &cap = p->onepass_cap[seg_rows == 32 ? 0 : 1];
    if (cap == 0) cap = onepass_capacity(seg_rows);
}

const SegRec *seg_cache_locked(pent_plan *p, int seg_rows, int *st, bool sync);
const GrpRec *grp_cache_locked(pent_plan *p, int seg_rows, int waves, int *st, bool sync);
bool tile_cache(pent_plan *p, int rows, const ScanRec **scan, const double **trec, int *st,
                bool sync);

// Factor the diagonals already in p->d_diag and build the per-schedule
// tables of the automatic schedule (segment constants for 64- and 32-row
// segments, and the resident tile's tables where n allows it), all on the
// null stream, then synchronise once to read the pivot check.  Later solves
// with the automatic schedule then allocate nothing for these tables.
// Consumes p on error.
pent_handle finish_factor(pent_plan *p)
{
    int64_t *d_bad = nullptr;
    int64_t bad = -1;
    int st = PENT_OK;
    hipError_t e = hipMalloc(&d_bad, sizeof(int64_t));
    if (e == hipSuccess) e = launch_factor(p->d_diag, p->n, p->npad, p->d_fac, p->d_fwd, p->d_bwd, d_bad, 0);
    if (e == hipSuccess) e = launch_anorm(p->d_diag, p->n, p->d_anorm, 0);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(p->mu);
        // and the group constants of the many-matrix single pass (64-row
        // segments, four per group)
        if (!seg_cache_locked(p, 64, &st, false) || !seg_cache_locked(p, 32, &st, false) ||
            !grp_cache_locked(p, 64, 4, &st, false))
            e = hipErrorUnknown;
    }
    if (e == hipSuccess && tile_rows_for(p->n) > 0) {
        const ScanRec *sc;
        const double *tr;
        if (!tile_cache(p, tile_rows_for(p->n), &sc, &tr, &st, false)) e = hipErrorUnknown;
    }
    if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (d_bad) (void)hipFree(d_bad);
    if (e != hipSuccess) {
        free_plan(p);
        ret(st != PENT_OK ? st : hip_status(e));
        return nullptr;
    }
    if (bad >= 0) {
        free_plan(p);
        g_pivot_row = bad;
        ret(PENT_ZERO_PIVOT);
        return nullptr;
    }
    query_onepass_cap(p, 64);  // occupancy only; lets the default pick the single pass
    p->magic = kMagic;
    ret(PENT_OK);
    return p;
}

// Per-segment constants for seg_rows, built once per handle on first use.
// The build runs on the null stream and synchronises it, so later solves on
// any stream see the finished constants.
const SegRec *seg_cache_locked(pent_plan *p, int seg_rows, int *st, bool sync = true)
{
    const int slot = seg_slot(seg_rows);
    SegCache &c = p->seg[slot];
    if (c.d_seg) {
        *st = PENT_OK;
        return c.d_seg;
    }
    const int64_t nseg = (p->n + seg_rows - 1) / seg_rows;
    // padded with all-zero records to a multiple of kSegPad segments, so
    // kernels that take segments in groups read no past-the-end record
    const int64_t nalloc = (nseg + kSegPad - 1) / kSegPad * kSegPad;
    SegRec *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(SegRec) * nalloc);
    if (e == hipSuccess) e = hipMemset(d, 0, sizeof(SegRec) * nalloc);
    if (e == hipSuccess) e = launch_seg_prep(p->d_fwd, p->d_bwd, p->n, seg_rows, d, 0);
    if (e == hipSuccess && sync) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        *st = hip_status(e);
        return nullptr;
    }
    c.seg_rows = seg_rows;
    c.nseg = nseg;
    c.d_seg = d;
    *st = PENT_OK;
    return d;
}

const SegRec *seg_cache(pent_plan *p, int seg_rows, int *st)
{
    std::lock_guard<std::mutex> lk(p->mu);
    return seg_cache_locked(p, seg_rows, st);
}

// Group constants of the single pass for seg_rows-row segments, `waves`
// per group, built once per handle from the segment constants (same stream
// and synchronisation rules as seg_cache_locked).
const GrpRec *grp_cache_locked(pent_plan *p, int seg_rows, int waves, int *st, bool sync = true)
{
    GrpCache *slot = nullptr;
    for (auto &c : p->grp) {
        if (c.d_grp && c.seg_rows == seg_rows && c.waves == waves) {
            *st = PENT_OK;
            return c.d_grp;
        }
        if (!c.d_grp && !slot) slot = &c;
    }
    if (!slot) {
        *st = PENT_NOT_SUPPORTED;
        return nullptr;
    }
    const SegRec *seg = seg_cache_locked(p, seg_rows, st, sync);
    if (!seg) return nullptr;
    const int64_t ngroups = (p->n + (int64_t)seg_rows * waves - 1) / ((int64_t)seg_rows * waves);
    GrpRec *d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(GrpRec) * ngroups);
    if (e == hipSuccess) e = launch_grp_prep(seg, waves, ngroups, d, 0);
    if (e == hipSuccess && sync) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (d) (void)hipFree(d);
        *st = hip_status(e);
        return nullptr;
    }
    slot->seg_rows = seg_rows;
    slot->waves = waves;
    slot->ngroups = ngroups;
    slot->d_grp = d;
    *st = PENT_OK;
    return d;
}

const GrpRec *grp_cache(pent_plan *p, int seg_rows, int waves, int *st)
{
    std::lock_guard<std::mutex> lk(p->mu);
    return grp_cache_locked(p, seg_rows, waves, st);
}

// Interface-scan constants and record image of the resident-tile schedule
// (built once per handle).
bool tile_cache(pent_plan *p, int rows, const ScanRec **scan, const double **trec, int *st,
                bool sync = true)
{
    std::lock_guard<std::mutex> lk(p->mu);
    if (!(p->d_scan && p->scan_rows == rows)) {
        const SegRec *seg = seg_cache_locked(p, rows, st, sync);
        if (!seg) return false;
        ScanRec *d = nullptr;
        double *t = nullptr;
        hipError_t e = hipMalloc(&d, sizeof(ScanRec) * 64);
        if (e == hipSuccess) e = hipMalloc(&t, sizeof(double) * tile_recs_doubles(rows));
        if (e == hipSuccess) e = launch_scan_prep(seg, (p->n + rows - 1) / rows, d, 0);
        if (e == hipSuccess) e = launch_tile_recs(p->d_fwd, p->d_bwd, rows, t, 0);
        if (e == hipSuccess && sync) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            if (d) (void)hipFree(d);
            if (t) (void)hipFree(t);
            *st = hip_status(e);
            return false;
        }
        if (p->d_scan) (void)hipFree(p->d_scan);
        if (p->d_trec) (void)hipFree(p->d_trec);
        p->d_scan = d;
        p->d_trec = t;
        p->scan_rows = rows;
    }
    *scan = p->d_scan;
    *trec = p->d_trec;
    *st = PENT_OK;
    return true;
}

// Automatic schedule (chosen from measured sweeps over sizes on MI355X): the
// resident tile for small solves, where launch count and latency dominate
// (it is one kernel, the partitioned sweep three); the single pass for
// large ones (f read once and x written once; measured ahead of the
// partitioned sweep from n = 1024 to 8192, FP64 and FP32 input), and the
// partitioned sweep where the single pass cannot run.
void choose_schedule(const pent_plan *p, int64_t batch, int *kind, int *seg_rows)
{
    if (p->sched_kind != 0) {
        *kind = p->sched_kind;
        *seg_rows = p->sched_seg;
    } else if (tile_rows_for(p->n) > 0 && p->n * batch <= (int64_t)8 << 20) {
        *kind = 3;
        *seg_rows = 0;
    } else if (p->onepass_cap[1] > 0 && p->n >= 1024) {
        *kind = 4;
        *seg_rows = 64;
    } else {
        *kind = 2;
        *seg_rows = p->n <= 2048 ? 32 : 64;
    }
    if (*kind == 3 && tile_rows_for(p->n) == 0) {
        *kind = 2;
        *seg_rows = 64;
    }
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }


// Scratch of the partitioned and single-pass schedules for `batch` systems
// (0 for the others).
size_t summ_bytes(const pent_plan *p, int kind, int seg_rows, int64_t batch)
{
    if (kind == 4) return onepass_scratch_bytes(p->n, seg_rows, batch);
    if (kind != 2) return 0;
    const int64_t nseg = (p->n + seg_rows - 1) / seg_rows;
    const int64_t summ_ld = (batch + 63) / 64 * 64;
    return align256(sizeof(double) * 4 * nseg * summ_ld);
}

// Effective schedule of an out-of-place / FP32-input solve (the one-lane
// schedule only works in place on FP64, so it maps to the partitioned one).
void io_schedule(const pent_plan *p, int64_t batch, bool inplace64, int *kind, int *seg_rows)
{
    choose_schedule(p, batch, kind, seg_rows);
    if (*kind == 4) {
        // every unit of one tile must fit on the device at once (with room
        // to spare for other work); else the three-kernel form
        const int cap = p->onepass_cap[*seg_rows == 32 ? 0 : 1];
        if (cap <= 0 || onepass_groups(p->n, *seg_rows) > cap / 4 ||
            onepass_units(p->n, *seg_rows, batch) > (int64_t)UINT32_MAX / 2)
            *kind = 2;
    }
    if (*kind == 2 && (p->n + *seg_rows - 1) / *seg_rows > 65535) {
        *kind = 1;
        *seg_rows = 16;
    }
    if (*kind == 1 && *seg_rows != 8 && *seg_rows != 32) *seg_rows = 16;  // prefetch depth
    if (*kind == 1 && !inplace64) {
        *kind = 2;
        *seg_rows = 64;
    }
}

// x = A^{-1} f with FP64 arithmetic; f FP32 or FP64; summ: scratch of
// summ_bytes() for the chosen schedule.
int solve_io(pent_plan *h, const void *f, bool f32, int64_t ldf, double *x, int64_t ldx,
             int64_t batch, void *summ, hipStream_t s, bool words_clear = false)
{
    const bool inplace64 = !f32 && (const void *)x == f && ldx == ldf;
    int kind, seg_rows, st;
    io_schedule(h, batch, inplace64, &kind, &seg_rows);
    if (kind == 1)
        return hip_status(launch_lane_sweep(h->d_fwd, h->d_bwd, h->n, x, batch, ldx, seg_rows, s));
    if (kind == 3) {
        const int rows = tile_rows_for(h->n);
        const ScanRec *scan;
        const double *trec;
        if (!tile_cache(h, rows, &scan, &trec, &st)) return st;
        return hip_status(launch_tile_sweep_io(trec, scan, h->n, rows, f, f32, ldf, x, ldx, batch, s));
    }
    const SegRec *seg = seg_cache(h, seg_rows, &st);
    if (!seg) return st;
    if (kind == 4)
        return hip_status(launch_onepass(h->d_fwd, h->d_bwd, seg, h->n, seg_rows, f, f32, ldf, x,
                                         ldx, batch, summ, h->d_err, s, 64, 64, words_clear));
    const int64_t summ_ld = (batch + 63) / 64 * 64;
    return hip_status(launch_part_sweep_io(h->d_fwd, h->d_bwd, seg, h->n, h->npad, seg_rows, f,
                                           f32, ldf, x, ldx, batch, (double *)summ, summ_ld, s));
}

// solve_io with its scratch taken from the stream-ordered allocator.
int solve_io_scratch(pent_plan *h, const double *f, int64_t ldf, double *x, int64_t ldx,
                     int64_t batch, hipStream_t s)
{
    int kind, seg_rows;
    io_schedule(h, batch, (const void *)f == (const void *)x && ldf == ldx, &kind, &seg_rows);
    const size_t bytes = summ_bytes(h, kind, seg_rows, batch);
    void *summ = nullptr;
    if (bytes) {
        hipError_t e = scratch_alloc(&summ, bytes, s);
        if (e != hipSuccess) return hip_status(e);
    }
    const int st = solve_io(h, f, false, ldf, x, ldx, batch, summ, s);
    if (summ) {
        hipError_t e = hipFreeAsync(summ, s);
        if (st == PENT_OK && e != hipSuccess) return hip_status(e);
    }
    return st;
}

constexpr int kMaxRefine = 16;

// Workspace of pent_solve_mixed: single-pass / partitioned scratch, the
// correction buffer r (three-kernel corrections only) and the backward-error
// accumulators (when eta is asked for or a tolerance is set).
struct MixedLayout {
    size_t summ = 0, r = 0, acc = 0;
    bool fused = false;  // corrections run as the fused single pass
    size_t total() const { return summ + r + acc; }
};

MixedLayout mixed_layout(pent_plan *h, int64_t batch, bool inplace64, int refine_steps, bool want_eta)
{
    MixedLayout L;
    int kind, seg_rows;
    io_schedule(h, batch, inplace64, &kind, &seg_rows);
    L.summ = summ_bytes(h, kind, seg_rows, batch);
    if (refine_steps > 0) {
        if (kind == 4) {
            if (h->fix_cap == 0) h->fix_cap = onepass_fix_capacity();
            L.fused = h->fix_cap > 0 && onepass_fix_groups(h->n) <= h->fix_cap / 4 &&
                      onepass_fix_scratch_bytes(h->n, batch) <= L.summ;
        }
        if (!L.fused) L.r = align256(sizeof(double) * (size_t)h->n * batch);
    }
    if (want_eta || h->refine_tol > 0.0) L.acc = align256(sizeof(unsigned long long) * 3 * (size_t)batch);
    return L;
}

}  // namespace

namespace {

// Device tables of one binding of a group: the buffer table, the work list
// of the persistent kernel and the unit table of the single pass.  Shared by
// the group and by every graph captured from that binding and freed when
// the last of them lets go, so rebinding or destroying the group never
// pulls them from under a graph that still launches kernels reading them.
struct GroupTables {
    GroupMat *d_mats = nullptr;
    GroupItem *d_items = nullptr;
    GroupUnit *d_units = nullptr;
    int nitems = 0;
    int64_t nunits = 0;
    int64_t max_groups = 0;    // deepest tile of the single pass, in units
    GroupTables() = default;
    GroupTables(const GroupTables &) = delete;
    GroupTables &operator=(const GroupTables &) = delete;
    ~GroupTables()
    {
        for (void *q : {(void *)d_mats, (void *)d_items, (void *)d_units})
            if (q) (void)hipFree(q);
    }
};

// The group's device words [next item, workgroups done, wait timed out],
// shared the same way (the kernels of a captured graph use them).
struct GroupCounters {
    unsigned int *d_ctr = nullptr;
    GroupCounters() = default;
    GroupCounters(const GroupCounters &) = delete;
    GroupCounters &operator=(const GroupCounters &) = delete;
    ~GroupCounters()
    {
        if (d_ctr) (void)hipFree(d_ctr);
    }
};

}  // namespace

struct pent_group_s {
    uint64_t magic = 0;
    int device = 0;
    std::vector<pent_plan *> plans;
    // bound buffers (host copies, to detect changes)
    bool bound = false;
    std::vector<double *> F;
    std::vector<int64_t> batch, ld;
    std::shared_ptr<GroupTables> tabs;
    std::shared_ptr<GroupCounters> ctr;
    int onepass_cap = 0;  // co-resident single-pass workgroups (0: not yet queried)
    int variant = 1;      // group kernel variant (pent_group_set_variant / autotune)
};

struct pent_graph_s {
    uint64_t magic = 0;
    hipGraphExec_t exec = nullptr;
    std::shared_ptr<GroupTables> tabs;  // kept alive while the graph exists
    std::shared_ptr<GroupCounters> ctr;
};

struct pent_cyclic_s {
    uint64_t magic = 0;
    int64_t n = 0;
    pent_plan *E = nullptr;     // factors of the leading (n-2) x (n-2) block
    double *d_cd = nullptr;     // cyclic diagonals, 5 blocks of cyc_ld(n), zero-padded
    double *d_Z = nullptr;      // E->npad x 2, ld 2: E^{-1} k (rows past n-2 zero)
    double *d_W = nullptr;      // E->npad x 2, ld 2: (h^T E^{-1})^T (rows past n-2 zero)
    CycAux *d_aux = nullptr;    // sparse h^T and [C2 - h^T Z]^{-1}
    int kind = 0;               // 0 automatic, 1 E-solve + update kernels, 2 single pass
    int seg_rows = 64;          // single-pass segment height
    int cap[2][2] = {{0, 0}, {0, 0}};  // co-resident single-pass units [seg 32/64][solve/CN]
    bool uni = false;           // each diagonal is the same in every row (bit for bit) ...
    double uc[5] = {0, 0, 0, 0, 0};  // ... with these values, a..e
};

namespace {

constexpr uint64_t kGroupMagic = 0x70656e7467727075ull;
constexpr uint64_t kGraphMagic = 0x70656e7467726166ull;

bool gvalid(pent_group g) { return g && g->magic == kGroupMagic; }

constexpr uint64_t kCyclicMagic = 0x70656e7463796369ull;

bool cvalid(pent_cyclic c) { return c && c->magic == kCyclicMagic; }

void free_cyclic(pent_cyclic c)
{
    if (!c) return;
    if (c->E) free_plan(c->E);
    if (c->d_cd) (void)hipFree(c->d_cd);
    if (c->d_Z) (void)hipFree(c->d_Z);
    if (c->d_W) (void)hipFree(c->d_W);
    if (c->d_aux) (void)hipFree(c->d_aux);
    c->magic = 0;
    delete c;
}

// Allocate a periodic handle whose cyclic diagonals (c->d_cd) the caller fills.
pent_cyclic new_cyclic(int64_t n, int *st)
{
    pent_cyclic c = new (std::nothrow) pent_cyclic_s();
    if (!c) {
        *st = PENT_OUT_OF_MEMORY;
        return nullptr;
    }
    c->n = n;
    c->E = new_plan(n - 2, st);
    if (!c->E) {
        free_cyclic(c);
        return nullptr;
    }
    hipError_t e = hipMalloc(&c->d_cd, sizeof(double) * 5 * cyc_ld(n));
    if (e == hipSuccess) e = hipMemset(c->d_cd, 0, sizeof(double) * 5 * cyc_ld(n));
    if (e == hipSuccess) e = hipMalloc(&c->d_Z, sizeof(double) * 2 * c->E->npad);
    if (e == hipSuccess) e = hipMalloc(&c->d_W, sizeof(double) * 2 * c->E->npad);
    if (e == hipSuccess) e = hipMalloc(&c->d_aux, sizeof(CycAux));
    if (e != hipSuccess) {
        free_cyclic(c);
        *st = hip_status(e);
        return nullptr;
    }
    *st = PENT_OK;
    return c;
}

// Bordering precomputation on the diagonals in c->d_cd: factor E, solve
// Z = E^{-1} k (two right-hand sides), then h^T and [C2 - h^T Z]^{-1}.
// Blocks; consumes c on error.
pent_cyclic finish_cyclic(pent_cyclic c)
{
    const int64_t n = c->n;
    hipError_t e = launch_cyc_build(c->d_cd, n, c->E->npad, c->E->d_diag, c->d_Z, 0);
    if (e != hipSuccess) {
        free_cyclic(c);
        ret(hip_status(e));
        return nullptr;
    }
    pent_plan *E = c->E;
    c->E = nullptr;           // finish_factor frees the plan itself on error
    c->E = finish_factor(E);
    if (!c->E) {
        free_cyclic(c);
        return nullptr;       // status (and pivot row) set by finish_factor
    }
    int st = solve_io_scratch(c->E, c->d_Z, 2, c->d_Z, 2, 2, 0);
    if (st == PENT_OK) st = hip_status(launch_cyc_finish(c->d_cd, n, c->d_Z, c->d_aux, 0));
    // (h^T E^{-1})^T = E^{-T} h: factor E^T (same leading minors as E) and
    // solve with the two border rows as right-hand sides
    if (st == PENT_OK) {
        pent_plan *Et = new_plan(n - 2, &st);
        if (Et) {
            hipError_t e2 = launch_cyc_build_transposed(c->d_cd, n, c->E->npad, Et->d_diag, c->d_W, 0);
            if (e2 != hipSuccess) {
                free_plan(Et);
                st = hip_status(e2);
            } else {
                Et = finish_factor(Et);  // frees Et itself on error
                if (!Et) {
                    st = g_status;
                } else {
                    st = solve_io_scratch(Et, c->d_W, 2, c->d_W, 2, 2, 0);
                    if (st == PENT_OK) st = hip_status(hipDeviceSynchronize());
                    free_plan(Et);
                }
            }
        }
    }
    CycAux aux;
    if (st == PENT_OK)
        st = hip_status(hipMemcpy(&aux, c->d_aux, sizeof(CycAux), hipMemcpyDeviceToHost));
    if (st != PENT_OK) {
        free_cyclic(c);
        ret(st);
        return nullptr;
    }
    if (aux.bad) {
        free_cyclic(c);
        g_pivot_row = n - 2;
        ret(PENT_ZERO_PIVOT);
        return nullptr;
    }
    // row-invariant diagonals (the constant-coefficient operators of the
    // paper's periodic problems): the CN step then reads them from its
    // arguments instead of five per-row loads
    {
        const int64_t ld = cyc_ld(n);
        std::vector<double> h((size_t)(5 * ld));
        if (hipMemcpy(h.data(), c->d_cd, sizeof(double) * 5 * ld, hipMemcpyDeviceToHost) != hipSuccess) {
            free_cyclic(c);
            ret(PENT_HIP_ERROR);
            return nullptr;
        }
        bool uni = true;
        for (int k = 0; k < 5 && uni; k++)
            for (int64_t i = 1; i < n && uni; i++)
                uni = std::memcmp(&h[k * ld + i], &h[k * ld], sizeof(double)) == 0;
        c->uni = uni;
        for (int k = 0; k < 5; k++) c->uc[k] = h[k * ld];
    }
    c->magic = kCyclicMagic;
    ret(PENT_OK);
    return c;
}

// Whether a periodic solve (cn: the Crank-Nicolson step) of `batch` systems
// runs as one pass: schedule kind 0 or 2, and every block of one 64-system
// tile fits on the device at once with room to spare.  Queries the device
// once per handle and variant.
bool cyc_single_pass(pent_cyclic c, int64_t batch, bool cn)
{
    if (c->kind == 1) return false;
    const int sr = c->seg_rows;
    int &cap = c->cap[sr == 32 ? 0 : 1][cn ? 1 : 0];
    if (cap == 0) cap = cyc_onepass_capacity(sr, cn);
    return cap > 0 && cyc_onepass_groups(c->n, sr) <= cap / 4 &&
           cyc_onepass_units(c->n, sr, batch) <= (int64_t)UINT32_MAX / 2;
}

int cyc_run_single(pent_cyclic c, bool cn, const double *F, int64_t ldf, double *X, int64_t ldx,
                   int64_t batch, hipStream_t s)
{
    int st;
    const SegRec *seg = seg_cache(c->E, c->seg_rows, &st);
    if (!seg) return st;
    void *xbuf = nullptr;
    hipError_t e = scratch_alloc(&xbuf, cyc_onepass_scratch_bytes(c->n, c->seg_rows, batch), s);
    if (e != hipSuccess) return hip_status(e);
    e = launch_cyc_onepass(c->E->d_fwd, c->E->d_bwd, seg, c->d_cd, c->d_Z, c->d_W, c->d_aux, c->n,
                           c->seg_rows, cn, F, ldf, X, ldx, batch, xbuf, c->E->d_err, s,
                           c->uni ? c->uc : nullptr);
    const hipError_t e2 = hipFreeAsync(xbuf, s);
    return hip_status(e != hipSuccess ? e : e2);
}

void free_group(pent_group g)
{
    if (!g) return;
    g->tabs.reset();  // graphs captured from the group keep their own references
    g->ctr.reset();
    g->magic = 0;
    delete g;
}

// Workspace of the persistent solve for these counts (doubles of segment
// summaries, 64-row segments).
int64_t group_summ_doubles(const pent_group g, const int64_t *batch)
{
    int64_t tot = 0;
    for (size_t k = 0; k < g->plans.size(); k++) {
        const int64_t nseg = (g->plans[k]->n + 63) / 64;
        tot += (batch[k] + 63) / 64 * nseg * 256;
    }
    return tot;
}

// Group kernel variants: 0 the persistent kernel (group.hip), 1 the single
// pass over all matrices (onepass.hip).
constexpr int kGroupPersistent = 0, kGroupOnepass = 1, kGroupVariants = 2;

// Group solve modes (pent_group_solve).
constexpr int kModeFP64 = 0, kModeMixed = 1, kModePerMatrix = 2;

int64_t group_onepass_units(const pent_group g, const int64_t *batch)
{
    const int64_t rows = group_onepass_rows();
    int64_t u = 0;
    for (size_t k = 0; k < g->plans.size(); k++)
        u += (batch[k] + 63) / 64 * ((g->plans[k]->n + rows - 1) / rows);
    return u;
}

// Whether the bound work list can run as one single pass: every workgroup of
// the deepest tile fits on the device at once, with room to spare.
bool group_onepass_ok(pent_group g)
{
    if (g->onepass_cap == 0) g->onepass_cap = group_onepass_capacity();
    return g->tabs && g->onepass_cap > 0 && g->tabs->max_groups <= g->onepass_cap / 4 &&
           g->tabs->nunits <= (int64_t)UINT32_MAX / 2;
}

size_t group_ws_bytes(const pent_group g, const int64_t *batch)
{
    size_t b = align256(sizeof(double) * (size_t)group_summ_doubles(g, batch));
    b = std::max(b, group_onepass_scratch_bytes(group_onepass_units(g, batch)));
    for (size_t k = 0; k < g->plans.size(); k++) {
        int kind, seg_rows;
        io_schedule(g->plans[k], batch[k], true, &kind, &seg_rows);
        b = std::max(b, summ_bytes(g->plans[k], kind, seg_rows, batch[k]));
    }
    return b;
}

// Upload the buffer table and the sorted work list if anything changed.
// Blocking; also builds every per-matrix cache a later solve could need, so
// the solves themselves never synchronise (graph capture).  The new tables
// replace the group's; graphs captured earlier keep the old ones.
int group_bind(pent_group g, double *const *F, const int64_t *batch, const int64_t *ld)
{
    const size_t cnt = g->plans.size();
    bool same = g->bound;
    for (size_t k = 0; same && k < cnt; k++)
        same = g->F[k] == F[k] && g->batch[k] == batch[k] && g->ld[k] == ld[k];
    if (same) return PENT_OK;
    std::vector<GroupMat> mats(cnt);
    std::vector<GroupItem> items;
    int st;
    for (size_t k = 0; k < cnt; k++) {
        pent_plan *p = g->plans[k];
        const SegRec *seg64 = seg_cache(p, 64, &st);
        if (!seg64) return st;
        const GrpRec *grp64 = grp_cache(p, 64, 4, &st);
        if (!grp64) return st;
        const SegRec *segp = seg_cache(p, kGroupSegRows, &st);
        if (!segp) return st;
        const GrpRec *grpp = grp_cache(p, kGroupSegRows, 4, &st);
        if (!grpp) return st;
        int kind, seg_rows;
        io_schedule(p, batch[k], true, &kind, &seg_rows);
        if ((kind == 2 || kind == 4) && !seg_cache(p, seg_rows, &st)) return st;
        if (kind == 3) {
            const ScanRec *sc;
            const double *tr;
            if (!tile_cache(p, tile_rows_for(p->n), &sc, &tr, &st)) return st;
        }
        mats[k] = GroupMat{p->d_fwd, p->d_bwd, seg64, grp64, F[k], p->n, p->npad, ld[k], batch[k],
                           segp, grpp};
    }
    for (size_t k = 0; k < cnt; k++)
        for (int64_t c0 = 0; c0 < batch[k]; c0 += 64)
            items.push_back(GroupItem{(int)k, (int)std::min<int64_t>(64, batch[k] - c0), c0, 0});
    // longest first: rows x systems of the item
    std::stable_sort(items.begin(), items.end(), [&](const GroupItem &a, const GroupItem &b) {
        return mats[a.mat].n * a.ncols > mats[b.mat].n * b.ncols;
    });
    int64_t off = 0;
    for (auto &it : items) {
        it.summ_off = off;
        off += (mats[it.mat].n + 63) / 64 * 256;
    }
    if (items.size() > (size_t)INT32_MAX / 2) return PENT_NOT_SUPPORTED;
    // unit table of the single pass: every item's row groups, consecutive;
    // items with the longest chains of groups (largest n) first, then the
    // widest (measured ~1% faster than the work-list order, whose per-item
    // balance is not what bounds the single pass)
    std::vector<size_t> uorder(items.size());
    for (size_t i = 0; i < items.size(); i++) uorder[i] = i;
    std::stable_sort(uorder.begin(), uorder.end(), [&](size_t a, size_t b) {
        const int64_t na = mats[items[a].mat].n, nb = mats[items[b].mat].n;
        if (na != nb) return na > nb;
        return items[a].ncols > items[b].ncols;
    });
    std::vector<GroupUnit> units;
    int64_t max_groups = 0;
    const int64_t orows = group_onepass_rows();
    for (size_t i : uorder) {
        const int64_t ng = (mats[items[i].mat].n + orows - 1) / orows;
        max_groups = std::max(max_groups, ng);
        const int64_t u0 = (int64_t)units.size();
        for (int64_t q = 0; q < ng; q++)
            units.push_back(GroupUnit{items[i].mat, (int)q, (int)ng, 0, items[i].col0, u0});
    }
    auto t = std::make_shared<GroupTables>();
    hipError_t e = hipMalloc(&t->d_mats, sizeof(GroupMat) * std::max<size_t>(cnt, 1));
    if (e == hipSuccess) e = hipMalloc(&t->d_items, sizeof(GroupItem) * std::max<size_t>(items.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&t->d_units, sizeof(GroupUnit) * std::max<size_t>(units.size(), 1));
    if (e == hipSuccess && !units.empty())
        e = hipMemcpy(t->d_units, units.data(), sizeof(GroupUnit) * units.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && cnt)
        e = hipMemcpy(t->d_mats, mats.data(), sizeof(GroupMat) * cnt, hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(t->d_items, items.data(), sizeof(GroupItem) * items.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_status(e);  // t frees what it holds
    t->nitems = (int)items.size();
    t->nunits = (int64_t)units.size();
    t->max_groups = max_groups;
    g->tabs = std::move(t);
    g->F.assign(F, F + cnt);
    g->batch.assign(batch, batch + cnt);
    g->ld.assign(ld, ld + cnt);
    g->bound = true;
    return PENT_OK;
}

// Enqueue one group solve of the bound buffers (no synchronisation).
int group_enqueue(pent_group g, int mode, void *work, hipStream_t s)
{
    if (mode == kModeFP64) {
        const GroupTables &t = *g->tabs;
        if (t.nitems == 0) return PENT_OK;
        if (g->variant == kGroupOnepass && group_onepass_ok(g))
            return hip_status(launch_group_onepass(t.d_mats, t.d_units, t.nunits, work,
                                                   &g->ctr->d_ctr[2], s));
        // the persistent kernel (chosen, or a tile too deep for the single pass)
        const int nblocks = std::max(1, std::min(t.nitems, group_max_blocks()));
        return hip_status(launch_group(t.d_mats, t.d_items, t.nitems, (double *)work, g->ctr->d_ctr,
                                       nblocks, s));
    }
    for (size_t k = 0; k < g->plans.size(); k++) {
        if (g->batch[k] == 0) continue;
        const int st = solve_io(g->plans[k], g->F[k], false, g->ld[k], g->F[k], g->ld[k],
                                g->batch[k], work, s);
        if (st != PENT_OK) return st;
    }
    return PENT_OK;
}

// ---- autotuning ----
// Results are kept per process, keyed by (device architecture, n, batch,
// element type of the solve), and optionally in a text file named by
// PENT_TUNE_CACHE ("arch n batch dtype kind seg_rows ms" per line), so a
// choice measured on one device or element type is never applied to another.
using TuneKey = std::tuple<std::string, int64_t, int64_t, int>;
std::mutex g_tune_mu;
std::map<TuneKey, std::tuple<int, int, double>> g_tune;
bool g_tune_loaded = false;

std::string device_arch(int dev)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a(prop.gcnArchName);
    const size_t colon = a.find(':');  // drop feature suffixes (":sramecc+:xnack-")
    return colon == std::string::npos ? a : a.substr(0, colon);
}

void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("PENT_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512], arch[128];
    long long n, b;
    int dt, kind, seg;
    double ms;
    while (std::fgets(line, sizeof(line), f)) {
        if (std::sscanf(line, "%127s %lld %lld %d %d %d %lf", arch, &n, &b, &dt, &kind, &seg, &ms) == 7)
            g_tune[TuneKey{arch, n, b, dt}] = std::make_tuple(kind, seg, ms);
    }
    std::fclose(f);
}

void tune_store_locked(const TuneKey &key, int kind, int seg, double ms)
{
    g_tune[key] = std::make_tuple(kind, seg, ms);
    const char *path = std::getenv("PENT_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %lld %lld %d %d %d %.6f\n", std::get<0>(key).c_str(),
                 (long long)std::get<1>(key), (long long)std::get<2>(key), std::get<3>(key), kind,
                 seg, ms);
    std::fclose(f);
}

__global__ void k_fill_const(double *p, int64_t count, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

hipError_t fill_const(double *p, int64_t count, double v, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_const, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p,
                       count, v);
    return hipGetLastError();
}

// Average milliseconds of `reps` calls of fn after one warm-up call.
template <typename Fn>
int time_ms(Fn fn, hipStream_t s, int reps, double *ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int st = e == hipSuccess ? fn() : hip_status(e);
    if (st == PENT_OK) e = hipEventRecord(e0, s);
    for (int r = 0; st == PENT_OK && e == hipSuccess && r < reps; r++) st = fn();
    if (st == PENT_OK && e == hipSuccess) e = hipEventRecord(e1, s);
    if (st == PENT_OK && e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (st == PENT_OK && e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st == PENT_OK && e != hipSuccess) st = hip_status(e);
    *ms = t / reps;
    return st;
}

int group_check_args(pent_group g, double *const *F, const int64_t *batch, const int64_t *ld,
                     int mode)
{
    if (!gvalid(g) || !batch || !ld || mode < kModeFP64 || mode > kModePerMatrix)
        return PENT_INVALID_VALUE;
    for (size_t k = 0; k < g->plans.size(); k++) {
        if (!valid(g->plans[k]) || batch[k] < 0 || ld[k] < batch[k]) return PENT_INVALID_VALUE;
        if (batch[k] > 0 && (!F || !F[k])) return PENT_INVALID_VALUE;
    }
    // the mixed group solve: a time-stepping state is the FP64 solution of
    // the previous step, so there is no FP32 stream to save bytes on
    if (mode == kModeMixed) return PENT_NOT_SUPPORTED;
    return PENT_OK;
}

// ---- allocation-free solve (pent_solve_noalloc) ----

// Scratch of pent_solve_noalloc: device memory that belongs to the library's
// code object, one copy per GPU (each GPU holds it until the process ends),
// used where pent_solve takes stream-ordered scratch.  72 MiB covers the
// single pass's status words and exchange area up to 18 000 units (64-system
// tiles x 256-row groups), e.g. n = 4096 with 72 000 systems.  In host code
// the name is only a stand-in for the symbol: kernels get the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchBytes = (size_t)72 << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_addr;  // device -> address of its copy of scratch

// Address of the current device's copy of scratch, looked up once per device
// (with that device current).
int noalloc_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) return e != hipSuccess ? hip_status(e) : PENT_HIP_ERROR;
        it = g_scratch_addr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return PENT_OK;
}

// The tables a schedule reads already exist (built by pent_factor or an
// earlier solve), so solve_io will not build (allocate) them.
bool tables_ready(pent_plan *p, int kind, int seg_rows)
{
    std::lock_guard<std::mutex> lk(p->mu);
    if (kind == 1) return true;
    if (kind == 3) {
        const int rows = tile_rows_for(p->n);
        return p->d_scan != nullptr && p->scan_rows == rows;
    }
    return p->seg[seg_slot(seg_rows)].d_seg != nullptr;
}

}  // namespace

extern "C" {

pent_handle pent_factor(int64_t n, const double *a, const double *b, const double *c,
                        const double *d, const double *e)
{
    g_pivot_row = -1;
    if (n < 1 || n > INT32_MAX || !a || !b || !c || !d || !e) {
        ret(PENT_INVALID_VALUE);
        return nullptr;
    }
    int st;
    pent_plan *p = new_plan(n, &st);
    if (!p) {
        ret(st);
        return nullptr;
    }
    // zero-pad the entries that fall outside the matrix, then copy
    double *h = new (std::nothrow) double[5 * n];
    if (!h) {
        free_plan(p);
        ret(PENT_OUT_OF_MEMORY);
        return nullptr;
    }
    for (int64_t i = 0; i < n; i++) {
        h[0 * n + i] = (i >= 2) ? a[i] : 0.0;
        h[1 * n + i] = (i >= 1) ? b[i] : 0.0;
        h[2 * n + i] = c[i];
        h[3 * n + i] = (i + 1 < n) ? d[i] : 0.0;
        h[4 * n + i] = (i + 2 < n) ? e[i] : 0.0;
    }
    hipError_t err = hipMemcpy(p->d_diag, h, sizeof(double) * 5 * n, hipMemcpyHostToDevice);
    delete[] h;
    if (err != hipSuccess) {
        free_plan(p);
        ret(hip_status(err));
        return nullptr;
    }
    return finish_factor(p);
}

pent_handle pent_factor_d4(int64_t n, double sigma)
{
    g_pivot_row = -1;
    if (n < 1 || n > INT32_MAX || !std::isfinite(sigma)) {
        ret(PENT_INVALID_VALUE);
        return nullptr;
    }
    int st;
    pent_plan *p = new_plan(n, &st);
    if (!p) {
        ret(st);
        return nullptr;
    }
    hipError_t err = launch_assemble_d4(p->d_diag, n, sigma, 0);
    if (err != hipSuccess) {
        free_plan(p);
        ret(hip_status(err));
        return nullptr;
    }
    return finish_factor(p);
}

int pent_destroy(pent_handle h)
{
    if (h == nullptr) return ret(PENT_OK);
    if (!valid(h)) return ret(PENT_INVALID_VALUE);
    free_plan(h);
    return ret(PENT_OK);
}

int pent_solve(pent_handle h, double *F, int64_t batch, int64_t ld, void *stream)
{
    if (!valid(h) || batch < 0 || ld < batch) return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!F) return ret(PENT_INVALID_VALUE);
    return ret(solve_io_scratch(h, F, ld, F, ld, batch, (hipStream_t)stream));
}

int pent_solve_tiled(pent_handle h, double *F, int64_t batch, int64_t ld, int64_t tile_stride,
                     void *stream)
{
    if (!valid(h) || batch < 0 || ld < 64 || tile_stride < (h->n - 1) * ld + 64)
        return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!F) return ret(PENT_INVALID_VALUE);
    int kind, seg_rows, st;
    io_schedule(h, batch, true, &kind, &seg_rows);
    if (kind != 4) return ret(PENT_NOT_SUPPORTED);
    const SegRec *seg = seg_cache(h, seg_rows, &st);
    if (!seg) return ret(st);
    hipStream_t s = (hipStream_t)stream;
    void *summ = nullptr;
    hipError_t e = scratch_alloc(&summ, summ_bytes(h, kind, seg_rows, batch), s);
    if (e != hipSuccess) return ret(hip_status(e));
    e = launch_onepass(h->d_fwd, h->d_bwd, seg, h->n, seg_rows, F, false, ld, F, ld, batch, summ,
                       h->d_err, s, tile_stride, tile_stride);
    const hipError_t e2 = hipFreeAsync(summ, s);
    return ret(hip_status(e != hipSuccess ? e : e2));
}

int pent_solve_noalloc(pent_handle h, double *F, int64_t batch, int64_t ld, void *stream)
{
    if (!valid(h) || batch < 0 || ld < batch) return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!F) return ret(PENT_INVALID_VALUE);
    int kind, seg_rows;
    io_schedule(h, batch, true, &kind, &seg_rows);
    if (!tables_ready(h, kind, seg_rows)) return ret(PENT_NOT_SUPPORTED);
    const size_t bytes = summ_bytes(h, kind, seg_rows, batch);
    if (bytes > kNoallocScratchBytes) return ret(PENT_NOT_SUPPORTED);
    void *ws = nullptr;
    if (bytes > 0) {
        const int st = noalloc_scratch(&ws);
        if (st != PENT_OK) return ret(st);
    }
    return ret(solve_io(h, F, false, ld, F, ld, batch, ws, (hipStream_t)stream));
}

size_t pent_mixed_workspace_size_ex(pent_handle h, int64_t batch, int refine_steps, int want_eta)
{
    if (!valid(h) || batch < 0 || refine_steps < 0 || refine_steps > kMaxRefine) {
        ret(PENT_INVALID_VALUE);
        return 0;
    }
    const MixedLayout L = mixed_layout(h, batch, false, refine_steps, want_eta != 0);
    ret(PENT_OK);
    return L.total();
}

size_t pent_mixed_workspace_size(pent_handle h, int64_t batch)
{
    return pent_mixed_workspace_size_ex(h, batch, kMaxRefine, 1);
}

int pent_solve_mixed(pent_handle h, const void *f, int f_dtype, int64_t ld_f, double *x,
                     int64_t ld_x, int64_t batch, int refine_steps, double *eta_out, void *work,
                     size_t work_bytes, void *stream)
{
    if (!valid(h) || batch < 0 || (f_dtype != PENT_DTYPE_FP64 && f_dtype != PENT_DTYPE_FP32) ||
        ld_f < batch || ld_x < batch || refine_steps < 0 || refine_steps > kMaxRefine)
        return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!f || !x) return ret(PENT_INVALID_VALUE);
    const bool f32 = f_dtype == PENT_DTYPE_FP32;
    const bool alias = (const void *)x == f;
    if (alias && (f32 || ld_x != ld_f || refine_steps > 0)) return ret(PENT_INVALID_VALUE);
    if (h->n > (int64_t)65535 * 32) return ret(PENT_NOT_SUPPORTED);
    const MixedLayout L = mixed_layout(h, batch, alias, refine_steps, eta_out != nullptr);
    const size_t need = L.total();
    if (need > 0 && (!work || work_bytes < need)) return ret(work ? PENT_SIZE_MISMATCH : PENT_INVALID_VALUE);
    char *w = (char *)work;
    void *summ = w;
    double *r = (double *)(w + L.summ);
    unsigned long long *acc = (unsigned long long *)(w + L.summ + L.r);
    hipStream_t s = (hipStream_t)stream;

    int st = solve_io(h, f, f32, ld_f, x, ld_x, batch, summ, s);
    if (st != PENT_OK) return ret(st);
    // Corrections: where the solve ran as a single pass and a tile of the
    // fused correction fits on the device, each correction is one fused pass
    // too (residual, solve and update of x in one kernel); else residual,
    // solve, x += d.
    if (refine_steps > 0 && L.fused) {
        const SegRec *seg64 = seg_cache(h, 64, &st);
        if (!seg64) return ret(st);
        for (int it = 0; it < refine_steps; it++) {
            hipError_t e = launch_onepass_fix(h->d_fwd, h->d_bwd, seg64, h->d_diag, h->n, f, f32, ld_f,
                                              x, ld_x, batch, summ, h->d_err, s);
            if (e != hipSuccess) return ret(hip_status(e));
        }
    } else {
        for (int it = 0; it < refine_steps; it++) {
            hipError_t e = launch_residual(h->d_diag, h->n, f, f32, ld_f, x, ld_x, r, batch, batch, s);
            if (e != hipSuccess) return ret(hip_status(e));
            st = solve_io(h, r, false, batch, r, batch, batch, summ, s);
            if (st != PENT_OK) return ret(st);
            e = launch_axpy(x, ld_x, r, batch, h->n, batch, s);
            if (e != hipSuccess) return ret(hip_status(e));
        }
    }
    // the backward error, when asked for or when a tolerance is set (a miss
    // sets the handle's status, reported by pent_check)
    if (L.acc) {
        hipError_t e = launch_eta(h->d_diag, h->d_anorm, h->n, f, f32, ld_f, x, ld_x, batch, acc,
                                  eta_out, h->refine_tol, h->d_err, s);
        if (e != hipSuccess) return ret(hip_status(e));
    }
    return ret(PENT_OK);
}

int pent_backward_error(pent_handle h, const void *f, int f_dtype, int64_t ld_f, const double *x,
                        int64_t ld_x, int64_t batch, double *eta_out, void *work,
                        size_t work_bytes, void *stream)
{
    if (!valid(h) || batch < 0 || (f_dtype != PENT_DTYPE_FP64 && f_dtype != PENT_DTYPE_FP32) ||
        ld_f < batch || ld_x < batch)
        return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!f || !x || !eta_out || !work) return ret(PENT_INVALID_VALUE);
    if (work_bytes < sizeof(unsigned long long) * 3 * (size_t)batch) return ret(PENT_SIZE_MISMATCH);
    if (h->n > (int64_t)65535 * 32) return ret(PENT_NOT_SUPPORTED);
    return ret(hip_status(launch_eta(h->d_diag, h->d_anorm, h->n, f, f_dtype == PENT_DTYPE_FP32,
                                     ld_f, x, ld_x, batch, (unsigned long long *)work, eta_out,
                                     0.0, nullptr, (hipStream_t)stream)));
}

pent_group pent_group_create(const pent_handle *hs, int64_t count)
{
    if (!hs || count < 1 || count > (1 << 20)) {
        ret(PENT_INVALID_VALUE);
        return nullptr;
    }
    for (int64_t k = 0; k < count; k++)
        if (!valid(hs[k])) {
            ret(PENT_INVALID_VALUE);
            return nullptr;
        }
    pent_group g = new (std::nothrow) pent_group_s();
    if (!g) {
        ret(PENT_OUT_OF_MEMORY);
        return nullptr;
    }
    g->plans.assign(hs, hs + count);
    hipError_t e = hipGetDevice(&g->device);
    try {
        g->ctr = std::make_shared<GroupCounters>();
        g->tabs = std::make_shared<GroupTables>();
    } catch (const std::bad_alloc &) {
        free_group(g);
        ret(PENT_OUT_OF_MEMORY);
        return nullptr;
    }
    if (e == hipSuccess) e = hipMalloc(&g->ctr->d_ctr, 3 * sizeof(unsigned int));
    if (e == hipSuccess) e = launch_group_init(g->ctr->d_ctr, 0);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_group(g);
        ret(hip_status(e));
        return nullptr;
    }
    g->magic = kGroupMagic;
    ret(PENT_OK);
    return g;
}

size_t pent_group_workspace_size(pent_group g, const int64_t *batch)
{
    if (!gvalid(g) || !batch) {
        ret(PENT_INVALID_VALUE);
        return 0;
    }
    for (size_t k = 0; k < g->plans.size(); k++)
        if (batch[k] < 0) {
            ret(PENT_INVALID_VALUE);
            return 0;
        }
    ret(PENT_OK);
    return group_ws_bytes(g, batch);
}

int pent_group_solve(pent_group g, double *const *F, const int64_t *batch, const int64_t *ld,
                     int mode, void *work, size_t work_bytes, void *stream)
{
    int st = group_check_args(g, F, batch, ld, mode);
    if (st != PENT_OK) return ret(st);
    const size_t need = group_ws_bytes(g, batch);
    if (need > 0 && !work) return ret(PENT_INVALID_VALUE);
    if (work_bytes < need) return ret(PENT_SIZE_MISMATCH);
    st = group_bind(g, F, batch, ld);
    if (st != PENT_OK) return ret(st);
    return ret(group_enqueue(g, mode, work, (hipStream_t)stream));
}

int pent_autotune(pent_handle h, int64_t batch, int *kind_out, int *seg_rows_out, double *ms_out,
                  void *stream)
{
    if (!valid(h) || batch < 1) return ret(PENT_INVALID_VALUE);
    hipStream_t s = (hipStream_t)stream;
    const TuneKey key{device_arch(h->device), h->n, batch, PENT_DTYPE_FP64};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            h->sched_kind = std::get<0>(it->second);
            h->sched_seg = std::get<1>(it->second);
            if (h->sched_kind == 4) query_onepass_cap(h, h->sched_seg);
            if (kind_out) *kind_out = h->sched_kind;
            if (seg_rows_out) *seg_rows_out = h->sched_seg;
            if (ms_out) *ms_out = std::get<2>(it->second);
            return ret(PENT_OK);
        }
    }
    // (kind, seg_rows): one lane per system at three prefetch depths, the
    // partitioned sweep at three segment heights, the resident tile, the
    // single pass at two segment heights
    const int cands[9][2] = {{1, 8}, {1, 16}, {1, 32}, {2, 16}, {2, 32}, {2, 64}, {3, 0}, {4, 32}, {4, 64}};
    double *F = nullptr;
    void *work = nullptr;
    const size_t nF = (size_t)h->n * batch;
    size_t wbytes = 0;
    for (const auto &c : cands)
        if (c[0] != 1) wbytes = std::max(wbytes, summ_bytes(h, c[0], c[1] ? c[1] : 64, batch));
    hipError_t e = hipMalloc(&F, sizeof(double) * nF);
    if (e == hipSuccess && wbytes) e = hipMalloc(&work, wbytes);
    if (e == hipSuccess) e = fill_const(F, (int64_t)nF, 1.0, s);
    int st = hip_status(e);
    const int saved_kind = h->sched_kind, saved_seg = h->sched_seg;
    int best_kind = 0, best_seg = 0;
    double best = 1e300;
    for (const auto &c : cands) {
        if (st != PENT_OK) break;
        if (c[0] == 3 && tile_rows_for(h->n) == 0) continue;
        if (c[0] == 2 && (h->n + c[1] - 1) / c[1] > 65535) continue;
        h->sched_kind = c[0];
        h->sched_seg = c[1];
        if (c[0] == 4) query_onepass_cap(h, c[1]);
        int ek, es;
        io_schedule(h, batch, true, &ek, &es);
        if (ek != c[0]) continue;  // not runnable at this size (falls back)
        double ms = 0.0;
        st = time_ms([&] { return solve_io(h, F, false, batch, F, batch, batch, work, s); }, s, 3, &ms);
        if (st == PENT_OK && ms < best) {
            best = ms;
            best_kind = c[0];
            best_seg = c[1];
        }
    }
    (void)hipStreamSynchronize(s);
    if (F) (void)hipFree(F);
    if (work) (void)hipFree(work);
    if (st != PENT_OK) {
        h->sched_kind = saved_kind;
        h->sched_seg = saved_seg;
        return ret(st);
    }
    h->sched_kind = best_kind;
    h->sched_seg = best_seg;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_store_locked(key, best_kind, best_seg, best);
    }
    if (kind_out) *kind_out = best_kind;
    if (seg_rows_out) *seg_rows_out = best_seg;
    if (ms_out) *ms_out = best;
    return ret(PENT_OK);
}

int pent_group_autotune(pent_group g, const int64_t *batch, int *variant_out, double *ms_out,
                        void *stream)
{
    if (!gvalid(g) || !batch) return ret(PENT_INVALID_VALUE);
    const size_t cnt = g->plans.size();
    for (size_t k = 0; k < cnt; k++)
        if (batch[k] < 0) return ret(PENT_INVALID_VALUE);
    hipStream_t s = (hipStream_t)stream;
    // scratch blocks of the same shapes (the caller's data is never touched),
    // rows padded to whole 128-byte lines as a caller would store them
    std::vector<double *> F(cnt, nullptr);
    std::vector<int64_t> ld(cnt);
    for (size_t k = 0; k < cnt; k++) ld[k] = (batch[k] + 15) / 16 * 16;
    void *work = nullptr;
    hipError_t e = hipSuccess;
    for (size_t k = 0; k < cnt && e == hipSuccess; k++) {
        const size_t m = (size_t)g->plans[k]->n * std::max<int64_t>(ld[k], 1);
        e = hipMalloc(&F[k], sizeof(double) * m);
        if (e == hipSuccess) e = fill_const(F[k], (int64_t)m, 1.0, s);
    }
    const size_t wbytes = group_ws_bytes(g, batch);
    if (e == hipSuccess && wbytes) e = hipMalloc(&work, wbytes);
    int st = hip_status(e);
    // keep the caller's binding (its tables stay alive through the shared
    // pointer) to restore afterwards
    const bool had = g->bound;
    std::vector<double *> oF = g->F;
    std::vector<int64_t> ob = g->batch, ol = g->ld;
    std::shared_ptr<GroupTables> otabs = g->tabs;
    if (st == PENT_OK) {
        g->bound = false;
        st = group_bind(g, F.data(), batch, ld.data());
    }
    const int saved = g->variant;
    int best_v = saved;
    double best = 1e300;
    for (int v = 0; st == PENT_OK && v < kGroupVariants; v++) {
        if (v == kGroupOnepass && !group_onepass_ok(g)) continue;
        g->variant = v;
        double ms = 0.0;
        st = time_ms([&] { return group_enqueue(g, kModeFP64, work, s); }, s, 3, &ms);
        if (st == PENT_OK && ms < best) {
            best = ms;
            best_v = v;
        }
    }
    g->variant = st == PENT_OK ? best_v : saved;
    (void)hipStreamSynchronize(s);
    // back to the caller's binding, without re-uploading it
    g->tabs = otabs;
    g->F = oF;
    g->batch = ob;
    g->ld = ol;
    g->bound = had;
    for (auto p : F)
        if (p) (void)hipFree(p);
    if (work) (void)hipFree(work);
    if (st != PENT_OK) return ret(st);
    if (variant_out) *variant_out = best_v;
    if (ms_out) *ms_out = best;
    return ret(PENT_OK);
}

int pent_group_set_variant(pent_group g, int variant)
{
    if (!gvalid(g) || variant < 0 || variant >= kGroupVariants) return ret(PENT_INVALID_VALUE);
    g->variant = variant;
    return ret(PENT_OK);
}

int pent_group_check(pent_group g)
{
    if (!gvalid(g)) return ret(PENT_INVALID_VALUE);
    unsigned int flag = 0;
    hipError_t e = hipMemcpy(&flag, &g->ctr->d_ctr[2], sizeof(flag), hipMemcpyDeviceToHost);
    if (e == hipSuccess && flag) e = hipMemset(&g->ctr->d_ctr[2], 0, sizeof(flag));
    if (e != hipSuccess) return ret(hip_status(e));
    return ret(flag ? PENT_TIMEOUT : PENT_OK);
}

int pent_group_destroy(pent_group g)
{
    if (!g) return ret(PENT_OK);
    if (!gvalid(g)) return ret(PENT_INVALID_VALUE);
    free_group(g);
    return ret(PENT_OK);
}

pent_graph pent_group_capture(pent_group g, double *const *F, const int64_t *batch,
                              const int64_t *ld, int mode, int steps, void *work,
                              size_t work_bytes, void *stream)
{
    int st = group_check_args(g, F, batch, ld, mode);
    if (st == PENT_OK && (steps < 1 || !stream)) st = PENT_INVALID_VALUE;
    if (st != PENT_OK) {
        ret(st);
        return nullptr;
    }
    const size_t need = group_ws_bytes(g, batch);
    if ((need > 0 && !work) || work_bytes < need) {
        ret(work ? PENT_SIZE_MISMATCH : PENT_INVALID_VALUE);
        return nullptr;
    }
    st = group_bind(g, F, batch, ld);
    if (st != PENT_OK) {
        ret(st);
        return nullptr;
    }
    pent_graph gr = new (std::nothrow) pent_graph_s();
    if (!gr) {
        ret(PENT_OUT_OF_MEMORY);
        return nullptr;
    }
    gr->tabs = g->tabs;
    gr->ctr = g->ctr;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete gr;
        ret(hip_status(e));
        return nullptr;
    }
    for (int i = 0; i < steps && st == PENT_OK; i++) st = group_enqueue(g, mode, work, s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (st == PENT_OK && e != hipSuccess) st = hip_status(e);
    hipGraphExec_t exec = nullptr;
    if (st == PENT_OK) {
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = hip_status(e);
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (st != PENT_OK) {
        if (exec) (void)hipGraphExecDestroy(exec);
        delete gr;
        ret(st);
        return nullptr;
    }
    gr->exec = exec;
    gr->magic = kGraphMagic;
    ret(PENT_OK);
    return gr;
}

int pent_graph_launch(pent_graph gr, void *stream)
{
    if (!gr || gr->magic != kGraphMagic) return ret(PENT_INVALID_VALUE);
    return ret(hip_status(hipGraphLaunch(gr->exec, (hipStream_t)stream)));
}

int pent_graph_destroy(pent_graph gr)
{
    if (!gr) return ret(PENT_OK);
    if (gr->magic != kGraphMagic) return ret(PENT_INVALID_VALUE);
    (void)hipGraphExecDestroy(gr->exec);
    gr->magic = 0;
    delete gr;  // drops its references to the tables it was captured with
    return ret(PENT_OK);
}

int pent_ch2d_rhs(const double *C, double *R, int64_t ny, int64_t ninst, int64_t nx,
                  const double *dt, double h, void *stream)
{
    if (!C || !R || !dt || ny < 1 || ninst < 1 || nx < 1 || !(h > 0.0) || ny > 65535 ||
        ninst > 65535 || C == R)
        return ret(PENT_INVALID_VALUE);
    return ret(hip_status(launch_ch2d_rhs(C, R, ny, ninst, nx, dt, h, (hipStream_t)stream)));
}

int pent_ch2d_step(pent_handle hx, pent_handle hy, double *C, double *R, int64_t ny,
                   int64_t ninst, int64_t nx, const double *dt, double h, void *stream)
{
    if (!valid(hx) || !valid(hy) || hx->n != nx || hy->n != ny) return ret(PENT_INVALID_VALUE);
    if (!C || !R || !dt || ny < 1 || ninst < 1 || nx < 1 || !(h > 0.0) || ny > 65535 ||
        ninst > 65535 || C == R)
        return ret(PENT_INVALID_VALUE);
    hipStream_t s = (hipStream_t)stream;
    const int64_t batch = ny * ninst, ybatch = ninst * nx;
    // the y sweeps' scratch comes first: where they run as a single pass
    // after the single-pass x sweeps, the x-sweep kernel zeroes their
    // status words, and the step needs no clearing kernel between the two
    int ykind, yseg;
    io_schedule(hy, ybatch, false, &ykind, &yseg);
    const size_t ybytes = summ_bytes(hy, ykind, yseg, ybatch);
    void *ybuf = nullptr;
    if (ybytes) {
        const hipError_t e = scratch_alloc(&ybuf, ybytes, s);
        if (e != hipSuccess) return ret(hip_status(e));
    }
    int st = PENT_OK;
    bool ywords_clear = false;
    // x sweeps, system (y, k) being nx contiguous values: the single pass
    // forms the explicit right-hand side from C itself where a tile of it
    // fits on the device; else the stencil pass writes it to R first
    if (hx->tst_cap == 0) hx->tst_cap = onepass_t_capacity(true);
    if (hx->tst_cap > 0 && onepass_t_groups(nx) <= hx->tst_cap / 4 &&
        (batch + 63) / 64 * onepass_t_groups(nx) <= (int64_t)UINT32_MAX / 2) {
        const SegRec *seg64 = seg_cache(hx, 64, &st);
        if (seg64) {
            void *xbuf = nullptr;
            hipError_t e = scratch_alloc(&xbuf, onepass_t_scratch_bytes(nx, batch), s);
            if (e == hipSuccess) {
                const bool clear = ykind == 4 &&
                                   onepass_words(hy->n, yseg, ybatch) <= onepass_t_threads(nx, batch);
                e = launch_onepass_t_ch2d(hx->d_fwd, hx->d_bwd, seg64, nx, C, R, ny, ninst, dt, h, xbuf,
                                          hx->d_err, s, clear ? (unsigned int *)ybuf : nullptr,
                                          clear ? onepass_words(hy->n, yseg, ybatch) : 0);
                const hipError_t e2 = hipFreeAsync(xbuf, s);
                if (e == hipSuccess) e = e2;
                ywords_clear = clear && e == hipSuccess;
            }
            if (e != hipSuccess) st = hip_status(e);
        }
    } else {
        st = pent_ch2d_rhs(C, R, ny, ninst, nx, dt, h, stream);
        if (st == PENT_OK) st = pent_solve_strided(hx, R, batch, nx, stream);
    }
    // y sweeps: batch-fastest over (k, x), read from R, written into C
    if (st == PENT_OK) st = solve_io(hy, R, false, ybatch, C, ybatch, ybatch, ybuf, s, ywords_clear);
    if (ybuf) {
        const hipError_t e = hipFreeAsync(ybuf, s);
        if (st == PENT_OK && e != hipSuccess) st = hip_status(e);
    }
    return ret(st);
}

pent_cyclic pent_cyclic_factor(int64_t n, const double *a, const double *b, const double *c,
                               const double *d, const double *e)
{
    g_pivot_row = -1;
    if (n < 5 || n > INT32_MAX || !a || !b || !c || !d || !e) {
        ret(PENT_INVALID_VALUE);
        return nullptr;
    }
    int st;
    pent_cyclic cy = new_cyclic(n, &st);
    if (!cy) {
        ret(st);
        return nullptr;
    }
    const double *src[5] = {a, b, c, d, e};
    hipError_t err = hipSuccess;
    for (int k = 0; k < 5 && err == hipSuccess; k++)
        err = hipMemcpy(cy->d_cd + k * cyc_ld(n), src[k], sizeof(double) * n, hipMemcpyHostToDevice);
    if (err != hipSuccess) {
        free_cyclic(cy);
        ret(hip_status(err));
        return nullptr;
    }
    return finish_cyclic(cy);
}

pent_cyclic pent_cyclic_factor_d4(int64_t n, double sigma)
{
    g_pivot_row = -1;
    if (n < 5 || n > INT32_MAX || !std::isfinite(sigma)) {
        ret(PENT_INVALID_VALUE);
        return nullptr;
    }
    int st;
    pent_cyclic cy = new_cyclic(n, &st);
    if (!cy) {
        ret(st);
        return nullptr;
    }
    hipError_t err = launch_cyc_assemble_d4(cy->d_cd, n, sigma, 0);
    if (err != hipSuccess) {
        free_cyclic(cy);
        ret(hip_status(err));
        return nullptr;
    }
    return finish_cyclic(cy);
}

int pent_cyclic_solve(pent_cyclic c, double *F, int64_t batch, int64_t ld, void *stream)
{
    if (!cvalid(c) || batch < 0 || ld < batch) return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!F) return ret(PENT_INVALID_VALUE);
    const hipStream_t s = (hipStream_t)stream;
    if (cyc_single_pass(c, batch, false)) return ret(cyc_run_single(c, false, F, ld, F, ld, batch, s));
    int st = solve_io_scratch(c->E, F, ld, F, ld, batch, s);
    if (st != PENT_OK) return ret(st);
    return ret(hip_status(launch_cyc_correct(c->d_aux, c->d_Z, F, c->n, batch, ld, s)));
}

int pent_cyclic_cn_step(pent_cyclic c, const double *C, int64_t ldc, double *X, int64_t ldx,
                        int64_t batch, void *stream)
{
    if (!cvalid(c) || batch < 0 || ldc < batch || ldx < batch) return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!C || !X || (const void *)C == (const void *)X) return ret(PENT_INVALID_VALUE);
    const hipStream_t s = (hipStream_t)stream;
    if (cyc_single_pass(c, batch, true)) return ret(cyc_run_single(c, true, C, ldc, X, ldx, batch, s));
    int st = hip_status(launch_cn_rhs(c->d_cd, c->n, C, ldc, X, ldx, batch, s));
    if (st != PENT_OK) return ret(st);
    return pent_cyclic_solve(c, X, batch, ldx, stream);
}

int pent_cyclic_set_schedule(pent_cyclic c, int kind, int seg_rows)
{
    if (!cvalid(c)) return ret(PENT_INVALID_VALUE);
    if (kind == 0 || kind == 1) {
        c->kind = kind;
        return ret(PENT_OK);
    }
    if (kind == 2 && (seg_rows == 32 || seg_rows == 64)) {
        c->kind = 2;
        c->seg_rows = seg_rows;
        return ret(PENT_OK);
    }
    return ret(PENT_INVALID_VALUE);
}

int pent_cyclic_query_schedule(pent_cyclic c, int64_t batch, int cn, int *kind, int *seg_rows)
{
    if (!cvalid(c) || batch < 0 || !kind || !seg_rows) return ret(PENT_INVALID_VALUE);
    const bool one = cyc_single_pass(c, batch, cn != 0);
    *kind = one ? 2 : 1;
    *seg_rows = one ? c->seg_rows : 0;
    return ret(PENT_OK);
}

int pent_cyclic_check(pent_cyclic c)
{
    if (!cvalid(c)) return ret(PENT_INVALID_VALUE);
    return pent_check(c->E);
}

int pent_cyclic_cn_rhs(pent_cyclic c, const double *C, int64_t ldc, double *R, int64_t ldr,
                       int64_t batch, void *stream)
{
    if (!cvalid(c) || batch < 0 || ldc < batch || ldr < batch) return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!C || !R || (const void *)C == (const void *)R) return ret(PENT_INVALID_VALUE);
    return ret(hip_status(launch_cn_rhs(c->d_cd, c->n, C, ldc, R, ldr, batch, (hipStream_t)stream)));
}

int pent_cyclic_bordering(pent_cyclic c, double *Z, double *minv)
{
    if (!cvalid(c) || !Z || !minv) return ret(PENT_INVALID_VALUE);
    CycAux aux;
    hipError_t e = hipMemcpy(Z, c->d_Z, sizeof(double) * 2 * (c->n - 2), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&aux, c->d_aux, sizeof(CycAux), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ret(hip_status(e));
    std::memcpy(minv, aux.minv, sizeof(aux.minv));
    return ret(PENT_OK);
}

int pent_cyclic_destroy(pent_cyclic c)
{
    if (c == nullptr) return ret(PENT_OK);
    if (!cvalid(c)) return ret(PENT_INVALID_VALUE);
    free_cyclic(c);
    return ret(PENT_OK);
}

size_t pent_rewrite_workspace_size(int64_t n, int64_t batch)
{
    if (n < 1 || batch < 0) return 0;
    return rewrite_workspace_bytes(n, batch);
}

int pent_solve_rewrite(int64_t n, const double *a, const double *b, const double *c,
                       const double *d, const double *e, int64_t ldm, double *F, int64_t batch,
                       int64_t ld, void *work, size_t work_bytes, void *stream)
{
    if (n < 1 || n > INT32_MAX || batch < 0 || ldm < batch || ld < batch)
        return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!a || !b || !c || !d || !e || !F || !work) return ret(PENT_INVALID_VALUE);
    if (work_bytes < rewrite_workspace_bytes(n, batch)) return ret(PENT_SIZE_MISMATCH);
    return ret(hip_status(launch_rewrite(a, b, c, d, e, ldm, n, F, batch, ld, work,
                                         (hipStream_t)stream)));
}

int pent_rewrite_check(const void *work, int64_t n, int64_t *system, int64_t *row)
{
    if (!work || n < 1) return ret(PENT_INVALID_VALUE);
    unsigned long long key = 0;
    hipError_t e = hipMemcpy(&key, work, sizeof(key), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return ret(hip_status(e));
    if (key == ~0ull) {
        if (system) *system = -1;
        if (row) *row = -1;
        return ret(PENT_OK);
    }
    if (system) *system = (int64_t)(key / (unsigned long long)n);
    if (row) *row = (int64_t)(key % (unsigned long long)n);
    g_pivot_row = (int64_t)(key % (unsigned long long)n);
    return ret(PENT_ZERO_PIVOT);
}

int pent_solve_strided(pent_handle h, double *F, int64_t batch, int64_t ld, void *stream)
{
    if (!valid(h) || batch < 0 || ld < h->n) return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!F) return ret(PENT_INVALID_VALUE);
    hipStream_t s = (hipStream_t)stream;
    // the single pass (blocks transposed through LDS) where a tile of it
    // fits on the device; else one lane per system
    if (h->t_cap == 0) h->t_cap = onepass_t_capacity();
    if (h->t_cap > 0 && onepass_t_groups(h->n) <= h->t_cap / 4 &&
        (batch + 63) / 64 * onepass_t_groups(h->n) <= (int64_t)UINT32_MAX / 2) {
        int st;
        const SegRec *seg64 = seg_cache(h, 64, &st);
        if (!seg64) return ret(st);
        void *xbuf = nullptr;
        hipError_t e = scratch_alloc(&xbuf, onepass_t_scratch_bytes(h->n, batch), s);
        if (e != hipSuccess) return ret(hip_status(e));
        e = launch_onepass_t(h->d_fwd, h->d_bwd, seg64, h->n, F, batch, ld, xbuf, h->d_err, s);
        const hipError_t e2 = hipFreeAsync(xbuf, s);
        return ret(hip_status(e != hipSuccess ? e : e2));
    }
    return ret(hip_status(launch_strided_sweep(h->d_fwd, h->d_bwd, h->n, F, batch, ld, s)));
}

int pent_get_factors(pent_handle h, double *alpha, double *beta, double *gamma, double *delta)
{
    if (!valid(h) || !alpha || !beta || !gamma || !delta) return ret(PENT_INVALID_VALUE);
    const int64_t n = h->n;
    double *outs[4] = {alpha, beta, gamma, delta};
    for (int k = 0; k < 4; k++) {
        hipError_t e = hipMemcpy(outs[k], h->d_fac + k * n, sizeof(double) * n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return ret(hip_status(e));
    }
    return ret(PENT_OK);
}

int pent_get_diagonals(pent_handle h, double *a, double *b, double *c, double *d, double *e)
{
    if (!valid(h) || !a || !b || !c || !d || !e) return ret(PENT_INVALID_VALUE);
    const int64_t n = h->n;
    double *outs[5] = {a, b, c, d, e};
    for (int k = 0; k < 5; k++) {
        hipError_t err = hipMemcpy(outs[k], h->d_diag + k * n, sizeof(double) * n, hipMemcpyDeviceToHost);
        if (err != hipSuccess) return ret(hip_status(err));
    }
    return ret(PENT_OK);
}

int64_t pent_size(pent_handle h)
{
    if (!valid(h)) {
        ret(PENT_INVALID_VALUE);
        return -1;
    }
    ret(PENT_OK);
    return h->n;
}

int pent_set_schedule(pent_handle h, int kind, int seg_rows)
{
    if (!valid(h)) return ret(PENT_INVALID_VALUE);
    if (kind == 0 || kind == 3) {
        h->sched_kind = kind;
        h->sched_seg = 0;
        return ret(PENT_OK);
    }
    if (kind == 1 && (seg_rows == 0 || seg_rows == 8 || seg_rows == 16 || seg_rows == 32)) {
        h->sched_kind = 1;
        h->sched_seg = seg_rows == 0 ? 16 : seg_rows;  // prefetch depth
        return ret(PENT_OK);
    }
    if (kind == 2 && (seg_rows == 16 || seg_rows == 32 || seg_rows == 64)) {
        h->sched_kind = 2;
        h->sched_seg = seg_rows;
        return ret(PENT_OK);
    }
    if (kind == 4 && (seg_rows == 32 || seg_rows == 64)) {
        query_onepass_cap(h, seg_rows);
        h->sched_kind = 4;
        h->sched_seg = seg_rows;
        return ret(PENT_OK);
    }
    return ret(PENT_INVALID_VALUE);
}

int pent_check(pent_handle h)
{
    if (!valid(h)) return ret(PENT_INVALID_VALUE);
    unsigned int w = 0;
    hipError_t e = hipMemcpy(&w, h->d_err, sizeof(w), hipMemcpyDeviceToHost);
    if (e == hipSuccess && w) e = hipMemset(h->d_err, 0, sizeof(w));
    if (e != hipSuccess) return ret(hip_status(e));
    if (w & 1u) return ret(PENT_TIMEOUT);
    if (w & 2u) return ret(PENT_NOT_CONVERGED);
    return ret(PENT_OK);
}

int pent_set_refine_tolerance(pent_handle h, double tol)
{
    if (!valid(h) || !(tol >= 0.0) || !std::isfinite(tol)) return ret(PENT_INVALID_VALUE);
    h->refine_tol = tol;
    return ret(PENT_OK);
}

int pent_query_schedule(pent_handle h, int64_t batch, int *kind, int *seg_rows)
{
    if (!valid(h) || batch < 0 || !kind || !seg_rows) return ret(PENT_INVALID_VALUE);
    io_schedule(h, batch, true, kind, seg_rows);  // what an in-place pent_solve runs
    if (*kind == 3) *seg_rows = 0;
    return ret(PENT_OK);
}

int pent_stream_copy(const double *src, int64_t ld_src, double *dst, int64_t ld_dst, int64_t n,
                     int64_t batch, void *stream)
{
    if (n < 1 || batch < 0 || ld_src < batch || ld_dst < batch) return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!src || !dst) return ret(PENT_INVALID_VALUE);
    return ret(hip_status(launch_block_copy(src, dst, n, batch, ld_src, ld_dst, (hipStream_t)stream)));
}

int pent_stream_copy_shaped(const double *src, int64_t ld_src, double *dst, int64_t ld_dst,
                            int64_t n, int64_t batch, int tiles_across, int waves_down,
                            void *stream)
{
    const bool shape = (tiles_across == 1 && (waves_down == 2 || waves_down == 4)) ||
                       (tiles_across == 2 && (waves_down == 1 || waves_down == 2)) ||
                       (tiles_across == 4 && waves_down == 1);
    if (!shape || n < 1 || batch < 0 || ld_src < batch || ld_dst < batch) return ret(PENT_INVALID_VALUE);
    if (batch == 0) return ret(PENT_OK);
    if (!src || !dst) return ret(PENT_INVALID_VALUE);
    return ret(hip_status(launch_block_copy(src, dst, n, batch, ld_src, ld_dst, (hipStream_t)stream,
                                            tiles_across, waves_down)));
}

int pent_last_status(void) { return g_status; }

int64_t pent_last_pivot_row(void) { return g_pivot_row; }

const char *pent_status_string(int status)
{
    switch (status) {
    case PENT_OK: return "success";
    case PENT_INVALID_VALUE: return "invalid argument";
    case PENT_ZERO_PIVOT: return "zero or non-finite pivot (matrix not factorable without pivoting)";
    case PENT_OUT_OF_MEMORY: return "device out of memory";
    case PENT_HIP_ERROR: return "HIP runtime error";
    case PENT_NOT_CONVERGED: return "iterative refinement did not converge";
    case PENT_SIZE_MISMATCH: return "buffer sizes disagree";
    case PENT_NOT_SUPPORTED: return "not supported";
    case PENT_TIMEOUT: return "a device-side wait ran out (work list not drained)";
    default: return "unknown status";
    }
}

}  // extern "C"
