// group.hip -- many matrices, each with its own right-hand sides, solved in
// one persistent launch.
//
// Work item = (matrix k, group of up to 64 consecutive systems of matrix k).
// Items are sorted longest first (rows x systems) and handed out through an
// atomic counter; every workgroup loops until the list is exhausted, and the
// last workgroup to leave resets the counters, so the next launch on the
// stream starts from a clean list without a memset (safe inside a captured
// graph).
//
// One workgroup (kGroupWaves waves) solves one item with the partitioned
// sweep of sweep.hip, entirely inside the workgroup: lane = system, each
// wave takes whole segments of 64 rows; pass 1 writes the segment summaries
// to the item's slice of the workspace, wave 0 runs the interface recurrence
// over the segments, pass 2 repeats the sweeps from the true incoming states
// and writes x in place.  No workgroup ever waits for another.
#include "lookback.h"

namespace pent {
namespace {


// Pointers read from the device table are generic; give them their address
// spaces back so records become scalar loads and data global (not flat) loads.
typedef __attribute__((address_space(4))) const FwdRec *CFwd;
typedef __attribute__((address_space(4))) const BwdRec *CBwd;
typedef __attribute__((address_space(4))) const SegRec *CSeg;
typedef __attribute__((address_space(1))) double *GDbl;

template <int kGK>
__device__ __forceinline__ void load_seg(double (&v)[kGK], GDbl base, int64_t ld, int L)
{
    if (L == kGK) {
#pragma unroll
        for (int k = 0; k < kGK; k++) v[k] = __builtin_nontemporal_load(base + k * ld);
    } else {
#pragma unroll
        for (int k = 0; k < kGK; k++) v[k] = (k < L) ? base[k * ld] : 0.0;
    }
}

// Sweeps over one segment; the per-row records are wave-uniform (every lane
// of the wave is on the same row), so they come through scalar loads.
// Rows past n have all-zero records and zero data, so no per-row guards.
template <int kGK>
__device__ __forceinline__ void fwd_seg(double (&v)[kGK], CFwd fwd, int64_t r0, double &p2,
                                        double &p1)
{
#pragma unroll
    for (int k = 0; k < kGK; k++) {
        const double ra = fwd[r0 + k].ra, ap = fwd[r0 + k].ap, bp = fwd[r0 + k].bp;
        const double g = fma(-bp, p1, fma(-ap, p2, ra * v[k]));
        v[k] = g;
        p2 = p1;
        p1 = g;
    }
}

template <int kGK>
__device__ __forceinline__ void bwd_seg(double (&v)[kGK], CBwd bwd, int64_t r0, double &q1,
                                        double &q2)
{
#pragma unroll
    for (int k = kGK - 1; k >= 0; k--) {
        const double gm = bwd[r0 + k].gm, dl = bwd[r0 + k].dl;
        const double x = fma(-gm, q1, fma(-dl, q2, v[k]));
        v[k] = x;
        q2 = q1;
        q1 = x;
    }
}

// kGK rows per segment, kGroupWaves waves per workgroup (tuned per group).
template <int kGK, int kGroupWaves>
__global__ __launch_bounds__(64 * kGroupWaves) void k_group(const GroupMat *__restrict__ mats,
                                                            const GroupItem *__restrict__ items,
                                                            int nitems, double *__restrict__ summ,
                                                            unsigned int *__restrict__ ctr)
{
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid / 64), lane = tid % 64;
    for (;;) {
        if (tid == 0) s_item = (int)atomicAdd(&ctr[0], 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);  // wave-uniform: scalar loads below
        __syncthreads();  // everyone has read s_item before it is reused
        if (it >= nitems) break;
        const GroupItem item = items[it];
        const GroupMat m = mats[item.mat];
        const CFwd fwd = (CFwd)m.fwd;
        const CBwd bwd = (CBwd)m.bwd;
        const CSeg segr = (CSeg)(kGK == 64 ? m.seg64 : m.seg32);
        const int64_t n = m.n;
        const int nseg = (int)((n + kGK - 1) / kGK);
        const bool act = lane < item.ncols;
        const int64_t j = item.col0 + (act ? lane : 0);
        GDbl col = (GDbl)m.F + j;
        GDbl S = (GDbl)summ + item.summ_off * (64 / kGK);  // [seg][4][64]

        // pass 1: zero-incoming sweeps per segment, outgoing states to S
        for (int sg = w; sg < nseg; sg += kGroupWaves) {
            const int64_t r0 = (int64_t)sg * kGK;
            const int L = (int)((n - r0) < kGK ? (n - r0) : kGK);
            double v[kGK];
            load_seg(v, col + r0 * m.ld, m.ld, act ? L : 0);
            double p2 = 0.0, p1 = 0.0, q1 = 0.0, q2 = 0.0;
            fwd_seg(v, fwd, r0, p2, p1);
            bwd_seg(v, bwd, r0, q1, q2);
            GDbl o = S + (int64_t)sg * 256 + lane;
            o[0] = p2;
            o[64] = p1;
            o[128] = q1;
            o[192] = q2;
        }
        __threadfence_block();
        __syncthreads();

        // interface recurrence (wave 0, lane = system)
        if (w == 0) interface_chain(S + lane, (int64_t)256, (int64_t)64, segr, (int64_t)nseg);
        __threadfence_block();
        __syncthreads();

        // pass 2: sweeps from the true incoming states, x in place
        for (int sg = w; sg < nseg; sg += kGroupWaves) {
            const int64_t r0 = (int64_t)sg * kGK;
            const int L = (int)((n - r0) < kGK ? (n - r0) : kGK);
            double v[kGK];
            GDbl base = col + r0 * m.ld;
            load_seg(v, base, m.ld, act ? L : 0);
            GDbl o = S + (int64_t)sg * 256 + lane;
            double p2 = o[0], p1 = o[64], q1 = o[128], q2 = o[192];
            fwd_seg(v, fwd, r0, p2, p1);
            bwd_seg(v, bwd, r0, q1, q2);
            if (act) {
                if (L == kGK) {
#pragma unroll
                    for (int k = 0; k < kGK; k++) __builtin_nontemporal_store(v[k], base + k * m.ld);
                } else {
#pragma unroll
                    for (int k = 0; k < kGK; k++)
                        if (k < L) base[k * m.ld] = v[k];
                }
            }
        }
        __syncthreads();  // the item's summaries are not reused, but keep waves together
    }
    // last workgroup out resets the counters for the next launch
    if (tid == 0) {
        __threadfence();
        const unsigned int done = atomicAdd(&ctr[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&ctr[0], 0u);
            atomicExch(&ctr[1], 0u);
            __threadfence();
        }
    }
}

// Decoupled variant: one-wave workgroups, each pulling (item, segment)
// tasks from one counter.  Tasks [0, T) are pass 1 of every segment of every
// item (items longest first), tasks [T, 2T) pass 2 in the same order.  The
// wave that completes the last pass-1 task of an item runs the item's
// interface recurrence and then publishes ready[item]; a pass-2 task waits
// for that flag.  Every pass-2 task is handed out only after all pass-1
// tasks have been handed to running waves, and those never wait on
// anything, so every flag is eventually published; the wait is bounded
// anyway and a timeout is reported through ctr[2] instead of hanging.
//
// No branch in this kernel depends on the lane index alone: the atomics are
// executed by every lane (lanes other than 0 add zero, stores repeat the same
// value) and lane 0's result is read back with readlane.  With a lane-0-only
// fetch the compiler may thread the loop's back edge round the fetch for
// the other lanes, which then re-run the previous task.
constexpr int kSpinLimit = 1 << 24;

__device__ __forceinline__ unsigned int wave_fetch_add(unsigned int *p, unsigned int v)
{
    const unsigned int r = atomicAdd(p, threadIdx.x == 0 ? v : 0u);
    return (unsigned int)__builtin_amdgcn_readlane((int)r, 0);
}

// Every lane polls the flag (one address); true once it reads non-zero.
// The flag and the summaries move with relaxed agent-scope accesses, ordered
// by waiting for the writer's own stores before its flag (as the single
// pass does): acquire / release operations would invalidate or write back a
// whole XCD L2 per poll.
__device__ __forceinline__ bool wait_flag(unsigned int *flag)
{
    for (int spins = 0; spins < kSpinLimit; spins++) {
        const unsigned int v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (__builtin_amdgcn_readlane((int)v, 0) != 0) return true;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

// Device-coherent element access for interface_chain over the summaries,
// which waves on other XCDs wrote.
struct CohRef {
    double *p;
    __device__ operator double() const { return lb::xload(p); }
    __device__ CohRef &operator=(double v)
    {
        lb::xstore(p, v);
        return *this;
    }
};
struct CohPtr {
    double *p;
    __device__ CohRef operator[](int64_t i) const { return CohRef{p + i}; }
};

template <int kGK>
__global__ __launch_bounds__(64) void k_group_tasks(const GroupMat *__restrict__ mats,
                                                    const GroupItem *__restrict__ items,
                                                    const int2 *__restrict__ tasks, int ntasks,
                                                    int nitems, double *__restrict__ summ,
                                                    unsigned int *__restrict__ ctr,
                                                    unsigned int *__restrict__ cnt,
                                                    unsigned int *__restrict__ ready)
{
    const int lane = threadIdx.x;
    for (;;) {
        const int t = (int)wave_fetch_add(&ctr[0], 1u);
        if (t >= 2 * ntasks) break;
        const bool pass1 = t < ntasks;
        const int2 task = tasks[pass1 ? t : t - ntasks];
        const int ii = __builtin_amdgcn_readfirstlane(task.x);
        const int sg = __builtin_amdgcn_readfirstlane(task.y);
        const GroupItem item = items[ii];
        const GroupMat m = mats[item.mat];
        const CFwd fwd = (CFwd)m.fwd;
        const CBwd bwd = (CBwd)m.bwd;
        const CSeg segr = (CSeg)(kGK == 64 ? m.seg64 : m.seg32);
        const int64_t n = m.n;
        const int nseg = (int)((n + kGK - 1) / kGK);
        const bool act = lane < item.ncols;
        const int64_t j = item.col0 + (act ? lane : 0);
        GDbl col = (GDbl)m.F + j;
        GDbl S = (GDbl)summ + item.summ_off * (64 / kGK);
        const int64_t r0 = (int64_t)sg * kGK;
        const int L = (int)((n - r0) < kGK ? (n - r0) : kGK);
        GDbl base = col + r0 * m.ld;
        GDbl o = S + (int64_t)sg * 256 + lane;
        double v[kGK];
        if (pass1) {
            load_seg(v, base, m.ld, act ? L : 0);
            double p2 = 0.0, p1 = 0.0, q1 = 0.0, q2 = 0.0;
            fwd_seg(v, fwd, r0, p2, p1);
            bwd_seg(v, bwd, r0, q1, q2);
            double *oc = (double *)o;
            lb::xstore(oc, p2);
            lb::xstore(oc + 64, p1);
            lb::xstore(oc + 128, q1);
            lb::xstore(oc + 192, q2);
            lb::store_fence();  // summaries complete before the count
            const int c = (int)wave_fetch_add(&cnt[ii], 1u);
            if (c == nseg - 1) {  // last segment of this item: resolve its interfaces
                // every other segment counted after storing its summaries
                interface_chain(CohPtr{(double *)(S + lane)}, (int64_t)256, (int64_t)64, segr,
                                (int64_t)nseg);
                lb::store_fence();
                __hip_atomic_store(&ready[ii], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else if (!wait_flag(&ready[ii])) {
            atomicExch(&ctr[2], 1u);
        } else {
            load_seg(v, base, m.ld, act ? L : 0);
            const double *oc = (const double *)o;
            double p2 = lb::xload(oc), p1 = lb::xload(oc + 64), q1 = lb::xload(oc + 128),
                   q2 = lb::xload(oc + 192);
            fwd_seg(v, fwd, r0, p2, p1);
            bwd_seg(v, bwd, r0, q1, q2);
            if (act) {
                if (L == kGK) {
#pragma unroll
                    for (int k = 0; k < kGK; k++) __builtin_nontemporal_store(v[k], base + k * m.ld);
                } else {
#pragma unroll
                    for (int k = 0; k < kGK; k++)
                        if (k < L) base[k * m.ld] = v[k];
                }
            }
        }
    }
    // last wave out resets the counters and flags for the next launch
    __threadfence();
    const unsigned int d = wave_fetch_add(&ctr[1], 1u);
    if (d == gridDim.x - 1) {
        __threadfence();
        for (int i = lane; i < nitems; i += 64) {
            cnt[i] = 0u;
            ready[i] = 0u;
        }
        __threadfence();
        atomicExch(&ctr[0], 0u);
        atomicExch(&ctr[1], 0u);
        __threadfence();
    }
}

__global__ void k_zero_u32(unsigned int *p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

}  // namespace

// variants 0..3: one workgroup per item (64/32 rows, 8/4 waves);
// variants 4, 5: decoupled one-wave tasks (64/32 rows).
int group_variants() { return 6; }

static void variant_shape(int v, int *K, int *W)
{
    if (v >= 4) {
        *K = v == 4 ? 64 : 32;
        *W = 1;
        return;
    }
    *K = (v & 1) ? 32 : 64;
    *W = (v & 2) ? 4 : 8;
}

bool group_variant_is_tasks(int v) { return v >= 4; }

int group_variant_seg_rows(int v)
{
    int K, W;
    variant_shape(v, &K, &W);
    return K;
}

static const void *variant_fn(int v)
{
    switch (v) {
    case 0: return (const void *)k_group<64, 8>;
    case 1: return (const void *)k_group<32, 8>;
    case 2: return (const void *)k_group<64, 4>;
    case 3: return (const void *)k_group<32, 4>;
    case 4: return (const void *)k_group_tasks<64>;
    default: return (const void *)k_group_tasks<32>;
    }
}

int group_max_blocks(int v)
{
    int dev = 0, cus = 0, per_cu = 0, K, W;
    variant_shape(v, &K, &W);
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, variant_fn(v), 64 * W, 0) != hipSuccess)
        return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
}

hipError_t launch_group_init(unsigned int *ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ctr, 3);
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int *p, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_group(int v, const GroupMat *mats, const GroupItem *items, int nitems,
                        const int2 *tasks, int ntasks, double *summ, unsigned int *ctr,
                        unsigned int *cnt, unsigned int *ready, int nblocks, hipStream_t s)
{
    int K, W;
    variant_shape(v, &K, &W);
    const dim3 grid((unsigned)nblocks), block(64 * W);
    switch (v) {
    case 0: hipLaunchKernelGGL((k_group<64, 8>), grid, block, 0, s, mats, items, nitems, summ, ctr); break;
    case 1: hipLaunchKernelGGL((k_group<32, 8>), grid, block, 0, s, mats, items, nitems, summ, ctr); break;
    case 2: hipLaunchKernelGGL((k_group<64, 4>), grid, block, 0, s, mats, items, nitems, summ, ctr); break;
    case 3: hipLaunchKernelGGL((k_group<32, 4>), grid, block, 0, s, mats, items, nitems, summ, ctr); break;
    case 4:
        hipLaunchKernelGGL((k_group_tasks<64>), grid, block, 0, s, mats, items, tasks, ntasks, nitems,
                           summ, ctr, cnt, ready);
        break;
    default:
        hipLaunchKernelGGL((k_group_tasks<32>), grid, block, 0, s, mats, items, tasks, ntasks, nitems,
                           summ, ctr, cnt, ready);
        break;
    }
    return hipGetLastError();
}

}  // namespace pent
