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
// and writes x in place.  No workgroup ever waits for another, so this
// kernel runs at any size; the single pass over all matrices (onepass.hip)
// is faster where its tiles fit on the device.
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
        static_assert(kGK == 64, "segment records are the 64-row ones");
        const CSeg segr = (CSeg)m.seg64;
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

__global__ void k_zero_u32(unsigned int *p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

}  // namespace

// The persistent kernel: 64-row segments, eight waves per workgroup (the
// shape that measured fastest of 64/32 rows x 8/4 waves).
constexpr int kPK = 64, kPW = 8;

int group_max_blocks()
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_group<kPK, kPW>, 64 * kPW,
                                                     0) != hipSuccess)
        return 0;
    return cus * (per_cu > 0 ? per_cu : 1);
}

hipError_t launch_group_init(unsigned int *ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, ctr, 3);
    return hipGetLastError();
}

hipError_t launch_group(const GroupMat *mats, const GroupItem *items, int nitems, double *summ,
                        unsigned int *ctr, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_group<kPK, kPW>), dim3((unsigned)nblocks), dim3(64 * kPW), 0, s, mats, items,
                       nitems, summ, ctr);
    return hipGetLastError();
}

}  // namespace pent
