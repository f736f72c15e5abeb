// sweep.hip -- FP64 forward / backward sweeps over batch-fastest right-hand
// sides (element (i, j) at F[i*ld + j], Sec. 2.6).
//
// Two schedules:
//  * lane:        one lane per system runs the forward sweep over all rows and
//                 then the back substitution (the paper's one-thread-per-system
//                 schedule, Sec. 2.4 last paragraph).  A wave covers 64
//                 consecutive systems, so every row access is one coalesced
//                 512-byte segment; the per-row factors are wave-uniform and
//                 come through scalar loads; the two carried values live in
//                 registers; rows are prefetched D at a time, double-buffered
//                 (D = 8, 16 or 32: the prefetch depth, a tuning knob).
//                 g is written over f between the sweeps.
//  * partitioned: the rows are cut into segments of K rows and every
//                 (segment, system) pair gets its own lane.  By linearity the
//                 solution on a segment is the solution with zero incoming
//                 states plus the responses to the two incoming forward values
//                 (g_{r0-2}, g_{r0-1}) and the two incoming backward values
//                 (x_{r1}, x_{r1+1}).  Pass 1 finds, per segment, the outgoing
//                 states of the zero-incoming sweeps; a short serial
//                 recurrence over the segments (2x2 transfer matrices that
//                 depend on A only) turns them into the true incoming states;
//                 pass 2 repeats the sweeps with those states and writes x.
//                 Reads f twice, writes x once, and never writes g.
#include "internal.h"

namespace pent {
namespace {

// ------------------------------------------------------------------ lane ----
template <int D>
__device__ __forceinline__ void load_block(double (&buf)[D], const double *col, int64_t ld,
                                           int i0)
{
#pragma unroll
    for (int k = 0; k < D; k++) buf[k] = __builtin_nontemporal_load(col + (int64_t)(i0 + k) * ld);
}

template <int D>
__device__ __forceinline__ void fwd_block(const double (&buf)[D], double *col, int64_t ld, int i0,
                                          const FwdRec *__restrict__ fwd, double &p2, double &p1)
{
#pragma unroll
    for (int k = 0; k < D; k++) {
        const FwdRec r = fwd[i0 + k];
        const double g = fma(-r.bp, p1, fma(-r.ap, p2, r.ra * buf[k]));
        col[(int64_t)(i0 + k) * ld] = g;
        p2 = p1;
        p1 = g;
    }
}

template <int D>
__device__ __forceinline__ void load_block_rev(double (&buf)[D], const double *col, int64_t ld,
                                               int i0)
{
    // buf[k] = row i0 - k  (descending)
#pragma unroll
    for (int k = 0; k < D; k++) buf[k] = col[(int64_t)(i0 - k) * ld];
}

template <int D>
__device__ __forceinline__ void bwd_block(const double (&buf)[D], double *col, int64_t ld, int i0,
                                          const BwdRec *__restrict__ bwd, double &q1, double &q2)
{
#pragma unroll
    for (int k = 0; k < D; k++) {
        const BwdRec r = bwd[i0 - k];
        const double x = fma(-r.gm, q1, fma(-r.dl, q2, buf[k]));
        __builtin_nontemporal_store(x, col + (int64_t)(i0 - k) * ld);
        q2 = q1;
        q1 = x;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_lane(const FwdRec *__restrict__ fwd,
                                              const BwdRec *__restrict__ bwd, int n,
                                              double *__restrict__ F, int64_t batch, int64_t ld)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;  // no barriers below: lanes past the batch just leave
    double *col = F + j;
    const int nb = n / D;

    // forward sweep, rows ascending
    double p2 = 0.0, p1 = 0.0;
    {
        double bufA[D], bufB[D];
        int b = 0;
        if (nb > 0) load_block<D>(bufA, col, ld, 0);
        for (; b + 1 < nb; b += 2) {
            load_block<D>(bufB, col, ld, (b + 1) * D);
            fwd_block<D>(bufA, col, ld, b * D, fwd, p2, p1);
            if (b + 2 < nb) load_block<D>(bufA, col, ld, (b + 2) * D);
            fwd_block<D>(bufB, col, ld, (b + 1) * D, fwd, p2, p1);
        }
        if (b < nb) fwd_block<D>(bufA, col, ld, b * D, fwd, p2, p1);
        for (int i = nb * D; i < n; i++) {
            const FwdRec r = fwd[i];
            const double g = fma(-r.bp, p1, fma(-r.ap, p2, r.ra * col[(int64_t)i * ld]));
            col[(int64_t)i * ld] = g;
            p2 = p1;
            p1 = g;
        }
    }

    // back substitution, rows descending: first the ragged tail, then blocks
    double q1 = 0.0, q2 = 0.0;
    for (int i = n - 1; i >= nb * D; i--) {
        const BwdRec r = bwd[i];
        const double x = fma(-r.gm, q1, fma(-r.dl, q2, col[(int64_t)i * ld]));
        col[(int64_t)i * ld] = x;
        q2 = q1;
        q1 = x;
    }
    {
        double bufA[D], bufB[D];
        int b = nb - 1;
        if (b >= 0) load_block_rev<D>(bufA, col, ld, b * D + D - 1);
        for (; b - 1 >= 0; b -= 2) {
            load_block_rev<D>(bufB, col, ld, (b - 1) * D + D - 1);
            bwd_block<D>(bufA, col, ld, b * D + D - 1, bwd, q1, q2);
            if (b - 2 >= 0) load_block_rev<D>(bufA, col, ld, (b - 2) * D + D - 1);
            bwd_block<D>(bufB, col, ld, (b - 1) * D + D - 1, bwd, q1, q2);
        }
        if (b >= 0) bwd_block<D>(bufA, col, ld, b * D + D - 1, bwd, q1, q2);
    }
}

// ------------------------------------------------------------ partitioned ----
// Summary layout: summ[(s*4 + q)*summ_ld + j], q = 0,1 forward state, 2,3
// backward state.  Pass 1 writes the zero-incoming outgoing states; the chain
// overwrites them with the true incoming states of the segment.

template <int K, typename TI>
__device__ __forceinline__ void seg_load(double (&v)[K], const TI *col, int64_t ld, int64_t r0,
                                         int L)
{
    const TI *base = col + r0 * ld;
    if (L == K) {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = (double)__builtin_nontemporal_load(base + k * ld);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = (k < L) ? (double)base[k * ld] : 0.0;
    }
}

// Row records of a segment: lane k of the wave loads the records of row
// r0 + k (one coalesced load per wave), and step k of a sweep takes them from
// lane k with v_readlane into scalar registers.  Rows past n have all-zero
// records, so the sweeps need no per-row guards.
__device__ __forceinline__ double lane_bcast(double v, int k)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

struct LaneRecs {
    double ra, ap, bp, gm, dl;
};

__device__ __forceinline__ LaneRecs load_lane_recs(const FwdRec *__restrict__ fwd,
                                                   const BwdRec *__restrict__ bwd, int64_t r0,
                                                   int K, int64_t npad)
{
    const int lane = threadIdx.x & 63;
    int64_t row = r0 + (lane < K ? lane : 0);
    row = row < npad ? row : npad - 1;
    const FwdRec f = fwd[row];
    const BwdRec b = bwd[row];
    return LaneRecs{f.ra, f.ap, f.bp, b.gm, b.dl};
}

// Same sweeps with the records taken from scalar loads (wave-uniform rows);
// fewer vector registers than the broadcast form.
template <int K>
__device__ __forceinline__ void seg_forward_s(double (&v)[K], const FwdRec *__restrict__ fwd,
                                              int64_t r0, double &p2, double &p1)
{
#pragma unroll
    for (int k = 0; k < K; k++) {
        const FwdRec r = fwd[r0 + k];
        const double g = fma(-r.bp, p1, fma(-r.ap, p2, r.ra * v[k]));
        v[k] = g;
        p2 = p1;
        p1 = g;
    }
}

template <int K>
__device__ __forceinline__ void seg_backward_s(double (&v)[K], const BwdRec *__restrict__ bwd,
                                               int64_t r0, double &q1, double &q2)
{
#pragma unroll
    for (int k = K - 1; k >= 0; k--) {
        const BwdRec r = bwd[r0 + k];
        const double x = fma(-r.gm, q1, fma(-r.dl, q2, v[k]));
        v[k] = x;
        q2 = q1;
        q1 = x;
    }
}

template <int K>
__device__ __forceinline__ void seg_forward(double (&v)[K], const LaneRecs &rc, double &p2,
                                            double &p1)
{
#pragma unroll
    for (int k = 0; k < K; k++) {
        const double ra = lane_bcast(rc.ra, k), ap = lane_bcast(rc.ap, k), bp = lane_bcast(rc.bp, k);
        const double g = fma(-bp, p1, fma(-ap, p2, ra * v[k]));
        v[k] = g;
        p2 = p1;
        p1 = g;
    }
}

template <int K>
__device__ __forceinline__ void seg_backward(double (&v)[K], const LaneRecs &rc, double &q1,
                                             double &q2)
{
#pragma unroll
    for (int k = K - 1; k >= 0; k--) {
        const double gm = lane_bcast(rc.gm, k), dl = lane_bcast(rc.dl, k);
        const double x = fma(-gm, q1, fma(-dl, q2, v[k]));
        v[k] = x;
        q2 = q1;
        q1 = x;
    }
}

template <int K, typename TI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_part_summary(const FwdRec *__restrict__ fwd,
                                                     const BwdRec *__restrict__ bwd, int64_t n,
                                                     int64_t npad, const TI *__restrict__ F,
                                                     int64_t batch, int64_t ld,
                                                     double *__restrict__ summ, int64_t summ_ld)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t s = blockIdx.y;
    const bool act = j < batch;  // every lane stays: records are read across lanes
    const int64_t r0 = s * K;
    const int L = (int)((n - r0) < K ? (n - r0) : K);
    double v[K];
    seg_load<K, TI>(v, F + (act ? j : 0), ld, r0, act ? L : 0);
    const LaneRecs rc = load_lane_recs(fwd, bwd, r0, K, npad);
    double p2 = 0.0, p1 = 0.0;
    seg_forward<K>(v, rc, p2, p1);
    double q1 = 0.0, q2 = 0.0;
    seg_backward<K>(v, rc, q1, q2);
    if (!act) return;
    double *o = summ + s * 4 * summ_ld + j;
    o[0] = p2;
    o[summ_ld] = p1;
    o[2 * summ_ld] = q1;
    o[3 * summ_ld] = q2;
}

// Serial interface recurrence (interface_chain), one lane per system.
__global__ __launch_bounds__(256) void k_part_chain(const SegRec *__restrict__ seg, int64_t nseg,
                                                    double *__restrict__ summ, int64_t summ_ld,
                                                    int64_t batch)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;
    interface_chain(summ + j, 4 * summ_ld, summ_ld, seg, nseg);
}

// Pass 2 reads f (type TI, leading dimension ldf) and writes x (FP64,
// leading dimension ldx); x may be f itself when TI is double and ldx == ldf.
template <int K, typename TI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_part_final(const FwdRec *__restrict__ fwd,
                                                   const BwdRec *__restrict__ bwd, int64_t n,
                                                   int64_t npad, const TI *Fin, int64_t ldf,
                                                   double *X, int64_t ldx, int64_t batch,
                                                   const double *__restrict__ summ,
                                                   int64_t summ_ld)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t s = blockIdx.y;
    const bool act = j < batch;  // every lane stays: records are read across lanes
    const int64_t jj = act ? j : 0;
    const int64_t r0 = s * K;
    const int L = (int)((n - r0) < K ? (n - r0) : K);
    double v[K];
    seg_load<K, TI>(v, Fin + jj, ldf, r0, act ? L : 0);
    double *col = X + jj;
    const int64_t ld = ldx;
    const double *o = summ + s * 4 * summ_ld + jj;
    double p2 = o[0], p1 = o[summ_ld];
    double q1 = o[2 * summ_ld], q2 = o[3 * summ_ld];
    seg_forward_s<K>(v, fwd, r0, p2, p1);
    seg_backward_s<K>(v, bwd, r0, q1, q2);
    if (!act) return;
    double *base = col + r0 * ld;
    if (L == K) {
#pragma unroll
        for (int k = 0; k < K; k++) __builtin_nontemporal_store(v[k], base + k * ld);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++)
            if (k < L) base[k * ld] = v[k];
    }
}

// -------------------------------------------------------------- strided ----
// System-major storage (system j = n contiguous doubles at F + j*ld).  One
// lane per system; rows are staged through LDS in blocks of T so that global
// accesses stay coalesced: a wave moves 64 systems x T rows with each
// system's T values contiguous.
template <int T>
__global__ __launch_bounds__(64) void k_strided(const FwdRec *__restrict__ fwd,
                                                const BwdRec *__restrict__ bwd, int n,
                                                double *__restrict__ F, int64_t batch, int64_t ld)
{
    __shared__ double tile[64][T + 1];
    const int lane = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int64_t nsys = (batch - j0) < 64 ? (batch - j0) : 64;
    // cooperative load of rows [i0, i0+L) for the wave's systems into tile
    auto load_tile = [&](int i0, int L) {
        for (int idx = lane; idx < 64 * T; idx += 64) {
            const int sys = idx / T, r = idx % T;
            double v = 0.0;
            if (sys < nsys && r < L) v = F[(j0 + sys) * ld + i0 + r];
            tile[sys][r] = v;
        }
        __syncthreads();
    };
    auto store_tile = [&](int i0, int L) {
        __syncthreads();
        for (int idx = lane; idx < 64 * T; idx += 64) {
            const int sys = idx / T, r = idx % T;
            if (sys < nsys && r < L) F[(j0 + sys) * ld + i0 + r] = tile[sys][r];
        }
        __syncthreads();
    };
    double p2 = 0.0, p1 = 0.0;
    for (int i0 = 0; i0 < n; i0 += T) {
        const int L = (n - i0) < T ? (n - i0) : T;
        load_tile(i0, L);
        for (int r = 0; r < L; r++) {
            const FwdRec rc = fwd[i0 + r];
            const double g = fma(-rc.bp, p1, fma(-rc.ap, p2, rc.ra * tile[lane][r]));
            tile[lane][r] = g;
            p2 = p1;
            p1 = g;
        }
        store_tile(i0, L);
    }
    double q1 = 0.0, q2 = 0.0;
    const int last0 = ((n - 1) / T) * T;
    for (int i0 = last0; i0 >= 0; i0 -= T) {
        const int L = (n - i0) < T ? (n - i0) : T;
        load_tile(i0, L);
        for (int r = L - 1; r >= 0; r--) {
            const BwdRec rc = bwd[i0 + r];
            const double x = fma(-rc.gm, q1, fma(-rc.dl, q2, tile[lane][r]));
            tile[lane][r] = x;
            q2 = q1;
            q1 = x;
        }
        store_tile(i0, L);
    }
}

}  // namespace

hipError_t launch_lane_sweep(const FwdRec *fwd, const BwdRec *bwd, int64_t n, double *F,
                             int64_t batch, int64_t ld, int depth, hipStream_t s)
{
    const int bs = 256;
    const dim3 grid((unsigned)((batch + bs - 1) / bs));
    switch (depth) {
    case 8: hipLaunchKernelGGL(k_lane<8>, grid, dim3(bs), 0, s, fwd, bwd, (int)n, F, batch, ld); break;
    case 32: hipLaunchKernelGGL(k_lane<32>, grid, dim3(bs), 0, s, fwd, bwd, (int)n, F, batch, ld); break;
    default: hipLaunchKernelGGL(k_lane<16>, grid, dim3(bs), 0, s, fwd, bwd, (int)n, F, batch, ld); break;
    }
    return hipGetLastError();
}

template <int K, typename TI>
static hipError_t part_sweep_k(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg, int64_t n,
                               int64_t npad, const TI *Fin, int64_t ldf, double *X, int64_t ldx,
                               int64_t batch, double *summ, int64_t summ_ld, hipStream_t s)
{
    const int64_t nseg = (n + K - 1) / K;
    const dim3 grid((unsigned)((batch + 63) / 64), (unsigned)nseg);
    const dim3 gridc((unsigned)((batch + 255) / 256));
    hipLaunchKernelGGL((k_part_summary<K, TI>), grid, dim3(64), 0, s, fwd, bwd, n, npad, Fin, batch,
                       ldf, summ, summ_ld);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_part_chain, gridc, dim3(256), 0, s, seg, nseg, summ, summ_ld, batch);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_part_final<K, TI>), grid, dim3(64), 0, s, fwd, bwd, n, npad, Fin, ldf, X,
                       ldx, batch, summ, summ_ld);
    return hipGetLastError();
}

hipError_t launch_part_sweep_io(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg,
                                int64_t n, int64_t npad, int seg_rows, const void *Fin, bool f32,
                                int64_t ldf, double *X, int64_t ldx, int64_t batch, double *summ,
                                int64_t summ_ld, hipStream_t s)
{
#define PENT_PART(KK)                                                                              \
    return f32 ? part_sweep_k<KK, float>(fwd, bwd, seg, n, npad, (const float *)Fin, ldf, X, ldx, \
                                         batch, summ, summ_ld, s)                                  \
               : part_sweep_k<KK, double>(fwd, bwd, seg, n, npad, (const double *)Fin, ldf, X,    \
                                          ldx, batch, summ, summ_ld, s)
    switch (seg_rows) {
    case 16: PENT_PART(16);
    case 32: PENT_PART(32);
    case 64: PENT_PART(64);
    default: return hipErrorInvalidValue;
    }
#undef PENT_PART
}

hipError_t launch_part_sweep(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg,
                             int64_t n, int64_t npad, int seg_rows, double *F, int64_t batch,
                             int64_t ld, double *summ, int64_t summ_ld, hipStream_t s)
{
    return launch_part_sweep_io(fwd, bwd, seg, n, npad, seg_rows, F, false, ld, F, ld, batch,
                                summ, summ_ld, s);
}

hipError_t launch_strided_sweep(const FwdRec *fwd, const BwdRec *bwd, int64_t n, double *F,
                                int64_t batch, int64_t ld, hipStream_t s)
{
    const dim3 grid((unsigned)((batch + 63) / 64));
    hipLaunchKernelGGL(k_strided<32>, grid, dim3(64), 0, s, fwd, bwd, (int)n, F, batch, ld);
    return hipGetLastError();
}

}  // namespace pent
