// onepass.hip -- the partitioned sweep in a single pass: f read once, x
// written once.
//
// The rows are cut into segments of K rows and the systems into tiles of 64
// (one lane per system); a unit = (tile, segment) is one one-wave workgroup
// that holds its K x 64 block of the right-hand side in registers from load
// to store.  By linearity (Sec. 2.4's recurrences are affine in the carried
// pair), a segment's outgoing forward state is
//     out_s = e_s + Tf_s y_s,        y_s = out_{s-1},  y_0 = 0,
// with e_s the outgoing state of a zero-start forward sweep, and its
// outgoing (upward) backward state is
//     up_s = a_s + Tb_s z_s,         z_s = up_{s+1},   z_{last} = 0,
// with a_s the top of a zero-start backward sweep over the TRUE forward
// values.  Tf and Tb depend on A only (SegRec).  The carries travel between
// the units of a tile through a small exchange area with decoupled
// look-back: a unit publishes its aggregate (e_s, or a_s) when its
// neighbour's inclusive value is not there yet, looks back (forward) or
// ahead (backward) composing aggregates with the transfer matrices until it
// meets an inclusive value, and publishes its own inclusive value.
//
// Units take tickets from a counter in ticket order (tile-major), so a unit
// only ever waits on units that already hold a slot (look-back) or on later
// units of its own tile (look-ahead).  While at least one whole tile of
// units fits on the device at once (checked on the host), every wait ends;
// each wait is also bounded, and a wait that runs out raises the plan's
// error word and lets the wave finish.
#include "internal.h"

namespace pent {
namespace {

typedef __attribute__((address_space(4))) const FwdRec *CFwd;
typedef __attribute__((address_space(4))) const BwdRec *CBwd;
typedef __attribute__((address_space(4))) const SegRec *CSeg;

constexpr int kSpin = 1 << 20;  // polls per wait before giving up

// Every lane joins the atomic (lanes other than 0 add zero) and lane 0's
// result is read back: no branch depends on the lane index alone.
__device__ __forceinline__ unsigned int take_ticket(unsigned int *p)
{
    const unsigned int r = atomicAdd(p, threadIdx.x == 0 ? 1u : 0u);
    return (unsigned int)__builtin_amdgcn_readlane((int)r, 0);
}

__device__ __forceinline__ unsigned int poll(unsigned int *p)
{
    const unsigned int v = __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    return (unsigned int)__builtin_amdgcn_readlane((int)v, 0);
}

__device__ __forceinline__ void publish(unsigned int *p, unsigned int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Status of a neighbour once it is non-zero (1 aggregate, 2 inclusive); on
// timeout the error word is raised and 2 is returned so the wave finishes.
__device__ __forceinline__ unsigned int wait_status(unsigned int *p, unsigned int *err)
{
    for (int i = 0; i < kSpin; i++) {
        const unsigned int v = poll(p);
        if (v != 0) return v;
        __builtin_amdgcn_s_sleep(1);
    }
    atomicOr(err, 1u);
    return 2;
}

template <int K, typename TI>
__device__ __forceinline__ void load_rows(double (&v)[K], const TI *base, int64_t ld, int L)
{
    if (L == K) {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = (double)__builtin_nontemporal_load(base + k * ld);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = (k < L) ? (double)base[k * ld] : 0.0;
    }
}

// Forward recurrence over the segment from (p2, p1); STORE writes g over v.
template <int K, bool STORE>
__device__ __forceinline__ void forward(double (&v)[K], CFwd fwd, int64_t r0, double &p2, double &p1)
{
#pragma unroll
    for (int k = 0; k < K; k++) {
        const double ra = fwd[r0 + k].ra, ap = fwd[r0 + k].ap, bp = fwd[r0 + k].bp;
        const double g = fma(-bp, p1, fma(-ap, p2, ra * v[k]));
        if (STORE) v[k] = g;
        p2 = p1;
        p1 = g;
    }
}

// Back substitution over the segment from (q1, q2) = (x_{r0+K}, x_{r0+K+1});
// on exit (q1, q2) = (x_{r0}, x_{r0+1}).  STORE writes x over v.
template <int K, bool STORE>
__device__ __forceinline__ void backward(double (&v)[K], CBwd bwd, int64_t r0, double &q1, double &q2)
{
#pragma unroll
    for (int k = K - 1; k >= 0; k--) {
        const double gm = bwd[r0 + k].gm, dl = bwd[r0 + k].dl;
        const double x = fma(-gm, q1, fma(-dl, q2, v[k]));
        if (STORE) v[k] = x;
        q2 = q1;
        q1 = x;
    }
}

// One link of the interface chain, (y0, y1) <- w + T (y0, y1), T column-major.
// Publishers and look-back use this one function with explicit fused
// multiply-adds, so a carry has the same bits whichever path produced it.
__device__ __forceinline__ void link(double w0, double w1, double t0, double t1, double t2,
                                     double t3, double &y0, double &y1)
{
    const double n0 = fma(t2, y1, fma(t0, y0, w0));
    const double n1 = fma(t3, y1, fma(t1, y0, w1));
    y0 = n0;
    y1 = n1;
}

// Exchange area of one unit: 8 rows of 64 doubles (lane = system):
// 0,1 forward aggregate e; 2,3 forward inclusive out; 4,5 backward
// aggregate a; 6,7 backward inclusive up.
constexpr int kExRows = 8;

// 64-row blocks need up to 256 vector registers (two waves per SIMD),
// 32-row blocks fit three waves per SIMD.
template <int K, typename TI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(K == 64 ? 2 : 3))) void k_onepass(
    const FwdRec *fwd_, const BwdRec *bwd_, const SegRec *seg_, int64_t n, int nseg,
    const TI *Fin, int64_t ldf, double *X, int64_t ldx, int64_t batch, unsigned int *ctr,
    unsigned int *fst, unsigned int *bst, double *ex, unsigned int *err)
{
    const CFwd fwd = (CFwd)fwd_;
    const CBwd bwd = (CBwd)bwd_;
    const CSeg seg = (CSeg)seg_;
    const int lane = threadIdx.x;
    const unsigned int u = take_ticket(&ctr[0]);
    const int t = (int)(u / (unsigned int)nseg), s = (int)(u % (unsigned int)nseg);
    const int64_t j = (int64_t)t * 64 + lane;
    const bool act = j < batch;
    const int64_t jj = act ? j : 0;
    const int64_t r0 = (int64_t)s * K;
    const int L = (int)((n - r0) < K ? (n - r0) : K);
    double v[K];
    load_rows<K, TI>(v, Fin + jj + r0 * ldf, ldf, act ? L : 0);
    double *me = ex + (int64_t)u * (kExRows * 64) + lane;

    // ---- forward: incoming state (y0, y1) = (g_{r0-2}, g_{r0-1})
    // Look-back: find the nearest earlier segment with an inclusive value
    // (segment 0 only ever publishes inclusive values), then replay the
    // chain from it through the aggregates in between, innermost first:
    // bit for bit the serial recurrence y_{p+1} = e_p + Tf_p y_p.
    const unsigned int u0 = u - (unsigned int)s;  // first unit of the tile
    double y0 = 0.0, y1 = 0.0;
    if (s > 0) {
        double e0 = 0.0, e1 = 0.0;
        forward<K, false>(v, fwd, r0, e0, e1);
        int p = s - 1;
        unsigned int st = poll(&fst[u0 + p]);
        if (st != 2) {
            me[0] = e0;
            me[64] = e1;
            publish(&fst[u], 1u);
            for (;;) {
                if (st == 0) st = wait_status(&fst[u0 + p], err);
                if (st == 2 || p == 0) break;
                p--;
                st = poll(&fst[u0 + p]);
            }
        }
        const double *nb = ex + (int64_t)(u0 + p) * (kExRows * 64) + lane;
        y0 = nb[2 * 64];
        y1 = nb[3 * 64];
        for (int q = p + 1; q < s; q++) {
            const double *ag = ex + (int64_t)(u0 + q) * (kExRows * 64) + lane;
            link(ag[0], ag[64], seg[q].tf[0], seg[q].tf[1], seg[q].tf[2], seg[q].tf[3], y0, y1);
        }
        if (s < nseg - 1) {
            double o0 = y0, o1 = y1;
            link(e0, e1, seg[s].tf[0], seg[s].tf[1], seg[s].tf[2], seg[s].tf[3], o0, o1);
            me[2 * 64] = o0;
            me[3 * 64] = o1;
            publish(&fst[u], 2u);
        }
        forward<K, true>(v, fwd, r0, y0, y1);
    } else {
        forward<K, true>(v, fwd, r0, y0, y1);  // zero start is the true start
        if (nseg > 1) {
            me[2 * 64] = y0;
            me[3 * 64] = y1;
            publish(&fst[u], 2u);
        }
    }

    // ---- backward: incoming state (z0, z1) = (x_{r0+K}, x_{r0+K+1}); the
    // mirror image (the last segment only ever publishes inclusive values)
    double z0 = 0.0, z1 = 0.0;
    if (s < nseg - 1) {
        double a0 = 0.0, a1 = 0.0;
        backward<K, false>(v, bwd, r0, a0, a1);
        int p = s + 1;
        unsigned int st = poll(&bst[u0 + p]);
        if (st != 2) {
            me[4 * 64] = a0;
            me[5 * 64] = a1;
            publish(&bst[u], 1u);
            for (;;) {
                if (st == 0) st = wait_status(&bst[u0 + p], err);
                if (st == 2 || p == nseg - 1) break;
                p++;
                st = poll(&bst[u0 + p]);
            }
        }
        const double *nb = ex + (int64_t)(u0 + p) * (kExRows * 64) + lane;
        z0 = nb[6 * 64];
        z1 = nb[7 * 64];
        for (int q = p - 1; q > s; q--) {
            const double *ag = ex + (int64_t)(u0 + q) * (kExRows * 64) + lane;
            link(ag[4 * 64], ag[5 * 64], seg[q].tb[0], seg[q].tb[1], seg[q].tb[2], seg[q].tb[3], z0,
                 z1);
        }
        if (s > 0) {
            double o0 = z0, o1 = z1;
            link(a0, a1, seg[s].tb[0], seg[s].tb[1], seg[s].tb[2], seg[s].tb[3], o0, o1);
            me[6 * 64] = o0;
            me[7 * 64] = o1;
            publish(&bst[u], 2u);
        }
        backward<K, true>(v, bwd, r0, z0, z1);
    } else {
        backward<K, true>(v, bwd, r0, z0, z1);  // nothing below the last segment
        if (s > 0) {
            me[6 * 64] = z0;
            me[7 * 64] = z1;
            publish(&bst[u], 2u);
        }
    }

    if (!act) return;
    double *base = X + jj + r0 * ldx;
    if (L == K) {
#pragma unroll
        for (int k = 0; k < K; k++) __builtin_nontemporal_store(v[k], base + k * ldx);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++)
            if (k < L) base[k * ldx] = v[k];
    }
}

__global__ void k_zero_words(unsigned int *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

template <int K>
const void *onepass_fn(bool f32)
{
    return f32 ? (const void *)k_onepass<K, float> : (const void *)k_onepass<K, double>;
}

}  // namespace

int64_t onepass_units(int64_t n, int seg_rows, int64_t batch)
{
    return (batch + 63) / 64 * ((n + seg_rows - 1) / seg_rows);
}

size_t onepass_scratch_bytes(int64_t n, int seg_rows, int64_t batch)
{
    const int64_t units = onepass_units(n, seg_rows, batch);
    const size_t words = (size_t)(2 * units + 4);
    const size_t wbytes = (words * sizeof(unsigned int) + 255) / 256 * 256;
    return wbytes + (size_t)units * kExRows * 64 * sizeof(double);
}

int onepass_capacity(int seg_rows)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const void *fn = seg_rows == 32 ? onepass_fn<32>(false) : onepass_fn<64>(false);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, 0) != hipSuccess) return 0;
    return cus * per_cu;
}

hipError_t launch_onepass(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg, int64_t n,
                          int seg_rows, const void *Fin, bool f32, int64_t ldf, double *X,
                          int64_t ldx, int64_t batch, void *scratch, unsigned int *err,
                          hipStream_t s)
{
    const int64_t nseg = (n + seg_rows - 1) / seg_rows;
    const int64_t units = onepass_units(n, seg_rows, batch);
    if (units > (int64_t)UINT32_MAX / 2) return hipErrorInvalidValue;
    const int64_t words = 2 * units + 4;
    unsigned int *w = (unsigned int *)scratch;
    unsigned int *ctr = w, *fst = w + 4, *bst = w + 4 + units;
    const size_t wbytes = ((size_t)words * sizeof(unsigned int) + 255) / 256 * 256;
    double *ex = (double *)((char *)scratch + wbytes);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, w, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define PENT_ONEPASS(KK, TT)                                                                       \
    hipLaunchKernelGGL((k_onepass<KK, TT>), dim3((unsigned)units), dim3(64), 0, s, fwd, bwd, seg, \
                       n, (int)nseg, (const TT *)Fin, ldf, X, ldx, batch, ctr, fst, bst, ex, err)
    if (seg_rows == 64) {
        if (f32) PENT_ONEPASS(64, float);
        else PENT_ONEPASS(64, double);
    } else if (seg_rows == 32) {
        if (f32) PENT_ONEPASS(32, float);
        else PENT_ONEPASS(32, double);
    } else {
        return hipErrorInvalidValue;
    }
#undef PENT_ONEPASS
    return hipGetLastError();
}

}  // namespace pent
