// tile.hip -- single-pass FP64 solve with the whole column tile resident in
// registers.
//
// A workgroup of 512 lanes owns W = 8 consecutive systems and all n rows of
// them: lane (c, s) holds rows [s*K, s*K + K) of system c (S = 64 segments
// per system, K <= 64 rows per lane, so n <= 64*K).  Every f is read from HBM
// once and every x written once; nothing else touches memory except the
// per-row factor records (L2-resident, shared by every workgroup).
//
// Per system, the sweeps of Sec. 2.4 are split at segment boundaries.  By
// linearity:
//   pass 1  each lane runs the forward sweep on its rows with zero incoming
//           state (g0, stored in place) and then the back substitution of g0
//           with zero incoming state, keeping only the two outgoing values:
//           e_s = last two g0, b_s = first two back-substituted values;
//   scan    wave c (lane = segment) resolves the segment interfaces of system
//           c: incoming forward states y_s from y_{s+1} = Tf_s y_s + e_s
//           (Hillis-Steele scan over the affine maps, whose 2x2 matrix
//           products depend on A only and are precomputed), then the incoming
//           backward states z_s from z_{s-1} = Tb_s z_s + (b_s + Cg_s y_s);
//   pass 2  g = g0 + (homogeneous forward response to y_s), then the back
//           substitution from z_s, in place; store x.
#include "internal.h"

namespace pent {
namespace {

constexpr int kTileSeg = 64;  // segments per system (= lanes of the scan wave)
constexpr int kTileW = 8;     // systems per workgroup
constexpr int kTileThreads = kTileSeg * kTileW;
constexpr int kFence = 8;     // rows between scheduling fences (bounds record lookahead)

__device__ __forceinline__ double shfl_up_d(double v, int d)
{
    return __shfl_up(v, d, 64);
}

__device__ __forceinline__ double shfl_down_d(double v, int d)
{
    return __shfl_down(v, d, 64);
}

// Block -> tile map: consecutive workgroup ids go round-robin over the 8
// XCDs, so tiles 2m and 2m+1 (which share 128-byte lines of every row) are
// given to two workgroups of the same XCD dispatched back to back.
__device__ __forceinline__ int64_t tile_of_block(int64_t b)
{
    const int64_t x = b & 7, i = b >> 3;
    return 2 * ((i >> 1) * 8 + x) + (i & 1);
}

// LDS image of the per-row records of one tile configuration: five
// components (ra, ap, bp, gm, dl), each stored step-major as [k][s] (row
// s*K + k), so at step k the eight segments a wave covers read eight
// adjacent doubles.
template <int K>
constexpr int tile_lds_bytes()
{
    return K == 64 ? 5 * kTileSeg * K * 8 : 5 * kTileSeg * K * 8 + 4 * kTileW * kTileSeg * 8;
}

// f is read with type TI (leading dimension ldf), x written as FP64 (ldx);
// x may be f itself when TI is double and ldx == ldf.
template <int K, typename TI>
__global__ __launch_bounds__(kTileThreads) void k_tile(const double *__restrict__ trec,
                                                      const ScanRec *__restrict__ scan, int n,
                                                      const TI *Fin, int64_t ldf, double *X,
                                                      int64_t ldx, int64_t batch, int64_t ntiles)
{
    extern __shared__ double lds[];
    constexpr int C = kTileSeg * K;  // doubles per record component
    const double *l_ra = lds, *l_ap = lds + C, *l_bp = lds + 2 * C, *l_gm = lds + 3 * C,
                 *l_dl = lds + 4 * C;
    // interface buffer: aliases the ra component (used by the first forward
    // pass only) when the records fill the LDS, else placed after them
    double *sh = (K == 64) ? lds : lds + 5 * C;
    auto SH = [&](int q, int col, int seg) -> double & { return sh[(q * kTileW + col) * kTileSeg + seg]; };

    const int64_t tile = tile_of_block(blockIdx.x);
    if (tile >= ntiles) return;  // whole workgroup leaves together
    const int tid = threadIdx.x;
    const int c = tid % kTileW;
    const int s = tid / kTileW;
    const int64_t j = tile * kTileW + c;
    const bool act = j < batch;
    const int r0 = s * K;
    const int L = max(0, min(K, n - r0));
    const bool full = act && L == K;
    // lane bases: row r0 of system j (rows past n / systems past the batch
    // are never dereferenced)
    const int64_t roff = (int64_t)(L > 0 ? r0 : 0);
    const TI *fbase = Fin + (act ? j : 0) + roff * ldf;

    double v[K];
    if (full) {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = (double)__builtin_nontemporal_load(fbase + k * ldf);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = (act && k < L) ? (double)fbase[k * ldf] : 0.0;
    }
    // stage the records into LDS: 1 KB per wave per instruction, straight
    // from global memory (no VGPRs)
    {
        const int w = tid / 64, lane = tid % 64;
        constexpr int chunks = 5 * C * 8 / 1024;
        for (int q = w; q < chunks; q += kTileThreads / 64) {
            __builtin_amdgcn_global_load_lds(
                (const void *)(trec + (size_t)q * 128 + lane * 2),
                (__attribute__((address_space(3))) void *)(lds + q * 128), 16, 0, 0);
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __syncthreads();

    // pass 1: forward with zero incoming state, g0 in place.  Rows past n
    // have all-zero records and zero data, so they stay zero and pass the
    // state through unchanged; no per-row guards are needed.
    double p2 = 0.0, p1 = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int o = k * kTileSeg + s;
        const double g = fma(-l_bp[o], p1, fma(-l_ap[o], p2, l_ra[o] * v[k]));
        v[k] = g;
        p2 = p1;
        p1 = g;
        if (k % kFence == kFence - 1) __builtin_amdgcn_sched_barrier(0);
    }
    // back substitution of g0 with zero incoming state, outgoing values only
    double q1 = 0.0, q2 = 0.0;
#pragma unroll
    for (int k = K - 1; k >= 0; k--) {
        const int o = k * kTileSeg + s;
        const double x = fma(-l_gm[o], q1, fma(-l_dl[o], q2, v[k]));
        q2 = q1;
        q1 = x;
        if (k % kFence == 0) __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // every lane is done with ra before sh may reuse it
    SH(0, c, s) = p2;
    SH(1, c, s) = p1;
    SH(2, c, s) = q1;
    SH(3, c, s) = q2;
    __syncthreads();

    // interface scans: wave w handles system w, lane = segment
    {
        const int w = tid / 64;
        const int ls = tid % 64;
        const ScanRec &sr = scan[ls];
        double y0 = SH(0, w, ls), y1 = SH(1, w, ls);
        const double b0 = SH(2, w, ls), b1 = SH(3, w, ls);
#pragma unroll
        for (int l = 0; l < 6; l++) {
            const int d = 1 << l;
            const double u0 = shfl_up_d(y0, d), u1 = shfl_up_d(y1, d);
            if (ls >= d) {
                const double *P = sr.p[l];
                const double n0 = y0 + fma(P[0], u0, P[2] * u1);
                const double n1 = y1 + fma(P[1], u0, P[3] * u1);
                y0 = n0;
                y1 = n1;
            }
        }
        // incoming forward state of segment ls = outgoing of segment ls-1
        double yi0 = shfl_up_d(y0, 1), yi1 = shfl_up_d(y1, 1);
        if (ls == 0) { yi0 = 0.0; yi1 = 0.0; }
        double z0 = b0 + fma(sr.cg[0], yi0, sr.cg[2] * yi1);
        double z1 = b1 + fma(sr.cg[1], yi0, sr.cg[3] * yi1);
#pragma unroll
        for (int l = 0; l < 6; l++) {
            const int d = 1 << l;
            const double u0 = shfl_down_d(z0, d), u1 = shfl_down_d(z1, d);
            if (ls + d < 64) {
                const double *Q = sr.q[l];
                const double n0 = z0 + fma(Q[0], u0, Q[2] * u1);
                const double n1 = z1 + fma(Q[1], u0, Q[3] * u1);
                z0 = n0;
                z1 = n1;
            }
        }
        double zi0 = shfl_down_d(z0, 1), zi1 = shfl_down_d(z1, 1);
        if (ls == 63) { zi0 = 0.0; zi1 = 0.0; }
        __syncthreads();  // everyone has read sh before it is overwritten
        SH(0, w, ls) = yi0;
        SH(1, w, ls) = yi1;
        SH(2, w, ls) = zi0;
        SH(3, w, ls) = zi1;
    }
    __syncthreads();

    // pass 2: add the response to the true incoming forward state, then the
    // back substitution from the true incoming backward state
    double h2 = SH(0, c, s), h1 = SH(1, c, s);
    q1 = SH(2, c, s);
    q2 = SH(3, c, s);
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int o = k * kTileSeg + s;
        const double h = fma(-l_bp[o], h1, -l_ap[o] * h2);
        v[k] += h;
        h2 = h1;
        h1 = h;
        if (k % kFence == kFence - 1) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = K - 1; k >= 0; k--) {
        const int o = k * kTileSeg + s;
        const double x = fma(-l_gm[o], q1, fma(-l_dl[o], q2, v[k]));
        v[k] = x;
        q2 = q1;
        q1 = x;
        if (k % kFence == 0) __builtin_amdgcn_sched_barrier(0);
    }
    double *base = X + (act ? j : 0) + roff * ldx;
    if (full) {
#pragma unroll
        for (int k = 0; k < K; k++) __builtin_nontemporal_store(v[k], base + k * ldx);
    } else if (act) {
#pragma unroll
        for (int k = 0; k < K; k++)
            if (k < L) base[k * ldx] = v[k];
    }
}

// Records in the LDS image layout: out[comp][k][s] = component comp of row
// s*K + k (comp: ra, ap, bp, gm, dl).
template <int K>
__global__ void k_tile_recs(const FwdRec *__restrict__ fwd, const BwdRec *__restrict__ bwd,
                            double *__restrict__ out)
{
    constexpr int C = kTileSeg * K;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 5 * C) return;
    const int comp = i / C, rem = i % C, k = rem / kTileSeg, sg = rem % kTileSeg;
    const int row = sg * K + k;
    double v;
    switch (comp) {
    case 0: v = fwd[row].ra; break;
    case 1: v = fwd[row].ap; break;
    case 2: v = fwd[row].bp; break;
    case 3: v = bwd[row].gm; break;
    default: v = bwd[row].dl; break;
    }
    out[i] = v;
}

// Scan matrices from the per-segment transfer matrices (one lane per
// segment, 64 segments).  p[l] = Tf_s Tf_{s-1} ... Tf_{max(0, s-2^l+1)},
// q[l] = Tb_s Tb_{s+1} ... Tb_{min(63, s+2^l-1)}; matrices column-major.
__device__ __forceinline__ void mul2(const double *A, const double *B, double *C)
{
    // C = A * B, column-major 2x2
    const double c0 = A[0] * B[0] + A[2] * B[1];
    const double c1 = A[1] * B[0] + A[3] * B[1];
    const double c2 = A[0] * B[2] + A[2] * B[3];
    const double c3 = A[1] * B[2] + A[3] * B[3];
    C[0] = c0; C[1] = c1; C[2] = c2; C[3] = c3;
}

__global__ void k_scan_prep(const SegRec *__restrict__ seg, int64_t nseg, ScanRec *__restrict__ out)
{
    const int s = threadIdx.x;
    if (s >= kTileSeg) return;
    ScanRec r;
    for (int l = 0; l < 6; l++) {
        const int len = 1 << l;
        double M[4] = {1.0, 0.0, 0.0, 1.0};
        for (int t = s; t >= 0 && t > s - len; t--) {  // M = M * Tf_t, t descending
            double T[4] = {1.0, 0.0, 0.0, 1.0};
            if (t < nseg) { T[0] = seg[t].tf[0]; T[1] = seg[t].tf[1]; T[2] = seg[t].tf[2]; T[3] = seg[t].tf[3]; }
            mul2(M, T, M);
        }
        for (int k = 0; k < 4; k++) r.p[l][k] = M[k];
        double Q[4] = {1.0, 0.0, 0.0, 1.0};
        for (int t = s; t < kTileSeg && t < s + len; t++) {  // Q = Q * Tb_t, t ascending
            double T[4] = {1.0, 0.0, 0.0, 1.0};
            if (t < nseg) { T[0] = seg[t].tb[0]; T[1] = seg[t].tb[1]; T[2] = seg[t].tb[2]; T[3] = seg[t].tb[3]; }
            mul2(Q, T, Q);
        }
        for (int k = 0; k < 4; k++) r.q[l][k] = Q[k];
    }
    for (int k = 0; k < 4; k++) r.cg[k] = (s < nseg) ? seg[s].cg[k] : 0.0;
    for (int k = 0; k < 4; k++) r.pad[k] = 0.0;
    out[s] = r;
}

}  // namespace

int tile_rows_for(int64_t n)
{
    if (n <= 16 * kTileSeg) return 16;
    if (n <= 32 * kTileSeg) return 32;
    if (n <= 64 * kTileSeg) return 64;
    return 0;
}

hipError_t launch_scan_prep(const SegRec *seg, int64_t nseg, ScanRec *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_prep, dim3(1), dim3(kTileSeg), 0, s, seg, nseg, out);
    return hipGetLastError();
}

size_t tile_recs_doubles(int rows) { return (size_t)5 * kTileSeg * rows; }

hipError_t launch_tile_recs(const FwdRec *fwd, const BwdRec *bwd, int rows, double *out,
                            hipStream_t s)
{
    const int total = 5 * kTileSeg * rows;
    const dim3 grid((total + 255) / 256), block(256);
    switch (rows) {
    case 16: hipLaunchKernelGGL(k_tile_recs<16>, grid, block, 0, s, fwd, bwd, out); break;
    case 32: hipLaunchKernelGGL(k_tile_recs<32>, grid, block, 0, s, fwd, bwd, out); break;
    case 64: hipLaunchKernelGGL(k_tile_recs<64>, grid, block, 0, s, fwd, bwd, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

namespace {
template <int K, typename TI>
hipError_t launch_tile_k(const double *trec, const ScanRec *scan, int64_t n, const TI *Fin,
                         int64_t ldf, double *X, int64_t ldx, int64_t batch, hipStream_t s)
{
    static bool attr_set = false;  // benign race: the attribute value is the same
    constexpr int lds = tile_lds_bytes<K>();
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_tile<K, TI>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t ntiles = (batch + kTileW - 1) / kTileW;
    const int64_t nblocks = (ntiles + 15) / 16 * 16;
    hipLaunchKernelGGL((k_tile<K, TI>), dim3((unsigned)nblocks), dim3(kTileThreads), lds, s, trec,
                       scan, (int)n, Fin, ldf, X, ldx, batch, ntiles);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_tile_sweep_io(const double *trec, const ScanRec *scan, int64_t n, int rows,
                                const void *Fin, bool f32, int64_t ldf, double *X, int64_t ldx,
                                int64_t batch, hipStream_t s)
{
#define PENT_TILE(KK)                                                                              \
    return f32 ? launch_tile_k<KK, float>(trec, scan, n, (const float *)Fin, ldf, X, ldx, batch, s) \
               : launch_tile_k<KK, double>(trec, scan, n, (const double *)Fin, ldf, X, ldx, batch, s)
    switch (rows) {
    case 16: PENT_TILE(16);
    case 32: PENT_TILE(32);
    case 64: PENT_TILE(64);
    default: return hipErrorInvalidValue;
    }
#undef PENT_TILE
}

hipError_t launch_tile_sweep(const double *trec, const ScanRec *scan, int64_t n, int rows,
                             double *F, int64_t batch, int64_t ld, hipStream_t s)
{
    return launch_tile_sweep_io(trec, scan, n, rows, F, false, ld, F, ld, batch, s);
}

}  // namespace pent
