// internal.h -- shared declarations of libpentbatch's host code and kernel
// launchers (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/pentbatch.h"

namespace pent {

// Read-only kernel data through the constant address space: uniform
// indexes then compile to scalar loads (a generic pointer gives per-lane
// flat loads, each waited for).
typedef __attribute__((address_space(4))) const double *CDbl;

// The same pointer, opaque to the optimiser (an empty asm that may have
// changed it): loads through the copy are neither merged with loads through
// the original nor moved above this point.
template <typename P>
__device__ __forceinline__ P fresh(P p)
{
    unsigned long long a = (unsigned long long)p;
    asm volatile("" : "+s"(a));
    return (P)a;
}

// max(m, v) that keeps a NaN once seen (fmax drops it): the maxima of the
// backward error must let a non-finite solution through.
__device__ __forceinline__ double nan_max(double m, double v) { return (v > m || v != v) ? v : m; }

// r_i of one row: f_i - sum_k coef_k * x_k, every product and partial sum
// carried with its rounding error (TwoProduct by fused multiply-add, TwoSum;
// the "Dot2" scheme of Ogita, Rump and Oishi, SIAM J. Sci. Comput. 26, 2005).
__device__ __forceinline__ double dot2_row(double f, const double (&cf)[5], const double (&xv)[5])
{
#pragma clang fp contract(off)
    double s = f, c = 0.0;
#pragma unroll
    for (int k = 0; k < 5; k++) {
        const double p = -cf[k] * xv[k];
        const double pe = __builtin_fma(-cf[k], xv[k], -p);
        const double t = s + p;
        const double z = t - s;
        const double te = (s - (t - z)) + (p - z);
        s = t;
        c = c + (te + pe);
    }
    return s + c;
}

// Per-row constants of the forward sweep, prescaled by 1/alpha_i so the
// recurrence g_i = (f_i - a_i g_{i-2} - beta_i g_{i-1}) / alpha_i (Sec. 2.4)
// becomes g_i = ra*f_i - ap*g_{i-2} - bp*g_{i-1}, one fused multiply-add on
// the g_{i-1} dependency chain.
struct alignas(32) FwdRec {
    double ra;  // 1 / alpha_i
    double ap;  // a_i / alpha_i      (a_i = epsilon_i)
    double bp;  // beta_i / alpha_i
    double pad;
};

// Per-row constants of the back substitution x_i = g_i - gamma_i x_{i+1}
// - delta_i x_{i+2} (Sec. 2.4).
struct alignas(16) BwdRec {
    double gm;  // gamma_i
    double dl;  // delta_i
};

// Per-segment constants of the partitioned sweep (segment = seg_rows
// consecutive rows).  Forward state entering a segment: (g_{r0-2}, g_{r0-1});
// leaving it: the last two g's.  Backward state entering from below:
// (x_{r1}, x_{r1+1}); leaving upward: (x_{r0}, x_{r0+1}).  Each 2x2 matrix is
// stored column-major: m[0] m[1] = image of the first unit state, m[2] m[3] =
// image of the second.
struct alignas(128) SegRec {
    double tf[4];  // forward state in  -> forward state out   (f = 0)
    double cg[4];  // forward state in  -> backward state out  (f = 0, x below = 0)
    double tb[4];  // backward state in -> backward state out  (g = 0)
    double pad[4];
};

// Per-group constants of the single-pass sweeps (a group = W consecutive
// segments), column-major 2x2 matrices as in SegRec:
//   tg  = Tf_last ... Tf_first: forward state in -> forward state out;
//   tbg = Tb_first ... Tb_last: backward state in (from below) -> out (top);
//   cg  = forward state in -> backward top state (zero right-hand side,
//         zero state below);
//   q   = response of the backward state entering the group from below to
//         the forward state leaving it, through all later groups:
//         q_last = 0, q_G = cg_{G+1} + tbg_{G+1} q_{G+1} tg_{G+1}.
struct alignas(128) GrpRec {
    double tg[4];
    double tbg[4];
    double cg[4];
    double q[4];
};

// Interface-scan constants of the resident-tile schedule, one record per
// segment (64 segments): p[l] and q[l] are the products of 2^l consecutive
// forward / backward transfer matrices ending (p) or starting (q) at the
// segment, cg the segment's forward-in -> backward-out matrix.
struct alignas(64) ScanRec {
    double p[6][4];
    double q[6][4];
    double cg[4];
    double pad[4];
};

// Factor records are stored for n rounded up to this many rows; the rows
// past n are all-zero records, which map a zero right-hand side to zero and
// let fixed-height kernels run without per-row guards.
constexpr int64_t kRecPad = 4096;

// One matrix of a group solve, as the persistent kernel sees it.
struct GroupMat {
    const FwdRec *fwd;
    const BwdRec *bwd;
    const SegRec *seg64;  // transfer matrices for 64-row segments
    const GrpRec *grp64;  // group constants for 64-row segments, four per group
    double *F;          // right-hand sides, batch-fastest, overwritten in place
    int64_t n, npad, ld, batch;
    const SegRec *segp;  // the single pass's segments (kGroupSegRows rows) ...
    const GrpRec *grpp;  // ... and its group constants (four segments per group)
};

// One work item: up to 64 consecutive systems of one matrix.
struct GroupItem {
    int mat;
    int ncols;
    int64_t col0;
    int64_t summ_off;  // offset (doubles) of the item's segment summaries in the workspace
};

// Bordering data of a periodic matrix: the at most ten non-zeros of h^T
// (row q of the trailing pair, column hcol, value hv) and [C2 - h^T Z]^{-1}
// row-major.  bad != 0 when that 2 x 2 matrix is singular or not finite.
struct CycAux {
    int nh;
    int bad;
    int hq[10];
    int64_t hcol[10];
    double hv[10];
    double minv[4];
};

// One unit of the single-pass group solve: rows [g*rows, (g+1)*rows) of
// the 64 systems of matrix `mat` that start at col0; u0 = index of the
// first unit of that tile (its units are consecutive).
struct GroupUnit {
    int mat;
    int g;
    int ngroups;
    int pad;
    int64_t col0;
    int64_t u0;
};

constexpr int kMaxSegCaches = 4;  // seg_rows 16, 32, 64 and the group single pass's
// Segment height of the many-matrix single pass (k_group_onepass): 56 rows
// leave its wave 0 enough registers for the chain work beside the block
// (64-row blocks spilled 11 of their rows around the wait, 18% more bytes).
constexpr int kGroupSegRows = 56;
inline int seg_slot(int seg_rows)
{
    return seg_rows == 16 ? 0 : seg_rows == 32 ? 1 : seg_rows == 64 ? 2 : 3;
}
constexpr int kSegPad = 16;       // segment records are padded to a multiple of this

struct SegCache {
    int seg_rows = 0;
    int64_t nseg = 0;
    SegRec *d_seg = nullptr;
};

// Group constants of the single pass for (seg_rows, waves per group).
constexpr int kMaxGrpCaches = 6;
struct GrpCache {
    int seg_rows = 0;
    int waves = 0;
    int64_t ngroups = 0;
    GrpRec *d_grp = nullptr;
};

}  // namespace pent

struct pent_plan {
    uint64_t magic;
    int64_t n;
    int device;
    double *d_diag;          // 5n: a, b, c, d, e (zero-padded outside the matrix)
    double *d_fac;           // 4n: alpha, beta, gamma, delta
    double *d_anorm;         // 1: ||A||_inf
    int64_t npad;            // record rows: n + 256 rounded up to kRecPad, rows >= n all zero
    pent::FwdRec *d_fwd;     // npad
    pent::BwdRec *d_bwd;     // npad
    int sched_kind;          // 0 auto, 1 lane, 2 partitioned, 3 resident tile, 4 single pass
    int sched_seg;           // seg_rows for kinds 2 and 4, prefetch depth for kind 1
    unsigned int *d_err;     // status bits since the last pent_check: 1 a single-pass wait
                             // ran out, 2 a refined solve missed its tolerance
    double refine_tol;       // backward-error tolerance of pent_solve_mixed (0: none)
    int onepass_cap[2];      // co-resident single-pass units (32, 64 rows), 0 = not yet queried
    int fix_cap;             // co-resident units of the fused correction, 0 = not yet queried
    int t_cap;               // ... of the system-major single pass
    int tst_cap;             // ... of its form with the 2-D Cahn-Hilliard stencil
    std::mutex mu;           // guards seg caches (lazy build)
    pent::SegCache seg[pent::kMaxSegCaches];
    pent::GrpCache grp[pent::kMaxGrpCaches];  // lazily built, guarded by mu
    pent::ScanRec *d_scan;   // resident-tile scan constants (64 records), lazily built
    double *d_trec;          // resident-tile record image (5 x 64 x rows doubles)
    int scan_rows;           // rows per lane they were built for
};

namespace pent {

// Serial interface recurrence over the segments of one system (one lane per
// system), shared by the partitioned and group kernels:
//   y_0 = 0,       y_{s+1} = e_s + Tf_s y_s
//   z_{S-1} = 0,   z_{s-1} = b_s + Cg_s y_s + Tb_s z_s
// Summary q of segment s lives at sum[s*sstride + q*qstride]; on entry it
// holds (e_s, b_s), on exit the incoming states (y_s, z_s).  The loads of a
// chunk of segments are issued before its arithmetic, so a chunk costs one
// memory latency instead of one per segment.
template <typename DP, typename SP>
__device__ __forceinline__ void interface_chain(DP sum, int64_t sstride, int64_t qstride,
                                                SP seg, int64_t nseg)
{
    constexpr int CH = 8;
    double y0 = 0.0, y1 = 0.0;
    for (int64_t s0 = 0; s0 < nseg; s0 += CH) {
        double e0[CH], e1[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            if (s0 + k < nseg) {
                e0[k] = sum[(s0 + k) * sstride];
                e1[k] = sum[(s0 + k) * sstride + qstride];
            }
        }
#pragma unroll
        for (int k = 0; k < CH; k++) {
            if (s0 + k < nseg) {
                const int64_t s = s0 + k;
                sum[s * sstride] = y0;
                sum[s * sstride + qstride] = y1;
                const double t0 = seg[s].tf[0], t1 = seg[s].tf[1], t2 = seg[s].tf[2], t3 = seg[s].tf[3];
                const double n0 = e0[k] + fma(t0, y0, t2 * y1);
                const double n1 = e1[k] + fma(t1, y0, t3 * y1);
                y0 = n0;
                y1 = n1;
            }
        }
    }
    double z0 = 0.0, z1 = 0.0;
    for (int64_t s1 = nseg - 1; s1 >= 0; s1 -= CH) {
        double b0[CH], b1[CH], ys0[CH], ys1[CH];
#pragma unroll
        for (int k = 0; k < CH; k++) {
            if (s1 - k >= 0) {
                const int64_t s = s1 - k;
                ys0[k] = sum[s * sstride];
                ys1[k] = sum[s * sstride + qstride];
                b0[k] = sum[s * sstride + 2 * qstride];
                b1[k] = sum[s * sstride + 3 * qstride];
            }
        }
#pragma unroll
        for (int k = 0; k < CH; k++) {
            if (s1 - k >= 0) {
                const int64_t s = s1 - k;
                sum[s * sstride + 2 * qstride] = z0;
                sum[s * sstride + 3 * qstride] = z1;
                const double c0 = seg[s].cg[0], c1 = seg[s].cg[1], c2 = seg[s].cg[2], c3 = seg[s].cg[3];
                const double u0 = seg[s].tb[0], u1 = seg[s].tb[1], u2 = seg[s].tb[2], u3 = seg[s].tb[3];
                const double n0 = b0[k] + fma(c0, ys0[k], c2 * ys1[k]) + fma(u0, z0, u2 * z1);
                const double n1 = b1[k] + fma(c1, ys0[k], c3 * ys1[k]) + fma(u1, z0, u3 * z1);
                z0 = n0;
                z1 = n1;
            }
        }
    }
}

constexpr uint64_t kMagic = 0x70656e7462617463ull;  // "pentbatc"

// ---- launchers (each returns a hipError_t from the launch) ----
hipError_t launch_assemble_d4(double *d_diag, int64_t n, double sigma, hipStream_t s);
hipError_t launch_factor(const double *d_diag, int64_t n, int64_t npad, double *d_fac,
                         FwdRec *d_fwd, BwdRec *d_bwd, int64_t *d_bad, hipStream_t s);
hipError_t launch_seg_prep(const FwdRec *d_fwd, const BwdRec *d_bwd, int64_t n, int seg_rows,
                           SegRec *d_seg, hipStream_t s);
// Group constants for groups of `waves` segments from the segment table
// (which holds at least ngroups * waves records).
hipError_t launch_grp_prep(const SegRec *d_seg, int waves, int64_t ngroups, GrpRec *d_grp,
                           hipStream_t s);

// depth: rows prefetched per block (8, 16 or 32; anything else means 16)
hipError_t launch_lane_sweep(const FwdRec *fwd, const BwdRec *bwd, int64_t n, double *F,
                             int64_t batch, int64_t ld, int depth, hipStream_t s);
hipError_t launch_part_sweep(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg,
                             int64_t n, int64_t npad, int seg_rows, double *F, int64_t batch,
                             int64_t ld, double *summ, int64_t summ_ld, hipStream_t s);
hipError_t launch_part_sweep_io(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg,
                                int64_t n, int64_t npad, int seg_rows, const void *Fin, bool f32,
                                int64_t ldf, double *X, int64_t ldx, int64_t batch, double *summ,
                                int64_t summ_ld, hipStream_t s);
int tile_rows_for(int64_t n);  // rows per lane of the resident tile, 0 if n is too large
hipError_t launch_scan_prep(const SegRec *seg, int64_t nseg, ScanRec *out, hipStream_t s);
size_t tile_recs_doubles(int rows);
hipError_t launch_tile_recs(const FwdRec *fwd, const BwdRec *bwd, int rows, double *out,
                            hipStream_t s);
hipError_t launch_tile_sweep(const double *trec, const ScanRec *scan, int64_t n, int rows,
                             double *F, int64_t batch, int64_t ld, hipStream_t s);
hipError_t launch_tile_sweep_io(const double *trec, const ScanRec *scan, int64_t n, int rows,
                                const void *Fin, bool f32, int64_t ldf, double *X, int64_t ldx,
                                int64_t batch, hipStream_t s);

// ---- precision extension (mixed.hip) ----
// r = f - A x in compensated FP64 (f of type float or double); r may not alias f or x.
hipError_t launch_residual(const double *d_diag, int64_t n, const void *f, bool f32, int64_t ldf,
                           const double *x, int64_t ldx, double *r, int64_t ldr, int64_t batch,
                           hipStream_t s);
// x += d
hipError_t launch_axpy(double *x, int64_t ldx, const double *d, int64_t ldd, int64_t n,
                       int64_t batch, hipStream_t s);
// eta[j] = ||f - A x||_inf / (||A||_inf ||x||_inf + ||f||_inf), compensated; acc is
// 3*batch uint64 of scratch.
// eta may be NULL (not stored); with tol > 0, a system whose eta exceeds tol
// or is not finite sets bit 2 of *err.
hipError_t launch_eta(const double *d_diag, const double *d_anorm, int64_t n, const void *f,
                      bool f32, int64_t ldf, const double *x, int64_t ldx, int64_t batch,
                      unsigned long long *acc, double *eta, double tol, unsigned int *err,
                      hipStream_t s);
hipError_t launch_anorm(const double *d_diag, int64_t n, double *d_anorm, hipStream_t s);

// ---- 2-D Cahn-Hilliard explicit term (ch2d.hip, and fused into k_onepass_t) ----
// R = C + dt_k * Lap_h(C^3 - C) at one point, from the point's C and the
// C^3 - C of itself and its four neighbours (zero outside the grid).  Both
// kernels that form it go through these two functions, so they agree bit
// for bit.
__device__ __forceinline__ double ch_wterm(double c) { return c * c * c - c; }
__device__ __forceinline__ double ch_point(double c, double w, double we, double ww, double wn,
                                           double ws, double dtk, double inv_h2)
{
    const double lap = (we + ww + wn + ws - 4.0 * w) * inv_h2;
    return c + dtk * lap;
}
hipError_t launch_ch2d_rhs(const double *C, double *R, int64_t ny, int64_t ninst, int64_t nx,
                           const double *dt, double h, hipStream_t s);

// ---- single-pass partitioned sweep (onepass.hip) ----
// Units = (64-system tile, segment); scratch = status words + exchange area.
int onepass_waves(int seg_rows);                     // segments (waves) per workgroup
int onepass_waves_override();
int64_t onepass_groups(int64_t n, int seg_rows);     // workgroups per 64-system tile
int64_t onepass_units(int64_t n, int seg_rows, int64_t batch);
// status words (tickets, forward and backward statuses) at the start of the
// scratch, which must be zero when the kernel starts
int64_t onepass_words(int64_t n, int seg_rows, int64_t batch);
size_t onepass_scratch_bytes(int64_t n, int seg_rows, int64_t batch);
int onepass_capacity(int seg_rows);  // co-resident workgroups on the current device
int onepass_t_capacity(bool stencil = false);
int64_t onepass_t_groups(int64_t n);
size_t onepass_t_scratch_bytes(int64_t n, int64_t batch);
hipError_t launch_onepass_t(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg64, int64_t n,
                            double *F, int64_t batch, int64_t ld, void *scratch, unsigned int *err,
                            hipStream_t s);
// The x sweeps of a 2-D Cahn-Hilliard step with its explicit right-hand side
// formed on the fly: grid C[y][k][x] (ny x ninst x nx, contiguous) in, the
// swept R (same layout) out; systems (y, k), nx rows each (n == nx).  The
// kernel also zeroes clear_words words at clear (the status words of the
// y sweeps' single pass, launched next on the stream), at most one word per
// thread of its grid (onepass_t_threads).
int64_t onepass_t_threads(int64_t n, int64_t batch);
hipError_t launch_onepass_t_ch2d(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg64,
                                 int64_t n, const double *C, double *R, int64_t ny, int64_t ninst,
                                 const double *dt, double h, void *scratch, unsigned int *err,
                                 hipStream_t s, unsigned int *clear = nullptr,
                                 int64_t clear_words = 0);
int onepass_fix_capacity();
int64_t onepass_fix_groups(int64_t n);
size_t onepass_fix_scratch_bytes(int64_t n, int64_t batch);
hipError_t launch_onepass_fix(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg64,
                              const double *diag, int64_t n, const void *F, bool f32, int64_t ldf,
                              double *X, int64_t ldx, int64_t batch, void *scratch,
                              unsigned int *err, hipStream_t s);
hipError_t launch_onepass(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg, int64_t n,
                          int seg_rows, const void *Fin, bool f32, int64_t ldf, double *X,
                          int64_t ldx, int64_t batch, void *scratch, unsigned int *err,
                          hipStream_t s, int64_t tsf = 64, int64_t tsx = 64,
                          bool words_clear = false);  // words_clear: the status words are zero already

// ---- measurement (copy.hip): dst = src through the single pass's blocks ----
hipError_t launch_block_copy(const double *src, double *dst, int64_t n, int64_t batch, int64_t lds,
                             int64_t ldd, hipStream_t s, int tiles_across = 1, int waves_down = 4);

// ---- per-system matrices, refactored every call (rewrite.hip) ----
// work: 256 bytes of header (first failing pivot key, system * n + row) and
// gamma, delta (n x batch each, row stride batch).
size_t rewrite_workspace_bytes(int64_t n, int64_t batch);
hipError_t launch_rewrite(const double *a, const double *b, const double *c, const double *d,
                          const double *e, int64_t ldm, int64_t n, double *F, int64_t batch,
                          int64_t ld, void *work, hipStream_t s);

// ---- single pass over many matrices (onepass.hip, group variant 6) ----
int group_onepass_rows();              // rows per unit (segments x 64 rows)
int group_onepass_capacity();          // co-resident workgroups on the current device
size_t group_onepass_scratch_bytes(int64_t units);
hipError_t launch_group_onepass(const GroupMat *mats, const GroupUnit *units, int64_t nunits,
                                void *scratch, unsigned int *err, hipStream_t s);

// ---- periodic matrices by bordering (cyclic.hip) ----
// cd: cyclic row-indexed diagonals on the device, five blocks (a, b, c, d, e)
// of cyc_ld(n) doubles each; entries past row n-1 are zero (so kernels may
// read coefficients of padded rows without a guard).
__host__ __device__ inline int64_t cyc_ld(int64_t n) { return (n + kRecPad - 1) / kRecPad * kRecPad; }
hipError_t launch_cyc_assemble_d4(double *cd, int64_t n, double sigma, hipStream_t s);
// ed: 5(n-2) diagonals of the leading block E; K: zrows x 2, ld 2 (rows past
// n-2 zero).
hipError_t launch_cyc_build(const double *cd, int64_t n, int64_t zrows, double *ed, double *K,
                            hipStream_t s);
// Single-pass bordered solve (cn = false: F in place allowed) or
// Crank-Nicolson step X = A^{-1} (2C - AC) (cn = true: Fin = C, X apart).
int64_t cyc_onepass_groups(int64_t n, int seg_rows);  // workgroups per 64-system tile
int64_t cyc_onepass_units(int64_t n, int seg_rows, int64_t batch);
size_t cyc_onepass_scratch_bytes(int64_t n, int seg_rows, int64_t batch);
int cyc_onepass_capacity(int seg_rows, bool cn);
// uni (host, 5 doubles, or null): the five cyclic diagonals when each is
// the same in every row; the CN step then takes them as arguments.
hipError_t launch_cyc_onepass(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg,
                              const double *cd, const double *Z, const double *Wt,
                              const CycAux *aux, int64_t n,
                              int seg_rows, bool cn, const double *Fin, int64_t ldf, double *X,
                              int64_t ldx, int64_t batch, void *scratch, unsigned int *err,
                              hipStream_t s, const double *uni = nullptr);
hipError_t launch_cyc_finish(const double *cd, int64_t n, const double *Z, CycAux *aux,
                             hipStream_t s);
// etd: 5(n-2) diagonals of E^T; H: zrows x 2, ld 2, H[i][q] = A[n-2+q][i]
// for i < n-2, zero below.
hipError_t launch_cyc_build_transposed(const double *cd, int64_t n, int64_t zrows, double *etd,
                                       double *H, hipStream_t s);
// F rows 0..n-3 hold y = E^{-1} f^ on entry; rows n-2, n-1 hold f's tail.
// On exit F holds x.  No scratch.
hipError_t launch_cyc_correct(const CycAux *aux, const double *Z, double *F, int64_t n,
                              int64_t batch, int64_t ld, hipStream_t s);
hipError_t launch_cn_rhs(const double *cd, int64_t n, const double *C, int64_t ldc, double *R,
                         int64_t ldr, int64_t batch, hipStream_t s);

// ---- group solve (group.hip): the persistent kernel ----
// Items (matrix, up to 64 systems) handed out longest first from ctr[0] to
// nblocks resident workgroups, each solving its item alone (summaries in
// summ at the item's offset); the last workgroup out clears ctr[0..1].
int group_max_blocks();  // co-resident workgroups on the current device
hipError_t launch_group_init(unsigned int *ctr, hipStream_t s);  // ctr[0..2] = 0
hipError_t launch_group(const GroupMat *mats, const GroupItem *items, int nitems, double *summ,
                        unsigned int *ctr, int nblocks, hipStream_t s);
hipError_t launch_strided_sweep(const FwdRec *fwd, const BwdRec *bwd, int64_t n, double *F,
                                int64_t batch, int64_t ld, hipStream_t s);

}  // namespace pent
