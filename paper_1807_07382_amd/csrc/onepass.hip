// onepass.hip -- the partitioned sweep in a single pass: f read once, x
// written once.
//
// The rows are cut into segments of K rows and the systems into tiles of 64
// (one lane per system); a unit = (tile, group of W consecutive segments) is
// one workgroup of W waves, each holding one K x 64 block of the right-hand
// side in registers from load to store; the waves pass their segment
// interface states through LDS, and the groups of a tile exchange theirs by
// decoupled look-back (lookback.h).  Variants: many matrices in one launch
// (k_group_onepass), system-major storage (k_onepass_t, also with the 2-D
// Cahn-Hilliard explicit term formed in the kernel), and one fused
// refinement correction (k_onepass_fix).
//
// Units take tickets from a counter in ticket order (tile-major), so a unit
// only ever waits on units that already hold a slot (look-back) or on later
// units of its own tile (look-ahead).  While at least one whole tile of
// units fits on the device at once (checked on the host), every wait ends;
// each wait is also bounded, and a wait that runs out raises the plan's
// error word and lets the wave finish.
#include <cstdlib>

#include "lookback.h"

namespace pent {
namespace {

using namespace lb;

// Grouped form: a workgroup of W waves holds W consecutive segments of one
// 64-system tile (K rows each); see lookback.h.  Three waves per SIMD (at
// most 168 vector registers): for 64-row blocks this spills a few values,
// and measured faster than two waves per SIMD without spills (more blocks
// resident while carries are in flight).
template <int K, int W, typename TI>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(3))) void k_onepass(
    const FwdRec *fwd_, const BwdRec *bwd_, const SegRec *seg_, int64_t n, int ngroups,
    const TI *Fin, int64_t ldf, double *X, int64_t ldx, int64_t batch, unsigned int *ctr,
    unsigned int *fst, unsigned int *bst, double *ex, unsigned int *err, int64_t tsf, int64_t tsx)
{
    PENT_GROUP_LDS(W);
    __shared__ unsigned int s_unit;
    const CFwd fwd = (CFwd)fwd_;
    const CBwd bwd = (CBwd)bwd_;
    const CSeg seg = (CSeg)seg_;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int lane = threadIdx.x & 63;
    if (w == 0) s_unit = take_unit(ctr);  // every lane of wave 0 stores the same value
    __syncthreads();
    const unsigned int u = (unsigned int)__builtin_amdgcn_readfirstlane((int)s_unit);
    const int t = (int)(u / (unsigned int)ngroups), g = (int)(u % (unsigned int)ngroups);
    const int64_t j = (int64_t)t * 64 + lane;
    const bool act = j < batch;
    // column j of tile t at t * ts + (j % 64); idle lanes read the tile's first column
    const int64_t jf = (int64_t)t * tsf + (act ? lane : 0), jx = (int64_t)t * tsx + (act ? lane : 0);
    const int64_t r0 = ((int64_t)g * W + w) * K;
    const int64_t rem = n - r0;
    const int L = (int)(rem < 0 ? 0 : rem < K ? rem : K);
    double v[K];
    load_rows<K, TI>(v, Fin + jf + (L > 0 ? r0 * ldf : 0), ldf, act ? L : 0);
    group_phases<K, W>(v, fwd, bwd, seg, r0, w, g, ngroups, u - (unsigned int)g, fst, bst, ex, err,
                       sh, agg, mat);
    if (!act || L == 0) return;
    double *base = X + jx + r0 * ldx;
    if (L == K) {
#pragma unroll
        for (int k = 0; k < K; k++) __builtin_nontemporal_store(v[k], base + k * ldx);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++)
            if (k < L) base[k * ldx] = v[k];
    }
}

// Many matrices in one launch: the unit table lists (matrix, 64-system
// tile, row group) with each tile's groups consecutive; otherwise as
// k_onepass, but with the single-wait phases (group_phases_1w): the many
// short matrices give tiles of few groups, where the chain latency, not
// the wait for the tile's loads, dominates.
template <int K, int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(3))) void k_group_onepass(
    const GroupMat *__restrict__ mats, const GroupUnit *__restrict__ units, unsigned int *ctr,
    unsigned int *fst, unsigned int *bst, double *ex, unsigned int *err)
{
    PENT_GROUP1W_LDS(W);
    __shared__ unsigned int s_unit;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int lane = threadIdx.x & 63;
    if (w == 0) s_unit = take_unit(ctr);  // every lane of wave 0 stores the same value
    __syncthreads();
    const unsigned int u = (unsigned int)__builtin_amdgcn_readfirstlane((int)s_unit);
    const GroupUnit un = units[u];
    const GroupMat m = mats[un.mat];
    const CFwd fwd = (CFwd)m.fwd;
    const CBwd bwd = (CBwd)m.bwd;
    const CSeg seg = (CSeg)m.segp;
    const CGrp gtab = (CGrp)m.grpp;
    const int64_t j = un.col0 + lane;
    const bool act = j < m.batch;
    const int64_t jj = act ? j : un.col0;  // idle lanes read the tile's first column (its own lines)
    const int64_t r0 = ((int64_t)un.g * W + w) * K;
    const int64_t rem = m.n - r0;
    const int L = (int)(rem < 0 ? 0 : rem < K ? rem : K);
    double v[K];
    // the sweeps' records from LDS (measured faster here, where the many
    // small matrices' record tables compete for the scalar cache; slower
    // in k_onepass, where the extra registers cost spills)
    __shared__ FwdRec lf[W][K];
    __shared__ BwdRec lb[W][K];
    stage_records<K>(m.fwd, m.bwd, r0, lf[w], lb[w]);
    load_rows<K, double>(v, m.F + jj + (L > 0 ? r0 * m.ld : 0), m.ld, act ? L : 0);
    rec_wait<K>(L == K);
    group_phases_1w<K, W, true>(v, fwd, bwd, seg, gtab, r0, w, un.g, un.ngroups, (unsigned int)un.u0,
                                fst, bst, ex, err, sh, agg, mat, ucon, lf[w], lb[w]);
    if (!act || L == 0) return;
    double *base = m.F + jj + r0 * m.ld;
    if (L == K) {
#pragma unroll
        for (int k = 0; k < K; k++) __builtin_nontemporal_store(v[k], base + k * m.ld);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++)
            if (k < L) base[k * m.ld] = v[k];
    }
}

// The double in lane l (a wave-uniform constant index) of v.
__device__ __forceinline__ double lane_double(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The double of lane l - 1 (UP) or l + 1 of the wave, by a DPP wave shift;
// the lane with no such neighbour (0, resp. 63) gets edge.  Every lane of
// the wave must be active.
template <bool UP>
__device__ __forceinline__ double lane_shift(double x, double edge)
{
    constexpr int ctrl = UP ? 0x138 : 0x130;  // wave_shr:1 / wave_shl:1
    const long long xi = __double_as_longlong(x), ei = __double_as_longlong(edge);
    const int lo = __builtin_amdgcn_update_dpp((int)ei, (int)xi, ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(ei >> 32), (int)(xi >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// r = f - A x over a block held in v (x on entry, r on exit), compensated
// (dot2_row); rows k >= L zero.  8 rows per batch, one batch ahead: f by
// row, and the batch's 5 x 8 diagonal entries by one gathering load (lane
// 8 d + q holds diagonal d of row q), read out lane by lane -- no scalar
// load latency per row.
template <int K, typename TI>
__device__ __forceinline__ void fix_residual(double (&v)[K], const double *diag, int64_t n,
                                             const TI *fc, int64_t ldf, int64_t r0, int L,
                                             double hm2, double hm1, double hp0, double hp1)
{
    constexpr int B = 8;
    const int lane = threadIdx.x & 63;
    auto frow = [&](int k) { return fc[(k < L ? k : 0) * ldf]; };
    auto coef = [&](int c) {  // rows past the matrix read its last row (dropped)
        const int l = lane < 5 * B ? lane : 0;
        const int64_t row = r0 + c * B + (l % B);
        return diag[(l / B) * n + (row < n ? row : n - 1)];
    };
    double p2 = hm2, p1 = hm1;
    TI fb[B], fn[B];
    double cb = coef(0), cn = 0.0;
#pragma unroll
    for (int q = 0; q < B; q++) fb[q] = frow(q);
#pragma unroll
    for (int c = 0; c < K / B; c++) {
        if (c + 1 < K / B) {
            cn = coef(c + 1);
#pragma unroll
            for (int q = 0; q < B; q++) fn[q] = frow((c + 1) * B + q);
        }
#pragma unroll
        for (int q = 0; q < B; q++) {
            const int k = c * B + q;
            const double xk = v[k];
            const double x1 = k + 1 < K ? v[k + 1] : hp0;
            const double x2 = k + 2 < K ? v[k + 2] : (k + 2 == K ? hp0 : hp1);
            const double cf[5] = {lane_double(cb, q), lane_double(cb, B + q), lane_double(cb, 2 * B + q),
                                  lane_double(cb, 3 * B + q), lane_double(cb, 4 * B + q)};
            const double xv[5] = {p2, p1, xk, x1, x2};
            const double r = dot2_row((double)fb[q], cf, xv);
            v[k] = k < L ? r : 0.0;
            p2 = p1;
            p1 = xk;
        }
        cb = cn;
#pragma unroll
        for (int q = 0; q < B; q++) fb[q] = fn[q];
    }
}

// System-major right-hand sides (element (row i, system s) at F[s*ld + i],
// e.g. the x sweeps of a grid stored x-fastest), in place: the single pass
// of k_onepass with each wave's K x 64 block transposed through LDS, 8 rows
// at a time.  Loads and stores move whole 128-byte runs of each system (8
// lanes per system, 16 bytes each, 8 systems per instruction); in registers
// every lane holds one system's rows, as in k_onepass.  Positions past the matrix or
// the batch load from clamped addresses (no load under a per-lane test) and
// are zeroed or never stored.
//
// ST: the x sweeps of a 2-D Cahn-Hilliard step (Sec. 2.1's semi-implicit
// scheme, split over x and y) with the explicit right-hand side formed here
// instead of in a pass of its own: C[y][k][x] is read, R = C + dt_k *
// Lap_h(C^3 - C) is formed in registers and swept, and the result is stored
// to F (same layout).  Systems are numbered instance-major, s = k * ny + y,
// so the 64 systems of a tile are consecutive y of one instance (where the
// tile does not straddle two): a system's y neighbours are the adjacent
// lanes, read back through the transpose buffer, plus one halo system above
// and below the tile (one row per lane); its x neighbours are the adjacent
// rows in registers, plus one value past each end of the block.  The y
// neighbours' terms come by DPP wave shifts of the row's own term (lanes 0
// and 63 take the halo systems' instead).  Three waves per SIMD in both
// forms.
template <int K, int W, bool ST>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(3))) void k_onepass_t(
    const FwdRec *fwd_, const BwdRec *bwd_, const SegRec *seg_, int64_t n, int ngroups, double *F,
    int64_t ld, int64_t batch, unsigned int *ctr, unsigned int *fst, unsigned int *bst, double *ex,
    unsigned int *err, const double *Cin, int64_t ny, int64_t ninst, const double *dt,
    double inv_h2, unsigned int *clr, int64_t nclr)
{
    static_assert(!ST || K == 64, "the halo rows are held one per lane");
    // status words of the launch that follows on the stream (nclr of them at
    // clr, at most one per thread of the grid), cleared here so that it
    // needs no clearing kernel of its own
    {
        const int64_t i = (int64_t)blockIdx.x * (64 * W) + threadIdx.x;
        if (i < nclr) clr[i] = 0u;
    }
    PENT_GROUP_LDS(W);
    __shared__ double tb[W][8][66];  // row stride 66: the transposing writes hit distinct banks
    __shared__ double xe[ST ? W : 1][2][64];  // ST: each block's first and last row of C
    __shared__ unsigned int s_unit;
    const CFwd fwd = (CFwd)fwd_;
    const CBwd bwd = (CBwd)bwd_;
    const CSeg seg = (CSeg)seg_;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int lane = threadIdx.x & 63;
    if (w == 0) s_unit = take_unit(ctr);  // every lane of wave 0 stores the same value
    __syncthreads();
    const unsigned int u = (unsigned int)__builtin_amdgcn_readfirstlane((int)s_unit);
    const int t = (int)(u / (unsigned int)ngroups), g = (int)(u % (unsigned int)ngroups);
    const int64_t s0 = (int64_t)t * 64;
    const int64_t r0 = ((int64_t)g * W + w) * K;
    const int64_t rem = n - r0;
    const int L = (int)(rem < 0 ? 0 : rem < K ? rem : K);
    const int sub = lane & 7, grp = lane >> 3;  // row in a chunk, system in an 8-system slice
    // first element of system s, and the distance between consecutive
    // systems of one run (ST: instance k's systems at y * ninst * ld + k * ld)
    auto sbase = [&](int64_t s) -> int64_t {
        if constexpr (ST) {
            const int64_t k = s / ny;
            return ((s - k * ny) * ninst + k) * ld;
        } else {
            return s * ld;
        }
    };
    const int64_t sst = ST ? ninst * ld : ld;
    const double *src = ST ? Cin : F;
    double v[K];
    // raw loads in 16-row chunks c: lane (sub, grp) takes rows 2 sub, 2 sub + 1
    // of the chunk of system s0 + 8q + grp (8 lanes cover a whole 128-byte
    // run of each system), into v[16c + 2q + e], e the row parity.  A full
    // block (all rows in the matrix, all 64 systems in the batch, and for ST
    // in one instance) is one per-lane base plus uniform offsets; a ragged
    // one clamps each address.  (the 16-byte accesses also need every
    // system's run 16-byte aligned: an even ld and F itself aligned)
    // ST: the values around the block, issued ahead of the block's loads
    // (they come from scattered lines; the stencil waits for them last)
    double xl = 0.0, xr = 0.0, h0 = 0.0, h1 = 0.0, dtk = 0.0;
    bool up = false, dn = false;
    if constexpr (ST) {
        const int64_t sl = s0 + lane < batch ? s0 + lane : batch - 1;  // this lane's system
        const int64_t kl = sl / ny, yl = sl - kl * ny;
        const int64_t bl = (yl * ninst + kl) * ld;
        up = yl >= 1;
        dn = yl + 1 < ny;
        // the rows just past the block: inside the workgroup they are its
        // neighbour waves' (exchanged below); only the group's first and
        // last wave load them (a block wholly past the matrix, r0 >= n,
        // clamps both to row n - 1)
        if (w == 0) xl = Cin[bl + (r0 < 1 ? 0 : r0 - 1 < n ? r0 - 1 : n - 1)];
        if (w == W - 1) xr = Cin[bl + (r0 + K < n ? r0 + K : n - 1)];
        dtk = dt[kl];
        // halo systems: s0 - 1 above lane 0, s0 + 64 below lane 63 (each used
        // only where that lane's own mask allows: same instance, inside the
        // grid), row r0 + lane of each
        const int64_t hrow = r0 + lane < n ? r0 + lane : n - 1;
        const int64_t sa = s0 >= 1 ? s0 - 1 : 0;
        const int64_t sb = s0 + 64 < batch ? s0 + 64 : batch - 1;
        h0 = Cin[sbase(sa) + hrow];
        h1 = Cin[sbase(sb) + hrow];
    }
    typedef double Dbl2 __attribute__((ext_vector_type(2)));
    bool full = L == K && s0 + 64 <= batch && ld % 2 == 0 && (uintptr_t)F % 16 == 0;
    if constexpr (ST) full = full && s0 % ny + 64 <= ny && (uintptr_t)Cin % 16 == 0;
    if (full) {
        const double *pl = src + sbase(s0) + grp * sst + r0 + 2 * sub;
#pragma unroll
        for (int c = 0; c < K / 16; c++)
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const Dbl2 p = __builtin_nontemporal_load((const Dbl2 *)(pl + 8 * q * sst + 16 * c));
                v[16 * c + 2 * q] = p.x;
                v[16 * c + 2 * q + 1] = p.y;
            }
    } else {
#pragma unroll
        for (int c = 0; c < K / 16; c++) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                int64_t sys = s0 + 8 * q + grp;
                sys = sys < batch ? sys : batch - 1;
                const int64_t sb = sbase(sys);
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    int64_t row = r0 + 16 * c + 2 * sub + e;
                    row = row < n ? row : n - 1;
                    v[16 * c + 2 * q + e] = src[sb + row];
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // 16 loads at a time: few addresses live
        }
    }
    // transpose in place, one row parity at a time (8 rows through the 8-row
    // buffer): afterwards v[k] = (row r0 + k, system s0 + lane)
    double(*tw)[66] = tb[w];
#pragma unroll
    for (int c = 0; c < K / 16; c++) {
#pragma unroll
        for (int e = 0; e < 2; e++) {
#pragma unroll
            for (int q = 0; q < 8; q++) tw[sub][8 * q + grp] = v[16 * c + 2 * q + e];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const int row = 16 * c + 2 * k + e;
                const double x = tw[k][lane];
                v[row] = row < L ? x : 0.0;  // rows past the matrix
            }
        }
    }
    if constexpr (ST) {
        // right-hand side in place, row by row: the y neighbours' C^3 - C by
        // wave shifts of the row's own (lanes 0 and 63 take the halo
        // systems', held lane = row and read out per row); x neighbours roll
        // along the rows
        const bool west = r0 >= 1, east = r0 + K < n;
        const double hs = ch_wterm(h0), hn = ch_wterm(h1);
        xe[w][0][lane] = v[0];
        xe[w][1][lane] = v[K - 1];
        __syncthreads();
        if (w > 0) xl = xe[w - 1][1][lane];
        if (w < W - 1) xr = xe[w + 1][0][lane];
        double wprev = west ? ch_wterm(xl) : 0.0;
        double wcur = ch_wterm(v[0]);
#pragma unroll
        for (int row = 0; row < K; row++) {
            const double ts = lane_shift<true>(wcur, lane_double(hs, row));
            const double tn = lane_shift<false>(wcur, lane_double(hn, row));
            const double wn = dn ? tn : 0.0;
            const double ws = up ? ts : 0.0;
            const double wnext = ch_wterm(row + 1 < K ? v[row + 1] : xr);
            const double we = (row + 1 < K ? r0 + row + 1 < n : east) ? wnext : 0.0;
            const double r = ch_point(v[row], wcur, we, wprev, wn, ws, dtk, inv_h2);
            wprev = wcur;
            wcur = wnext;
            v[row] = row < L ? r : 0.0;
        }
    }
    group_phases<K, W>(v, fwd, bwd, seg, r0, w, g, ngroups, u - (unsigned int)g, fst, bst, ex, err,
                       sh, agg, mat);
    // transpose back (per row parity) and store whole 128-byte runs
#pragma unroll
    for (int c = 0; c < K / 16; c++) {
#pragma unroll
        for (int e = 0; e < 2; e++) {
#pragma unroll
            for (int k = 0; k < 8; k++) tw[k][lane] = v[16 * c + 2 * k + e];
#pragma unroll
            for (int q = 0; q < 8; q++) v[16 * c + 2 * q + e] = tw[sub][8 * q + grp];
        }
    }
    if (full) {
        double *pl = F + sbase(s0) + grp * sst + r0 + 2 * sub;
#pragma unroll
        for (int c = 0; c < K / 16; c++)
#pragma unroll
            for (int q = 0; q < 8; q++)
                __builtin_nontemporal_store(Dbl2{v[16 * c + 2 * q], v[16 * c + 2 * q + 1]},
                                            (Dbl2 *)(pl + 8 * q * sst + 16 * c));
    } else {
#pragma unroll
        for (int c = 0; c < K / 16; c++)
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const int64_t sys = s0 + 8 * q + grp;
                const int64_t sb = sbase(sys < batch ? sys : batch - 1);
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    const int64_t row = r0 + 16 * c + 2 * sub + e;
                    if (row < n && sys < batch) F[sb + row] = v[16 * c + 2 * q + e];
                }
            }
    }
}

// One refinement correction in a single pass: each block forms the
// residual r = f - A x of its rows from f and x (x with two halo rows each
// side, zero outside the matrix; compensated, dot2_row), solves A d = r by
// the same look-back sweeps, and adds d to x in place.  The update cannot
// race the neighbours' halo reads: a block stores only after its tile's
// carries have passed through both neighbours, which post them only after
// their loads have completed.  x = A^{-1} f to one more correction.
// 2 waves per SIMD: the halo and residual terms need more registers.
template <int K, int W, typename TI>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(2))) void k_onepass_fix(
    const FwdRec *fwd_, const BwdRec *bwd_, const SegRec *seg_, const double *__restrict__ diag,
    int64_t n, int ngroups, const TI *F, int64_t ldf, double *X, int64_t ldx, int64_t batch,
    unsigned int *ctr, unsigned int *fst, unsigned int *bst, double *ex, unsigned int *err)
{
    PENT_GROUP_LDS(W);
    __shared__ unsigned int s_unit;
    const CFwd fwd = (CFwd)fwd_;
    const CBwd bwd = (CBwd)bwd_;
    const CSeg seg = (CSeg)seg_;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
    const int lane = threadIdx.x & 63;
    if (w == 0) s_unit = take_unit(ctr);  // every lane of wave 0 stores the same value
    __syncthreads();
    const unsigned int u = (unsigned int)__builtin_amdgcn_readfirstlane((int)s_unit);
    const int t = (int)(u / (unsigned int)ngroups), g = (int)(u % (unsigned int)ngroups);
    const int64_t j = (int64_t)t * 64 + lane;
    const bool act = j < batch;
    const int64_t jj = act ? j : 0;
    const int64_t r0 = ((int64_t)g * W + w) * K;
    const int64_t rem = n - r0;
    const int L = (int)(rem < 0 ? 0 : rem < K ? rem : K);
    double v[K];
    // x of the block, and its halo rows (zero outside the matrix)
    load_rows<K, double>(v, X + jj + (L > 0 ? r0 * ldx : 0), ldx, act ? L : 0);
    // Every load below is unconditional, from a row clamped into the matrix
    // (a load whose value is used under a per-lane condition gets sunk into
    // that branch and waited for there).  No select is needed: a halo row
    // outside the matrix meets a zero diagonal entry (the stored diagonals
    // are zero there), rows past L are zeroed after the residual, and lanes
    // past the batch store nothing.
    auto xrow = [&](int64_t i) { return X[(i < 0 ? 0 : i >= n ? n - 1 : i) * ldx + jj]; };
    const double hm2 = xrow(r0 - 2), hm1 = xrow(r0 - 1), hp0 = xrow(r0 + K), hp1 = xrow(r0 + K + 1);
    // r over x, row by row, the two overwritten x values kept rolling; rows
    // past the matrix (k >= L) give zero
    fix_residual<K, TI>(v, diag, n, F + jj + (L > 0 ? r0 * ldf : 0), ldf, r0, L, hm2, hm1, hp0, hp1);
    group_phases<K, W>(v, fwd, bwd, seg, r0, w, g, ngroups, u - (unsigned int)g, fst, bst, ex, err,
                       sh, agg, mat);
    if (!act || L == 0) return;
    // x += d, 32 rows at a time: every load of a batch is issued before its
    // stores (one round trip per batch; the compiler cannot tell the rows
    // apart, so an interleaved read-modify-write would wait per row)
    double *base = X + jj + r0 * ldx;
#pragma unroll
    for (int b = 0; b < K; b += 32) {
        double xo[32];
#pragma unroll
        for (int q = 0; q < 32; q++) xo[q] = base[(b + q < L ? b + q : 0) * ldx];
#pragma unroll
        for (int q = 0; q < 32; q++)
            if (b + q < L) base[(b + q) * ldx] = xo[q] + v[b + q];
    }
}

__global__ void k_zero_words(unsigned int *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

template <int K, int W>
const void *onepass_fn(bool f32)
{
    return f32 ? (const void *)k_onepass<K, W, float> : (const void *)k_onepass<K, W, double>;
}

const void *onepass_fn_kw(int K, int W, bool f32)
{
    if (K == 64) return W == 2 ? onepass_fn<64, 2>(f32) : W == 4 ? onepass_fn<64, 4>(f32) : onepass_fn<64, 8>(f32);
    return W == 2 ? onepass_fn<32, 2>(f32) : W == 4 ? onepass_fn<32, 4>(f32) : onepass_fn<32, 8>(f32);
}

}  // namespace

// Waves per workgroup forced by PENT_ONEPASS_WAVES (2, 4 or 8; read once),
// or 0.
int onepass_waves_override()
{
    static const int env = [] {
        const char *e = std::getenv("PENT_ONEPASS_WAVES");
        const int v = e ? std::atoi(e) : 0;
        return (v == 2 || v == 4 || v == 8) ? v : 0;
    }();
    return env;
}

// Waves (segments) per workgroup of the single-pass kernel: 4 measured best
// for both segment lengths (shorter interface chains than 2, and unlike 8
// still three workgroups per CU).
int onepass_waves(int seg_rows)
{
    (void)seg_rows;
    const int o = onepass_waves_override();
    return o ? o : 4;
}

int64_t onepass_groups(int64_t n, int seg_rows)
{
    const int64_t rows = (int64_t)seg_rows * onepass_waves(seg_rows);
    return (n + rows - 1) / rows;
}

int64_t onepass_units(int64_t n, int seg_rows, int64_t batch)
{
    return (batch + 63) / 64 * onepass_groups(n, seg_rows);
}

int64_t onepass_words(int64_t n, int seg_rows, int64_t batch)
{
    return kTicketWords + 2 * onepass_units(n, seg_rows, batch);
}

size_t onepass_scratch_bytes(int64_t n, int seg_rows, int64_t batch)
{
    const int64_t units = onepass_units(n, seg_rows, batch);
    const size_t words = (size_t)onepass_words(n, seg_rows, batch);
    const size_t wbytes = (words * sizeof(unsigned int) + 255) / 256 * 256;
    return wbytes + (size_t)units * kExRows * 64 * sizeof(double);
}

int onepass_capacity(int seg_rows)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int W = onepass_waves(seg_rows);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, onepass_fn_kw(seg_rows, W, false),
                                                     64 * W, 0) != hipSuccess)
        return 0;
    return cus * per_cu;
}

hipError_t launch_onepass(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg, int64_t n,
                          int seg_rows, const void *Fin, bool f32, int64_t ldf, double *X,
                          int64_t ldx, int64_t batch, void *scratch, unsigned int *err,
                          hipStream_t s, int64_t tsf, int64_t tsx, bool words_clear)
{
    if (seg_rows != 32 && seg_rows != 64) return hipErrorInvalidValue;
    const int W = onepass_waves(seg_rows);
    const int64_t ngroups = onepass_groups(n, seg_rows);
    const int64_t units = onepass_units(n, seg_rows, batch);
    // segment records exist for ngroups * W segments: the cache is padded to
    // a multiple of kSegPad, which W divides
    if (units > (int64_t)UINT32_MAX / 2 || kSegPad % W != 0) return hipErrorInvalidValue;
    const int64_t words = onepass_words(n, seg_rows, batch);
    unsigned int *w = (unsigned int *)scratch;
    unsigned int *ctr = w, *fst = w + kTicketWords, *bst = w + kTicketWords + units;
    const size_t wbytes = ((size_t)words * sizeof(unsigned int) + 255) / 256 * 256;
    double *ex = (double *)((char *)scratch + wbytes);
    hipError_t e = hipSuccess;
    if (!words_clear) {
        hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, w, words);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const void *fn = onepass_fn_kw(seg_rows, W, f32);
    const SegRec *segp = seg;
    int ng = (int)ngroups;
    void *args[] = {(void *)&fwd, (void *)&bwd, (void *)&segp, (void *)&n, (void *)&ng, (void *)&Fin,
                    (void *)&ldf, (void *)&X, (void *)&ldx, (void *)&batch, (void *)&ctr,
                    (void *)&fst, (void *)&bst, (void *)&ex, (void *)&err, (void *)&tsf, (void *)&tsx};
    e = hipLaunchKernel(fn, dim3((unsigned)units), dim3(64 * W), args, 0, s);
    return e;
}

// The single pass over system-major right-hand sides (k_onepass_t): 64-row
// segments, four per workgroup; scratch as launch_onepass.
constexpr int kTK = 64, kTW = 4;

int onepass_t_capacity(bool stencil)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const void *fn = stencil ? (const void *)k_onepass_t<kTK, kTW, true>
                             : (const void *)k_onepass_t<kTK, kTW, false>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kTW, 0) != hipSuccess) return 0;
    return cus * per_cu;
}

int64_t onepass_t_groups(int64_t n) { return (n + kTK * kTW - 1) / (kTK * kTW); }

int64_t onepass_t_threads(int64_t n, int64_t batch)
{
    return (batch + 63) / 64 * onepass_t_groups(n) * 64 * kTW;
}

size_t onepass_t_scratch_bytes(int64_t n, int64_t batch)
{
    const int64_t units = (batch + 63) / 64 * onepass_t_groups(n);
    const size_t words = (size_t)(kTicketWords + 2 * units);
    const size_t wbytes = (words * sizeof(unsigned int) + 255) / 256 * 256;
    return wbytes + (size_t)units * kExRows * 64 * sizeof(double);
}

namespace {

hipError_t launch_t(bool stencil, const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg64,
                    int64_t n, double *F, int64_t batch, int64_t ld, void *scratch,
                    unsigned int *err, const double *Cin, int64_t ny, int64_t ninst,
                    const double *dt, double inv_h2, hipStream_t s, unsigned int *clr,
                    int64_t nclr)
{
    const int64_t ngroups = onepass_t_groups(n);
    const int64_t units = (batch + 63) / 64 * ngroups;
    if (units > (int64_t)UINT32_MAX / 2 || kSegPad % kTW != 0) return hipErrorInvalidValue;
    const int64_t words = kTicketWords + 2 * units;
    unsigned int *w = (unsigned int *)scratch;
    unsigned int *ctr = w, *fst = w + kTicketWords, *bst = w + kTicketWords + units;
    const size_t wbytes = ((size_t)words * sizeof(unsigned int) + 255) / 256 * 256;
    double *ex = (double *)((char *)scratch + wbytes);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, w, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int ng = (int)ngroups;
    void *args[] = {(void *)&fwd, (void *)&bwd, (void *)&seg64, (void *)&n,   (void *)&ng,
                    (void *)&F,   (void *)&ld,  (void *)&batch, (void *)&ctr, (void *)&fst,
                    (void *)&bst, (void *)&ex,  (void *)&err,   (void *)&Cin, (void *)&ny,
                    (void *)&ninst, (void *)&dt, (void *)&inv_h2, (void *)&clr, (void *)&nclr};
    const void *fn = stencil ? (const void *)k_onepass_t<kTK, kTW, true>
                             : (const void *)k_onepass_t<kTK, kTW, false>;
    return hipLaunchKernel(fn, dim3((unsigned)units), dim3(64 * kTW), args, 0, s);
}

}  // namespace

hipError_t launch_onepass_t(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg64, int64_t n,
                            double *F, int64_t batch, int64_t ld, void *scratch, unsigned int *err,
                            hipStream_t s)
{
    return launch_t(false, fwd, bwd, seg64, n, F, batch, ld, scratch, err, F, batch, 1, nullptr, 0.0, s,
                    nullptr, 0);
}

hipError_t launch_onepass_t_ch2d(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg64,
                                 int64_t n, const double *C, double *R, int64_t ny, int64_t ninst,
                                 const double *dt, double h, void *scratch, unsigned int *err,
                                 hipStream_t s, unsigned int *clear, int64_t clear_words)
{
    if (clear_words < 0 || (clear_words > 0 && !clear) || clear_words > onepass_t_threads(n, ny * ninst))
        return hipErrorInvalidValue;
    return launch_t(true, fwd, bwd, seg64, n, R, ny * ninst, n, scratch, err, C, ny, ninst, dt,
                    1.0 / (h * h), s, clear, clear_words);
}

// One fused refinement correction (k_onepass_fix): x += A^{-1}(f - A x).
// diag: the 5n row-indexed diagonals; scratch and capacity as launch_onepass
// (64-row segments, four per workgroup).
constexpr int kFixK = 64, kFixW = 4;

int onepass_fix_capacity()
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void *)k_onepass_fix<kFixK, kFixW, double>, 64 * kFixW, 0) != hipSuccess)
        return 0;
    return cus * per_cu;
}

int64_t onepass_fix_groups(int64_t n) { return (n + kFixK * kFixW - 1) / (kFixK * kFixW); }

size_t onepass_fix_scratch_bytes(int64_t n, int64_t batch)
{
    const int64_t units = (batch + 63) / 64 * onepass_fix_groups(n);
    const size_t words = (size_t)(kTicketWords + 2 * units);
    const size_t wbytes = (words * sizeof(unsigned int) + 255) / 256 * 256;
    return wbytes + (size_t)units * kExRows * 64 * sizeof(double);
}

hipError_t launch_onepass_fix(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg64,
                              const double *diag, int64_t n, const void *F, bool f32, int64_t ldf,
                              double *X, int64_t ldx, int64_t batch, void *scratch,
                              unsigned int *err, hipStream_t s)
{
    const int64_t ngroups = onepass_fix_groups(n);
    const int64_t units = (batch + 63) / 64 * ngroups;
    if (units > (int64_t)UINT32_MAX / 2 || kSegPad % kFixW != 0) return hipErrorInvalidValue;
    const int64_t words = kTicketWords + 2 * units;
    unsigned int *w = (unsigned int *)scratch;
    unsigned int *ctr = w, *fst = w + kTicketWords, *bst = w + kTicketWords + units;
    const size_t wbytes = ((size_t)words * sizeof(unsigned int) + 255) / 256 * 256;
    double *ex = (double *)((char *)scratch + wbytes);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, w, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void *fn = f32 ? (const void *)k_onepass_fix<kFixK, kFixW, float>
                         : (const void *)k_onepass_fix<kFixK, kFixW, double>;
    int ng = (int)ngroups;
    void *args[] = {(void *)&fwd, (void *)&bwd, (void *)&seg64, (void *)&diag, (void *)&n,
                    (void *)&ng, (void *)&F, (void *)&ldf, (void *)&X, (void *)&ldx,
                    (void *)&batch, (void *)&ctr, (void *)&fst, (void *)&bst, (void *)&ex,
                    (void *)&err};
    return hipLaunchKernel(fn, dim3((unsigned)units), dim3(64 * kFixW), args, 0, s);
}

// ---- group variant 6: kGroupSegRows-row segments, four per workgroup
constexpr int kGroupK = kGroupSegRows, kGroupW = 4;

int group_onepass_rows() { return kGroupK * kGroupW; }

int group_onepass_capacity()
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, (const void *)k_group_onepass<kGroupK, kGroupW>, 64 * kGroupW, 0) != hipSuccess)
        return 0;
    return cus * per_cu;
}

size_t group_onepass_scratch_bytes(int64_t units)
{
    const size_t words = (size_t)(kTicketWords + 2 * units);
    const size_t wbytes = (words * sizeof(unsigned int) + 255) / 256 * 256;
    return wbytes + (size_t)units * kExRows * 64 * sizeof(double);
}

hipError_t launch_group_onepass(const GroupMat *mats, const GroupUnit *units, int64_t nunits,
                                void *scratch, unsigned int *err, hipStream_t s)
{
    if (nunits <= 0) return hipSuccess;
    if (nunits > (int64_t)UINT32_MAX / 2) return hipErrorInvalidValue;
    const int64_t words = kTicketWords + 2 * nunits;
    unsigned int *w = (unsigned int *)scratch;
    unsigned int *ctr = w, *fst = w + kTicketWords, *bst = w + kTicketWords + nunits;
    const size_t wbytes = ((size_t)words * sizeof(unsigned int) + 255) / 256 * 256;
    double *ex = (double *)((char *)scratch + wbytes);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, w, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_group_onepass<kGroupK, kGroupW>), dim3((unsigned)nunits), dim3(64 * kGroupW),
                       0, s, mats, units, ctr, fst, bst, ex, err);
    return hipGetLastError();
}

}  // namespace pent
