// cyclic.hip -- periodic (cyclic) pentadiagonal matrices through Navon's
// bordering (Sec. 2.3), and the explicit half of the Crank-Nicolson step.
//
// With E the leading (n-2) x (n-2) block, k the last two columns of the
// first n-2 rows, h^T the first n-2 columns of the last two rows and C2 the
// trailing 2 x 2 block:
//     (x_{n-2}, x_{n-1}) = [C2 - h^T E^{-1} k]^{-1} ((f_{n-2}, f_{n-1}) - h^T E^{-1} f^)
//     x^               = E^{-1} f^ - (E^{-1} k) (x_{n-2}, x_{n-1})
// (0-based rows).  Z = E^{-1} k and the 2 x 2 inverse are computed once per
// matrix.  Per solve this library runs ONE batched pentadiagonal solve
// y = E^{-1} f^ in place, then h^T y (h^T has at most ten non-zeros, so it
// reads a handful of rows of y), then the update x^ = y - Z x_tail -- the
// same quantities as the paper's formula, with the E-solve shared by both
// uses of E^{-1} f^.
//
// Cyclic row-indexed diagonals: row i holds a[i] at column (i-2) mod n,
// b[i] at (i-1) mod n, c[i] at i, d[i] at (i+1) mod n, e[i] at (i+2) mod n.
#include "lookback.h"

namespace pent {
namespace {

__device__ __forceinline__ double cyc_coef(const double *cd, int64_t n, int64_t i, int o)
{
    return cd[(o + 2) * cyc_ld(n) + i];  // o in -2..2 -> a, b, c, d, e
}

__global__ void k_cyc_assemble_d4(double *__restrict__ cd, int64_t n, double sigma)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t ld = cyc_ld(n);
    cd[i] = sigma;
    cd[ld + i] = -4.0 * sigma;
    cd[2 * ld + i] = 1.0 + 6.0 * sigma;
    cd[3 * ld + i] = -4.0 * sigma;
    cd[4 * ld + i] = sigma;
}

// E's diagonals (m = n-2 rows), zero outside the (m x m) block.
__global__ void k_cyc_build_E(const double *__restrict__ cd, int64_t n, double *__restrict__ ed)
{
    const int64_t m = n - 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t ld = cyc_ld(n);
    ed[i] = (i >= 2) ? cd[i] : 0.0;
    ed[m + i] = (i >= 1) ? cd[ld + i] : 0.0;
    ed[2 * m + i] = cd[2 * ld + i];
    ed[3 * m + i] = (i + 1 < m) ? cd[3 * ld + i] : 0.0;
    ed[4 * m + i] = (i + 2 < m) ? cd[4 * ld + i] : 0.0;
}

// K (m x 2, batch-fastest, ld 2): column s = entries of A in column m + s;
// rows m .. rows-1 are zero padding (the single-pass kernel reads Z = E^{-1} K
// by row without guards).
__global__ void k_cyc_build_k(const double *__restrict__ cd, int64_t n, int64_t rows,
                              double *__restrict__ K)
{
    const int64_t m = n - 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    if (i >= m) {
        K[2 * i] = 0.0;
        K[2 * i + 1] = 0.0;
        return;
    }
    double k0 = 0.0, k1 = 0.0;
    for (int o = -2; o <= 2; o++) {
        const int64_t col = ((i + o) % n + n) % n;
        if (col == m) k0 += cyc_coef(cd, n, i, o);
        if (col == m + 1) k1 += cyc_coef(cd, n, i, o);
    }
    K[2 * i] = k0;
    K[2 * i + 1] = k1;
}

// E^T's diagonals: row i of E^T is column i of E.
__global__ void k_cyc_build_Et(const double *__restrict__ cd, int64_t n, double *__restrict__ etd)
{
    const int64_t m = n - 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int64_t ld = cyc_ld(n);
    etd[i] = (i >= 2) ? cd[4 * ld + i - 2] : 0.0;            // E[i-2][i]
    etd[m + i] = (i >= 1) ? cd[3 * ld + i - 1] : 0.0;        // E[i-1][i]
    etd[2 * m + i] = cd[2 * ld + i];                          // E[i][i]
    etd[3 * m + i] = (i + 1 < m) ? cd[ld + i + 1] : 0.0;     // E[i+1][i]
    etd[4 * m + i] = (i + 2 < m) ? cd[i + 2] : 0.0;          // E[i+2][i]
}

// H (rows x 2, ld 2): H[i][q] = A[m+q][i] for i < m (the border rows h^T),
// zero for i >= m.
__global__ void k_cyc_build_H(const double *__restrict__ cd, int64_t n, int64_t rows,
                              double *__restrict__ H)
{
    const int64_t m = n - 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    double h0 = 0.0, h1 = 0.0;
    if (i < m) {
        for (int o = -2; o <= 2; o++) {
            if (((m + o) % n + n) % n == i) h0 += cyc_coef(cd, n, m, o);
            if (((m + 1 + o) % n + n) % n == i) h1 += cyc_coef(cd, n, m + 1, o);
        }
    }
    H[2 * i] = h0;
    H[2 * i + 1] = h1;
}

// Sparse h^T, C2 and [C2 - h^T Z]^{-1}, one lane.
__global__ void k_cyc_finish(const double *__restrict__ cd, int64_t n, const double *__restrict__ Z,
                             CycAux *__restrict__ aux)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int64_t m = n - 2;
    CycAux a;
    a.nh = 0;
    double C2[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    double HZ[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int q = 0; q < 2; q++) {
        const int64_t r = m + q;
        for (int o = -2; o <= 2; o++) {
            const int64_t col = ((r + o) % n + n) % n;
            const double v = cyc_coef(cd, n, r, o);
            if (col >= m) {
                C2[q][col - m] += v;
            } else {
                a.hq[a.nh] = q;
                a.hcol[a.nh] = col;
                a.hv[a.nh] = v;
                a.nh++;
                HZ[q][0] += v * Z[2 * col];
                HZ[q][1] += v * Z[2 * col + 1];
            }
        }
    }
    const double m00 = C2[0][0] - HZ[0][0], m01 = C2[0][1] - HZ[0][1];
    const double m10 = C2[1][0] - HZ[1][0], m11 = C2[1][1] - HZ[1][1];
    const double det = m00 * m11 - m01 * m10;
    a.minv[0] = m11 / det;
    a.minv[1] = -m01 / det;
    a.minv[2] = -m10 / det;
    a.minv[3] = m00 / det;
    a.bad = !(det != 0.0) || !__builtin_isfinite(det);
    *aux = a;
}

// Per system: x_tail = Minv ((f_m, f_{m+1}) - h^T y), written over f_m, f_{m+1}
// (each lane reads and writes only its own column).
__global__ void k_cyc_tail(const CycAux *__restrict__ aux, double *__restrict__ F, int64_t m,
                           int64_t batch, int64_t ld)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;
    double t0 = F[m * ld + j], t1 = F[(m + 1) * ld + j];
    const int nh = aux->nh;
    for (int k = 0; k < nh; k++) {
        const double v = aux->hv[k] * F[aux->hcol[k] * ld + j];
        if (aux->hq[k] == 0) t0 -= v;
        else t1 -= v;
    }
    F[m * ld + j] = aux->minv[0] * t0 + aux->minv[1] * t1;
    F[(m + 1) * ld + j] = aux->minv[2] * t0 + aux->minv[3] * t1;
}

// x_i = y_i - Z_i0 x_tail0 - Z_i1 x_tail1 for i < m.
__global__ void k_cyc_fix(const double *__restrict__ Z, double *__restrict__ F, int64_t m,
                          int64_t batch, int64_t ld)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;
    const double x0 = F[m * ld + j], x1 = F[(m + 1) * ld + j];
    for (int64_t i = blockIdx.y; i < m; i += gridDim.y)
        F[i * ld + j] = F[i * ld + j] - Z[2 * i] * x0 - Z[2 * i + 1] * x1;
}

// R = 2 C - A C (explicit half of Crank-Nicolson for A = I + S), periodic.
__global__ void k_cn_rhs(const double *__restrict__ cd, int64_t n, const double *__restrict__ C,
                         int64_t ldc, double *__restrict__ R, int64_t ldr, int64_t batch)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        double acc = 2.0 * C[i * ldc + j];
        for (int o = -2; o <= 2; o++) {
            int64_t col = i + o;  // n >= 5: one wrap at most
            col += col < 0 ? n : 0;
            col -= col >= n ? n : 0;
            acc -= cyc_coef(cd, n, i, o) * C[col * ldc + j];
        }
        R[i * ldr + j] = acc;
    }
}

// ---- single pass: the bordered solve (and the Crank-Nicolson step) in one
// kernel.  Workgroups (64-system tile, W consecutive segments of the E rows,
// one per wave) hold their rows in registers from load to store; the E-solve
// runs by look-back (lookback.h).  The last two unknowns need
// h^T E^{-1} f^ = sum over rows of (h^T E^{-1})[q][i] f_i: every block forms
// its part from the precomputed (h^T E^{-1})^T while f is in registers, every
// group posts the sum of its waves' parts, and the tile's last group adds
// the groups' parts in order while its wave 0 waits for the forward carry
// (the sum needs only the loaded blocks), forms
// x_tail = Minv ((f_{n-2}, f_{n-1}) - h^T E^{-1} f^) and posts it.  Every
// block applies x^ = y - Z x_tail in its back substitution, as the y rows
// are formed (TailCorr).  This is the paper's bordering formula with
// hT E^{-1} precomputed.
//
// With CN the block loads C rows r0-2 .. r0+K+1 (periodic) instead of f and
// forms f = 2C - AC in registers (the explicit half of the step); C and X
// must then be different buffers.  The last group forms f's tail the same
// way.
using namespace lb;


// f_i = 2 C_i - (A C)_i for row i, C rows i-2 .. i+2 in c0..c4; the
// coefficients are wave-uniform (scalar loads), ld = cyc_ld(n).
__device__ __forceinline__ double cn_row(CDbl cd, int64_t ld, int64_t i, double c0, double c1,
                                         double c2, double c3, double c4)
{
    double acc = 2.0 * c2;
    acc = fma(-cd[i], c0, acc);
    acc = fma(-cd[ld + i], c1, acc);
    acc = fma(-cd[2 * ld + i], c2, acc);
    acc = fma(-cd[3 * ld + i], c3, acc);
    acc = fma(-cd[4 * ld + i], c4, acc);
    return acc;
}

// r mod n for a window index r in [-2, n + K + 1]; the division only runs
// when n is smaller than the window (wave-uniform, so scalar code).
__device__ __forceinline__ int64_t wrap(int64_t r, int64_t n)
{
    if (r < 0) r += n;
    if (r >= n) r -= n;
    if (r < 0 || r >= n) {
        r %= n;
        if (r < 0) r += n;
    }
    return r;
}

// f_i = 2 C_i - (A C)_i with row-invariant diagonals u (same operations in
// the same order as cn_row).
struct CycUni {
    double c[5];
};
__device__ __forceinline__ double cn_row_u(const CycUni &u, double c0, double c1, double c2,
                                           double c3, double c4)
{
    double acc = 2.0 * c2;
    acc = fma(-u.c[0], c0, acc);
    acc = fma(-u.c[1], c1, acc);
    acc = fma(-u.c[2], c2, acc);
    acc = fma(-u.c[3], c3, acc);
    acc = fma(-u.c[4], c4, acc);
    return acc;
}

// Waits until *p >= want; false (and *err raised) if the wait ran out.
__device__ __forceinline__ bool wait_nonzero(unsigned int *p, unsigned int want, unsigned int *err)
{
    for (int i = 0; i < kSpin; i++) {
        const unsigned int v = poll(p);
        if (v >= want) return true;
        __builtin_amdgcn_s_sleep(1);
    }
    atomicOr(err, 1u);
    return false;
}

// The bordering correction, run inside group_phases.  early(): on the
// tile's last group, by a wave that waits for nothing else then, adds the
// groups' partial products in group order (they need only the loaded
// blocks), forms x_tail = Minv ((f_{n-2}, f_{n-1}) - h^T E^{-1} f^), posts it
// (status tst, values tx) and stores it as rows n-2, n-1 of x.  fetch(): the
// group's last wave reads x_tail while wave 0 waits for the backward carry
// and leaves it in LDS (xt).  The back substitution then stores
// x^_i = y_i - Z_i x_tail as it forms y_i.
struct TailCorr {
    static constexpr bool on = true;
    CDbl Z;
    unsigned int *tst;
    double *tx;  // the tile's x_tail (rows 0 and 64, a column per lane)
    unsigned int *err;
    double (*xt)[64];  // LDS, 2 x 64
    bool last;         // this group forms x_tail
    unsigned int *pst;
    const double *pex;
    unsigned int u0;  // the tile's first unit
    int ngroups;
    const double (*sft)[64];  // LDS: f_{n-2}, f_{n-1} of the tile
    const CycAux *aux;
    double *xt_rows;  // X + the tile's first column
    int64_t m, ldx;
    bool act;
    __device__ void early(int lane) const
    {
        if (!last) return;
        // every group's partial products, in group order (windows of 64)
        bool timed_out = false;
        for (int b0 = 0; b0 < ngroups; b0 += 64) {
            for (int spin = 0;; spin++) {
                const bool in = b0 + lane < ngroups;
                const unsigned int st = lane_status(pst, (int64_t)u0 + b0 + lane, in);
                if (__ballot(in && st == 0) == 0) break;
                if (spin >= kSpin) {
                    atomicOr(err, 1u);
                    timed_out = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        double d0 = 0.0, d1 = 0.0;
        for (int q0 = 0; q0 < ngroups; q0 += 8) {
            double a0[8], a1[8];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const double *pp = pex + (int64_t)(u0 + q0 + i) * 128 + lane;
                a0[i] = q0 + i < ngroups ? xload(&pp[0]) : 0.0;
                a1[i] = q0 + i < ngroups ? xload(&pp[64]) : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 8; i++) {
                if (q0 + i < ngroups) {
                    d0 += a0[i];
                    d1 += a1[i];
                }
            }
        }
        if (timed_out) {  // partial products never seen: poison the tail
            d0 = __builtin_nan("");
            d1 = __builtin_nan("");
        }
        const double r0v = sft[0][lane] - d0, r1v = sft[1][lane] - d1;
        const double xt0 = fma(aux->minv[1], r1v, aux->minv[0] * r0v);
        const double xt1 = fma(aux->minv[3], r1v, aux->minv[2] * r0v);
        xstore(&tx[lane], xt0);
        xstore(&tx[64 + lane], xt1);
        publish(tst, 1u);
        if (act) {
            xt_rows[m * ldx + lane] = xt0;
            xt_rows[(m + 1) * ldx + lane] = xt1;
        }
    }
    __device__ void fetch(int lane) const
    {
        const bool seen = wait_nonzero(tst, 1u, err);
        double a = xload(&tx[lane]), b = xload(&tx[64 + lane]);
        if (!seen) {  // the tail never arrived: NaN instead of stale values
            a = __builtin_nan("");
            b = __builtin_nan("");
        }
        xt[0][lane] = a;
        xt[1][lane] = b;
    }
    __device__ void get(int lane, double &c0, double &c1) const
    {
        c0 = xt[0][lane];
        c1 = xt[1][lane];
    }
};

template <int K, int W, bool CN, bool UNI>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(3))) void k_cyc_onepass(
    const FwdRec *fwd_, const BwdRec *bwd_, const SegRec *seg_, const double *__restrict__ cd_,
    const double *__restrict__ Z_, const double *__restrict__ Wt_, const CycAux *__restrict__ aux,
    int64_t n, int ngroups, const double *Fin, int64_t ldf, double *X, int64_t ldx, int64_t batch,
    unsigned int *ctr, unsigned int *fst, unsigned int *bst, unsigned int *pst, unsigned int *tst,
    double *ex, double *pex, double *tex, unsigned int *err, CycUni uc)
{
    PENT_GROUP_LDS(W);
    __shared__ double sp[W][2][64];
    __shared__ double sft[2][64];  // f_m, f_{m+1} of the tile (tail block), kept out of registers
    __shared__ unsigned int s_unit;
    const CFwd fwd = (CFwd)fwd_;
    const CBwd bwd = (CBwd)bwd_;
    const CSeg seg = (CSeg)seg_;
    const CDbl Z = (CDbl)Z_;
    const CDbl Wt = (CDbl)Wt_;
    const CDbl cd = (CDbl)cd_;
    const int64_t m = n - 2;
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
    const int64_t rem = m - r0;
    const int L = (int)(rem < 0 ? 0 : rem < K ? rem : K);  // E rows in this block
    const bool last = g == ngroups - 1;  // forms x_tail for the tile
    const double *col = Fin + jj;
    double v[K];
    if (CN) {
        // C rows r0 .. r0+K-1 into v (two rows past the block's last E row are
        // needed by the stencil: for a short last block they sit in v, else in
        // the halo h2, h3), rows r0-2, r0-1 in h0, h1; all periodic.  f is then
        // formed in place with the two overwritten originals kept rolling.
        const int Lc = L + 2 < K ? L + 2 : K;
        double h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0;
        // Halo rows held by a neighbouring wave of the group come through
        // LDS: rows r0-2, r0-1 are the last two rows of wave w-1's full
        // block; rows r0+K, r0+K+1 are the first two of wave w+1's when that
        // wave has E rows (then this block is full and needs both).  The
        // group's edge halos, and the border rows m, m+1 past a last E row,
        // are read from memory.
        const bool top_lds = w > 0;
        const bool bot_lds = w < W - 1 && m > r0 + K;
        if (act && L > 0) {
            if (!top_lds) {
                h0 = col[wrap(r0 - 2, n) * ldf];
                h1 = col[wrap(r0 - 1, n) * ldf];
            }
            if (!bot_lds) {
                if (L + 1 >= K) h2 = col[wrap(r0 + K, n) * ldf];
                if (L + 2 >= K) h3 = col[wrap(r0 + K + 1, n) * ldf];
            }
        }
        // rows r0 .. r0+Lc-1 <= m+1 never wrap (only the halo rows can)
        const double *base = col + (L > 0 ? r0 * ldf : 0);
        if (Lc == K) {
#pragma unroll
            for (int k = 0; k < K; k++) v[k] = act ? __builtin_nontemporal_load(base + k * ldf) : 0.0;
        } else {
#pragma unroll
            for (int k = 0; k < K; k++) v[k] = (act && k < Lc) ? base[k * ldf] : 0.0;
        }
        {
            // every wave's first and last two rows, through the look-back's
            // staging area (W x 4 x 64 of its kStage x 128 doubles; the
            // look-back first writes it after the barrier that follows the
            // partial products, when every wave has read its halo)
            static_assert(W * 4 * 64 <= kStage * 128, "the halo rows fit the staging area");
            double (*hx)[4][64] = (double (*)[4][64])&agg[0][0];
            hx[w][0][lane] = v[0];
            hx[w][1][lane] = v[1];
            hx[w][2][lane] = v[K - 2];
            hx[w][3][lane] = v[K - 1];
            __syncthreads();
            if (top_lds && L > 0) {
                h0 = hx[w - 1][2][lane];
                h1 = hx[w - 1][3][lane];
            }
            if (bot_lds) {
                h2 = hx[w + 1][0][lane];
                h3 = hx[w + 1][1][lane];
            }
        }
        if (last && w == 0) {
            const double cm2 = act ? col[(m - 2) * ldf] : 0.0, cm1 = act ? col[(m - 1) * ldf] : 0.0;
            const double c_m = act ? col[m * ldf] : 0.0, c_m1 = act ? col[(m + 1) * ldf] : 0.0;
            const double c0 = act ? col[0] : 0.0, c1 = act ? col[ldf] : 0.0;
            sft[0][lane] = UNI ? cn_row_u(uc, cm2, cm1, c_m, c_m1, c0)
                               : cn_row(cd, cyc_ld(n), m, cm2, cm1, c_m, c_m1, c0);
            sft[1][lane] = UNI ? cn_row_u(uc, cm1, c_m, c_m1, c0, c1)
                               : cn_row(cd, cyc_ld(n), m + 1, cm1, c_m, c_m1, c0, c1);
        }
        double c2 = h0, c1 = h1;  // C_{k-2}, C_{k-1}
        CDbl cdf = cd;
        // a copy of L the compiler cannot match with the later k < L tests,
        // so it does not keep 64 row masks live from here to the stores
        int Ls = L;
        asm volatile("" : "+s"(Ls));
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (!UNI && k % kSchedRows == 0) {
                __builtin_amdgcn_sched_barrier(0);
                cdf = fresh(cdf);
            }
            const double ck = v[k];
            const double n1 = k + 1 < K ? v[k + 1] : h2;
            const double n2 = k + 2 < K ? v[k + 2] : (k + 2 == K ? h2 : h3);
            // rows past the E rows read zero padding (no select: the
            // addresses stay affine in k, scalar loads with immediate offsets)
            const double f = UNI ? cn_row_u(uc, c2, c1, ck, n1, n2)
                                 : cn_row(cdf, cyc_ld(n), r0 + k, c2, c1, ck, n1, n2);
            v[k] = k < Ls ? f : 0.0;
            c2 = c1;
            c1 = ck;
        }
    } else {
        const double *base = col + (L > 0 ? r0 * ldf : 0);
        if (L == K) {
#pragma unroll
            for (int k = 0; k < K; k++) v[k] = act ? __builtin_nontemporal_load(base + k * ldf) : 0.0;
        } else {
#pragma unroll
            for (int k = 0; k < K; k++) v[k] = (act && k < L) ? base[k * ldf] : 0.0;
        }
        if (last && w == 0) {
            sft[0][lane] = act ? col[m * ldf] : 0.0;
            sft[1][lane] = act ? col[(m + 1) * ldf] : 0.0;
        }
    }

    // partial products of the border rows with the block: p_q = sum over its
    // rows of (h^T E^{-1})[q][i] f_i, rows in order; the group's sum (waves
    // in order) is posted for the tile's last group, which adds the groups
    // in order: h^T E^{-1} f^ with one fixed summation order.
    double p0 = 0.0, p1 = 0.0;
    {
        CDbl Wf = Wt;
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (k % kSchedRows == 0) {
                __builtin_amdgcn_sched_barrier(0);
                Wf = fresh(Wf);
            }
            const int64_t i = r0 + k;
            p0 = fma(Wf[2 * i], v[k], p0);
            p1 = fma(Wf[2 * i + 1], v[k], p1);
        }
    }
    sp[w][0][lane] = p0;
    sp[w][1][lane] = p1;
    __syncthreads();
    if (w == 0) {
        double P0 = 0.0, P1 = 0.0;
#pragma unroll
        for (int i = 0; i < W; i++) {
            P0 += sp[i][0][lane];
            P1 += sp[i][1][lane];
        }
        double *mp = pex + (int64_t)u * 128 + lane;
        xstore(&mp[0], P0);
        xstore(&mp[64], P1);
        publish(&pst[u], 1u);
    }

    const TailCorr corr{Z,   &tst[t], tex + (int64_t)t * 128, err, sp[0], last, pst, pex,
                        u - (unsigned int)g, ngroups, sft, aux, X + (int64_t)t * 64, m, ldx, act};
    group_phases<K, W, false, TailCorr>(v, fwd, bwd, seg, r0, w, g, ngroups, u - (unsigned int)g, fst,
                                        bst, ex, err, sh, agg, mat, nullptr, nullptr, corr);
    if (!act || L == 0) return;
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

__global__ void k_cyc_zero(unsigned int *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

}  // namespace

// Waves per workgroup of the periodic single pass: 2 for 64-row segments
// (measured ahead of 4 here: the kernel carries more state per wave than
// the plain single pass), else 4; PENT_ONEPASS_WAVES overrides.
static int cyc_waves(int seg_rows)
{
    const int o = onepass_waves_override();
    return o ? o : seg_rows == 64 ? 2 : 4;
}

static int64_t cyc_groups(int64_t n, int seg_rows)
{
    const int64_t rows = (int64_t)seg_rows * cyc_waves(seg_rows);
    return (n - 2 + rows - 1) / rows;
}

int64_t cyc_onepass_groups(int64_t n, int seg_rows) { return cyc_groups(n, seg_rows); }

int64_t cyc_onepass_units(int64_t n, int seg_rows, int64_t batch)
{
    return (batch + 63) / 64 * cyc_groups(n, seg_rows);
}

// words: tickets, forward / backward / partial-product statuses per unit,
// x_tail status per tile
static size_t cyc_words(int64_t n, int seg_rows, int64_t batch)
{
    const int64_t units = cyc_onepass_units(n, seg_rows, batch);
    const int64_t tiles = (batch + 63) / 64;
    return (size_t)(kTicketWords + 3 * units + tiles);
}

size_t cyc_onepass_scratch_bytes(int64_t n, int seg_rows, int64_t batch)
{
    const int64_t units = cyc_onepass_units(n, seg_rows, batch);
    const int64_t tiles = (batch + 63) / 64;
    const size_t wbytes = (cyc_words(n, seg_rows, batch) * sizeof(unsigned int) + 255) / 256 * 256;
    return wbytes + (size_t)(units * (8 + 2) * 64 + tiles * 2 * 64) * sizeof(double);
}

template <int K, int W>
static const void *cyc_fn(bool cn, bool uni)
{
    if (!cn) return (const void *)k_cyc_onepass<K, W, false, false>;
    return uni ? (const void *)k_cyc_onepass<K, W, true, true> : (const void *)k_cyc_onepass<K, W, true, false>;
}

static const void *cyc_fn_kw(int K, int W, bool cn, bool uni = false)
{
    if (K == 64) return W == 2 ? cyc_fn<64, 2>(cn, uni) : W == 4 ? cyc_fn<64, 4>(cn, uni) : cyc_fn<64, 8>(cn, uni);
    return W == 2 ? cyc_fn<32, 2>(cn, uni) : W == 4 ? cyc_fn<32, 4>(cn, uni) : cyc_fn<32, 8>(cn, uni);
}

int cyc_onepass_capacity(int seg_rows, bool cn)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int W = cyc_waves(seg_rows);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cyc_fn_kw(seg_rows, W, cn), 64 * W, 0) !=
        hipSuccess)
        return 0;
    return cus * per_cu;
}

hipError_t launch_cyc_onepass(const FwdRec *fwd, const BwdRec *bwd, const SegRec *seg,
                              const double *cd, const double *Z, const double *Wt,
                              const CycAux *aux, int64_t n,
                              int seg_rows, bool cn, const double *Fin, int64_t ldf, double *X,
                              int64_t ldx, int64_t batch, void *scratch, unsigned int *err,
                              hipStream_t s, const double *uni)
{
    if (seg_rows != 32 && seg_rows != 64) return hipErrorInvalidValue;
    const int W = cyc_waves(seg_rows);
    const int64_t ngroups = cyc_groups(n, seg_rows);
    const int64_t units = cyc_onepass_units(n, seg_rows, batch);
    if (units > (int64_t)UINT32_MAX / 2 || kSegPad % W != 0) return hipErrorInvalidValue;
    const int64_t words = (int64_t)cyc_words(n, seg_rows, batch);
    unsigned int *w = (unsigned int *)scratch;
    unsigned int *ctr = w, *fst = w + kTicketWords, *bst = w + kTicketWords + units,
                 *pst = w + kTicketWords + 2 * units, *tst = w + kTicketWords + 3 * units;
    const size_t wbytes = ((size_t)words * sizeof(unsigned int) + 255) / 256 * 256;
    double *ex = (double *)((char *)scratch + wbytes);
    double *pex = ex + units * 8 * 64;
    double *tex = pex + units * 2 * 64;
    hipLaunchKernelGGL(k_cyc_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, w, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int ng = (int)ngroups;
    CycUni uc = {{0.0, 0.0, 0.0, 0.0, 0.0}};
    if (uni)
        for (int k = 0; k < 5; k++) uc.c[k] = uni[k];
    void *args[] = {(void *)&fwd, (void *)&bwd, (void *)&seg, (void *)&cd, (void *)&Z, (void *)&Wt,
                    (void *)&aux, (void *)&n, (void *)&ng, (void *)&Fin, (void *)&ldf, (void *)&X,
                    (void *)&ldx, (void *)&batch, (void *)&ctr, (void *)&fst, (void *)&bst,
                    (void *)&pst, (void *)&tst, (void *)&ex, (void *)&pex, (void *)&tex,
                    (void *)&err, (void *)&uc};
    return hipLaunchKernel(cyc_fn_kw(seg_rows, W, cn, uni != nullptr), dim3((unsigned)units),
                           dim3(64 * W), args, 0, s);
}

hipError_t launch_cyc_assemble_d4(double *cd, int64_t n, double sigma, hipStream_t s)
{
    hipLaunchKernelGGL(k_cyc_assemble_d4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cd, n,
                       sigma);
    return hipGetLastError();
}

hipError_t launch_cyc_build(const double *cd, int64_t n, int64_t zrows, double *ed, double *K,
                            hipStream_t s)
{
    const int64_t m = n - 2;
    hipLaunchKernelGGL(k_cyc_build_E, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, cd, n, ed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cyc_build_k, dim3((unsigned)((zrows + 255) / 256)), dim3(256), 0, s, cd, n,
                       zrows, K);
    return hipGetLastError();
}

hipError_t launch_cyc_build_transposed(const double *cd, int64_t n, int64_t zrows, double *etd,
                                       double *H, hipStream_t s)
{
    const int64_t m = n - 2;
    hipLaunchKernelGGL(k_cyc_build_Et, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, cd, n, etd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cyc_build_H, dim3((unsigned)((zrows + 255) / 256)), dim3(256), 0, s, cd, n,
                       zrows, H);
    return hipGetLastError();
}

hipError_t launch_cyc_finish(const double *cd, int64_t n, const double *Z, CycAux *aux, hipStream_t s)
{
    hipLaunchKernelGGL(k_cyc_finish, dim3(1), dim3(64), 0, s, cd, n, Z, aux);
    return hipGetLastError();
}

hipError_t launch_cyc_correct(const CycAux *aux, const double *Z, double *F, int64_t n,
                              int64_t batch, int64_t ld, hipStream_t s)
{
    const int64_t m = n - 2;
    hipLaunchKernelGGL(k_cyc_tail, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, aux, F, m,
                       batch, ld);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)((batch + 255) / 256), (unsigned)(m < 4096 ? m : 4096));
    hipLaunchKernelGGL(k_cyc_fix, grid, dim3(256), 0, s, Z, F, m, batch, ld);
    return hipGetLastError();
}

hipError_t launch_cn_rhs(const double *cd, int64_t n, const double *C, int64_t ldc, double *R,
                         int64_t ldr, int64_t batch, hipStream_t s)
{
    const dim3 grid((unsigned)((batch + 255) / 256), (unsigned)(n < 4096 ? n : 4096));
    hipLaunchKernelGGL(k_cn_rhs, grid, dim3(256), 0, s, cd, n, C, ldc, R, ldr, batch);
    return hipGetLastError();
}

}  // namespace pent
