// factor.hip -- assembly of I + sigma*D4, the A = L R factorisation and the
// per-segment constants of the partitioned sweep.
#include "internal.h"

namespace pent {
namespace {

// I + sigma*D4 (Sec. 2.3 coefficient list), truncated at both ends.  The
// products and the sum 1 + 6 sigma are rounded separately (no contraction)
// so the diagonals are the IEEE values of the printed formulas.
__global__ void k_assemble_d4(double *__restrict__ diag, int64_t n, double sigma)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s4 = -4.0 * sigma;
    diag[0 * n + i] = (i >= 2) ? sigma : 0.0;
    diag[1 * n + i] = (i >= 1) ? s4 : 0.0;
    diag[2 * n + i] = 1.0 + 6.0 * sigma;
    diag[3 * n + i] = (i + 1 < n) ? s4 : 0.0;
    diag[4 * n + i] = (i + 2 < n) ? sigma : 0.0;
}

// A = L R (Sec. 2.4).  The recurrence is serial in the row index:
//   beta_i  = b_i - a_i gamma_{i-2}
//   alpha_i = c_i - a_i delta_{i-2} - beta_i gamma_{i-1}
//   gamma_i = (d_i - beta_i delta_{i-1}) / alpha_i
//   delta_i = e_i / alpha_i
// (the paper's first and last rows are the general step with zero padding).
// Operations are rounded one by one in the written order (no contraction,
// IEEE division), so the factors are the correctly rounded values of that
// sequence.  One workgroup: its threads bring the diagonals into LDS a chunk
// of kFC rows at a time (the next chunk while the current one is worked on)
// and write the factors out coalesced; one lane runs the recurrence from
// LDS, kFU rows per batch with the batch's diagonal entries read ahead of
// its arithmetic, so a row costs the latency of its dependent arithmetic
// (one product, one difference, one division) and no memory round trip.
//
// Where the diagonals repeat (the interior of a constant-coefficient matrix
// such as I + sigma D4) the rounded recurrence falls into an exact cycle: a
// row's factors are a function of its diagonals and the previous two rows'
// factors, so once two consecutive rows equal, bit for bit, the rows p
// earlier, every following row whose diagonals equal those p rows earlier
// repeats the row p earlier too.  Every kFCheck rows the wave looks for such
// a period p <= 63 among the rows it has just produced; when one holds, the
// block finds the first later row whose diagonals break the period and
// copies the p-periodic rows up to it in parallel, then the serial lane
// resumes there.  The factors are the same bits as without the shortcut; a
// matrix with no repeating stretch runs fully serial.
//
// The loop has no branch on the pivot: the first row with a zero or
// non-finite pivot is recorded and the rows from it on are overwritten
// afterwards (no shortcut is taken after such a row).  *bad receives that
// row, or -1.
constexpr int kFC = 512;     // rows per chunk
constexpr int kFU = 8;       // rows per batch of the serial lane
constexpr int kFCheck = 64;  // rows between checks for a period

__global__ __launch_bounds__(256) void k_factor_serial(const double *__restrict__ diag, int64_t n,
                                                       double *__restrict__ fac,
                                                       int64_t *__restrict__ bad)
{
#pragma clang fp contract(off)
    __shared__ double din[2][5][kFC];  // diagonals a..e of the chunk (zero outside the matrix)
    __shared__ double dout[4][kFC];    // alpha, beta, gamma, delta of the chunk
    __shared__ long long s_bad;
    __shared__ int s_period;           // period found by the serial wave (0: none)
    __shared__ int s_done;             // rows of the chunk computed when it was found
    __shared__ unsigned long long s_until;
    const int tid = threadIdx.x, lane = tid & 63;
    double *alpha = fac, *beta = fac + n, *gamma = fac + 2 * n, *delta = fac + 3 * n;
    // diagonal q of row i (zero outside the matrix)
    auto dg = [&](int q, int64_t i) -> double {
        if (i < 0 || i >= n) return 0.0;
        const bool in = q == 0 ? i >= 2 : q == 1 ? i >= 1 : q == 3 ? i + 1 < n : q == 4 ? i + 2 < n : true;
        return in ? diag[(int64_t)q * n + i] : 0.0;
    };
    // threads [t0, t0 + nt) fetch rows r0 .. r0 + kFC - 1 into din[buf]
    auto load_chunk = [&](int64_t r0, int buf, int t0, int nt) {
        for (int k = tid - t0; k < 5 * kFC; k += nt) {
            const int q = k / kFC, r = k % kFC;
            din[buf][q][r] = dg(q, r0 + r);
        }
    };
    if (tid == 0) s_bad = -1;
    double gam2 = 0.0, del2 = 0.0, gam1 = 0.0, del1 = 0.0;  // the serial lane's state
    long long badrow = -1;
    int64_t start = 0;
    while (start < n) {
        // serial phase from row `start`
        const int64_t nch = (n - start + kFC - 1) / kFC;
        if (tid == 0) s_period = 0;
        load_chunk(start, 0, 0, 256);
        __syncthreads();
        int64_t next = n;
        for (int64_t c = 0; c < nch; c++) {
            const int buf = (int)(c & 1);
            const int64_t c0 = start + c * kFC;
            const int rows = (int)(n - c0 < kFC ? n - c0 : kFC);
            if (tid >= 64) {
                if (c + 1 < nch) load_chunk(c0 + kFC, buf ^ 1, 64, 192);  // waves 1..3 fetch ahead
            } else {
                const double(*d)[kFC] = din[buf];
                for (int sb = 0; sb < kFC; sb += kFCheck) {
                    if (lane == 0) {
                        for (int r0 = sb; r0 < sb + kFCheck; r0 += kFU) {
                            double a[kFU], b[kFU], cc[kFU], dd[kFU], e[kFU];
#pragma unroll
                            for (int k = 0; k < kFU; k++) {
                                a[k] = d[0][r0 + k];
                                b[k] = d[1][r0 + k];
                                cc[k] = d[2][r0 + k];
                                dd[k] = d[3][r0 + k];
                                e[k] = d[4][r0 + k];
                            }
#pragma unroll
                            for (int k = 0; k < kFU; k++) {
                                const double be = b[k] - a[k] * gam2;
                                const double al = cc[k] - a[k] * del2 - be * gam1;
                                const double ga = (dd[k] - be * del1) / al;
                                const double de = e[k] / al;
                                const int64_t i = c0 + r0 + k;
                                const bool pivot_bad = !(al != 0.0) || !__builtin_isfinite(al);
                                badrow = (badrow < 0 && pivot_bad && i < n) ? (long long)i : badrow;
                                dout[0][r0 + k] = al;
                                dout[1][r0 + k] = be;
                                dout[2][r0 + k] = ga;
                                dout[3][r0 + k] = de;
                                gam2 = gam1;
                                del2 = del1;
                                gam1 = ga;
                                del1 = de;
                            }
                        }
                    }
                    // a period: the chunk's last two rows equal, bit for bit, the
                    // rows p earlier (lane p tests period p)
                    const int eb = sb + kFCheck < rows ? sb + kFCheck : rows;
                    const long long brow = __builtin_amdgcn_readfirstlane((int)badrow);
                    bool ok = lane >= 1 && eb - 2 - lane >= 0 && brow < 0 && c0 + eb < n;
                    if (ok) {
#pragma unroll
                        for (int q = 0; q < 4; q++)
                            ok = ok &&
                                 __double_as_longlong(dout[q][eb - 1]) == __double_as_longlong(dout[q][eb - 1 - lane]) &&
                                 __double_as_longlong(dout[q][eb - 2]) == __double_as_longlong(dout[q][eb - 2 - lane]);
                    }
                    const unsigned long long hit = __ballot(ok);
                    if (hit != 0) {
                        if (lane == 0) {
                            s_period = __builtin_ctzll(hit);
                            s_done = eb;
                        }
                        break;
                    }
                    if (eb >= rows) break;
                }
            }
            __syncthreads();
            const int done = s_period ? s_done : rows;
            for (int k = tid; k < 4 * kFC; k += 256) {
                const int q = k / kFC, r = k % kFC;
                if (r < done) fac[(int64_t)q * n + c0 + r] = dout[q][r];
            }
            __syncthreads();  // dout and the next chunk's buffer are reused
            if (s_period) {
                next = c0 + done;
                break;
            }
        }
        if (next >= n) break;
        // copy phase: rows next .. m-1 repeat the rows p earlier, m the first
        // row whose diagonals differ from those p rows before it (or n)
        const int p = s_period;
        if (tid == 0) s_until = (unsigned long long)n;
        __syncthreads();
        for (int64_t i = next + tid; i < n; i += 256) {
            bool same = true;
#pragma unroll
            for (int q = 0; q < 5; q++)
                same = same && __double_as_longlong(dg(q, i)) == __double_as_longlong(dg(q, i - p));
            if (!same) atomicMin(&s_until, (unsigned long long)i);
        }
        __syncthreads();
        const int64_t m = (int64_t)s_until;
        for (int64_t i = next + tid; i < m; i += 256) {
            const int64_t src = next - p + (i - next) % p;
            alpha[i] = alpha[src];
            beta[i] = beta[src];
            gamma[i] = gamma[src];
            delta[i] = delta[src];
        }
        __syncthreads();
        // the serial lane resumes at row m from the rows m-2, m-1
        if (tid == 0 && m < n) {
            gam2 = gamma[m - 2];
            del2 = delta[m - 2];
            gam1 = gamma[m - 1];
            del1 = delta[m - 1];
        }
        start = m;
        __syncthreads();
    }
    if (tid == 0) s_bad = badrow;
    __syncthreads();
    const long long b0 = s_bad;
    if (b0 >= 0) {
        // leave defined values behind: gamma, delta zero from the bad row on,
        // alpha 1 and beta 0 past it (as if the factorisation had stopped)
        for (int64_t i = b0 + tid; i < n; i += 256) {
            gamma[i] = 0.0;
            delta[i] = 0.0;
            if (i > b0) {
                alpha[i] = 1.0;
                beta[i] = 0.0;
            }
        }
    }
    if (tid == 0) *bad = b0;
}

// Sweep records from the factors (row-parallel).
__global__ void k_records(const double *__restrict__ diag, const double *__restrict__ fac,
                          int64_t n, int64_t npad, FwdRec *__restrict__ fwd,
                          BwdRec *__restrict__ bwd)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i >= n) {  // padding rows: all zero
        fwd[i] = FwdRec{0.0, 0.0, 0.0, 0.0};
        bwd[i] = BwdRec{0.0, 0.0};
        return;
    }
    const double al = fac[i];
    const double be = (i >= 1) ? fac[n + i] : 0.0;
    const double ai = (i >= 2) ? diag[i] : 0.0;
    FwdRec r;
    r.ra = 1.0 / al;
    r.ap = ai / al;
    r.bp = be / al;
    r.pad = 0.0;
    fwd[i] = r;
    BwdRec q;
    q.gm = (i + 1 < n) ? fac[2 * n + i] : 0.0;
    q.dl = (i + 2 < n) ? fac[3 * n + i] : 0.0;
    bwd[i] = q;
}

// Per-segment transfer matrices of the partitioned sweep.  For segment s
// (rows r0 .. r0+L-1, L = min(K, n-r0)):
//   u, v  = forward responses to the incoming states (1,0) and (0,1) with f = 0;
//   tf    = outgoing forward state of u, v;
//   cg    = outgoing backward state of the zero-incoming back substitution of u, v;
//   tb    = outgoing backward state of the back substitution of g = 0 from the
//           incoming states (1,0) and (0,1).
// The recurrences are the same prescaled ones the sweeps use.
template <int K>
__global__ void k_seg_prep(const FwdRec *__restrict__ fwd, const BwdRec *__restrict__ bwd,
                           int64_t n, int64_t nseg, SegRec *__restrict__ seg)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const int64_t r0 = s * K;
    const int L = (int)((n - r0) < K ? (n - r0) : K);
    double u[K], v[K];
    SegRec out;
    // forward responses
    {
        double up2 = 1.0, up1 = 0.0, vp2 = 0.0, vp1 = 1.0;
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (k < L) {
                const FwdRec r = fwd[r0 + k];
                const double gu = fma(-r.bp, up1, -r.ap * up2);
                const double gv = fma(-r.bp, vp1, -r.ap * vp2);
                u[k] = gu; v[k] = gv;
                up2 = up1; up1 = gu;
                vp2 = vp1; vp1 = gv;
            } else {
                u[k] = 0.0; v[k] = 0.0;
            }
        }
        out.tf[0] = up2; out.tf[1] = up1;
        out.tf[2] = vp2; out.tf[3] = vp1;
    }
    // backward: zero-incoming over u, v; and g = 0 from unit incoming states
    {
        double uq1 = 0.0, uq2 = 0.0, vq1 = 0.0, vq2 = 0.0;
        double aq1 = 1.0, aq2 = 0.0, bq1 = 0.0, bq2 = 1.0;
#pragma unroll
        for (int k = K - 1; k >= 0; k--) {
            if (k < L) {
                const BwdRec q = bwd[r0 + k];
                const double xu = fma(-q.gm, uq1, fma(-q.dl, uq2, u[k]));
                const double xv = fma(-q.gm, vq1, fma(-q.dl, vq2, v[k]));
                const double xa = fma(-q.gm, aq1, -q.dl * aq2);
                const double xb = fma(-q.gm, bq1, -q.dl * bq2);
                uq2 = uq1; uq1 = xu;
                vq2 = vq1; vq1 = xv;
                aq2 = aq1; aq1 = xa;
                bq2 = bq1; bq1 = xb;
            }
        }
        out.cg[0] = uq1; out.cg[1] = uq2;
        out.cg[2] = vq1; out.cg[3] = vq2;
        out.tb[0] = aq1; out.tb[1] = aq2;
        out.tb[2] = bq1; out.tb[3] = bq2;
    }
    out.pad[0] = out.pad[1] = out.pad[2] = out.pad[3] = 0.0;
    seg[s] = out;
}

// C = A B for column-major 2x2 matrices, explicit fused multiply-adds.
__device__ __forceinline__ void mat2_mul(const double *a, const double *b, double *c)
{
    const double c0 = fma(a[2], b[1], a[0] * b[0]), c1 = fma(a[3], b[1], a[1] * b[0]);
    const double c2 = fma(a[2], b[3], a[0] * b[2]), c3 = fma(a[3], b[3], a[1] * b[2]);
    c[0] = c0;
    c[1] = c1;
    c[2] = c2;
    c[3] = c3;
}

// Group constants of the single pass (GrpRec) from the segment records of
// segments [G*W, G*W + W) of each group G (the segment table is padded with
// all-zero records past the matrix).  One lane, serial over the groups; a
// few hundred matrix products per matrix, once per handle.
__global__ void k_grp_prep(const SegRec *__restrict__ seg, int W, int64_t ngroups,
                           GrpRec *__restrict__ grp)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int64_t G = 0; G < ngroups; G++) {
        const SegRec *sg = seg + G * W;
        // tg = Tf_{W-1} ... Tf_0, tbg = Tb_0 ... Tb_{W-1},
        // cg = sum_i (Tb_0 ... Tb_{i-1}) Cg_i (Tf_{i-1} ... Tf_0)
        double tg[4] = {1.0, 0.0, 0.0, 1.0}, bp[4] = {1.0, 0.0, 0.0, 1.0}, cg[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < W; i++) {
            double t[4], u[4];
            mat2_mul(sg[i].cg, tg, t);  // Cg_i M_i
            mat2_mul(bp, t, u);         // (Tb_0 ... Tb_{i-1}) Cg_i M_i
            for (int k = 0; k < 4; k++) cg[k] = cg[k] + u[k];
            mat2_mul(sg[i].tf, tg, tg);
            mat2_mul(bp, sg[i].tb, bp);
        }
        for (int k = 0; k < 4; k++) {
            grp[G].tg[k] = tg[k];
            grp[G].tbg[k] = bp[k];
            grp[G].cg[k] = cg[k];
        }
    }
    // q_last = 0, q_G = cg_{G+1} + tbg_{G+1} q_{G+1} tg_{G+1}
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t G = ngroups - 1; G >= 0; G--) {
        for (int k = 0; k < 4; k++) grp[G].q[k] = q[k];
        if (G == 0) break;
        double t[4], u[4];
        mat2_mul(q, grp[G].tg, t);
        mat2_mul(grp[G].tbg, t, u);
        for (int k = 0; k < 4; k++) q[k] = grp[G].cg[k] + u[k];
    }
}

}  // namespace

hipError_t launch_grp_prep(const SegRec *d_seg, int waves, int64_t ngroups, GrpRec *d_grp,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_grp_prep, dim3(1), dim3(64), 0, s, d_seg, waves, ngroups, d_grp);
    return hipGetLastError();
}

hipError_t launch_assemble_d4(double *d_diag, int64_t n, double sigma, hipStream_t s)
{
    const int bs = 256;
    const int64_t grid = (n + bs - 1) / bs;
    hipLaunchKernelGGL(k_assemble_d4, dim3((unsigned)grid), dim3(bs), 0, s, d_diag, n, sigma);
    return hipGetLastError();
}

hipError_t launch_factor(const double *d_diag, int64_t n, int64_t npad, double *d_fac,
                         FwdRec *d_fwd, BwdRec *d_bwd, int64_t *d_bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_factor_serial, dim3(1), dim3(256), 0, s, d_diag, n, d_fac, d_bad);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int bs = 256;
    const int64_t grid = (npad + bs - 1) / bs;
    hipLaunchKernelGGL(k_records, dim3((unsigned)grid), dim3(bs), 0, s, d_diag, d_fac, n, npad,
                       d_fwd, d_bwd);
    return hipGetLastError();
}

hipError_t launch_seg_prep(const FwdRec *d_fwd, const BwdRec *d_bwd, int64_t n, int seg_rows,
                           SegRec *d_seg, hipStream_t s)
{
    const int64_t nseg = (n + seg_rows - 1) / seg_rows;
    const int bs = 64;
    const dim3 grid((unsigned)((nseg + bs - 1) / bs));
    switch (seg_rows) {
    case 16: hipLaunchKernelGGL(k_seg_prep<16>, grid, dim3(bs), 0, s, d_fwd, d_bwd, n, nseg, d_seg); break;
    case 32: hipLaunchKernelGGL(k_seg_prep<32>, grid, dim3(bs), 0, s, d_fwd, d_bwd, n, nseg, d_seg); break;
    case 64: hipLaunchKernelGGL(k_seg_prep<64>, grid, dim3(bs), 0, s, d_fwd, d_bwd, n, nseg, d_seg); break;
    case kGroupSegRows:
        hipLaunchKernelGGL(k_seg_prep<kGroupSegRows>, grid, dim3(bs), 0, s, d_fwd, d_bwd, n, nseg, d_seg);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pent
