// rewrite.hip -- every system with its own matrix, factored and solved in
// one call: the paper's refactor-every-step mode (Sec. 3), in which the
// matrix may change between time steps, measured against a general batched
// pentadiagonal solver.
//
// One lane per system (the factorisation recurrence is not linear in its
// carried values, so the segment decomposition of the constant-matrix
// schedules does not apply).  Downward pass: the Sec. 2.4 factorisation and
// forward sweep of row i together (beta, alpha, gamma, delta, then g), with
// gamma and delta written to the workspace and g over f; upward pass: back
// substitution.  Every stream is batch-fastest, so a wave's access to one
// row is one coalesced 512-byte segment; rows come in blocks of D,
// double-buffered, so the loads of the next block are in flight while the
// current one is computed.  HBM: 6 x 8 B read + 3 x 8 B written downward,
// 3 x 8 B read + 8 B written upward = 104 B per unknown.
#include "internal.h"

namespace pent {
namespace {

template <int D>
struct DownBlock {
    double a[D], b[D], c[D], d[D], e[D], f[D];
};

template <int D>
__device__ __forceinline__ void load_down(DownBlock<D> &blk, const double *A, const double *B,
                                          const double *C, const double *Dg, const double *E,
                                          int64_t ldm, const double *F, int64_t ld, int i0, int n)
{
#pragma unroll
    for (int k = 0; k < D; k++) {
        const int i = i0 + k;
        const bool in = i < n;
        const int64_t om = (int64_t)(in ? i : 0) * ldm, of = (int64_t)(in ? i : 0) * ld;
        blk.a[k] = in ? __builtin_nontemporal_load(A + om) : 0.0;
        blk.b[k] = in ? __builtin_nontemporal_load(B + om) : 0.0;
        blk.c[k] = in ? __builtin_nontemporal_load(C + om) : 1.0;
        blk.d[k] = in ? __builtin_nontemporal_load(Dg + om) : 0.0;
        blk.e[k] = in ? __builtin_nontemporal_load(E + om) : 0.0;
        blk.f[k] = in ? F[of] : 0.0;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_rewrite(const double *__restrict__ A,
                                                 const double *__restrict__ B,
                                                 const double *__restrict__ C,
                                                 const double *__restrict__ Dg,
                                                 const double *__restrict__ E, int64_t ldm, int n,
                                                 double *__restrict__ F, int64_t batch, int64_t ld,
                                                 double *__restrict__ Gm, double *__restrict__ Dl,
                                                 unsigned long long *__restrict__ bad)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;  // no barriers: lanes past the batch just leave
    A += j;
    B += j;
    C += j;
    Dg += j;
    E += j;
    double *col = F + j;
    double *gcol = Gm + j, *dcol = Dl + j;  // workspace rows have stride batch
    // downward: factorisation and forward sweep
    double gm2 = 0.0, gm1 = 0.0, dl2 = 0.0, dl1 = 0.0, g2 = 0.0, g1 = 0.0;
    bool ok = true;
    DownBlock<D> cur, nxt;
    load_down<D>(cur, A, B, C, Dg, E, ldm, col, ld, 0, n);
    for (int i0 = 0; i0 < n; i0 += D) {
        if (i0 + D < n) load_down<D>(nxt, A, B, C, Dg, E, ldm, col, ld, i0 + D, n);
#pragma unroll
        for (int k = 0; k < D; k++) {
            const int i = i0 + k;
            if (i < n) {
                // entries outside the matrix are ignored (read as zero)
                const double ai = i >= 2 ? cur.a[k] : 0.0, bi = i >= 1 ? cur.b[k] : 0.0;
                const double di = i + 1 < n ? cur.d[k] : 0.0, ei = i + 2 < n ? cur.e[k] : 0.0;
                const double beta = fma(-ai, gm2, bi);
                const double alpha = fma(-beta, gm1, fma(-ai, dl2, cur.c[k]));
                if (ok && (!(alpha != 0.0) || !__builtin_isfinite(alpha))) {
                    ok = false;
                    atomicMin(bad, (unsigned long long)j * (unsigned long long)n + (unsigned long long)i);
                }
                const double r = 1.0 / alpha;
                const double gam = fma(-beta, dl1, di) * r;
                const double del = ei * r;
                const double g = fma(-beta, g1, fma(-ai, g2, cur.f[k])) * r;
                __builtin_nontemporal_store(gam, gcol + (int64_t)i * batch);
                __builtin_nontemporal_store(del, dcol + (int64_t)i * batch);
                col[(int64_t)i * ld] = g;
                gm2 = gm1;
                gm1 = gam;
                dl2 = dl1;
                dl1 = del;
                g2 = g1;
                g1 = g;
            }
        }
        cur = nxt;
    }
    // upward: back substitution x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2}
    double x1 = 0.0, x2 = 0.0;
    const int top = ((n - 1) / D) * D;
    double cg[D], cgm[D], cdl[D], ng[D], ngm[D], ndl[D];
    auto load_up = [&](double(&g)[D], double(&gmv)[D], double(&dlv)[D], int b0) {
#pragma unroll
        for (int k = 0; k < D; k++) {
            const int i = b0 + k;
            const bool in = i < n;
            const int64_t ii = in ? i : 0;
            g[k] = in ? col[ii * ld] : 0.0;
            gmv[k] = in ? __builtin_nontemporal_load(gcol + ii * batch) : 0.0;
            dlv[k] = in ? __builtin_nontemporal_load(dcol + ii * batch) : 0.0;
        }
    };
    load_up(cg, cgm, cdl, top);
    for (int b0 = top; b0 >= 0; b0 -= D) {
        if (b0 - D >= 0) load_up(ng, ngm, ndl, b0 - D);
#pragma unroll
        for (int k = D - 1; k >= 0; k--) {
            const int i = b0 + k;
            if (i < n) {
                const double x = fma(-cdl[k], x2, fma(-cgm[k], x1, cg[k]));
                col[(int64_t)i * ld] = x;
                x2 = x1;
                x1 = x;
            }
        }
#pragma unroll
        for (int k = 0; k < D; k++) {
            cg[k] = ng[k];
            cgm[k] = ngm[k];
            cdl[k] = ndl[k];
        }
    }
}

__global__ void k_rewrite_init(unsigned long long *bad)
{
    if (threadIdx.x == 0) *bad = ~0ull;
}

}  // namespace

size_t rewrite_workspace_bytes(int64_t n, int64_t batch)
{
    return 256 + sizeof(double) * 2 * (size_t)n * (size_t)batch;
}

hipError_t launch_rewrite(const double *a, const double *b, const double *c, const double *d,
                          const double *e, int64_t ldm, int64_t n, double *F, int64_t batch,
                          int64_t ld, void *work, hipStream_t s)
{
    unsigned long long *bad = (unsigned long long *)work;
    double *G = (double *)((char *)work + 256);
    double *H = G + n * batch;
    hipLaunchKernelGGL(k_rewrite_init, dim3(1), dim3(64), 0, s, bad);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int bs = 256;
    hipLaunchKernelGGL(k_rewrite<8>, dim3((unsigned)((batch + bs - 1) / bs)), dim3(bs), 0, s, a, b, c,
                       d, e, ldm, (int)n, F, batch, ld, G, H, bad);
    return hipGetLastError();
}

}  // namespace pent
