// mixed.hip -- kernels of the precision extension: compensated FP64 residual
// r = f - A x, the update x += d, the per-system backward error and ||A||_inf.
//
// The residual carries every product and partial sum with its rounding error
// (TwoProduct by fused multiply-add, TwoSum; the "Dot2" scheme of Ogita, Rump
// and Oishi, SIAM J. Sci. Comput. 26, 2005), so r is accurate to about one
// rounding of its own size even when it is 1e-16 of the terms.
#include "internal.h"

namespace pent {
namespace {

constexpr int kRB = 32;  // rows per lane in the residual / backward-error kernels

template <typename TI>
__device__ __forceinline__ double ld_in(const TI *p)
{
    return (double)*p;
}

// One lane = one system and kRB consecutive rows; x rows i0-2 .. i0+kRB+1 are
// held in registers.  Diagonal entries are wave-uniform (scalar loads).
template <typename TI, bool STORE_R>
__device__ __forceinline__ void residual_block(const double *__restrict__ diag, int64_t n,
                                               const TI *f, int64_t ldf, const double *x,
                                               int64_t ldx, int64_t j, int64_t i0, double (&r)[kRB],
                                               double (&fv)[kRB], double (&xw)[kRB + 4])
{
#pragma unroll
    for (int k = 0; k < kRB + 4; k++) {
        const int64_t i = i0 - 2 + k;
        xw[k] = (i >= 0 && i < n) ? x[i * ldx + j] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kRB; k++) {
        const int64_t i = i0 + k;
        fv[k] = (i < n) ? ld_in(f + i * ldf + j) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kRB; k++) {
        const int64_t i = i0 + k;
        if (i < n) {
            const double cf[5] = {diag[i], diag[n + i], diag[2 * n + i], diag[3 * n + i],
                                  diag[4 * n + i]};
            const double xv[5] = {xw[k], xw[k + 1], xw[k + 2], xw[k + 3], xw[k + 4]};
            r[k] = dot2_row(fv[k], cf, xv);
        } else {
            r[k] = 0.0;
        }
    }
}

// Interior block (rows i0-2 .. i0+kRB+1 all inside the matrix): no bounds
// tests, and the diagonal entries come 4 rows at a time through a fresh
// pointer, so their scalar loads neither pile up at the start (out of scalar
// registers) nor wait one row at a time.  r is formed over f (rv holds f on
// entry).
// MAXES: also fold max |x| and max |f| over the block's rows into xm, fm.
template <typename TI, bool MAXES = false>
__device__ __forceinline__ void residual_interior(const double *__restrict__ diag, int64_t n,
                                                  const TI *f, int64_t ldf, const double *x,
                                                  int64_t ldx, int64_t j, int64_t i0,
                                                  double (&fv)[kRB], double *xm = nullptr,
                                                  double *fm = nullptr)
{
    double xw[kRB + 4];
    const double *xc = x + (i0 - 2) * ldx + j;
    const TI *fc = f + i0 * ldf + j;
#pragma unroll
    for (int k = 0; k < kRB + 4; k++) xw[k] = __builtin_nontemporal_load(xc + k * ldx);
#pragma unroll
    for (int k = 0; k < kRB; k++) fv[k] = (double)__builtin_nontemporal_load(fc + k * ldf);
    if (MAXES) {
#pragma unroll
        for (int k = 0; k < kRB; k++) {
            *xm = nan_max(*xm, fabs(xw[k + 2]));
            *fm = nan_max(*fm, fabs(fv[k]));
        }
    }
    CDbl dg = (CDbl)diag;
#pragma unroll
    for (int k = 0; k < kRB; k++) {
        if (k % 4 == 0) {
            __builtin_amdgcn_sched_barrier(0);
            dg = fresh(dg);
        }
        const int64_t i = i0 + k;
        const double cf[5] = {dg[i], dg[n + i], dg[2 * n + i], dg[3 * n + i], dg[4 * n + i]};
        const double xv[5] = {xw[k], xw[k + 1], xw[k + 2], xw[k + 3], xw[k + 4]};
        fv[k] = dot2_row(fv[k], cf, xv);
    }
}

template <typename TI>
__global__ __launch_bounds__(64) void k_residual(const double *__restrict__ diag, int64_t n,
                                                 const TI *__restrict__ f, int64_t ldf,
                                                 const double *__restrict__ x, int64_t ldx,
                                                 double *__restrict__ r, int64_t ldr,
                                                 int64_t batch)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (j >= batch) return;
    const int64_t i0 = (int64_t)blockIdx.y * kRB;
    double rv[kRB];
    if (i0 >= 2 && i0 + kRB + 2 <= n) {
        residual_interior<TI>(diag, n, f, ldf, x, ldx, j, i0, rv);
        double *rc = r + i0 * ldr + j;
#pragma unroll
        for (int k = 0; k < kRB; k++) __builtin_nontemporal_store(rv[k], rc + k * ldr);
        return;
    }
    double xw[kRB + 4];
    residual_block<TI, true>(diag, n, f, ldf, x, ldx, j, i0, rv, rv, xw);  // r over f
#pragma unroll
    for (int k = 0; k < kRB; k++)
        if (i0 + k < n) r[(i0 + k) * ldr + j] = rv[k];
}

__global__ void k_axpy(double *__restrict__ x, int64_t ldx, const double *__restrict__ d,
                       int64_t ldd, int64_t n, int64_t batch)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) x[i * ldx + j] += d[i * ldd + j];
}

__global__ void k_fill_u64(unsigned long long *__restrict__ p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

// Non-negative doubles order like their bit patterns, so the maxima are
// taken with integer atomics on the bits; a (positive) NaN's bits exceed
// every number's, so a NaN in any block survives the atomics.
template <typename TI>
__global__ __launch_bounds__(64) void k_eta_partial(const double *__restrict__ diag, int64_t n,
                                                    const TI *__restrict__ f, int64_t ldf,
                                                    const double *__restrict__ x, int64_t ldx,
                                                    int64_t batch, unsigned long long *acc)
{
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (j >= batch) return;
    // row blocks blockIdx.y, blockIdx.y + gridDim.y, ...: maxima in
    // registers, one set of atomics per lane
    double rm = 0.0, xm = 0.0, fm = 0.0;
    const int64_t nblk = (n + kRB - 1) / kRB;
    for (int64_t b = blockIdx.y; b < nblk; b += gridDim.y) {
        const int64_t i0 = b * kRB;
        double rv[kRB];
        if (i0 >= 2 && i0 + kRB + 2 <= n) {
            residual_interior<TI, true>(diag, n, f, ldf, x, ldx, j, i0, rv, &xm, &fm);
        } else {
            double fv[kRB], xw[kRB + 4];
            residual_block<TI, false>(diag, n, f, ldf, x, ldx, j, i0, rv, fv, xw);
#pragma unroll
            for (int k = 0; k < kRB; k++) {
                xm = nan_max(xm, fabs(xw[k + 2]));
                fm = nan_max(fm, fabs(fv[k]));
            }
        }
#pragma unroll
        for (int k = 0; k < kRB; k++) rm = nan_max(rm, fabs(rv[k]));
    }
    atomicMax(acc + 3 * j + 0, (unsigned long long)__double_as_longlong(rm));
    atomicMax(acc + 3 * j + 1, (unsigned long long)__double_as_longlong(xm));
    atomicMax(acc + 3 * j + 2, (unsigned long long)__double_as_longlong(fm));
}

// eta from the maxima; eta may be NULL.  tol > 0: a system with eta > tol,
// or a non-finite eta, raises bit 2 of *err (the refinement missed its
// tolerance).
__global__ void k_eta_final(const unsigned long long *__restrict__ acc,
                            const double *__restrict__ anorm, int64_t batch,
                            double *__restrict__ eta, double tol, unsigned int *err)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;
    const double rm = __longlong_as_double((long long)acc[3 * j]);
    const double xm = __longlong_as_double((long long)acc[3 * j + 1]);
    const double fm = __longlong_as_double((long long)acc[3 * j + 2]);
    const double den = anorm[0] * xm + fm;
    // den == 0 only for x = 0 and f = 0 (then r = 0); NaN reaches eta
    const double e = (den > 0.0 || den != den) ? rm / den : rm;
    if (eta) eta[j] = e;
    if (tol > 0.0 && !(e <= tol)) atomicOr(err, 2u);
}

// ||A||_inf = max_i sum_k |A_ik| over the (zero-padded) diagonals.
__global__ __launch_bounds__(256) void k_anorm(const double *__restrict__ diag, int64_t n,
                                               double *__restrict__ out)
{
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double sum = fabs(diag[i]) + fabs(diag[n + i]) + fabs(diag[2 * n + i]) +
                           fabs(diag[3 * n + i]) + fabs(diag[4 * n + i]);
        m = fmax(m, sum);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

hipError_t launch_residual(const double *d_diag, int64_t n, const void *f, bool f32, int64_t ldf,
                           const double *x, int64_t ldx, double *r, int64_t ldr, int64_t batch,
                           hipStream_t s)
{
    const dim3 grid((unsigned)((batch + 63) / 64), (unsigned)((n + kRB - 1) / kRB));
    if (f32)
        hipLaunchKernelGGL(k_residual<float>, grid, dim3(64), 0, s, d_diag, n, (const float *)f,
                           ldf, x, ldx, r, ldr, batch);
    else
        hipLaunchKernelGGL(k_residual<double>, grid, dim3(64), 0, s, d_diag, n, (const double *)f,
                           ldf, x, ldx, r, ldr, batch);
    return hipGetLastError();
}

hipError_t launch_axpy(double *x, int64_t ldx, const double *d, int64_t ldd, int64_t n,
                       int64_t batch, hipStream_t s)
{
    const dim3 grid((unsigned)((batch + 255) / 256), (unsigned)(n < 4096 ? n : 4096));
    hipLaunchKernelGGL(k_axpy, grid, dim3(256), 0, s, x, ldx, d, ldd, n, batch);
    return hipGetLastError();
}

hipError_t launch_eta(const double *d_diag, const double *d_anorm, int64_t n, const void *f,
                      bool f32, int64_t ldf, const double *x, int64_t ldx, int64_t batch,
                      unsigned long long *acc, double *eta, double tol, unsigned int *err,
                      hipStream_t s)
{
    const int64_t cnt = 3 * batch;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, acc, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nblk = (n + kRB - 1) / kRB;
    const dim3 grid((unsigned)((batch + 63) / 64), (unsigned)(nblk < 32 ? nblk : 32));
    if (f32)
        hipLaunchKernelGGL(k_eta_partial<float>, grid, dim3(64), 0, s, d_diag, n, (const float *)f,
                           ldf, x, ldx, batch, acc);
    else
        hipLaunchKernelGGL(k_eta_partial<double>, grid, dim3(64), 0, s, d_diag, n,
                           (const double *)f, ldf, x, ldx, batch, acc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_eta_final, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, acc,
                       d_anorm, batch, eta, tol, err);
    return hipGetLastError();
}

hipError_t launch_anorm(const double *d_diag, int64_t n, double *d_anorm, hipStream_t s)
{
    hipLaunchKernelGGL(k_anorm, dim3(1), dim3(256), 0, s, d_diag, n, d_anorm);
    return hipGetLastError();
}

}  // namespace pent
