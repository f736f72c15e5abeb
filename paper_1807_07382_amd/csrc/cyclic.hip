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
#include "internal.h"

namespace pent {
namespace {

__device__ __forceinline__ double cyc_coef(const double *cd, int64_t n, int64_t i, int o)
{
    return cd[(o + 2) * n + i];  // o in -2..2 -> a, b, c, d, e
}

__global__ void k_cyc_assemble_d4(double *__restrict__ cd, int64_t n, double sigma)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cd[i] = sigma;
    cd[n + i] = -4.0 * sigma;
    cd[2 * n + i] = 1.0 + 6.0 * sigma;
    cd[3 * n + i] = -4.0 * sigma;
    cd[4 * n + i] = sigma;
}

// E's diagonals (m = n-2 rows), zero outside the (m x m) block.
__global__ void k_cyc_build_E(const double *__restrict__ cd, int64_t n, double *__restrict__ ed)
{
    const int64_t m = n - 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    ed[i] = (i >= 2) ? cd[i] : 0.0;
    ed[m + i] = (i >= 1) ? cd[n + i] : 0.0;
    ed[2 * m + i] = cd[2 * n + i];
    ed[3 * m + i] = (i + 1 < m) ? cd[3 * n + i] : 0.0;
    ed[4 * m + i] = (i + 2 < m) ? cd[4 * n + i] : 0.0;
}

// K (m x 2, batch-fastest, ld 2): column s = entries of A in column m + s.
__global__ void k_cyc_build_k(const double *__restrict__ cd, int64_t n, double *__restrict__ K)
{
    const int64_t m = n - 2;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double k0 = 0.0, k1 = 0.0;
    for (int o = -2; o <= 2; o++) {
        const int64_t col = ((i + o) % n + n) % n;
        if (col == m) k0 += cyc_coef(cd, n, i, o);
        if (col == m + 1) k1 += cyc_coef(cd, n, i, o);
    }
    K[2 * i] = k0;
    K[2 * i + 1] = k1;
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
            const int64_t col = ((i + o) % n + n) % n;
            acc -= cyc_coef(cd, n, i, o) * C[col * ldc + j];
        }
        R[i * ldr + j] = acc;
    }
}

}  // namespace

hipError_t launch_cyc_assemble_d4(double *cd, int64_t n, double sigma, hipStream_t s)
{
    hipLaunchKernelGGL(k_cyc_assemble_d4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cd, n,
                       sigma);
    return hipGetLastError();
}

hipError_t launch_cyc_build(const double *cd, int64_t n, double *ed, double *K, hipStream_t s)
{
    const int64_t m = n - 2;
    hipLaunchKernelGGL(k_cyc_build_E, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, cd, n, ed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cyc_build_k, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, cd, n, K);
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
