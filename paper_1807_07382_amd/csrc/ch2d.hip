// ch2d.hip -- explicit part of the split-implicit 2-D Cahn-Hilliard step.
//
// Semi-implicit Cahn-Hilliard (Sec. 2.1): the nonlinear term D*Lap(C^3 - C)
// is taken explicitly, the fourth-order term implicitly.  On a 2-D grid the
// implicit part is split into an x sweep and a y sweep of (I + sigma*D4)
// solves; this kernel forms the right-hand side of the x sweep:
//     R = C + dt_k * Lap_h(C^3 - C),
// Lap_h the 5-point Laplacian with zero values outside the grid (matching the
// truncated D4 rows), one dt per instance.  Layout [y][inst][x], contiguous:
// element (y, k, x) at y*ninst*nx + k*nx + x.
#include "internal.h"

namespace pent {
namespace {

__device__ __forceinline__ double wterm(double c) { return c * c * c - c; }

__global__ __launch_bounds__(256) void k_ch2d_rhs(const double *__restrict__ C,
                                                  double *__restrict__ R, int64_t ny,
                                                  int64_t ninst, int64_t nx,
                                                  const double *__restrict__ dt, double inv_h2)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = blockIdx.y;
    const int64_t y = blockIdx.z;
    if (x >= nx) return;
    const int64_t sy = ninst * nx;
    const int64_t i = y * sy + k * nx + x;
    const double c = C[i];
    const double w = wterm(c);
    const double we = (x + 1 < nx) ? wterm(C[i + 1]) : 0.0;
    const double ww = (x >= 1) ? wterm(C[i - 1]) : 0.0;
    const double wn = (y + 1 < ny) ? wterm(C[i + sy]) : 0.0;
    const double ws = (y >= 1) ? wterm(C[i - sy]) : 0.0;
    const double lap = (we + ww + wn + ws - 4.0 * w) * inv_h2;
    R[i] = c + dt[k] * lap;
}

}  // namespace

hipError_t launch_ch2d_rhs(const double *C, double *R, int64_t ny, int64_t ninst, int64_t nx,
                           const double *dt, double h, hipStream_t s)
{
    const dim3 grid((unsigned)((nx + 255) / 256), (unsigned)ninst, (unsigned)ny);
    hipLaunchKernelGGL(k_ch2d_rhs, grid, dim3(256), 0, s, C, R, ny, ninst, nx, dt, 1.0 / (h * h));
    return hipGetLastError();
}

}  // namespace pent
