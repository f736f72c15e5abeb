// ch2d.hip -- explicit part of the split-implicit 2-D Cahn-Hilliard step.
//
// Semi-implicit Cahn-Hilliard (Sec. 2.1): the nonlinear term D*Lap(C^3 - C)
// is taken explicitly, the fourth-order term implicitly.  On a 2-D grid the
// implicit part is split into an x sweep and a y sweep of (I + sigma*D4)
// solves; this kernel forms the right-hand side of the x sweep (the step
// itself forms it inside the x-sweep kernel; this pass serves pent_ch2d_rhs
// and the step where that kernel cannot run):
//     R = C + dt_k * Lap_h(C^3 - C),
// Lap_h the 5-point Laplacian with zero values outside the grid (matching the
// truncated D4 rows), one dt per instance.  Layout [y][inst][x], contiguous:
// element (y, k, x) at y*ninst*nx + k*nx + x.
#include "internal.h"

namespace pent {
namespace {

// One thread per (x, instance) walks kRows consecutive y rows, keeping the
// y-neighbours' C^3 - C in registers, so each element of C comes from memory
// once (the x-neighbours are the adjacent lanes' elements, cache hits).
constexpr int kRows = 16;

__global__ __launch_bounds__(256) void k_ch2d_rhs(const double *__restrict__ C,
                                                  double *__restrict__ R, int64_t ny,
                                                  int64_t ninst, int64_t nx,
                                                  const double *__restrict__ dt, double inv_h2)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = blockIdx.y;
    const int64_t y0 = (int64_t)blockIdx.z * kRows;
    if (x >= nx) return;
    const int64_t sy = ninst * nx;
    const double dtk = dt[k];
    int64_t i = y0 * sy + k * nx + x;
    if (y0 + kRows < ny && y0 >= 1) {
        // interior run: every load of the run issued up front (one round
        // trip instead of one per row)
        // (x-neighbours load unconditionally, from the column itself at the
        // grid's edge, and are masked by a multiply: a load under a per-lane
        // test would be waited for inside its branch)
        double cc[kRows + 2], ce[kRows], cw[kRows];
        const double *col = C + i - sy;
        const int de = x + 1 < nx ? 1 : 0, dw = x >= 1 ? 1 : 0;
#pragma unroll
        for (int r = 0; r < kRows + 2; r++) cc[r] = col[r * sy];
#pragma unroll
        for (int r = 0; r < kRows; r++) {
            ce[r] = col[(r + 1) * sy + de];
            cw[r] = col[(r + 1) * sy - dw];
        }
#pragma unroll
        for (int r = 0; r < kRows; r++) {
            const double we = de ? ch_wterm(ce[r]) : 0.0;
            const double ww = dw ? ch_wterm(cw[r]) : 0.0;
            R[i + r * sy] = ch_point(cc[r + 1], ch_wterm(cc[r + 1]), we, ww, ch_wterm(cc[r + 2]),
                                     ch_wterm(cc[r]), dtk, inv_h2);
        }
        return;
    }
    double ws = y0 >= 1 ? ch_wterm(C[i - sy]) : 0.0;
    double c = C[i];
    double w = ch_wterm(c);
    const int64_t y1 = y0 + kRows < ny ? y0 + kRows : ny;
    for (int64_t y = y0; y < y1; y++) {
        const double cn = y + 1 < ny ? C[i + sy] : 0.0;
        const double wn = y + 1 < ny ? ch_wterm(cn) : 0.0;
        const double we = (x + 1 < nx) ? ch_wterm(C[i + 1]) : 0.0;
        const double ww = (x >= 1) ? ch_wterm(C[i - 1]) : 0.0;
        R[i] = ch_point(c, w, we, ww, wn, ws, dtk, inv_h2);
        ws = w;
        w = wn;
        c = cn;
        i += sy;
    }
}

}  // namespace

hipError_t launch_ch2d_rhs(const double *C, double *R, int64_t ny, int64_t ninst, int64_t nx,
                           const double *dt, double h, hipStream_t s)
{
    const dim3 grid((unsigned)((nx + 255) / 256), (unsigned)ninst, (unsigned)((ny + kRows - 1) / kRows));
    hipLaunchKernelGGL(k_ch2d_rhs, grid, dim3(256), 0, s, C, R, ny, ninst, nx, dt, 1.0 / (h * h));
    return hipGetLastError();
}

}  // namespace pent
