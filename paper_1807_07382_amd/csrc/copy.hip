// copy.hip -- the attainable-bandwidth reference for the batch-fastest
// single pass: a plain copy of an (n x batch) block that moves memory
// exactly as k_onepass does (a wave loads 64 systems x 64 rows, one 512-byte
// row segment per load, four waves down the rows per workgroup, workgroups
// tile-major), with no arithmetic and no exchange.  A solve cannot beat it;
// its time is the copy ceiling the single pass's roofline fraction is read
// against.  Other workgroup shapes (tiles side by side, fewer waves down)
// are there to measure what the block shape alone does to the bandwidth.
#include "internal.h"

namespace pent {
namespace {

constexpr int kCK = 64;

// TW tiles side by side x WR waves down the rows per workgroup: wave w
// takes tile q TW + w / WR and rows (g WR + w % WR) kCK .. + kCK - 1 of
// workgroup (q, g), workgroups tile-major.  (1, 4) is the single pass's
// pattern; the others show how the block shape alone moves the bandwidth.
template <int TW, int WR>
__global__ __launch_bounds__(64 * TW * WR) void k_block_copy(const double *src, double *dst, int64_t n,
                                                             int64_t batch, int64_t lds, int64_t ldd,
                                                             int ngroups)
{
    const int w = threadIdx.x / 64, lane = threadIdx.x & 63;
    const int64_t q = blockIdx.x / ngroups, g = blockIdx.x % ngroups;
    const int64_t j = (q * TW + w / WR) * 64 + lane;
    const int64_t r0 = (g * WR + w % WR) * kCK;
    if (j >= batch || r0 >= n) return;
    const int L = (int)(n - r0 < kCK ? n - r0 : kCK);
    const double *s = src + r0 * lds + j;
    double *d = dst + r0 * ldd + j;
    double v[kCK];
    if (L == kCK) {
#pragma unroll
        for (int k = 0; k < kCK; k++) v[k] = __builtin_nontemporal_load(s + k * lds);
#pragma unroll
        for (int k = 0; k < kCK; k++) __builtin_nontemporal_store(v[k], d + k * ldd);
    } else {
#pragma unroll
        for (int k = 0; k < kCK; k++) v[k] = k < L ? s[k * lds] : 0.0;
#pragma unroll
        for (int k = 0; k < kCK; k++)
            if (k < L) d[k * ldd] = v[k];
    }
}

template <int TW, int WR>
hipError_t block_copy(const double *src, double *dst, int64_t n, int64_t batch, int64_t lds,
                      int64_t ldd, hipStream_t s)
{
    const int64_t ngroups = (n + kCK * WR - 1) / (kCK * WR);
    const int64_t quads = ((batch + 63) / 64 + TW - 1) / TW;
    const int64_t blocks = quads * ngroups;
    if (blocks > (int64_t)UINT32_MAX / 2 || ngroups > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_block_copy<TW, WR>), dim3((unsigned)blocks), dim3(64 * TW * WR), 0, s, src,
                       dst, n, batch, lds, ldd, (int)ngroups);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_block_copy(const double *src, double *dst, int64_t n, int64_t batch, int64_t lds,
                             int64_t ldd, hipStream_t s, int tiles_across, int waves_down)
{
    if (tiles_across == 1 && waves_down == 4) return block_copy<1, 4>(src, dst, n, batch, lds, ldd, s);
    if (tiles_across == 2 && waves_down == 2) return block_copy<2, 2>(src, dst, n, batch, lds, ldd, s);
    if (tiles_across == 1 && waves_down == 2) return block_copy<1, 2>(src, dst, n, batch, lds, ldd, s);
    if (tiles_across == 2 && waves_down == 1) return block_copy<2, 1>(src, dst, n, batch, lds, ldd, s);
    if (tiles_across == 4 && waves_down == 1) return block_copy<4, 1>(src, dst, n, batch, lds, ldd, s);
    return hipErrorInvalidValue;
}

}  // namespace pent
