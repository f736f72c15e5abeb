// copy.hip -- the attainable-bandwidth reference for the batch-fastest
// single pass: a plain copy of an (n x batch) block that moves memory
// exactly as k_onepass does (a wave loads 64 systems x 64 rows, one 512-byte
// row segment per load, four waves down the rows per workgroup, workgroups
// tile-major), with no arithmetic and no exchange.  A solve cannot beat it;
// its time is the copy ceiling the single pass's roofline fraction is read
// against.
#include "internal.h"

namespace pent {
namespace {

constexpr int kCK = 64, kCW = 4;

__global__ __launch_bounds__(64 * kCW) void k_block_copy(const double *src, double *dst, int64_t n,
                                                         int64_t batch, int64_t lds, int64_t ldd,
                                                         int ngroups)
{
    const int w = threadIdx.x / 64, lane = threadIdx.x & 63;
    const int64_t t = blockIdx.x / ngroups, g = blockIdx.x % ngroups;
    const int64_t j = t * 64 + lane;
    const int64_t r0 = (g * kCW + w) * kCK;
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

}  // namespace

hipError_t launch_block_copy(const double *src, double *dst, int64_t n, int64_t batch, int64_t lds,
                             int64_t ldd, hipStream_t s)
{
    const int64_t ngroups = (n + kCK * kCW - 1) / (kCK * kCW);
    const int64_t blocks = (batch + 63) / 64 * ngroups;
    if (blocks > (int64_t)UINT32_MAX / 2) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_copy, dim3((unsigned)blocks), dim3(64 * kCW), 0, s, src, dst, n, batch,
                       lds, ldd, (int)ngroups);
    return hipGetLastError();
}

}  // namespace pent
