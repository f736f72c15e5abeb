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

// ---- single pass: the bordered solve (and the Crank-Nicolson step) in one
// kernel.  Blocks (64-system tile, segment of the E rows) hold their rows in
// registers from load to store; the E-solve runs by look-back (lookback.h);
// then the blocks holding rows m-2 and m-1 post y there, the tile's first
// block (which holds y_0, y_1 after the backward chain) forms
// x_tail = Minv (f_tail - h^T y) and posts it, and every block applies
// x^ = y - Z x_tail to its rows before the one store.
//
// With CN the block loads C rows r0-2 .. r0+K+1 (periodic) instead of f and
// forms f = 2C - AC in registers (the explicit half of the step); C and X
// must then be different buffers.  The first block forms f_tail the same way.
//
// Tile words (per tile): [0] x_tail posted, [1] number of posted end rows (2).
// Tile exchange (per tile, 4 x 64 doubles): x_tail (2), y_{m-2}, y_{m-1}.
using namespace lb;

// f_i = 2 C_i - (A C)_i for row i, C rows i-2 .. i+2 in c0..c4.
__device__ __forceinline__ double cn_row(const double *__restrict__ cd, int64_t n, int64_t i,
                                         double c0, double c1, double c2, double c3, double c4)
{
    double acc = 2.0 * c2;
    acc = fma(-cd[i], c0, acc);
    acc = fma(-cd[n + i], c1, acc);
    acc = fma(-cd[2 * n + i], c2, acc);
    acc = fma(-cd[3 * n + i], c3, acc);
    acc = fma(-cd[4 * n + i], c4, acc);
    return acc;
}

__device__ __forceinline__ int64_t wrap(int64_t r, int64_t n)
{
    r %= n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ unsigned int wait_nonzero(unsigned int *p, unsigned int want,
                                                     unsigned int *err)
{
    for (int i = 0; i < kSpin; i++) {
        const unsigned int v = poll(p);
        if (v >= want) return v;
        __builtin_amdgcn_s_sleep(1);
    }
    atomicOr(err, 1u);
    return want;
}

template <int K, int W, bool CN>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(K == 64 ? 2 : 3))) void k_cyc_onepass(
    const FwdRec *fwd_, const BwdRec *bwd_, const SegRec *seg_, const double *__restrict__ cd_,
    const double *__restrict__ Z_, const CycAux *__restrict__ aux, int64_t n, int ngroups,
    const double *Fin, int64_t ldf, double *X, int64_t ldx, int64_t batch, unsigned int *ctr,
    unsigned int *fst, unsigned int *bst, unsigned int *tst, double *ex, double *tex,
    unsigned int *err)
{
    typedef __attribute__((address_space(4))) const double *CDbl;
    __shared__ double sh[W + 1][2][64];
    __shared__ unsigned int s_unit;
    const CFwd fwd = (CFwd)fwd_;
    const CBwd bwd = (CBwd)bwd_;
    const CSeg seg = (CSeg)seg_;
    const CDbl Z = (CDbl)Z_;
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
    const bool first = g == 0 && w == 0;                  // holds rows 0, 1
    const double *col = Fin + jj;
    double v[K];
    double ft0 = 0.0, ft1 = 0.0;  // f_m, f_{m+1} (first block only)
    if (CN) {
        double wv[K + 4];
#pragma unroll
        for (int k = 0; k < K + 4; k++)
            wv[k] = (act && k < L + 4 && L > 0) ? col[wrap(r0 - 2 + k, n) * ldf] : 0.0;
        if (first) {
            const double cm2 = act ? col[(m - 2) * ldf] : 0.0;
            const double cm1 = act ? col[(m - 1) * ldf] : 0.0;
            // rows m, m+1 = wv[0], wv[1]; rows 0, 1 = wv[2], wv[3]
            ft0 = cn_row(cd_, n, m, cm2, cm1, wv[0], wv[1], wv[2]);
            ft1 = cn_row(cd_, n, m + 1, cm1, wv[0], wv[1], wv[2], wv[3]);
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            const double f = cn_row(cd_, n, k < L ? r0 + k : 0, wv[k], wv[k + 1], wv[k + 2], wv[k + 3],
                                    wv[k + 4]);
            wv[k] = k < L ? f : 0.0;  // wv[k] is not needed by later rows
        }
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = wv[k];
    } else {
        const double *base = col + (L > 0 ? r0 * ldf : 0);
        if (L == K) {
#pragma unroll
            for (int k = 0; k < K; k++) v[k] = act ? __builtin_nontemporal_load(base + k * ldf) : 0.0;
        } else {
#pragma unroll
            for (int k = 0; k < K; k++) v[k] = (act && k < L) ? base[k * ldf] : 0.0;
        }
        if (first) {
            ft0 = act ? col[m * ldf] : 0.0;
            ft1 = act ? col[(m + 1) * ldf] : 0.0;
        }
    }

    group_phases<K, W>(v, fwd, bwd, seg, r0, w, g, ngroups, u - (unsigned int)g, fst, bst, ex, err,
                       sh);

    // post y_{m-2}, y_{m-1} if this block holds them
    double *tx = tex + (int64_t)t * 256 + lane;
    const int64_t k2 = m - 2 - r0, k1 = m - 1 - r0;
    const bool has2 = k2 >= 0 && k2 < L, has1 = k1 >= 0 && k1 < L;
    if (has2 || has1) {
        double y2 = 0.0, y1 = 0.0;
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (k == k2) y2 = v[k];
            if (k == k1) y1 = v[k];
        }
        if (has2) xstore(&tx[128], y2);
        if (has1) xstore(&tx[192], y1);
        store_fence();
        atomicAdd(&tst[2 * t + 1], threadIdx.x % 64 == 0 ? (unsigned int)(has2 + has1) : 0u);
    }

    double xt0, xt1;
    if (first) {
        wait_nonzero(&tst[2 * t + 1], 2u, err);
        const double ym2 = xload(&tx[128]), ym1 = xload(&tx[192]);
        double r0v = ft0, r1v = ft1;
        const int nh = aux->nh;
        for (int q = 0; q < nh; q++) {
            const int64_t c = aux->hcol[q];
            const double y = c == 0 ? v[0] : c == 1 ? v[1] : c == m - 2 ? ym2 : ym1;
            if (aux->hq[q] == 0) r0v = fma(-aux->hv[q], y, r0v);
            else r1v = fma(-aux->hv[q], y, r1v);
        }
        xt0 = fma(aux->minv[1], r1v, aux->minv[0] * r0v);
        xt1 = fma(aux->minv[3], r1v, aux->minv[2] * r0v);
        xstore(&tx[0], xt0);
        xstore(&tx[64], xt1);
        publish(&tst[2 * t], 1u);
        if (act) {
            X[jj + m * ldx] = xt0;
            X[jj + (m + 1) * ldx] = xt1;
        }
    } else {
        wait_nonzero(&tst[2 * t], 1u, err);
        xt0 = xload(&tx[0]);
        xt1 = xload(&tx[64]);
    }
    if (!act || L == 0) return;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int64_t i = r0 + k;
        v[k] = fma(-Z[2 * i + 1], xt1, fma(-Z[2 * i], xt0, v[k]));
    }
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

static int cyc_waves(int seg_rows) { return onepass_waves(seg_rows); }

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

static size_t cyc_words(int64_t n, int seg_rows, int64_t batch)
{
    const int64_t units = cyc_onepass_units(n, seg_rows, batch);
    const int64_t tiles = (batch + 63) / 64;
    return (size_t)(kTicketWords + 2 * units + 2 * tiles);
}

size_t cyc_onepass_scratch_bytes(int64_t n, int seg_rows, int64_t batch)
{
    const int64_t units = cyc_onepass_units(n, seg_rows, batch);
    const int64_t tiles = (batch + 63) / 64;
    const size_t wbytes = (cyc_words(n, seg_rows, batch) * sizeof(unsigned int) + 255) / 256 * 256;
    return wbytes + (size_t)(units * 8 * 64 + tiles * 4 * 64) * sizeof(double);
}

template <int K, int W>
static const void *cyc_fn(bool cn)
{
    return cn ? (const void *)k_cyc_onepass<K, W, true> : (const void *)k_cyc_onepass<K, W, false>;
}

static const void *cyc_fn_kw(int K, int W, bool cn)
{
    if (K == 64) return W == 2 ? cyc_fn<64, 2>(cn) : W == 4 ? cyc_fn<64, 4>(cn) : cyc_fn<64, 8>(cn);
    return W == 2 ? cyc_fn<32, 2>(cn) : W == 4 ? cyc_fn<32, 4>(cn) : cyc_fn<32, 8>(cn);
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
                              const double *cd, const double *Z, const CycAux *aux, int64_t n,
                              int seg_rows, bool cn, const double *Fin, int64_t ldf, double *X,
                              int64_t ldx, int64_t batch, void *scratch, unsigned int *err,
                              hipStream_t s)
{
    if (seg_rows != 32 && seg_rows != 64) return hipErrorInvalidValue;
    const int W = cyc_waves(seg_rows);
    const int64_t ngroups = cyc_groups(n, seg_rows);
    const int64_t units = cyc_onepass_units(n, seg_rows, batch);
    if (units > (int64_t)UINT32_MAX / 2 || kSegPad % W != 0) return hipErrorInvalidValue;
    const int64_t words = (int64_t)cyc_words(n, seg_rows, batch);
    unsigned int *w = (unsigned int *)scratch;
    unsigned int *ctr = w, *fst = w + kTicketWords, *bst = w + kTicketWords + units,
                 *tst = w + kTicketWords + 2 * units;
    const size_t wbytes = ((size_t)words * sizeof(unsigned int) + 255) / 256 * 256;
    double *ex = (double *)((char *)scratch + wbytes);
    double *tex = ex + units * 8 * 64;
    hipLaunchKernelGGL(k_cyc_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, w, words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int ng = (int)ngroups;
    void *args[] = {(void *)&fwd, (void *)&bwd, (void *)&seg, (void *)&cd, (void *)&Z, (void *)&aux,
                    (void *)&n, (void *)&ng, (void *)&Fin, (void *)&ldf, (void *)&X, (void *)&ldx,
                    (void *)&batch, (void *)&ctr, (void *)&fst, (void *)&bst, (void *)&tst,
                    (void *)&ex, (void *)&tex, (void *)&err};
    return hipLaunchKernel(cyc_fn_kw(seg_rows, W, cn), dim3((unsigned)units), dim3(64 * W), args, 0,
                           s);
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
