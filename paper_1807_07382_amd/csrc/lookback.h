// lookback.h -- device pieces of the single-pass sweeps (onepass.hip,
// cyclic.hip): ticketing, status words, the interface link, the sweeps of a
// block held in registers, and the phases of a workgroup of W such blocks in
// two forms: two-phase (group_phases, with its look-back and look-ahead
// group_carry) and single-wait (group_phases_1w, group_wait).
//
// By linearity (Sec. 2.4's recurrences are affine in the carried pair), a
// segment's outgoing forward state is
//     out_s = e_s + Tf_s y_s,        y_s = out_{s-1},  y_0 = 0,
// with e_s the outgoing state of a zero-start forward sweep, and its
// outgoing (upward) backward state is
//     up_s = a_s + Tb_s z_s,         z_s = up_{s+1},   z_{last} = 0,
// with a_s the top of a zero-start backward sweep over the TRUE forward
// values.  Tf and Tb depend on A only (SegRec).  The carries travel between
// the blocks of a tile through a small exchange area with decoupled
// look-back: a block publishes its aggregate (e_s, or a_s) when its
// neighbour's inclusive value is not there yet, looks back (forward) or
// ahead (backward) until it meets an inclusive value, replays the chain from
// there, and publishes its own inclusive value.
#pragma once

#include "internal.h"

namespace pent {
namespace lb {

typedef __attribute__((address_space(4))) const FwdRec *CFwd;
typedef __attribute__((address_space(4))) const BwdRec *CBwd;
typedef __attribute__((address_space(4))) const SegRec *CSeg;

constexpr int kSpin = 1 << 20;  // polls per wait before giving up

// Units are numbered through kTicketLines counters, one per 128-byte line,
// counter c serving the blocks with blockIdx % kTicketLines == c: ticket k
// of counter c is unit k * kTicketLines + c, so the grid (one block per
// unit) hands out every unit exactly once.  Blocks of one counter start in
// ticket order, and the counters advance together, so a unit only ever
// waits on units that hold a slot or on later units of its own tile; one
// counter for all blocks would serialise every block start on one address.
constexpr int kTicketLines = 64;
constexpr int kTicketStride = 32;  // words per counter line
constexpr int kTicketWords = kTicketLines * kTicketStride;

// Every lane joins the atomic (lanes other than 0 add zero) and lane 0's
// result is read back: no branch depends on the lane index alone.
__device__ __forceinline__ unsigned int take_unit(unsigned int *ctr)
{
    const unsigned int c = blockIdx.x % kTicketLines;
    const unsigned int r = atomicAdd(&ctr[c * kTicketStride], threadIdx.x == 0 ? 1u : 0u);
    return (unsigned int)__builtin_amdgcn_readlane((int)r, 0) * kTicketLines + c;
}

// Exchanged values and status words move with agent-scope relaxed atomics
// (loads and stores with the agent-coherence bit), never with acquire /
// release operations: on this GPU those write back or invalidate the whole
// L2 of the calling XCD, and with thousands of waves polling they flush
// everyone's cached records.  Ordering comes from waiting for the wave's
// own stores to complete before the status store (store_fence), and on the
// reading side from loading the values only after the status was seen.
__device__ __forceinline__ void xstore(double *p, double v)
{
    __hip_atomic_store((unsigned long long *)p, (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double xload(const double *p)
{
    return __longlong_as_double((long long)__hip_atomic_load(
        (unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Every earlier memory operation of the wave has completed (s_waitcnt
// vmcnt(0)); the compiler moves no memory operation across it.
__device__ __forceinline__ void store_fence()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ unsigned int poll(unsigned int *p)
{
    const unsigned int v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return (unsigned int)__builtin_amdgcn_readlane((int)v, 0);
}

// The wave's exchange stores (xstore) are complete before the status is.
__device__ __forceinline__ void publish(unsigned int *p, unsigned int v)
{
    store_fence();
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int K, typename TI>
__device__ __forceinline__ void load_rows(double (&v)[K], const TI *base, int64_t ld, int L)
{
    if (L == K) {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = (double)__builtin_nontemporal_load(base + k * ld);
    } else {
#pragma unroll
        for (int k = 0; k < K; k++) v[k] = (k < L) ? (double)base[k * ld] : 0.0;
    }
}

// The coefficient rows come in through scalar loads, kSchedRows rows at a
// time: each batch reads through a fresh copy of the pointer (fresh(),
// internal.h) behind a scheduling barrier, so the compiler can neither keep
// the zero-start sweep's coefficients (and their products with the block)
// alive until the true sweep nor hoist all of a sweep's loads to its start;
// both run out of scalar registers and spill into vector ones.
constexpr int kSchedRows = 8;

// Forward recurrence over the segment from (p2, p1); STORE writes g over v.
// LREC: the block's records were staged in LDS (lf[k], row r0 + k) instead.
template <int K, bool STORE, bool LREC = false>
__device__ __forceinline__ void forward(double (&v)[K], CFwd fwd, int64_t r0, double &p2, double &p1,
                                        const FwdRec *lf = nullptr)
{
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (!LREC && k % kSchedRows == 0) {
            __builtin_amdgcn_sched_barrier(0);
            fwd = fresh(fwd);
        }
        const double ra = LREC ? lf[k].ra : fwd[r0 + k].ra, ap = LREC ? lf[k].ap : fwd[r0 + k].ap,
                     bp = LREC ? lf[k].bp : fwd[r0 + k].bp;
        const double g = fma(-bp, p1, fma(-ap, p2, ra * v[k]));
        if (STORE) v[k] = g;
        p2 = p1;
        p1 = g;
    }
}

// Adds to v the forward sweep's response to the incoming state (p2, p1)
// with a zero right-hand side: g = g0 + h, h_k = -ap h_{k-2} - bp h_{k-1}
// (the sweep is affine in its incoming state).
template <int K, bool LREC = false>
__device__ __forceinline__ void respond(double (&v)[K], CFwd fwd, int64_t r0, double p2, double p1,
                                        const FwdRec *lf = nullptr)
{
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (!LREC && k % kSchedRows == 0) {
            __builtin_amdgcn_sched_barrier(0);
            fwd = fresh(fwd);
        }
        const double ap = LREC ? lf[k].ap : fwd[r0 + k].ap, bp = LREC ? lf[k].bp : fwd[r0 + k].bp;
        const double h = fma(-bp, p1, -ap * p2);
        v[k] += h;
        p2 = p1;
        p1 = h;
    }
}

// Back substitution over the segment from (q1, q2) = (x_{r0+K}, x_{r0+K+1});
// on exit (q1, q2) = (x_{r0}, x_{r0+1}).  STORE writes x over v.  CORR
// (periodic bordering) stores x_i - Z_i (c0, c1) instead, Z_i = rows 2i,
// 2i+1 of Z, while the recurrence carries x itself; its Z rows come in the
// same scalar batches as the records.
template <int K, bool STORE, bool LREC = false, bool CORR = false>
__device__ __forceinline__ void backward(double (&v)[K], CBwd bwd, int64_t r0, double &q1, double &q2,
                                         const BwdRec *lb = nullptr, CDbl Z = nullptr,
                                         double c0 = 0.0, double c1 = 0.0)
{
#pragma unroll
    for (int k = K - 1; k >= 0; k--) {
        if (!LREC && (k + 1) % kSchedRows == 0) {
            __builtin_amdgcn_sched_barrier(0);
            bwd = fresh(bwd);
            if (CORR) Z = fresh(Z);
        }
        const double gm = LREC ? lb[k].gm : bwd[r0 + k].gm, dl = LREC ? lb[k].dl : bwd[r0 + k].dl;
        const double x = fma(-gm, q1, fma(-dl, q2, v[k]));
        if (STORE) v[k] = CORR ? fma(-Z[2 * (r0 + k) + 1], c1, fma(-Z[2 * (r0 + k)], c0, x)) : x;
        q2 = q1;
        q1 = x;
    }
}

// No correction in group_phases (the plain single pass).
struct NoCorr {
    static constexpr bool on = false;
    CDbl Z = nullptr;
    __device__ void early(int) const {}
    __device__ void fetch(int) const {}
    __device__ void get(int, double &, double &) const {}
};

// One link of the interface chain, (y0, y1) <- w + T (y0, y1), T column-major.
// Publishers and look-back use this one function with explicit fused
// multiply-adds, so a carry has the same bits whichever path produced it.
__device__ __forceinline__ void link(double w0, double w1, double t0, double t1, double t2,
                                     double t3, double &y0, double &y1)
{
    const double n0 = fma(t2, y1, fma(t0, y0, w0));
    const double n1 = fma(t3, y1, fma(t1, y0, w1));
    y0 = n0;
    y1 = n1;
}

// Exchange area of one unit: 8 rows of 64 doubles (lane = system):
// 0,1 forward aggregate e; 2,3 forward inclusive out; 4,5 backward
// aggregate a; 6,7 backward inclusive up.
constexpr int kExRows = 8;

// One status word per lane: lane l reads word[base + l] when it is in
// [lo, hi], else reports 0 (not counted as missing).
__device__ __forceinline__ unsigned int lane_status(unsigned int *word, int64_t idx, bool in)
{
    const unsigned int v = in ? __hip_atomic_load(word + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return v;
}

// ---- grouped form: a workgroup of W waves takes W consecutive segments
// (one per wave) of one tile; the waves exchange their carries through LDS,
// and only the group's carries go through device memory.  The chain is
// canonical at two levels, so results do not depend on timing:
//   group level:   Y_{g+1} = E_g + TG_g Y_g,  E_g = the group's zero-start
//                  aggregate (its segments linked innermost first),
//                  TG_g = Tf of its segments multiplied in one fixed order;
//   inside a group: y of wave w = Y_g linked through e_0 .. e_{w-1};
// and the mirror image backward (TBG_g = Tb_{s0} ... Tb_{s0+W-1}).

// M <- T M for 2x2 column-major matrices, explicit fused multiply-adds.
__device__ __forceinline__ void mat_lmul(double t0, double t1, double t2, double t3, double &m0,
                                         double &m1, double &m2, double &m3)
{
    const double n0 = fma(t2, m1, t0 * m0), n1 = fma(t3, m1, t1 * m0);
    const double n2 = fma(t2, m3, t0 * m2), n3 = fma(t3, m3, t1 * m2);
    m0 = n0;
    m1 = n1;
    m2 = n2;
    m3 = n3;
}

// TG = Tf_{s0+W-1} ... Tf_{s0} (forward) or TBG = Tb_{s0} ... Tb_{s0+W-1},
// t(i, k) = entry k of the matrix of segment s0 + i.  Every caller forms a
// group's matrix through this one function, so it has the same bits
// wherever its factors were read from.
template <int W, bool FWD, typename Get>
__device__ __forceinline__ void group_product(Get t, double &m0, double &m1, double &m2, double &m3)
{
    m0 = 1.0;
    m1 = 0.0;
    m2 = 0.0;
    m3 = 1.0;
#pragma unroll
    for (int i = 0; i < W; i++) {
        const int q = FWD ? i : W - 1 - i;
        mat_lmul(t(q, 0), t(q, 1), t(q, 2), t(q, 3), m0, m1, m2, m3);
    }
}

template <int W, bool FWD>
__device__ __forceinline__ void group_matrix(CSeg seg, int64_t s0, double &m0, double &m1,
                                             double &m2, double &m3)
{
    group_product<W, FWD>([&](int i, int k) { return FWD ? seg[s0 + i].tf[k] : seg[s0 + i].tb[k]; },
                          m0, m1, m2, m3);
}

// Aggregates staged in LDS per round trip of the replay.
constexpr int kStage = 16;
constexpr int kCoherentLoad = 16;  // cache-policy bits of a direct load: sc1, as xload

// LDS of a group of W waves (declared by each kernel, as arrays: the direct
// loads need plain LDS addresses): sh [W + 1][2][64], the waves' carries;
// agg [kStage][128] and mat [kStage][W][4], the replay's staging area
// (aggregate pairs of the tile's 64 systems, and the W segment matrices of
// each of those groups).
#define PENT_GROUP_LDS(W)                          \
    __shared__ double sh[(W) + 1][2][64];          \
    __shared__ double agg[pent::lb::kStage][128];  \
    __shared__ double mat[pent::lb::kStage][(W)][4]

// The same for the single-wait form (group_phases_1w): sh [W + 1][4][64],
// per wave its forward and backward states (row W: the group's); mat
// [2 kStage][4], one group matrix per staged group; ucon, the group's W
// segment records and its group record (stage_consts).
#define PENT_GROUP1W_LDS(W)                                    \
    __shared__ double sh[(W) + 1][4][64];                      \
    __shared__ double agg[pent::lb::kStage][128];              \
    __shared__ double mat[2 * pent::lb::kStage][4];            \
    __shared__ double ucon[((W) * 16 + 16 + 127) / 128 * 128]

typedef __attribute__((address_space(4))) const GrpRec *CGrp;

// One group's aggregate pair for the tile's 64 systems (1 KB: row ra then
// row ra+1 of its exchange block) straight into LDS row dst, without
// passing through registers: lane l moves values 2l, 2l+1.  dst goes in as
// its LDS offset, the low half of its generic address (a cast to the LDS
// address space would add a null check the backend cannot encode here).
__device__ __forceinline__ void stage_load(const double *blk, double *dst)
{
    __builtin_amdgcn_global_load_lds(
        (const __attribute__((address_space(1))) void *)(blk + 2 * (threadIdx.x & 63)),
        (__attribute__((address_space(3))) void *)(uint32_t)(uintptr_t)dst, 16, 0, kCoherentLoad);
}

// Group-level look-back (FWD) or look-ahead: the incoming carry of group g
// of the tile whose first group unit is u0, given this group's aggregate
// (c0, c1), which is posted first.  A wait that runs out raises *err and
// returns a NaN carry.  Statuses: 1 aggregate posted, 2
// inclusive posted; the first group (forward) and the last group (backward)
// post only inclusive values.  Exchange rows: forward 0,1 aggregate, 2,3
// inclusive; backward 4,5 aggregate, 6,7 inclusive.
template <int W, bool FWD>
__device__ __forceinline__ void group_carry(CSeg seg, int g, int ngroups, unsigned int u0,
                                            unsigned int *st_word, double *ex, unsigned int *err,
                                            double c0, double c1, double &y0, double &y1,
                                            double (*agg)[128], double (*mat)[W][4])
{
    const int lane = threadIdx.x & 63;
    const int ra = FWD ? 0 : 4;  // aggregate rows
    double *me = ex + (int64_t)(u0 + g) * (kExRows * 64) + lane;
    // the aggregate goes out first: later groups can use it while this one
    // is still looking
    xstore(&me[ra * 64], c0);
    xstore(&me[(ra + 1) * 64], c1);
    publish(&st_word[u0 + g], 1u);
    int base = FWD ? g - 1 : g + 1, pstar = base;
    bool timed_out = false;
    for (int spin = 0;; spin++) {
        const int p = FWD ? base - lane : base + lane;
        const bool in = FWD ? p >= 0 : p < ngroups;
        const unsigned int st = lane_status(st_word, (int64_t)u0 + p, in);
        const unsigned long long incl = __ballot(st == 2);
        const unsigned long long none = __ballot(in && st == 0);
        if (incl != 0) {
            const int l = __builtin_ctzll(incl);
            if ((none & ((1ull << l) - 1)) == 0) {
                pstar = FWD ? base - l : base + l;
                break;
            }
        } else if (none == 0 && (FWD ? base >= 64 : base + 64 < ngroups)) {
            base = FWD ? base - 64 : base + 64;
            continue;
        }
        if (spin >= kSpin) {
            atomicOr(err, 1u);
            timed_out = true;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    // replay the groups between pstar and g, innermost first.  The replay
    // is latency-bound and registers hold the block, so each round trip
    // brings up to kStage groups' aggregates and segment matrices into LDS
    // at once; they are then linked in order.
    const int cnt = FWD ? g - 1 - pstar : pstar - g - 1;
    auto group_at = [&](int i) { return FWD ? pstar + 1 + i : pstar - 1 - i; };
    const double *nb = ex + (int64_t)(u0 + pstar) * (kExRows * 64) + lane;
    y0 = xload(&nb[(ra + 2) * 64]);
    y1 = xload(&nb[(ra + 3) * 64]);
    for (int c = 0; c < cnt; c += kStage) {
        const int m = cnt - c < kStage ? cnt - c : kStage;
#pragma unroll
        for (int i = 0; i < kStage; i++)
            if (i < m) stage_load(ex + (int64_t)(u0 + group_at(c + i)) * (kExRows * 64) + ra * 64, agg[i]);
        // segment matrices, half a matrix (16 bytes) per lane and load: slot
        // e = (i * W + q) * 2 + h lands at LDS byte 16 e of mat
#pragma unroll
        for (int k = 0; k < (kStage * W * 2 + 63) / 64; k++) {
            const int e = k * 64 + lane;
            const int i = e / (2 * W) < m ? e / (2 * W) : 0;  // slots past the chunk reload its first group
            const int64_t q = (int64_t)group_at(c + i) * W + (e / 2) % W;
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void *)(FWD ? &seg[q].tf[2 * (e % 2)] : &seg[q].tb[2 * (e % 2)]),
                (__attribute__((address_space(3))) void *)(uint32_t)(uintptr_t)&mat[(32 / W) * k][0][0], 16, 0, 0);
        }
        store_fence();  // the direct loads have landed in LDS
        // lane i < kStage forms group i's matrix (the same function as every
        // other path, so the same bits) and leaves it in mat[i][0]
        if (lane < kStage) {
            double m0, m1, m2, m3;
            group_product<W, FWD>([&](int q, int k) { return mat[lane][q][k]; }, m0, m1, m2, m3);
            mat[lane][0][0] = m0;
            mat[lane][0][1] = m1;
            mat[lane][0][2] = m2;
            mat[lane][0][3] = m3;
        }
        // the serial links, without branches (slots past the chunk are
        // computed and dropped), so the reads can run ahead of the chain
#pragma unroll
        for (int i = 0; i < kStage; i++) {
            double n0 = y0, n1 = y1;
            link(agg[i][lane], agg[i][64 + lane], mat[i][0][0], mat[i][0][1], mat[i][0][2], mat[i][0][3],
                 n0, n1);
            y0 = i < m ? n0 : y0;
            y1 = i < m ? n1 : y1;
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);  // LDS reads before the next chunk's loads
        __builtin_amdgcn_s_waitcnt(0xC07F);       // lgkmcnt(0)
    }
    // a wait that ran out replayed from a status it never saw: the carry is
    // NaN, so every value that depends on it (this tile's x, the carries it
    // publishes) comes out NaN instead of a plausible wrong number
    if (timed_out) {
        y0 = __builtin_nan("");
        y1 = __builtin_nan("");
    }
}

// The records of rows r0 .. r0+K-1 into LDS (lf: K FwdRec, lb: K BwdRec) by
// direct loads, to be issued before the block's own loads; rec_wait()
// before the first sweep then waits for them alone while the block is still
// arriving.  The sweeps then read their coefficients as LDS broadcasts
// instead of a scalar-load round trip per batch of rows.  K is 32 or 64.
template <int K>
__device__ __forceinline__ void stage_records(const FwdRec *fwd, const BwdRec *bwd, int64_t r0,
                                              FwdRec *lf, BwdRec *lb)
{
    const int lane = threadIdx.x & 63;
    const char *fs = (const char *)(fwd + r0) + 16 * lane;
    const uint32_t fl = (uint32_t)(uintptr_t)lf;
    // 1 KB per load; lanes past the block's records stay idle in the last
    // (partial) one, so nothing lands past lf
#pragma unroll
    for (int c = 0; c < (K * (int)sizeof(FwdRec) + 1023) / 1024; c++)
        if ((c + 1) * 1024 <= K * (int)sizeof(FwdRec) || 64 * c + lane < K * (int)sizeof(FwdRec) / 16)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(fs + 1024 * c),
                                             (__attribute__((address_space(3))) void *)(fl + 1024u * c), 16, 0, 0);
    const char *bs = (const char *)(bwd + r0) + 16 * lane;
    if (K * (int)sizeof(BwdRec) >= 1024 || lane < K * (int)sizeof(BwdRec) / 16)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)bs,
                                         (__attribute__((address_space(3))) void *)(uint32_t)(uintptr_t)lb,
                                         16, 0, 0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_sched_barrier(0);
}

// s_waitcnt immediate for vmcnt(vm) alone (vm <= 63; gfx9 encoding: low
// four bits at 3:0, high two at 15:14, expcnt and lgkmcnt at their maxima).
constexpr int vmcnt_imm(int vm) { return (vm & 15) | ((vm >> 4) << 14) | 0x0F70; }

// Waits for the staged records.  full (wave-uniform): a full block's K loads
// were issued after them, so at most K - 1 outstanding operations means
// they have landed while most of the block is still arriving; else wait for
// everything.
template <int K>
__device__ __forceinline__ void rec_wait(bool full)
{
    static_assert(K >= 1 && K <= 64, "vmcnt holds at most 63");
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (full) __builtin_amdgcn_s_waitcnt(vmcnt_imm(K - 1));
    else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Both sweeps of the block held by wave w of group g (rows r0 .. r0+K-1):
// on exit v holds x.
template <int K, int W, bool LREC = false, typename Corr = NoCorr>
__device__ __forceinline__ void group_phases(double (&v)[K], CFwd fwd, CBwd bwd, CSeg seg,
                                             int64_t r0, int w, int g, int ngroups,
                                             unsigned int u0, unsigned int *fst,
                                             unsigned int *bst, double *ex, unsigned int *err,
                                             double (*sh)[2][64], double (*agg)[128],
                                             double (*mat)[W][4], const FwdRec *lf = nullptr,
                                             const BwdRec *lb = nullptr, Corr corr = Corr())
{
    const int lane = threadIdx.x & 63;
    const int64_t s0 = (int64_t)g * W;
    // forward: zero-start aggregates of the waves, then the group's carry
    {
        double e0 = 0.0, e1 = 0.0;
        forward<K, false, LREC>(v, fwd, r0, e0, e1, lf);
        sh[w][0][lane] = e0;
        sh[w][1][lane] = e1;
    }
    __syncthreads();
    if (W == 1) corr.early(lane);
    if (w == 0) {
        double E0 = 0.0, E1 = 0.0;
#pragma unroll
        for (int i = 0; i < W; i++)
            link(sh[i][0][lane], sh[i][1][lane], seg[s0 + i].tf[0], seg[s0 + i].tf[1],
                 seg[s0 + i].tf[2], seg[s0 + i].tf[3], E0, E1);
        double Y0 = 0.0, Y1 = 0.0;
        if (g > 0) group_carry<W, true>(seg, g, ngroups, u0, fst, ex, err, E0, E1, Y0, Y1, agg, mat);
        if (g < ngroups - 1) {
            double m0, m1, m2, m3, o0 = Y0, o1 = Y1;
            group_matrix<W, true>(seg, s0, m0, m1, m2, m3);
            link(E0, E1, m0, m1, m2, m3, o0, o1);
            double *me = ex + (int64_t)(u0 + g) * (kExRows * 64) + lane;
            xstore(&me[2 * 64], o0);
            xstore(&me[3 * 64], o1);
            publish(&fst[u0 + g], 2u);
        }
        sh[W][0][lane] = Y0;
        sh[W][1][lane] = Y1;
    } else if (w == W - 1) {
        corr.early(lane);  // work that needs only the loaded blocks (an idle wave)
    }
    __syncthreads();
    {
        double y0 = sh[W][0][lane], y1 = sh[W][1][lane];
        for (int i = 0; i < w; i++)
            link(sh[i][0][lane], sh[i][1][lane], seg[s0 + i].tf[0], seg[s0 + i].tf[1],
                 seg[s0 + i].tf[2], seg[s0 + i].tf[3], y0, y1);
        forward<K, true, LREC>(v, fwd, r0, y0, y1, lf);
    }
    __syncthreads();  // sh is reused below
    // backward: zero-start aggregates over the true g, then the group's carry
    {
        double a0 = 0.0, a1 = 0.0;
        backward<K, false, LREC>(v, bwd, r0, a0, a1, lb);
        sh[w][0][lane] = a0;
        sh[w][1][lane] = a1;
    }
    __syncthreads();
    if (w == 0) {
        double A0 = 0.0, A1 = 0.0;
#pragma unroll
        for (int i = W - 1; i >= 0; i--)
            link(sh[i][0][lane], sh[i][1][lane], seg[s0 + i].tb[0], seg[s0 + i].tb[1],
                 seg[s0 + i].tb[2], seg[s0 + i].tb[3], A0, A1);
        double Z0 = 0.0, Z1 = 0.0;
        if (g < ngroups - 1) group_carry<W, false>(seg, g, ngroups, u0, bst, ex, err, A0, A1, Z0, Z1, agg, mat);
        if (g > 0) {
            double m0, m1, m2, m3, o0 = Z0, o1 = Z1;
            group_matrix<W, false>(seg, s0, m0, m1, m2, m3);
            link(A0, A1, m0, m1, m2, m3, o0, o1);
            double *me = ex + (int64_t)(u0 + g) * (kExRows * 64) + lane;
            xstore(&me[6 * 64], o0);
            xstore(&me[7 * 64], o1);
            publish(&bst[u0 + g], 2u);
        }
        sh[W][0][lane] = Z0;
        sh[W][1][lane] = Z1;
    }
    if (w == W - 1) corr.fetch(lane);  // the correction's coefficients into LDS (an idle wave)
    __syncthreads();
    {
        double z0 = sh[W][0][lane], z1 = sh[W][1][lane];
        for (int i = W - 1; i > w; i--)
            link(sh[i][0][lane], sh[i][1][lane], seg[s0 + i].tb[0], seg[s0 + i].tb[1],
                 seg[s0 + i].tb[2], seg[s0 + i].tb[3], z0, z1);
        double c0 = 0.0, c1 = 0.0;
        corr.get(lane, c0, c1);
        backward<K, true, LREC, Corr::on>(v, bwd, r0, z0, z1, lb, corr.Z, c0, c1);
    }
    // x is complete here: keep the compiler from sinking the sweep into the
    // block that stores x (past a caller's waits, with every coefficient
    // held live across them)
#pragma unroll
    for (int k = 0; k < K; k++) asm volatile("" : "+v"(v[k]));
}


// ---- single-wait form (group_phases_1w), used where tiles have few groups
// (the many-matrix kernel).  In the two-phase form above the backward
// look-ahead waits for the forward chain to resolve first; here both chains
// are resolved from quantities every group forms from its own block alone,
// so a group waits once, for its tile's other groups to have loaded their
// blocks, and never for another group's carries.  With segment i of a group entered by forward state y_i and left (upward) by
// backward state up_i = a0_i + Cg_i y_i + Tb_i z_i, where a0_i is the top of
// a zero-start back substitution over the zero-start forward values g0 (the
// true forward values are g0 + the response to y_i), the groups G of a tile
// satisfy
//     Y_{G+1} = E_G + TG_G Y_G,                   Y_0 = 0,
//     Zin_G   = A0_{G+1} + CG_{G+1} Y_{G+1} + TBG_{G+1} Zin_{G+1},
//                                                 Zin_last = 0,
// with E_G, A0_G the group's states for zero carries, Zin_G the backward
// state entering G from below and TG, TBG, CG constants of A (GrpRec).
// Writing Zin_G = P_G + Q_G Y_{G+1} (Q constant) gives
//     P_G = A'_{G+1} + TBG_{G+1} P_{G+1},   A'_H = A0_H + TBG_H Q_H E_H,
// a scan of the same form as the forward one, over aggregates A' that need
// no forward carry.  So every group posts (E_G, A'_G) right after its
// zero-start sweeps, then looks back for Y_G and ahead for P_G (decoupled:
// it replays aggregates back to the nearest posted inclusive value, Y_{G'}
// or P_{G'}), and posts its own inclusive values.  Each link is evaluated by
// one function in one order, with the group constants from one table, so a
// carry has the same bits whichever group produced it.

// The W segment records of group g (from segment s0) and its group record
// into LDS (ucon: W x 16 doubles, then 16), by direct loads of 1 KB: lane l
// of load k moves 16-byte chunk 64 k + l (chunks past the records repeat
// the group record into the unused tail).  Issued after the block's loads,
// they land with them (loads complete in order).
template <int W>
__device__ __forceinline__ void stage_consts(const SegRec *seg, const GrpRec *grp, int64_t s0, int g,
                                             double *ucon)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < (W * 8 + 8 + 63) / 64; k++) {
        const int c = 64 * k + lane;  // 16-byte chunk of ucon
        const char *src = c < W * 8 ? (const char *)(seg + s0) + 16 * c
                                    : (const char *)(grp + g) + 16 * ((c - W * 8) & 7);
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                         (__attribute__((address_space(3))) void *)(uint32_t)(uintptr_t)(ucon + 128 * k),
                                         16, 0, 0);
    }
}

// (z0, z1) <- (a0, a1) + C (y0, y1) + T (z0, z1): the upward state of a
// segment from its zero-start top state a, its forward state in y and the
// backward state below it z, one fixed order of fused multiply-adds.
__device__ __forceinline__ void up_link(double a0, double a1, double c0, double c1, double c2,
                                        double c3, double y0, double y1, double t0, double t1,
                                        double t2, double t3, double &z0, double &z1)
{
    const double n0 = fma(t2, z1, fma(t0, z0, fma(c2, y1, fma(c0, y0, a0))));
    const double n1 = fma(t3, z1, fma(t1, z0, fma(c3, y1, fma(c1, y0, a1))));
    z0 = n0;
    z1 = n1;
}

// Group-level look-back (FWD: the forward state Y_g entering group g) or
// look-ahead (P_g of the backward scan) of the tile whose first unit is u0,
// once every group has posted its aggregates.  Waits until a contiguous run
// of posted statuses reaches an inclusive one (2), then replays the
// aggregates between, innermost first.  A wait that runs out raises *err
// and returns a NaN carry, so every value that depends on it (this tile's
// x, the carries it posts) comes out NaN instead of a plausible wrong
// number.  Exchange rows: forward 0,1 aggregate E, 2,3 inclusive Y;
// backward 4,5 aggregate A', 6,7 inclusive P.
template <bool FWD>
__device__ __forceinline__ void group_wait(CGrp grp, int g, int ngroups, unsigned int u0,
                                           unsigned int *st_word, double *ex, unsigned int *err,
                                           double &y0, double &y1, double (*agg)[128],
                                           double (*mat)[4])
{
    const int lane = threadIdx.x & 63;
    const int ra = FWD ? 0 : 4;  // aggregate rows
    int base = FWD ? g - 1 : g + 1, pstar = base;
    bool timed_out = false;
    for (int spin = 0;; spin++) {
        const int p = FWD ? base - lane : base + lane;
        const bool in = FWD ? p >= 0 : p < ngroups;
        const unsigned int st = lane_status(st_word, (int64_t)u0 + p, in);
        const unsigned long long incl = __ballot(st == 2);
        const unsigned long long none = __ballot(in && st == 0);
        if (incl != 0) {
            const int l = __builtin_ctzll(incl);
            if ((none & ((1ull << l) - 1)) == 0) {
                pstar = FWD ? base - l : base + l;
                break;
            }
        } else if (none == 0 && (FWD ? base >= 64 : base + 64 < ngroups)) {
            base = FWD ? base - 64 : base + 64;
            continue;
        }
        if (spin >= kSpin) {
            atomicOr(err, 1u);
            timed_out = true;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    // replay the groups between pstar and g, innermost first.  The replay
    // is latency-bound and registers hold the block, so each round trip
    // brings up to kStage groups' aggregates and link matrices into LDS at
    // once; they are then linked in order.
    const int cnt = FWD ? g - 1 - pstar : pstar - g - 1;
    auto group_at = [&](int i) { return FWD ? pstar + 1 + i : pstar - 1 - i; };
    const double *nb = ex + (int64_t)(u0 + pstar) * (kExRows * 64) + lane;
    y0 = xload(&nb[(ra + 2) * 64]);
    y1 = xload(&nb[(ra + 3) * 64]);
    for (int c = 0; c < cnt; c += kStage) {
        const int m = cnt - c < kStage ? cnt - c : kStage;
#pragma unroll
        for (int i = 0; i < kStage; i++)
            if (i < m) stage_load(ex + (int64_t)(u0 + group_at(c + i)) * (kExRows * 64) + ra * 64, agg[i]);
        {
            // link matrices, half a matrix (16 bytes) per lane: lane l lands
            // at LDS byte 16 l of mat, so lanes 2i, 2i+1 fill mat[i] (lanes
            // 32..63 repeat lanes 0..31 into the upper half); slots past the
            // chunk reload its first group
            const int i = (lane >> 1) & (kStage - 1);
            const int q = group_at(c + (i < m ? i : 0));
            const CDbl src = FWD ? &grp[q].tg[2 * (lane & 1)] : &grp[q].tbg[2 * (lane & 1)];
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                             (__attribute__((address_space(3))) void *)(uint32_t)(uintptr_t)&mat[0][0],
                                             16, 0, 0);
        }
        store_fence();  // the direct loads have landed in LDS
        // the serial links, without branches (slots past the chunk are
        // computed and dropped), so the reads can run ahead of the chain
#pragma unroll
        for (int i = 0; i < kStage; i++) {
            double n0 = y0, n1 = y1;
            link(agg[i][lane], agg[i][64 + lane], mat[i][0], mat[i][1], mat[i][2], mat[i][3], n0, n1);
            y0 = i < m ? n0 : y0;
            y1 = i < m ? n1 : y1;
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);  // LDS reads before the next chunk's loads
        __builtin_amdgcn_s_waitcnt(0xC07F);       // lgkmcnt(0)
    }
    if (timed_out) {
        y0 = __builtin_nan("");
        y1 = __builtin_nan("");
    }
}

// The single-wait form of group_phases (see above): on exit v holds x.
// Sweeps: zero-start forward (v becomes g0), zero-start
// back substitution over g0 (its top state only), then, once the carries
// are known, g = g0 + the response to the incoming forward state, and the
// back substitution over g from the state below, which leaves x in v.
template <int K, int W, bool LREC = false>
__device__ __forceinline__ void group_phases_1w(double (&v)[K], CFwd fwd, CBwd bwd, CSeg seg, CGrp grp,
                                             int64_t r0, int w, int g, int ngroups,
                                             unsigned int u0, unsigned int *fst,
                                             unsigned int *bst, double *ex, unsigned int *err,
                                             double (*sh)[4][64], double (*agg)[128],
                                             double (*mat)[4], double *ucon,
                                             const FwdRec *lf = nullptr, const BwdRec *lb = nullptr)
{
    const int lane = threadIdx.x & 63;
    const int64_t s0 = (int64_t)g * W;
    if (w == 0) stage_consts<W>((const SegRec *)seg, (const GrpRec *)grp, s0, g, ucon);
    // segment record i (tf at 0, cg at 4, tb at 8) and the group record (tg
    // at 0, tbg at 4, q at 12) as staged in LDS
    auto sc = [&](int i, int k) { return ucon[16 * i + k]; };
    auto gc = [&](int k) { return ucon[16 * W + k]; };
    {
        double e0 = 0.0, e1 = 0.0, a0 = 0.0, a1 = 0.0;
        forward<K, true, LREC>(v, fwd, r0, e0, e1, lf);
        backward<K, false, LREC>(v, bwd, r0, a0, a1, lb);
        sh[w][0][lane] = e0;
        sh[w][1][lane] = e1;
        sh[w][2][lane] = a0;
        sh[w][3][lane] = a1;
    }
    __syncthreads();
    if (w == 0) {
        store_fence();  // the staged records have landed (they came in with the block)
        // the group's states for zero carries: E (forward out) and A0
        // (backward top, over the group's own forward values)
        double yi0[W], yi1[W];
        double E0 = 0.0, E1 = 0.0;
#pragma unroll
        for (int i = 0; i < W; i++) {
            yi0[i] = E0;
            yi1[i] = E1;
            link(sh[i][0][lane], sh[i][1][lane], sc(i, 0), sc(i, 1), sc(i, 2), sc(i, 3), E0, E1);
        }
        double A0 = 0.0, A1 = 0.0;
#pragma unroll
        for (int i = W - 1; i >= 0; i--)
            up_link(sh[i][2][lane], sh[i][3][lane], sc(i, 4), sc(i, 5), sc(i, 6), sc(i, 7), yi0[i],
                    yi1[i], sc(i, 8), sc(i, 9), sc(i, 10), sc(i, 11), A0, A1);
        // the backward scan's aggregate A' = A0 + TBG (Q E)
        double B0 = E0, B1 = E1;
        link(0.0, 0.0, gc(12), gc(13), gc(14), gc(15), B0, B1);
        link(A0, A1, gc(4), gc(5), gc(6), gc(7), B0, B1);
        // post both aggregates (the first group's forward value and the last
        // group's backward value are already inclusive)
        const bool first = g == 0, last = g == ngroups - 1;
        double *me = ex + (int64_t)(u0 + g) * (kExRows * 64) + lane;
        xstore(&me[(first ? 2 : 0) * 64], E0);
        xstore(&me[(first ? 3 : 1) * 64], E1);
        xstore(&me[(last ? 6 : 4) * 64], B0);
        xstore(&me[(last ? 7 : 5) * 64], B1);
        store_fence();
        __hip_atomic_store(&fst[u0 + g], first ? 2u : 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&bst[u0 + g], last ? 2u : 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // forward: Y_g, then Y_{g+1} = E + TG Y_g, posted as inclusive
        double Y0 = 0.0, Y1 = 0.0;
        if (!first) group_wait<true>(grp, g, ngroups, u0, fst, ex, err, Y0, Y1, agg, mat);
        double N0 = Y0, N1 = Y1;
        link(E0, E1, gc(0), gc(1), gc(2), gc(3), N0, N1);
        if (!first && !last) {
            xstore(&me[2 * 64], N0);
            xstore(&me[3 * 64], N1);
            publish(&fst[u0 + g], 2u);
        }
        // backward: P_g, then P_{g-1} = A' + TBG P_g, posted as inclusive
        double P0 = 0.0, P1 = 0.0;
        if (!last) group_wait<false>(grp, g, ngroups, u0, bst, ex, err, P0, P1, agg, mat);
        if (!first && !last) {
            double O0 = P0, O1 = P1;
            link(B0, B1, gc(4), gc(5), gc(6), gc(7), O0, O1);
            xstore(&me[6 * 64], O0);
            xstore(&me[7 * 64], O1);
            publish(&bst[u0 + g], 2u);
        }
        // the state entering the group from below: Zin = P + Q Y_{g+1}
        double Z0 = N0, Z1 = N1;
        link(P0, P1, gc(12), gc(13), gc(14), gc(15), Z0, Z1);
        // every wave's states: forward through the waves above it, backward
        // through the waves below it (over their true forward states); sh
        // row i then holds wave i's (y, z)
#pragma unroll
        for (int i = 0; i < W; i++) {
            yi0[i] = Y0;
            yi1[i] = Y1;
            if (i + 1 < W)
                link(sh[i][0][lane], sh[i][1][lane], sc(i, 0), sc(i, 1), sc(i, 2), sc(i, 3), Y0, Y1);
        }
#pragma unroll
        for (int i = W - 1; i >= 0; i--) {
            const double a0 = sh[i][2][lane], a1 = sh[i][3][lane];
            sh[i][0][lane] = yi0[i];
            sh[i][1][lane] = yi1[i];
            sh[i][2][lane] = Z0;
            sh[i][3][lane] = Z1;
            if (i > 0)
                up_link(a0, a1, sc(i, 4), sc(i, 5), sc(i, 6), sc(i, 7), yi0[i], yi1[i], sc(i, 8),
                        sc(i, 9), sc(i, 10), sc(i, 11), Z0, Z1);
        }
    }
    __syncthreads();
    respond<K, LREC>(v, fwd, r0, sh[w][0][lane], sh[w][1][lane], lf);
    {
        double z0 = sh[w][2][lane], z1 = sh[w][3][lane];
        backward<K, true, LREC>(v, bwd, r0, z0, z1, lb);
    }
    // x is complete here: keep the compiler from sinking the sweep into the
    // block that stores x (past a caller's waits, with every coefficient
    // held live across them)
#pragma unroll
    for (int k = 0; k < K; k++) asm volatile("" : "+v"(v[k]));
}

}  // namespace lb
}  // namespace pent
