/*
 * pentbatch.h -- C ABI of libpentbatch.so, a batched pentadiagonal solver for
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Gloster, O Naraigh and Pang, "cuPentBatch -- A batched pentadiagonal
 * solver for NVIDIA GPUs" (arXiv:1807.07382).  One N x N pentadiagonal matrix
 * A is factored once, A = L R without pivoting (Sec. 2.4), and the factors
 * are reused to solve A x_j = f_j for very many right-hand sides held in the
 * interleaved layout of Sec. 2.6.
 *
 * Conventions shared by every entry point
 *  - Rows are 0-based: row i of this API is row i+1 of the paper.
 *  - Diagonals are row-indexed (Sec. 2.4): row i holds a[i] (column i-2),
 *    b[i] (column i-1), c[i] (column i), d[i] (column i+1), e[i] (column i+2).
 *    a[0], a[1], b[0], d[n-1], e[n-2] and e[n-1] fall outside the matrix and
 *    are never read.
 *  - Batch-fastest ("interleaved", Sec. 2.6) right-hand sides: element
 *    (row i, system j) lives at F[i*ld + j], 0 <= i < n, 0 <= j < batch,
 *    ld >= batch, in elements (not bytes).
 *  - Device pointers are HIP device (or managed) memory on the device that
 *    was current when the handle was made; host pointers are ordinary host
 *    memory.  The caller owns every buffer it passes and must keep it alive
 *    until the stream work that uses it has finished.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Solves are asynchronous: they only enqueue kernels.
 *  - "Stream-ordered scratch" below is allocated on `stream` and freed on it
 *    after the kernels that use it, from a memory pool of the library's own
 *    on each device.  That pool keeps up to 4 GiB reserved after the stream
 *    synchronises (the device's default pool hands freed memory back at
 *    every synchronisation, and the next call would map it again), so a
 *    program that synchronises after every solve pays no allocation on the
 *    next one.  The reserve lasts until the process ends.
 *  - Errors are returned as a pent_status; nothing throws across the ABI.
 *    Argument checks run before any HIP call, so a bad argument never leaves
 *    work queued.  pent_last_status() repeats the status of the calling
 *    thread's last call.
 *  - Stability: no pivoting, as in the paper.  The method is stable for
 *    symmetric positive definite or diagonally dominant A (Sec. 2.6); other
 *    matrices with non-zero pivots are solved but may be inaccurate.
 */
#ifndef PENTBATCH_H
#define PENTBATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pent_plan *pent_handle;

typedef enum pent_status {
    PENT_OK = 0,
    PENT_INVALID_VALUE = 1, /* bad argument (null pointer, n < 1, ld < batch, ...) */
    PENT_ZERO_PIVOT = 2,    /* alpha_i == 0 or non-finite; row in pent_last_pivot_row() */
    PENT_OUT_OF_MEMORY = 3, /* a device allocation failed */
    PENT_HIP_ERROR = 4,     /* a HIP runtime call or kernel launch failed */
    PENT_NOT_CONVERGED = 5, /* refinement did not reach its tolerance */
    PENT_SIZE_MISMATCH = 6, /* buffers of one call disagree in size */
    PENT_NOT_SUPPORTED = 7, /* a valid request this build does not handle */
    PENT_TIMEOUT = 8        /* a bounded device-side wait ran out (see pent_group_check) */
} pent_status;

/* ---------------------------------------------------------------- factor --
 * Factor A = L R once (Sec. 2.4, factorisation steps; Sec. 2.6 splits the
 * factorisation from the solve so a constant matrix is factored only once).
 * a..e: HOST arrays of n doubles (row-indexed, see above); copied, the caller
 * keeps ownership.  The factorisation runs on the current device and the call
 * blocks until it has finished (one synchronisation, to read the pivot
 * check).  Returns a handle, or NULL with pent_last_status() set to
 * PENT_INVALID_VALUE, PENT_ZERO_PIVOT (see pent_last_pivot_row()),
 * PENT_OUT_OF_MEMORY or PENT_HIP_ERROR.  Limits: 1 <= n <= 2^31 - 1. */
pent_handle pent_factor(int64_t n, const double *a, const double *b, const double *c,
                        const double *d, const double *e);

/* Same, for the matrix of the implicit hyperdiffusion step I + sigma*D4
 * (Sec. 2.3, coefficient list a = e = sigma, b = d = -4 sigma,
 * c = 1 + 6 sigma), non-periodic: the row stencil is truncated at both ends.
 * The diagonals are assembled on the device. */
pent_handle pent_factor_d4(int64_t n, double sigma);

/* Free a handle.  NULL is a no-op.  The caller must have synchronised every
 * stream with work that uses the handle. */
int pent_destroy(pent_handle h);

/* ----------------------------------------------------------------- solve --
 * Overwrite F (DEVICE, FP64, batch-fastest, element (i, j) at F[i*ld + j])
 * with X = A^{-1} F: forward sweep L g = f, then back substitution R x = g
 * (Sec. 2.4), every system independent (Sec. 2.6).  Asynchronous on
 * `stream`.  batch == 0 is a no-op (F may then be NULL).  Returns
 * PENT_INVALID_VALUE for a bad handle, batch < 0, ld < batch or F == NULL.
 * The schedule (one lane per system, or several lanes per system through a
 * partitioned sweep) is chosen by the library; it may allocate stream-ordered
 * scratch memory on `stream`. */
int pent_solve(pent_handle h, double *F, int64_t batch, int64_t ld, void *stream);

/* Same solve, allocating nothing: for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, schedule, kernels and results (bit
 * for bit) as pent_solve; the scratch that pent_solve takes from the
 * stream-ordered allocator comes instead from a fixed 72 MiB buffer in the
 * library's device memory, one per GPU, held until the process ends.
 * Returns PENT_NOT_SUPPORTED, before any HIP call, when the schedule needs
 * more scratch than that (e.g. the single pass beyond about 18 000
 * 64-system x 256-row units: n = 4096 with more than 72 000 systems) or
 * tables that do not exist yet (a schedule forced by pent_set_schedule and
 * not yet used by pent_solve; pent_factor builds the automatic schedule's).
 * Every call on one GPU shares that GPU's buffer and the buffer keeps the
 * last call's contents (the kernels clear what must start at zero), so
 * calls that may overlap in time on one GPU (other streams, other threads)
 * race: serialise them. */
int pent_solve_noalloc(pent_handle h, double *F, int64_t batch, int64_t ld, void *stream);

/* Same solve for right-hand sides stored in tiles of 64 systems, each tile
 * its own interleaved block (the layout of Sec. 2.6 applied per tile):
 * element (i, j) at F[(j / 64) * tile_stride + i * ld + j % 64], with
 * ld >= 64 and tile_stride >= (n - 1) * ld + 64; with ld = 64 and
 * tile_stride = 64 n a tile's n rows are one contiguous run, which the
 * single pass streams with fewer open DRAM pages than rows a whole batch
 * apart.  A partial last tile needs its 64 columns of storage; columns past
 * the batch are not written.  Results are the bits pent_solve gives the
 * same systems.  Runs as the single pass only: PENT_NOT_SUPPORTED (before
 * any HIP call) where pent_solve would use another schedule.
 * PENT_INVALID_VALUE for a bad handle, batch < 0, ld or tile_stride too
 * small, or F == NULL with batch > 0.  Allocates stream-ordered scratch on
 * `stream`; a wait that runs out is reported by pent_check. */
int pent_solve_tiled(pent_handle h, double *F, int64_t batch, int64_t ld, int64_t tile_stride,
                     void *stream);

/* Same solve for system-major storage: system j occupies n contiguous
 * doubles at F + j*ld (element (i, j) at F[j*ld + i]), ld >= n.  This is the
 * layout of the second direction of an alternating-direction (ADI-style)
 * sweep over a 2-D grid (Sec. 4 names ADI as the route to 2-D and 3-D
 * problems).  Runs as the single pass (blocks of 64 systems transposed
 * through LDS so that memory moves in contiguous runs of each system),
 * allocating stream-ordered scratch on `stream`, when one tile of it fits on
 * the device; else one lane per system.  A single-pass wait that runs out is
 * reported by pent_check, as for pent_solve. */
int pent_solve_strided(pent_handle h, double *F, int64_t batch, int64_t ld, void *stream);

/* ------------------------------------------------- precision extension --
 * Element types of the right-hand sides. */
#define PENT_DTYPE_FP64 0
#define PENT_DTYPE_FP32 1

/* Solve A x = f with f streamed in FP32 or FP64 and x written in FP64.  The
 * factors and every operation stay FP64 (the paper computes in FP64, Sec. 3);
 * only the stored precision of the right-hand-side stream changes, so an
 * FP32 f costs 4 instead of 8 bytes per unknown and the result is the FP64
 * solution of the system with the FP32 values as right-hand side.
 *   f, ld_f : DEVICE, batch-fastest, element (i, j) at f[i*ld_f + j], of
 *             type f_dtype (PENT_DTYPE_FP32 or PENT_DTYPE_FP64).
 *   x, ld_x : DEVICE FP64 output, same layout.  x may be f itself only for
 *             FP64 f with ld_x == ld_f and refine_steps == 0.
 *   refine_steps (0..16): iterative-refinement corrections after the solve;
 *             each evaluates r = f - A x in compensated FP64 (every product
 *             and sum carried with its rounding error), solves A d = r and
 *             sets x += d.  Where the solve runs as the single pass (kind 4)
 *             each correction is one fused pass too (the residual formed as
 *             the blocks load, x updated in place as they store); else three
 *             kernels (residual, solve, update).
 *   eta_out : optional DEVICE array of batch doubles; receives each system's
 *             backward error ||f - A x||_inf / (||A||_inf ||x||_inf +
 *             ||f||_inf) with the residual evaluated compensated (NaN or Inf
 *             when x has a non-finite entry).
 *   work    : DEVICE scratch of at least
 *             pent_mixed_workspace_size_ex(h, batch, refine_steps, eta_out != NULL)
 *             bytes (pent_mixed_workspace_size(h, batch) covers every
 *             refine_steps and eta_out), caller-owned (NULL allowed when
 *             that size is 0).
 * With a tolerance set (pent_set_refine_tolerance) the backward error is
 * evaluated after the corrections even when eta_out is NULL, and a system
 * whose eta exceeds the tolerance (or is not finite) makes the next
 * pent_check return PENT_NOT_CONVERGED; nothing waits on the host.
 * Asynchronous on `stream`; allocates nothing once the handle's per-schedule
 * tables exist (pent_factor builds those of the automatic schedule; a
 * schedule forced later builds its own on first use, blocking once).
 * Returns PENT_INVALID_VALUE for bad arguments, PENT_SIZE_MISMATCH for a
 * workspace that is too small, PENT_NOT_SUPPORTED for n > 2097120. */
int pent_solve_mixed(pent_handle h, const void *f, int f_dtype, int64_t ld_f, double *x,
                     int64_t ld_x, int64_t batch, int refine_steps, double *eta_out, void *work,
                     size_t work_bytes, void *stream);
/* Workspace of pent_solve_mixed for `batch` systems, enough for any
 * refine_steps (0..16) with eta_out and a tolerance; 0 on a bad argument. */
size_t pent_mixed_workspace_size(pent_handle h, int64_t batch);
/* Workspace for one configuration: refine_steps corrections, want_eta != 0
 * when eta_out will be passed (a tolerance set on h counts as want_eta). */
size_t pent_mixed_workspace_size_ex(pent_handle h, int64_t batch, int refine_steps, int want_eta);

/* Backward-error tolerance of h's refined solves (pent_solve_mixed): tol > 0
 * turns the check on, 0 (the default) off.  PENT_INVALID_VALUE for a
 * negative or non-finite tol.  Host-only. */
int pent_set_refine_tolerance(pent_handle h, double tol);

/* Per-system backward error of a computed solution x (same definition and
 * layouts as eta_out above).  work: DEVICE scratch of at least
 * 24*batch bytes.  Asynchronous on `stream`. */
int pent_backward_error(pent_handle h, const void *f, int f_dtype, int64_t ld_f, const double *x,
                        int64_t ld_x, int64_t batch, double *eta_out, void *work,
                        size_t work_bytes, void *stream);

/* -------------------------------------------------- batching extension --
 * Many matrices of uneven size, each with its own block of right-hand sides,
 * solved in ONE persistent kernel launch (the paper's batch is one matrix,
 * Sec. 2.6; a group extends it to a parameter study with several operators). */
typedef struct pent_group_s *pent_group;

/* Make a group of `count` factored handles (HOST array; the handles must stay
 * alive while the group exists).  Blocking.  NULL on error (pent_last_status). */
pent_group pent_group_create(const pent_handle *hs, int64_t count);

/* Scratch the group solves need for these right-hand-side counts (HOST array
 * batch[count]); 0 on error. */
size_t pent_group_workspace_size(pent_group g, const int64_t *batch);

/* Group solve modes. */
#define PENT_GROUP_FP64 0      /* one launch for all matrices, FP64 streams */
#define PENT_GROUP_MIXED 1     /* FP32 streams: not supported, see below */
#define PENT_GROUP_PER_MATRIX 2 /* one solve per matrix, the baseline */

/* Solve every matrix k on its own block: F[k] (DEVICE pointer, FP64,
 * batch-fastest, element (i, j) at F[k][i*ld[k] + j]) is overwritten with
 * A_k^{-1} F[k].  F, batch and ld are HOST arrays of `count` entries.
 * mode PENT_GROUP_FP64: one launch for all matrices (the kernel variant set
 *         by pent_group_set_variant or pent_group_autotune);
 * mode PENT_GROUP_MIXED: returns PENT_NOT_SUPPORTED after the argument
 *         checks.  In a time-stepping group the right-hand side of a step is
 *         the FP64 solution of the previous one, so there is no FP32 stream
 *         whose bytes could be saved; pent_solve_mixed covers right-hand
 *         sides that arrive in FP32;
 * mode PENT_GROUP_PER_MATRIX: one solve per matrix (the library's
 *         single-matrix schedules, one after the other on `stream`), the
 *         baseline the single launch is compared with.
 * work: DEVICE scratch of at least pent_group_workspace_size() bytes.
 * The buffer table is uploaded (blocking) only when F/batch/ld differ from
 * the previous call, so repeated calls with the same buffers only enqueue
 * kernels and may be captured into a graph.  Calls on one group must not
 * overlap in time (they share the group's work counter).  The handles must
 * outlive the group and every graph captured from it. */
int pent_group_solve(pent_group g, double *const *F, const int64_t *batch, const int64_t *ld,
                     int mode, void *work, size_t work_bytes, void *stream);
int pent_group_destroy(pent_group g); /* NULL is a no-op; graphs captured from g stay valid */

/* Autotune the group kernel for these right-hand-side counts (HOST array
 * batch[count]): every variant that can run is timed on scratch blocks of
 * the same shapes, rows padded to a multiple of 16 doubles (the caller's
 * data and binding are not touched) and the
 * fastest is kept for later PENT_GROUP_FP64 solves.  Blocking; allocates
 * scratch for the duration of the call.  variant_out / ms_out (HOST,
 * optional) receive the choice and its time. */
int pent_group_autotune(pent_group g, const int64_t *batch, int *variant_out, double *ms_out,
                        void *stream);

/* Force the kernel variant of later PENT_GROUP_FP64 solves:
 *   0: persistent: resident workgroups take work items (matrix, 64
 *      consecutive systems) longest first from a device counter and solve
 *      each alone with the partitioned sweep (f read twice, x written once);
 *      runs at any size;
 *   1 (default): the single pass over all matrices (pent_set_schedule kind
 *      4 with 64-row segments, four per workgroup, the units of every matrix
 *      in one launch; f read once, x written once); falls back to variant 0
 *      when the deepest 64-system tile would not fit on the device at once.
 * PENT_INVALID_VALUE for an unknown variant. */
int pent_group_set_variant(pent_group g, int variant);

/* Blocking check of the group's device status after its solves: PENT_OK, or
 * PENT_TIMEOUT if a bounded wait of the single pass ran out since the last
 * check (the flag is then cleared; the values of that launch that depend on
 * the missed carry are NaN). */
int pent_group_check(pent_group g);

/* Capture `steps` consecutive group solves (mode as above) on `stream` into
 * an executable HIP graph (one graph launch = `steps` implicit time steps).
 * `stream` must be a created stream (not the null stream).  The buffers are
 * bound first, outside the capture.  The graph keeps its own reference to
 * the group's device tables of that binding, so a later rebinding, autotune
 * or pent_group_destroy leaves it valid; F and work are the caller's and
 * must stay alive (and keep their shapes) while the graph may launch.
 * NULL on error. */
typedef struct pent_graph_s *pent_graph;
pent_graph pent_group_capture(pent_group g, double *const *F, const int64_t *batch,
                              const int64_t *ld, int mode, int steps, void *work,
                              size_t work_bytes, void *stream);
int pent_graph_launch(pent_graph gr, void *stream);
int pent_graph_destroy(pent_graph gr); /* NULL is a no-op; no launch of gr may still run */

/* ------------------------------------------ 2-D Cahn-Hilliard workload --
 * Split-implicit step of the 2-D Cahn-Hilliard equation on ninst independent
 * ny x nx grids (the semi-implicit scheme of Sec. 2.1 applied direction by
 * direction; Sec. 4 names this alternating-direction route to 2-D).
 * C, R: DEVICE FP64, layout [y][inst][x] contiguous (element (y, k, x) at
 * (y*ninst + k)*nx + x); dt: DEVICE, ninst time steps; h: grid spacing.
 * pent_ch2d_rhs:  R = C + dt_k * Lap_h(C^3 - C) (5-point Laplacian, zero
 *                 values outside the grid); C and R must not overlap.
 * pent_ch2d_step: the x sweeps (I + sigma D4_x) R* = RHS (hx: n = nx,
 *                 system-major) with RHS the right-hand side above, formed
 *                 inside the sweep kernel from C (it never goes to memory;
 *                 where one tile of that kernel would not fit on the device,
 *                 pent_ch2d_rhs writes it to R first and R is swept in
 *                 place), then the y sweeps (I + sigma D4_y) C = R* (hy:
 *                 n = ny, batch-fastest over ninst*nx systems), so C holds
 *                 the next state and R is scratch.  R* is the same, bit for
 *                 bit, either way.  May allocate stream-ordered scratch.
 *                 Limits: ny, ninst <= 65535. */
int pent_ch2d_rhs(const double *C, double *R, int64_t ny, int64_t ninst, int64_t nx,
                  const double *dt, double h, void *stream);
int pent_ch2d_step(pent_handle hx, pent_handle hy, double *C, double *R, int64_t ny,
                   int64_t ninst, int64_t nx, const double *dt, double h, void *stream);

/* ------------------------------------------- per-system matrices --
 * Every system with its own matrix, factored and solved in one call: the
 * paper's refactor-every-step mode (Sec. 3), for matrices that change
 * between time steps (or differ between systems).  a..e: DEVICE FP64, the
 * row-indexed diagonals of system j at a[i*ldm + j] (same convention as
 * pent_factor; a[0], a[1], b[0], d[n-1], e[n-2], e[n-1] of each system are
 * ignored); read only.  F: DEVICE FP64, F[i*ld + j], overwritten with X.
 * ldm, ld >= batch.  work: DEVICE, at least pent_rewrite_workspace_size(n,
 * batch) bytes (16 n batch + 256), caller-owned; asynchronous on `stream`.
 * No pivoting (Sec. 2.4): a zero or non-finite pivot leaves that system's
 * X non-finite; pent_rewrite_check (blocking, after the solve) reports the
 * lowest-numbered such system and its row as PENT_ZERO_PIVOT.
 * Returns PENT_INVALID_VALUE / PENT_SIZE_MISMATCH synchronously before any
 * HIP call. */
size_t pent_rewrite_workspace_size(int64_t n, int64_t batch);
int pent_solve_rewrite(int64_t n, const double *a, const double *b, const double *c,
                       const double *d, const double *e, int64_t ldm, double *F, int64_t batch,
                       int64_t ld, void *work, size_t work_bytes, void *stream);
int pent_rewrite_check(const void *work, int64_t n, int64_t *system, int64_t *row);

/* ------------------------------------------------ periodic matrices --
 * Cyclic pentadiagonal matrices (Sec. 2.3): the periodic fourth-derivative
 * matrix wraps round the corners, so row i couples columns (i-2) mod n ..
 * (i+2) mod n.  Solved by Navon's bordering (Sec. 2.3): with E the leading
 * (n-2) x (n-2) block, k its two border columns, h^T its two border rows
 * and C2 the trailing 2 x 2 block, the last two unknowns are
 * [C2 - h^T E^{-1} k]^{-1} ((f_{n-2}, f_{n-1}) - h^T E^{-1} f^) and the rest
 * E^{-1} f^ - (E^{-1} k)(x_{n-2}, x_{n-1}) (rows 0-based).  E is factored as
 * in Sec. 2.4; E^{-1} k and the 2 x 2 inverse are computed once, at factor
 * time.  A solve is either one single-pass kernel (the E-solve by
 * decoupled look-back, the last two unknowns formed by the first block of
 * every 64-system tile, the update applied before the one store) or the
 * E-solve followed by two light kernels; both take stream-ordered scratch.
 *
 * pent_cyclic_factor: a..e HOST FP64 arrays of length n, row-indexed and
 *   wrapped: row i holds a[i] at column (i-2) mod n, b[i] at (i-1) mod n,
 *   c[i] at i, d[i] at (i+1) mod n, e[i] at (i+2) mod n; every entry is
 *   used.  n >= 5.  Copied; blocking.  NULL on failure: PENT_INVALID_VALUE,
 *   PENT_ZERO_PIVOT (pent_last_pivot_row: the failing row of E, or n-2 when
 *   the 2 x 2 bordered block is singular), PENT_OUT_OF_MEMORY,
 *   PENT_HIP_ERROR.  No pivoting, so the matrix should be SPD or diagonally
 *   dominant (the periodic I + sigma D4 is SPD for sigma >= 0).
 * pent_cyclic_factor_d4: the Crank-Nicolson matrix of Sec. 2.3,
 *   a = e = sigma, b = d = -4 sigma, c = 1 + 6 sigma in every row.
 * pent_cyclic_solve: overwrite F (DEVICE FP64, element (i, j) at F[i*ld+j],
 *   ld >= batch) with A^{-1} F, asynchronously on `stream`.
 * pent_cyclic_cn_rhs: R = 2 C - A C, the explicit half of the
 *   Crank-Nicolson step (Sec. 2.3: for A = I + sigma D4 this is
 *   (I - sigma D4) C), same layout; C and R DEVICE, must not overlap.
 * pent_cyclic_bordering: copy Z = E^{-1} k ((n-2) x 2, row-major) and
 *   [C2 - h^T Z]^{-1} (2 x 2, row-major) to HOST arrays (blocking).
 * pent_cyclic_destroy: NULL is a no-op; no queued work may still use c. */
typedef struct pent_cyclic_s *pent_cyclic;
pent_cyclic pent_cyclic_factor(int64_t n, const double *a, const double *b, const double *c,
                               const double *d, const double *e);
pent_cyclic pent_cyclic_factor_d4(int64_t n, double sigma);
int pent_cyclic_solve(pent_cyclic c, double *F, int64_t batch, int64_t ld, void *stream);
int pent_cyclic_cn_rhs(pent_cyclic c, const double *C, int64_t ldc, double *R, int64_t ldr,
                       int64_t batch, void *stream);
int pent_cyclic_bordering(pent_cyclic c, double *Z, double *minv);
int pent_cyclic_destroy(pent_cyclic c);

/* pent_cyclic_cn_step: X = A^{-1} (2C - AC), one Crank-Nicolson step of
 *   Sec. 2.3 for A = I + sigma D4 (for a general periodic A the same
 *   formula).  C, X DEVICE FP64, layout as above, different buffers (C is
 *   read with two rows of halo on each side).  In the single-pass form the
 *   right-hand side never goes to memory: C is read once and X written once.
 *   Where each of the five diagonals is the same in every row, bit for bit
 *   (checked when the handle is made; I + sigma D4 is), the single pass
 *   takes them as values instead of reading them per row (same results).
 * pent_cyclic_set_schedule: kind 0 automatic (single pass when every block
 *   of one 64-system tile fits on the device at once), kind 1 the E-solve
 *   followed by the update kernels (and, for the step, a separate stencil
 *   kernel), kind 2 single pass with seg_rows in {32, 64} (still falls back
 *   to kind 1 when the blocks would not fit).
 * pent_cyclic_query_schedule: the form a solve (cn = 0) or step (cn = 1) of
 *   `batch` systems runs: kind 1 or 2, seg_rows 0 unless kind 2.
 * pent_cyclic_check: blocking; PENT_TIMEOUT if a single-pass wait on this
 *   handle ran out since the last check (values of that call are wrong). */
int pent_cyclic_cn_step(pent_cyclic c, const double *C, int64_t ldc, double *X, int64_t ldx,
                        int64_t batch, void *stream);
int pent_cyclic_set_schedule(pent_cyclic c, int kind, int seg_rows);
int pent_cyclic_query_schedule(pent_cyclic c, int64_t batch, int cn, int *kind, int *seg_rows);
int pent_cyclic_check(pent_cyclic c);

/* ----------------------------------------------------------- inspection --
 * Copy the handle's data to HOST arrays of n doubles each (blocking).
 * pent_get_factors: alpha, beta, gamma, delta of Sec. 2.4 (epsilon = a).
 * pent_get_diagonals: the (zero-padded) diagonals the handle factored. */
int pent_get_factors(pent_handle h, double *alpha, double *beta, double *gamma, double *delta);
int pent_get_diagonals(pent_handle h, double *a, double *b, double *c, double *d, double *e);
int64_t pent_size(pent_handle h); /* n, or -1 for a bad handle */

/* Force a schedule for this handle (tests and tuning):
 *   kind 0: automatic (default): the resident tile for small solves
 *           (n <= 4096 and n * batch <= 8M), else the single pass (kind 4,
 *           64 rows) for n >= 1024 when a tile of its blocks fits on the
 *           device, else the partitioned form (kind 2);
 *   kind 1: one lane per system, both sweeps in one kernel (the paper's
 *           one-thread-per-system schedule, Sec. 2.4 last paragraph), rows
 *           prefetched seg_rows at a time (the prefetch depth: 8, 16 or 32;
 *           0 means 16);
 *   kind 2: partitioned: seg_rows consecutive rows per lane, several lanes
 *           per system, with a reduced interface recurrence between the
 *           segments (seg_rows in {16, 32, 64});
 *   kind 3: resident tile: 8 systems per workgroup held whole in registers
 *           (n <= 4096), one read of f and one write of x; seg_rows ignored.
 *           For larger n a solve falls back to kind 2.
 *   kind 4: single pass: the partitioned sweep of kind 2 in one kernel, each
 *           (64-system, seg_rows-row) block held in registers from load to
 *           store, the segment interface states exchanged between blocks
 *           through device memory (decoupled look-back); f read once, x
 *           written once (seg_rows in {32, 64}).  Falls back to kind 2 when
 *           the blocks of one 64-system tile could not all be resident at
 *           once.  Its waits are bounded; a wait that runs out (only possible
 *           when other work holds most of the device) leaves wrong values in
 *           that solve and is reported by pent_check.  The number of
 *           segments per workgroup (4) can be set to 2, 4 or 8 with the
 *           environment variable PENT_ONEPASS_WAVES, read once per process
 *           (tuning).
 * Returns PENT_INVALID_VALUE for an unknown kind or seg_rows. */
int pent_set_schedule(pent_handle h, int kind, int seg_rows);

/* Blocking check of the handle's status word since the last check (then
 * cleared): PENT_TIMEOUT if a single-pass solve on this handle gave up a
 * wait (the values that depend on the missed carry are NaN), else
 * PENT_NOT_CONVERGED if a refined solve missed the tolerance set by
 * pent_set_refine_tolerance, else PENT_OK. */
int pent_check(pent_handle h);

/* Autotune the schedule of this handle for `batch` systems: one lane per
 * system at prefetch depths 8/16/32, partitioned with 16/32/64 rows per
 * lane, (n <= 4096) the resident tile, and the single pass with 32/64-row
 * segments are timed on a scratch buffer of n x batch (allocated and freed
 * here) and the fastest is set as the handle's schedule (for every later
 * batch size).  Results are kept per process, keyed by (device
 * architecture, n, batch, element type), and appended to the text file named
 * by the environment variable PENT_TUNE_CACHE, which later processes read
 * back (a line measured on another architecture is never used).  Blocking.
 * kind_out, seg_rows_out, ms_out (HOST, optional) receive the choice and its
 * time. */
int pent_autotune(pent_handle h, int64_t batch, int *kind_out, int *seg_rows_out, double *ms_out,
                  void *stream);

/* The schedule pent_solve would use for `batch` systems on this handle
 * (kind as above; seg_rows is the segment height for kinds 2 and 4, the
 * prefetch depth for kind 1, 0 for kind 3).  Host-only, no HIP call. */
int pent_query_schedule(pent_handle h, int64_t batch, int *kind, int *seg_rows);

/* ---------------------------------------------------------- measurement --
 * The copy ceiling of the batch-fastest single pass: dst = src for an
 * (n x batch) block (DEVICE FP64, element (i, j) at src[i*ld_src + j] and
 * dst[i*ld_dst + j]; src == dst with equal ld is an in-place copy), moved
 * exactly as the single pass moves its right-hand sides (64 systems x 64
 * rows per wave, one 512-byte row segment per load, four waves down the
 * rows per workgroup) with no arithmetic and no exchange.  Its bandwidth is
 * what a solve on that layout can at best reach (Sec. 2.6 layout; the
 * measurement behind the roofline fractions).  Asynchronous on `stream`. */
int pent_stream_copy(const double *src, int64_t ld_src, double *dst, int64_t ld_dst, int64_t n,
                     int64_t batch, void *stream);

/* The same copy with another workgroup shape: tiles_across 64-system tiles
 * side by side, each covered by waves_down waves of 64 rows, (tiles_across,
 * waves_down) in {(1, 4), (1, 2), (2, 2), (2, 1), (4, 1)}; (1, 4) is
 * pent_stream_copy.  Wider shapes read longer runs of each row at once and
 * copy faster on the batch-fastest layout; a solve would pay for them with
 * longer interface chains (more, shorter groups per tile).  Measurement
 * only.  PENT_INVALID_VALUE for another shape or the arguments rejected by
 * pent_stream_copy. */
int pent_stream_copy_shaped(const double *src, int64_t ld_src, double *dst, int64_t ld_dst,
                            int64_t n, int64_t batch, int tiles_across, int waves_down,
                            void *stream);

/* --------------------------------------------------------------- status -- */
int pent_last_status(void);
int64_t pent_last_pivot_row(void); /* row of the last PENT_ZERO_PIVOT, else -1 */
const char *pent_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* PENTBATCH_H */
