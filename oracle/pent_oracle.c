/*
 * pent_oracle.c -- TEST INFRASTRUCTURE ONLY (the CPU oracle).
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the batched
 * pentadiagonal solve of Gloster, O Naraigh and Pang, "cuPentBatch -- A
 * batched pentadiagonal solver for NVIDIA GPUs" (arXiv:1807.07382).
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library.  It shares no code, header or
 * constant with the HIP library and must never be used as a fallback for it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (IEEE FP64, no fast
 * math, every division written as a division, no fused multiply-add except
 * the explicit fma() calls of the compensated residual).
 *
 * Index convention: rows are 0-based here (row i of this file is row i+1 of
 * the paper).  Diagonals are row-indexed as in Sec. 2.4: row i holds
 * a[i] (column i-2), b[i] (i-1), c[i] (i), d[i] (i+1), e[i] (i+2).
 * Entries that would fall outside the matrix (a[0], a[1], b[0], d[n-1],
 * e[n-2], e[n-1]) are never read; they are taken as zero.
 *
 * Right-hand sides use the interleaved (batch-fastest) layout of Sec. 2.6:
 * element (row i, system j) lives at F[i*ld + j].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_INVALID 1
#define ORC_ZERO_PIVOT 2

/* Coefficients of the implicit hyperdiffusion operator, Sec. 2.3 (the matrix
 * system and its coefficient list): a = e = sigma, b = d = -4 sigma,
 * c = 1 + 6 sigma.  The non-periodic (truncated) form keeps the same row
 * stencil and drops the entries that fall outside the matrix. */
int orc_assemble_d4(int64_t n, double sigma, double *a, double *b, double *c,
                    double *d, double *e)
{
    if (n < 1 || !a || !b || !c || !d || !e) return ORC_INVALID;
    for (int64_t i = 0; i < n; i++) {
        a[i] = (i >= 2) ? sigma : 0.0;
        b[i] = (i >= 1) ? -4.0 * sigma : 0.0;
        c[i] = 1.0 + 6.0 * sigma;
        d[i] = (i + 1 < n) ? -4.0 * sigma : 0.0;
        e[i] = (i + 2 < n) ? sigma : 0.0;
    }
    return ORC_OK;
}

/* A = L R (Sec. 2.4, "Factor A = LR" and its explicit factorisation steps).
 * L is lower triangular with diagonal alpha, first sub-diagonal beta and
 * second sub-diagonal epsilon (= a); R is unit upper triangular with first
 * super-diagonal gamma and second super-diagonal delta.
 *
 * The paper writes the first two rows and the last two rows as separate
 * steps; they are exactly the general step with the out-of-range quantities
 * (a, b of the first rows, d, e of the last rows, and gamma/delta of rows
 * before the first) set to zero, so one uniform loop is used here:
 *     beta_i  = b_i - a_i gamma_{i-2}
 *     alpha_i = c_i - a_i delta_{i-2} - beta_i gamma_{i-1}
 *     gamma_i = (d_i - beta_i delta_{i-1}) / alpha_i
 *     delta_i = e_i / alpha_i
 * No pivoting: a zero or non-finite alpha_i stops the factorisation and
 * reports row i (the method needs an SPD or diagonally dominant A, Sec. 2.6).
 */
int orc_factor(int64_t n, const double *a, const double *b, const double *c,
               const double *d, const double *e, double *alpha, double *beta,
               double *gamma, double *delta, int64_t *bad_row)
{
    if (bad_row) *bad_row = -1;
    if (n < 1 || !a || !b || !c || !d || !e || !alpha || !beta || !gamma || !delta)
        return ORC_INVALID;
    for (int64_t i = 0; i < n; i++) {
        double ai = (i >= 2) ? a[i] : 0.0;
        double bi = (i >= 1) ? b[i] : 0.0;
        double di = (i + 1 < n) ? d[i] : 0.0;
        double ei = (i + 2 < n) ? e[i] : 0.0;
        double gam2 = (i >= 2) ? gamma[i - 2] : 0.0;
        double del2 = (i >= 2) ? delta[i - 2] : 0.0;
        double gam1 = (i >= 1) ? gamma[i - 1] : 0.0;
        double del1 = (i >= 1) ? delta[i - 1] : 0.0;
        beta[i] = bi - ai * gam2;
        alpha[i] = c[i] - ai * del2 - beta[i] * gam1;
        if (!(alpha[i] != 0.0) || !isfinite(alpha[i])) {
            if (bad_row) *bad_row = i;
            return ORC_ZERO_PIVOT;
        }
        gamma[i] = (di - beta[i] * del1) / alpha[i];
        delta[i] = ei / alpha[i];
    }
    return ORC_OK;
}

/* Forward sweep L g = f then back substitution R x = g (Sec. 2.4, the steps
 * that find g and x), applied to every column of F in place: f is replaced
 * by g and then by x, as the paper does with its right-hand-side vector.
 *     g_i = (f_i - epsilon_i g_{i-2} - beta_i g_{i-1}) / alpha_i,  i ascending
 *     x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2},                i descending
 * epsilon_i = a_i (the last factorisation step).  Columns are independent;
 * the batch loop is innermost and the column range is split over OpenMP
 * threads (the paper's OpenMP variant parallelises the batch loop, Sec. 3.3).
 */
int orc_solve(int64_t n, const double *a, const double *alpha, const double *beta,
              const double *gamma, const double *delta, double *F, int64_t batch,
              int64_t ld)
{
    if (n < 1 || batch < 0 || ld < batch || !a || !alpha || !beta || !gamma || !delta)
        return ORC_INVALID;
    if (batch == 0) return ORC_OK;
    if (!F) return ORC_INVALID;
    const int64_t blk = 64;
    const int64_t nblk = (batch + blk - 1) / blk;
#pragma omp parallel for schedule(static)
    for (int64_t cb = 0; cb < nblk; cb++) {
        int64_t j0 = cb * blk;
        int64_t j1 = j0 + blk < batch ? j0 + blk : batch;
        for (int64_t i = 0; i < n; i++) {
            double eps = (i >= 2) ? a[i] : 0.0;
            double bet = (i >= 1) ? beta[i] : 0.0;
            double *row = F + i * ld;
            const double *row1 = (i >= 1) ? F + (i - 1) * ld : NULL;
            const double *row2 = (i >= 2) ? F + (i - 2) * ld : NULL;
            for (int64_t j = j0; j < j1; j++) {
                double g1 = row1 ? row1[j] : 0.0;
                double g2 = row2 ? row2[j] : 0.0;
                row[j] = (row[j] - eps * g2 - bet * g1) / alpha[i];
            }
        }
        for (int64_t i = n - 1; i >= 0; i--) {
            double gam = (i + 1 < n) ? gamma[i] : 0.0;
            double del = (i + 2 < n) ? delta[i] : 0.0;
            double *row = F + i * ld;
            const double *row1 = (i + 1 < n) ? F + (i + 1) * ld : NULL;
            const double *row2 = (i + 2 < n) ? F + (i + 2) * ld : NULL;
            for (int64_t j = j0; j < j1; j++) {
                double x1 = row1 ? row1[j] : 0.0;
                double x2 = row2 ? row2[j] : 0.0;
                row[j] = row[j] - gam * x1 - del * x2;
            }
        }
    }
    return ORC_OK;
}

/* ---- residual and backward error (test evaluators, not part of the method) ----
 * r = f - A x with every product and sum carried compensated: TwoProduct by
 * fma and TwoSum (the "Dot2" scheme of Ogita, Rump and Oishi, SIAM J. Sci.
 * Comput. 26 (2005)), so r is accurate to about one rounding of its own
 * magnitude even when it is 1e-16 of the terms it comes from. */
static inline void two_sum(double x, double y, double *s, double *err)
{
    double t = x + y;
    double z = t - x;
    *err = (x - (t - z)) + (y - z);
    *s = t;
}

static inline void two_prod(double x, double y, double *p, double *err)
{
    double t = x * y;
    *err = fma(x, y, -t);
    *p = t;
}

/* Per column j: eta[j] = ||r||_inf / (||A||_inf ||x||_inf + ||f||_inf) and
 * rho[j] = ||r||_2 / ||f||_2, with r = f - A x evaluated compensated.
 * X and Fo (the original right-hand sides) share the same layout; ldx, ldf
 * are their leading dimensions.  Either output may be NULL. */
int orc_residual(int64_t n, const double *a, const double *b, const double *c,
                 const double *d, const double *e, const double *X, int64_t ldx,
                 const double *Fo, int64_t ldf, int64_t batch, double *eta,
                 double *rho)
{
    if (n < 1 || batch < 0 || ldx < batch || ldf < batch || !a || !b || !c || !d || !e)
        return ORC_INVALID;
    if (batch == 0) return ORC_OK;
    if (!X || !Fo) return ORC_INVALID;
    double anorm = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double s = fabs(c[i]);
        if (i >= 2) s += fabs(a[i]);
        if (i >= 1) s += fabs(b[i]);
        if (i + 1 < n) s += fabs(d[i]);
        if (i + 2 < n) s += fabs(e[i]);
        if (s > anorm) anorm = s;
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < batch; j++) {
        double rmax = 0.0, xmax = 0.0, fmax = 0.0, r2 = 0.0, f2 = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double coef[5], xv[5];
            int m = 0;
            if (i >= 2) { coef[m] = a[i]; xv[m] = X[(i - 2) * ldx + j]; m++; }
            if (i >= 1) { coef[m] = b[i]; xv[m] = X[(i - 1) * ldx + j]; m++; }
            coef[m] = c[i]; xv[m] = X[i * ldx + j]; m++;
            if (i + 1 < n) { coef[m] = d[i]; xv[m] = X[(i + 1) * ldx + j]; m++; }
            if (i + 2 < n) { coef[m] = e[i]; xv[m] = X[(i + 2) * ldx + j]; m++; }
            /* Dot2 of (f, -coef) . (1, x): start from f exactly. */
            double s = Fo[i * ldf + j], comp = 0.0;
            for (int k = 0; k < m; k++) {
                double p, pe, t, te;
                two_prod(-coef[k], xv[k], &p, &pe);
                two_sum(s, p, &t, &te);
                s = t;
                comp += te + pe;
            }
            double r = s + comp;
            double ar = fabs(r), ax = fabs(X[i * ldx + j]), af = fabs(Fo[i * ldf + j]);
            /* maxima that keep a NaN: a non-finite x has no finite backward error */
            if (ar > rmax || ar != ar) rmax = ar;
            if (ax > xmax || ax != ax) xmax = ax;
            if (af > fmax || af != af) fmax = af;
            r2 += r * r;
            f2 += Fo[i * ldf + j] * Fo[i * ldf + j];
        }
        double den = anorm * xmax + fmax;
        /* den == 0 only for x = 0 and f = 0, where r = 0 too; a NaN in either
         * maximum reaches eta */
        if (eta) eta[j] = (den > 0.0 || den != den) ? rmax / den : rmax;
        if (rho) rho[j] = f2 > 0.0 ? sqrt(r2) / sqrt(f2) : sqrt(r2);
    }
    return ORC_OK;
}

/* Plain FP64 banded product y = A x (same layout), used by the workload
 * oracles to build manufactured right-hand sides.  Terms are added in
 * column order a, b, c, d, e. */
int orc_matvec(int64_t n, const double *a, const double *b, const double *c,
               const double *d, const double *e, const double *X, int64_t ldx,
               double *Y, int64_t ldy, int64_t batch)
{
    if (n < 1 || batch < 0 || ldx < batch || ldy < batch || !a || !b || !c || !d || !e)
        return ORC_INVALID;
    if (batch == 0) return ORC_OK;
    if (!X || !Y) return ORC_INVALID;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int64_t j = 0; j < batch; j++) {
            double s = 0.0;
            if (i >= 2) s += a[i] * X[(i - 2) * ldx + j];
            if (i >= 1) s += b[i] * X[(i - 1) * ldx + j];
            s += c[i] * X[i * ldx + j];
            if (i + 1 < n) s += d[i] * X[(i + 1) * ldx + j];
            if (i + 2 < n) s += e[i] * X[(i + 2) * ldx + j];
            Y[i * ldy + j] = s;
        }
    }
    return ORC_OK;
}

int orc_num_threads(void)
{
    int t = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        t = omp_get_num_threads();
    }
#endif
    return t;
}
