/*
 * FP64 CPU oracle for adaptive FSAI: the setup of G, its application z = G^T (G r), and
 * the preconditioned conjugate gradient method that uses it.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load this library; the product path never does.  It shares no code, header,
 * constant or helper with the HIP library.  Plain loops, FP64 throughout, built with
 * -ffp-contract=off so that every a*b+c is a rounded product followed by a rounded sum.
 *
 * Method (Isotton, Janna, Bernaschi, "A GPU-accelerated adaptive FSAI preconditioner for
 * massively parallel simulations", Sec. 2):
 *   - G is lower triangular and M^-1 = G^T G approximates A^-1 (eq. prec).
 *   - Row i of G on the pattern P_i (i last) is the solution of the dense SPD system
 *     A[P_i,P_i] y = e_m (eq. DensSys), scaled so that (G A G^T)_ii = 1 (eq. diagScal).
 *     With A[P_i,P_i] = L L^T this row equals L^-T e_m (the last row of L^-1), and
 *     psi_i = g~_i^T A g~_i of the unit-diagonal row equals L_mm^2, the Schur complement
 *     A_ii - A[i,Pbar] A[Pbar,Pbar]^-1 A[Pbar,i].
 *   - The pattern starts from the identity (G_0 = I, Sec. 2, adaptive part) and grows by
 *     the s lower positions j < i with the largest |d psi_i / d G~_ij| (eq. grapsi), which is
 *     proportional to |(A g_i)_j| for the current scaled row g_i; k_max such steps at most,
 *     and row i stops early when psi_{k,i} / psi_{0,i} <= eps (eq. exit_crit).
 *
 * Readings where the paper is silent or garbled (each is also listed in the design notes):
 *   - eq. diagScal2 prints D_G[i,i] = 1/psi_i; eqs. diagScal and kap1 need psi_i^{-1/2}.
 *     The scaled row used here is g_i = psi_i^{-1/2} g~_i (so G_ii = 1/L_mm).
 *   - eq. grapsi counts the diagonal twice if read literally; the gradient used is the one of
 *     psi(g~) = g~^T A g~, i.e. 2 (A g~)_j, ranked by |(A g)_j| over j < i, j not in P_i.
 *   - ties: every candidate with |v_j| >= (1 - tau) * max counts as tied and the smallest
 *     column index wins; s > 1 positions are taken one at a time with the maximum recomputed
 *     over the candidates left; candidates with |v_j| <= 2^-40 * max are not eligible; a row
 *     with no eligible candidate stops growing.
 *   - psi_{0,i} = a_ii (G_0 = I); the exit test is applied after each step's solve.
 *   - the paper treats P_i as a set and names only a batched Cholesky decomposition (Sec. 3).
 *     Here the off-diagonal positions are ordered by when they joined the pattern (step by
 *     step, within a step in selection order) with i last, and A[P,P] is factorised in that
 *     order in the column-scaling form: each pivot's reciprocal is formed once and the entries
 *     below it are multiplied by it (as in LAPACK's unblocked Cholesky); the back substitution
 *     multiplies by the same reciprocals.  In exact arithmetic neither choice changes G; they
 *     fix the rounding sequence.  Rows of G are returned with ascending columns.
 *   - PCG: textbook PCG with x0 given, stopping when ||r_k||_2 <= rtol ||b||_2 on the
 *     recursively updated residual (the paper only says the initial residual is reduced by
 *     eight orders of magnitude).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    OR_OK = 0,
    OR_ERR_INVALID_ARG = 1,
    OR_ERR_BAD_MATRIX = 2,
    OR_ERR_NOT_SPD = 3,
    OR_ERR_NO_MEMORY = 4,
    OR_ERR_NOT_CONVERGED = 5
};

enum { OR_STOP_KMAX = 0, OR_STOP_EPS = 1, OR_STOP_NOCAND = 2 };

/* A[r][c], or 0 when the entry is not stored: binary search in the ascending row r */
static double csr_entry(const int32_t *rp, const int32_t *ci, const double *av, int32_t r, int32_t c)
{
    int32_t lo = rp[r], hi = rp[r + 1] - 1;
    while (lo <= hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (ci[mid] == c) return av[mid];
        if (ci[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return 0.0;
}

static int in_pattern(const int32_t *P, int m, int32_t j)
{
    for (int t = 0; t < m; ++t)
        if (P[t] == j) return 1;
    return 0;
}

/* structural checks: row pointers monotone from 0, columns in range and strictly ascending
 * within each row, diagonal present in every row */
int oracle_check_csr(int32_t n, const int32_t *rp, const int32_t *ci)
{
    if (n <= 0 || rp[0] != 0) return OR_ERR_BAD_MATRIX;
    for (int32_t i = 0; i < n; ++i) {
        if (rp[i + 1] < rp[i]) return OR_ERR_BAD_MATRIX;
        int has_diag = 0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] < 0 || ci[e] >= n) return OR_ERR_BAD_MATRIX;
            if (e > rp[i] && ci[e] <= ci[e - 1]) return OR_ERR_BAD_MATRIX;
            if (ci[e] == i) has_diag = 1;
        }
        if (!has_diag) return OR_ERR_BAD_MATRIX;
    }
    return OR_OK;
}

typedef struct {
    double *v;        /* gradient accumulator, indexed by column, length n */
    char *mark;       /* column touched in this step, length n */
    int32_t *touched; /* touched columns, in first-touch order */
    int32_t *elig;    /* eligible candidates */
    double *B;        /* gathered dense block, mmax*mmax, row-major */
    double *L;        /* Cholesky factor, mmax*mmax, row-major, lower part */
    double *dinv;     /* reciprocals of the pivots L[c][c], mmax */
    int32_t *P;       /* pattern in growth order, i last, mmax */
    double *g;        /* scaled row on P, mmax */
} work_t;

/*
 * One row of the adaptive FSAI setup (Sec. 2).  While the row grows, w->P[0..m-1] holds the
 * pattern in growth order (i last) and w->g the scaled row on it.  On return cols[0..m-1]
 * (ascending) and vals[0..m-1] hold row i of the scaled factor G; psi_hist[k] holds psi_{k,i}
 * for the steps taken (psi_hist[0] = a_ii).
 */
static int afsai_row(int32_t i, const int32_t *rp, const int32_t *ci, const double *av,
                     int32_t kmax, int32_t s, double eps, double tau, work_t *w,
                     int32_t *cols, double *vals, int32_t *m_out, double *psi_hist,
                     int32_t *steps_out, int32_t *reason_out)
{
    int32_t *P = w->P;
    double *g = w->g;
    /* G_0 = I scaled (Sec. 2, adaptive part; eq. diagScal): P = {i}, g = a_ii^{-1/2} */
    double aii = csr_entry(rp, ci, av, i, i);
    if (!(aii > 0.0) || !isfinite(aii)) return OR_ERR_NOT_SPD;
    int32_t m = 1;
    P[0] = i;
    g[0] = 1.0 / sqrt(aii);
    double psi0 = aii;
    psi_hist[0] = psi0;
    int32_t steps = 0, reason = OR_STOP_KMAX;

    for (int32_t k = 1; k <= kmax; ++k) {
        /* Kaporin gradient (eq. grapsi): v_j = sum_{r in P} a_rj g_r for j < i, accumulated
         * over r in pattern order; a_rj = a_jr by symmetry, so this is (A g)_j. */
        int32_t nt = 0;
        for (int32_t t = 0; t < m; ++t) {
            int32_t r = P[t];
            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
                int32_t j = ci[e];
                if (j >= i) continue;
                if (!w->mark[j]) {
                    w->mark[j] = 1;
                    w->v[j] = 0.0;
                    w->touched[nt++] = j;
                }
                w->v[j] = w->v[j] + av[e] * g[t];
            }
        }
        /* candidates: touched columns outside the pattern; largest |v| */
        double M = 0.0;
        int32_t ncand = 0;
        for (int32_t q = 0; q < nt; ++q) {
            int32_t j = w->touched[q];
            if (in_pattern(P, m, j)) continue;
            ++ncand;
            double a = fabs(w->v[j]);
            if (a > M) M = a;
        }
        int32_t nel = 0;
        if (ncand > 0 && M > 0.0) {
            double thr = 0x1.0p-40 * M;
            for (int32_t q = 0; q < nt; ++q) {
                int32_t j = w->touched[q];
                if (in_pattern(P, m, j)) continue;
                if (fabs(w->v[j]) > thr) w->elig[nel++] = j;
            }
        }
        /* top-s selection, one position at a time: largest |v|, ties within relative tau
         * resolved towards the smallest column */
        int32_t S[64];
        int32_t ns = 0;
        while (ns < s && nel > 0) {
            double Mp = 0.0;
            for (int32_t q = 0; q < nel; ++q) {
                double a = fabs(w->v[w->elig[q]]);
                if (a > Mp) Mp = a;
            }
            double band = (1.0 - tau) * Mp;
            int32_t best = -1;
            for (int32_t q = 0; q < nel; ++q) {
                int32_t j = w->elig[q];
                if (fabs(w->v[j]) >= band && (best < 0 || j < w->elig[best])) best = q;
            }
            S[ns++] = w->elig[best];
            w->elig[best] = w->elig[--nel];
        }
        for (int32_t q = 0; q < nt; ++q) w->mark[w->touched[q]] = 0;
        if (ns == 0) {
            reason = OR_STOP_NOCAND;
            break;
        }
        /* enlarge the pattern: the new positions follow the old ones in selection order, and
         * i moves to the end */
        for (int32_t q = 0; q < ns; ++q) {
            P[m - 1] = S[q];
            P[m] = i;
            ++m;
        }
        /* systems gather: B = A[P,P] (lower part, row P[p] column P[q], q <= p) */
        for (int32_t p = 0; p < m; ++p)
            for (int32_t q = 0; q <= p; ++q) w->B[p * m + q] = csr_entry(rp, ci, av, P[p], P[q]);
        /* Cholesky A[P,P] = L L^T, one column after another; inner products in ascending
         * position order; the entries below a pivot are multiplied by its reciprocal */
        double *L = w->L;
        double *dinv = w->dinv;
        for (int32_t c = 0; c < m; ++c) {
            for (int32_t r = c; r < m; ++r) {
                double acc = w->B[r * m + c];
                for (int32_t t = 0; t < c; ++t) acc = acc - L[r * m + t] * L[c * m + t];
                if (r == c) {
                    if (!(acc > 0.0) || !isfinite(acc)) return OR_ERR_NOT_SPD;
                    L[c * m + c] = sqrt(acc);
                    dinv[c] = 1.0 / L[c * m + c];
                } else {
                    L[r * m + c] = acc * dinv[c];
                }
            }
        }
        /* g = L^-T e_m by back substitution (eq. DensSys scaled by eq. diagScal);
         * sums over l taken from the last position down */
        g[m - 1] = dinv[m - 1];
        for (int32_t t = m - 2; t >= 0; --t) {
            double acc = 0.0;
            for (int32_t l = m - 1; l > t; --l) acc = acc + L[l * m + t] * g[l];
            g[t] = -(acc * dinv[t]);
        }
        double lmm = L[(m - 1) * m + (m - 1)];
        double psi = lmm * lmm;
        steps = k;
        psi_hist[k] = psi;
        /* per-row exit test (eq. exit_crit) */
        if (psi <= eps * psi0) {
            reason = OR_STOP_EPS;
            break;
        }
    }
    /* the row of G with ascending columns */
    for (int32_t t = 0; t < m; ++t) {
        int32_t u = t;
        while (u > 0 && cols[u - 1] > P[t]) {
            cols[u] = cols[u - 1];
            vals[u] = vals[u - 1];
            --u;
        }
        cols[u] = P[t];
        vals[u] = g[t];
    }
    *m_out = m;
    *steps_out = steps;
    *reason_out = reason;
    return OR_OK;
}

/*
 * Adaptive FSAI setup for the rows listed in `rows` (all rows 0..nrows-1 when rows == NULL).
 * Outputs per listed row q: m_out[q], cols_out[q*mmax ...], vals_out[q*mmax ...],
 * psi_out[q*(kmax+1) ...] (NaN for steps not taken), steps_out[q], reason_out[q].
 * mmax must be at least 1 + kmax*s.  Returns the status of the lowest listed row that fails,
 * or OR_OK.  Rows are independent (Sec. 2), so they are spread over `nthreads` threads
 * (<= 0: the OpenMP default); results do not depend on the thread count.
 */
int oracle_afsai_rows(int32_t n, const int32_t *rp, const int32_t *ci, const double *av,
                      int32_t kmax, int32_t s, double eps, double tau, int32_t nrows,
                      const int32_t *rows, int32_t mmax, int32_t *m_out, int32_t *cols_out,
                      double *vals_out, double *psi_out, int32_t *steps_out, int32_t *reason_out,
                      int32_t nthreads)
{
    if (n <= 0 || kmax < 0 || (kmax > 0 && s < 1) || s > 64 || eps < 0.0 || !(tau >= 0.0 && tau < 1.0) ||
        mmax < 1 + kmax * s || nrows < 0)
        return OR_ERR_INVALID_ARG;
    int32_t maxlen = 1;
    for (int32_t r = 0; r < n; ++r)
        if (rp[r + 1] - rp[r] > maxlen) maxlen = rp[r + 1] - rp[r];
    int32_t *status = (int32_t *)calloc((size_t)(nrows > 0 ? nrows : 1), sizeof(int32_t));
    if (!status) return OR_ERR_NO_MEMORY;
    int nomem = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
#pragma omp parallel num_threads(nthreads)
    {
        work_t w;
        w.v = (double *)malloc(sizeof(double) * (size_t)n);
        w.mark = (char *)calloc((size_t)n, 1);
        /* distinct touched columns per step: at most n, and at most mmax full rows */
        size_t cap = (size_t)mmax * (size_t)maxlen;
        if (cap > (size_t)n) cap = (size_t)n;
        w.touched = (int32_t *)malloc(sizeof(int32_t) * cap);
        w.elig = (int32_t *)malloc(sizeof(int32_t) * cap);
        w.B = (double *)malloc(sizeof(double) * (size_t)mmax * mmax);
        w.L = (double *)malloc(sizeof(double) * (size_t)mmax * mmax);
        w.dinv = (double *)malloc(sizeof(double) * (size_t)mmax);
        w.P = (int32_t *)malloc(sizeof(int32_t) * (size_t)mmax);
        w.g = (double *)malloc(sizeof(double) * (size_t)mmax);
        double *psi = (double *)malloc(sizeof(double) * (size_t)(kmax + 1));
        if (!w.v || !w.mark || !w.touched || !w.elig || !w.B || !w.L || !w.dinv || !w.P || !w.g || !psi) {
#pragma omp atomic write
            nomem = 1;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int32_t q = 0; q < nrows; ++q) {
                int32_t i = rows ? rows[q] : q;
                if (i < 0 || i >= n) { status[q] = OR_ERR_INVALID_ARG; continue; }
                for (int32_t k = 0; k <= kmax; ++k) psi[k] = NAN;
                int32_t m = 0, st = 0, rs = 0;
                int rc = afsai_row(i, rp, ci, av, kmax, s, eps, tau, &w, cols_out + (size_t)q * mmax,
                                   vals_out + (size_t)q * mmax, &m, psi, &st, &rs);
                status[q] = rc;
                m_out[q] = m;
                if (steps_out) steps_out[q] = st;
                if (reason_out) reason_out[q] = rs;
                if (psi_out) memcpy(psi_out + (size_t)q * (kmax + 1), psi, sizeof(double) * (size_t)(kmax + 1));
            }
        }
        free(w.v); free(w.mark); free(w.touched); free(w.elig); free(w.B); free(w.L);
        free(w.dinv); free(w.P); free(w.g); free(psi);
    }
    int rc = nomem ? OR_ERR_NO_MEMORY : OR_OK;
    for (int32_t q = 0; q < nrows && rc == OR_OK; ++q)
        if (status[q] != OR_OK) rc = status[q];
    free(status);
    return rc;
}

/* threads of the parallel loops started afterwards by the calling thread (the products and
 * the setup without an explicit count); no effect on any result */
void oracle_set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* y = A x: each row summed in ascending column order */
void oracle_spmv(int32_t n, const int32_t *rp, const int32_t *ci, const double *av,
                 const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) acc = acc + av[e] * x[ci[e]];
        y[i] = acc;
    }
}

/* y = A^T x by scattering row after row (row index ascending) */
void oracle_spmv_t(int32_t n, const int32_t *rp, const int32_t *ci, const double *av,
                   const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) y[i] = 0.0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) y[ci[e]] = y[ci[e]] + av[e] * x[i];
}

/* z = G^T (G r), the preconditioner application M^-1 r (eq. prec); t is scratch */
void oracle_apply(int32_t n, const int32_t *grp, const int32_t *gci, const double *gv,
                  const double *r, double *z, double *t)
{
    oracle_spmv(n, grp, gci, gv, r, t);
    oracle_spmv_t(n, grp, gci, gv, t, z);
}

static double dot(int32_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int32_t i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
}

/*
 * Preconditioned conjugate gradient with M^-1 = G^T G (G == NULL: M = I, plain CG).
 * x holds x0 on entry and the last iterate on return.  Stops when ||r_k|| <= rtol ||b||.
 * res_hist (optional, maxit+1 entries) receives ||r_k|| / ||b|| for k = 0..iters.
 */
int oracle_pcg(int32_t n, const int32_t *rp, const int32_t *ci, const double *av,
               const int32_t *grp, const int32_t *gci, const double *gv, const double *b,
               double *x, double rtol, int32_t maxit, int32_t *iters_out, double *relres_out,
               double *true_relres_out, double *res_hist)
{
    if (n <= 0 || !(rtol > 0.0) || maxit < 0) return OR_ERR_INVALID_ARG;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !p || !q || !t) {
        free(r); free(z); free(p); free(q); free(t);
        return OR_ERR_NO_MEMORY;
    }
    int rc = OR_ERR_NOT_CONVERGED;
    int32_t it = 0;
    double nb = sqrt(dot(n, b, b));
    double rn = 0.0;
    if (nb == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        rc = OR_OK;
        if (res_hist) res_hist[0] = 0.0;
        goto done;
    }
    oracle_spmv(n, rp, ci, av, x, q);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    rn = sqrt(dot(n, r, r));
    if (res_hist) res_hist[0] = rn / nb;
    if (rn <= rtol * nb) { rc = OR_OK; goto done; }
    if (grp) oracle_apply(n, grp, gci, gv, r, z, t);
    else memcpy(z, r, sizeof(double) * (size_t)n);
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rho = dot(n, r, z);
    for (it = 1; it <= maxit; ++it) {
        oracle_spmv(n, rp, ci, av, p, q);
        double sigma = dot(n, p, q);
        if (!(sigma > 0.0)) { rc = OR_ERR_NOT_SPD; break; }
        double alpha = rho / sigma;
        for (int32_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        rn = sqrt(dot(n, r, r));
        if (res_hist) res_hist[it] = rn / nb;
        if (rn <= rtol * nb) { rc = OR_OK; break; }
        if (grp) oracle_apply(n, grp, gci, gv, r, z, t);
        else memcpy(z, r, sizeof(double) * (size_t)n);
        double rho1 = dot(n, r, z);
        double beta = rho1 / rho;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho1;
    }
    if (it > maxit) it = maxit;
done:
    if (iters_out) *iters_out = it;
    if (relres_out) *relres_out = (nb == 0.0) ? 0.0 : rn / nb;
    if (true_relres_out) {
        if (nb == 0.0) *true_relres_out = 0.0;
        else {
            oracle_spmv(n, rp, ci, av, x, q);
            for (int32_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
            *true_relres_out = sqrt(dot(n, q, q)) / nb;
        }
    }
    free(r); free(z); free(p); free(q); free(t);
    return rc;
}
