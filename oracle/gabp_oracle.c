/*
 * FP64 CPU oracle for the GaBP SVM solver -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain C + OpenMP.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * does, and the two share no code.
 *
 * Bickson, Yom-Tov, Dolev, "A Gaussian Belief Propagation Solver for Large
 * Scale Support Vector Machines" (arXiv 0810.1648):
 *   - D_ij = y_i y_j K(x_i, x_j)                  (eq. dual)
 *   - RBF kernel; bias by augmenting with lambda   (section "Proposed
 *     Solution of SVM Solver Based on GaBP"), read as K' = K + lambda^2
 *   - diagonal weighted to dominance; 2-norm soft margin adds 1/C
 *     (subsection "GaBP Algorithm Convergence")
 *   - Algorithm 2 (broadcast aggregates, message = aggregate minus the
 *     recipient's own term), synchronous rounds (section "Experimental
 *     Results"), messages in information form E_ij = P_ij mu_ij.
 *
 * Layout: incoming-message matrices Pin[j*N + i] = P_{i->j} and
 * Ein[j*N + i] = E_{i->j}, so that node j's aggregate is a contiguous row
 * sum.  Each unordered pair {i, j} is updated by one loop iteration from
 * the previous sweep's values, so the schedule is synchronous.  Aggregates
 * are Neumaier-compensated sums in index order: results do not depend on
 * the number of threads.
 *
 * Pinned by tests/test_oracle_pins.py (closed forms for N = 1, 2, the
 * first sweep, tree exactness, LAPACK Cholesky, divergence).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

enum { OR_DIAG_NONE = 0, OR_DIAG_SOFTMARGIN = 1, OR_DIAG_DOMINANT_ROW = 2,
       OR_DIAG_DOMINANT_UNIFORM = 3 };
enum { OR_CONVERGED = 0, OR_NOT_CONVERGED = 3, OR_DIVERGED = 4, OR_NOMEM = 2,
       OR_INVALID = 1 };

typedef struct { double s, c; } nsum_t;

static inline void nsum_add(nsum_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nsum_get(const nsum_t *a) { return a->s + a->c; }

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* K'_ij = exp(-gamma ||x_i - x_j||^2) + lam^2 for j = 0..N-1 (direct
 * differences in FP64 from the float32 features). */
void oracle_kernel_row(const float *X, int64_t N, int64_t m, double gamma,
                       double lam, int64_t i, double *out)
{
    const float *xi = X + i * m;
    for (int64_t j = 0; j < N; ++j) {
        const float *xj = X + j * m;
        double d2 = 0.0;
        for (int64_t k = 0; k < m; ++k) {
            double d = (double)xi[k] - (double)xj[k];
            d2 += d * d;
        }
        out[j] = exp(-gamma * d2) + lam * lam;
    }
}

/* Weighted diagonal entry from D_ii and r_i = sum_{j != i} |D_ij|. */
static double diag_rule(int mode, double dii, double r, double C, double delta)
{
    double soft = dii + 1.0 / C;
    double dom = (1.0 + delta) * r;
    switch (mode) {
    case OR_DIAG_NONE: return dii;
    case OR_DIAG_SOFTMARGIN: return soft;
    default: return soft > dom ? soft : dom;
    }
}

/* Synchronous GaBP (Algorithm 2, information form) on a dense symmetric A
 * given as its full N*N row-major array.  b is the right-hand side.
 * Outputs alpha (N), ptilde (N), deltas (max_sweeps), *sweeps.
 * Returns OR_CONVERGED / OR_NOT_CONVERGED / OR_DIVERGED / OR_NOMEM. */
static int gabp_run(const double *A, const double *b, int64_t N,
                    int max_sweeps, double tol_abs, double tol_rel,
                    double *alpha, double *Pt, double *deltas, int *sweeps,
                    double *sweep_seconds)
{
    size_t nn = (size_t)N * (size_t)N;
    double *Pin = calloc(nn, sizeof(double));
    double *Ein = calloc(nn, sizeof(double));
    double *S = malloc((size_t)N * sizeof(double));
    if (!Pin || !Ein || !S) { free(Pin); free(Ein); free(S); return OR_NOMEM; }

    for (int64_t i = 0; i < N; ++i) {
        Pt[i] = A[(size_t)i * N + i];
        S[i] = b[i];
        alpha[i] = S[i] / Pt[i];
    }
    int status = OR_NOT_CONVERGED;
    int t;
    double t0 = omp_get_wtime();
    *sweeps = 0;
    for (t = 1; t <= max_sweeps; ++t) {
        int bad = 0;
        /* internal scalars of every pair from the previous sweep */
#pragma omp parallel for schedule(dynamic, 8) reduction(| : bad)
        for (int64_t i = 0; i < N; ++i) {
            for (int64_t j = i + 1; j < N; ++j) {
                double a = A[(size_t)i * N + j];
                double pij = Pin[(size_t)j * N + i], pji = Pin[(size_t)i * N + j];
                double eij = Ein[(size_t)j * N + i], eji = Ein[(size_t)i * N + j];
                double qij = Pt[i] - pji;     /* P_{i\j} = P~_i - P_ji */
                double qji = Pt[j] - pij;
                if (!(qij > 0.0) || !(qji > 0.0) || !isfinite(qij) || !isfinite(qji))
                    bad = 1;
                Pin[(size_t)j * N + i] = -a * a / qij;
                Ein[(size_t)j * N + i] = -a * (S[i] - eji) / qij;
                Pin[(size_t)i * N + j] = -a * a / qji;
                Ein[(size_t)i * N + j] = -a * (S[j] - eij) / qji;
            }
        }
        if (bad) { status = OR_DIVERGED; break; }
        /* broadcast aggregates */
        double dmax = 0.0, amax = 0.0;
#pragma omp parallel for schedule(static) reduction(max : dmax, amax) reduction(| : bad)
        for (int64_t j = 0; j < N; ++j) {
            nsum_t sp = {0.0, 0.0}, se = {0.0, 0.0};
            nsum_add(&sp, A[(size_t)j * N + j]);
            nsum_add(&se, b[j]);
            const double *pr = Pin + (size_t)j * N, *er = Ein + (size_t)j * N;
            for (int64_t i = 0; i < N; ++i) {
                if (i == j) continue;
                nsum_add(&sp, pr[i]);
                nsum_add(&se, er[i]);
            }
            double p = nsum_get(&sp), s = nsum_get(&se);
            if (!(p > 0.0) || !isfinite(p) || !isfinite(s)) bad = 1;
            Pt[j] = p;
            S[j] = s;
            double an = s / p;
            double d = fabs(an - alpha[j]);
            alpha[j] = an;
            if (d > dmax) dmax = d;
            if (fabs(an) > amax) amax = fabs(an);
        }
        *sweeps = t;
        if (bad) { status = OR_DIVERGED; break; }
        if (deltas) deltas[t - 1] = dmax;
        if (dmax <= tol_abs + tol_rel * amax) { status = OR_CONVERGED; break; }
    }
    if (sweep_seconds) *sweep_seconds = omp_get_wtime() - t0;
    free(Pin); free(Ein); free(S);
    return status;
}

/* GaBP on an explicit matrix (pins: trees, equicorrelated systems, N = 2). */
int oracle_matrix_solve(const double *A, const double *b, int64_t N,
                        int max_sweeps, double tol_abs, double tol_rel,
                        double *alpha, double *ptilde, double *deltas,
                        int *sweeps)
{
    if (N < 1) return OR_INVALID;
    return gabp_run(A, b, N, max_sweeps, tol_abs, tol_rel, alpha, ptilde,
                    deltas, sweeps, NULL);
}

/* Builds A = weighted(Y K' Y) as a dense FP64 matrix. */
static double *build_svm_matrix(const float *X, const float *y, int64_t N,
                                int64_t m, double gamma, double C, double lam,
                                int diag_mode, double delta)
{
    double *A = malloc((size_t)N * (size_t)N * sizeof(double));
    if (!A) return NULL;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        double *row = A + (size_t)i * N;
        oracle_kernel_row(X, N, m, gamma, lam, i, row);
        for (int64_t j = 0; j < N; ++j) row[j] *= (double)y[i] * (double)y[j];
    }
    double *w = malloc((size_t)N * sizeof(double));
    if (!w) { free(A); return NULL; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        const double *row = A + (size_t)i * N;
        nsum_t r = {0.0, 0.0};
        for (int64_t j = 0; j < N; ++j)
            if (j != i) nsum_add(&r, fabs(row[j]));
        w[i] = diag_rule(diag_mode, row[i], nsum_get(&r), C, delta);
    }
    if (diag_mode == OR_DIAG_DOMINANT_UNIFORM) {
        double shift = -INFINITY;
        for (int64_t i = 0; i < N; ++i) {
            double s = w[i] - A[(size_t)i * N + i];
            if (s > shift) shift = s;
        }
        for (int64_t i = 0; i < N; ++i) w[i] = A[(size_t)i * N + i] + shift;
    }
    for (int64_t i = 0; i < N; ++i) A[(size_t)i * N + i] = w[i];
    free(w);
    return A;
}

/* Full SVM solve: alpha solves A alpha = 1 with A = weighted(Y K' Y).
 * adiag receives the weighted diagonal; timing[0] = system build seconds,
 * timing[1] = sweep-loop seconds. */
int oracle_svm_solve(const float *X, const float *y, int64_t N, int64_t m,
                     double gamma, double C, double lam, int diag_mode,
                     double delta, int max_sweeps, double tol_abs,
                     double tol_rel, double *alpha, double *ptilde,
                     double *adiag, double *deltas, int *sweeps,
                     double *timing)
{
    if (N < 1 || m < 1 || !(gamma > 0) || !(C > 0)) return OR_INVALID;
    double t0 = omp_get_wtime();
    double *A = build_svm_matrix(X, y, N, m, gamma, C, lam, diag_mode, delta);
    if (!A) return OR_NOMEM;
    double t1 = omp_get_wtime();
    if (adiag)
        for (int64_t i = 0; i < N; ++i) adiag[i] = A[(size_t)i * N + i];
    double *b = malloc((size_t)N * sizeof(double));
    if (!b) { free(A); return OR_NOMEM; }
    for (int64_t i = 0; i < N; ++i) b[i] = 1.0;
    double sweep_s = 0.0;
    int st = gabp_run(A, b, N, max_sweeps, tol_abs, tol_rel, alpha, ptilde,
                      deltas, sweeps, &sweep_s);
    if (timing) { timing[0] = t1 - t0; timing[1] = sweep_s; }
    free(b);
    free(A);
    return st;
}

/* Residual rows (1 - A alpha)_i for the rows listed in `rows`, computed one
 * row at a time from the features (O(N m) per row), plus the weighted
 * diagonal entry A_ii of each listed row.  Not defined for the uniform
 * diagonal rule, whose shift depends on every row. */
int oracle_svm_residual_rows(const float *X, const float *y, int64_t N,
                             int64_t m, double gamma, double C, double lam,
                             int diag_mode, double delta, const double *alpha,
                             const int64_t *rows, int64_t nrows,
                             double *resid, double *adiag_rows)
{
    if (diag_mode == OR_DIAG_DOMINANT_UNIFORM) return OR_INVALID;
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        double *row = malloc((size_t)N * sizeof(double));
        if (!row) err = 1;
        else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t r = 0; r < nrows; ++r) {
                int64_t i = rows[r];
                oracle_kernel_row(X, N, m, gamma, lam, i, row);
                nsum_t rs = {0.0, 0.0}, acc = {0.0, 0.0};
                for (int64_t j = 0; j < N; ++j) {
                    if (j == i) continue;
                    double dij = (double)y[i] * (double)y[j] * row[j];
                    nsum_add(&rs, fabs(dij));
                    nsum_add(&acc, dij * alpha[j]);
                }
                double aii = diag_rule(diag_mode, row[i], nsum_get(&rs), C, delta);
                nsum_add(&acc, aii * alpha[i]);
                resid[r] = 1.0 - nsum_get(&acc);
                if (adiag_rows) adiag_rows[r] = aii;
            }
            free(row);
        }
    }
    return err ? OR_NOMEM : OR_CONVERGED;
}

/* Times `nsweeps` synchronous sweeps of the solver on the first N points
 * (system build excluded).  Returns the sweep-loop seconds through *secs
 * and the number of threads used through *threads. */
int oracle_time_sweeps(const float *X, const float *y, int64_t N, int64_t m,
                       double gamma, double C, double lam, int diag_mode,
                       double delta, int nsweeps, double *secs, int *threads)
{
    double *A = build_svm_matrix(X, y, N, m, gamma, C, lam, diag_mode, delta);
    if (!A) return OR_NOMEM;
    double *b = malloc((size_t)N * sizeof(double));
    double *alpha = malloc((size_t)N * sizeof(double));
    double *pt = malloc((size_t)N * sizeof(double));
    if (!b || !alpha || !pt) { free(A); free(b); free(alpha); free(pt); return OR_NOMEM; }
    for (int64_t i = 0; i < N; ++i) b[i] = 1.0;
    int sw = 0;
    int st = gabp_run(A, b, N, nsweeps, 0.0, 0.0, alpha, pt, NULL, &sw, secs);
    *threads = omp_get_max_threads();
    free(A); free(b); free(alpha); free(pt);
    return st;
}
