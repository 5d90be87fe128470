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
 * Large systems (the 100k and 300k point workloads) never form A: the
 * matrix-free product A v recomputes every kernel row from the features
 * (feeding the conjugate-gradient reference solution alpha* = A^-1 1 and the
 * residual certificate), and the stateless sweep rebuilds each message from
 * the aggregate history by unrolling the message recursion, one target row
 * at a time.
 *
 * Pinned by tests/test_oracle_pins.py (closed forms for N = 1, 2, the
 * first sweep, tree exactness, LAPACK Cholesky, divergence, the dense
 * product A v, the stored-state sweep for the stateless form).
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

/* ------------------------------------------------------------------------
 * Matrix-free forms for large N
 * ------------------------------------------------------------------------ */

/* Features transposed to XT[k*N + j], so that one kernel row is built with
 * the point index innermost.  The distance of each pair is still summed over
 * k = 0..m-1 in order, as in oracle_kernel_row, so the entries are the same
 * bit for bit. */
static float *transpose_features(const float *X, int64_t N, int64_t m)
{
    float *XT = malloc((size_t)N * (size_t)m * sizeof(float));
    if (!XT) return NULL;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j)
        for (int64_t k = 0; k < m; ++k) XT[(size_t)k * N + j] = X[(size_t)j * m + k];
    return XT;
}

/* Row i of A = weighted(Y K' Y) from the features, into row[0..N): the
 * off-diagonal entries y_i y_j K'_ij and, at j = i, the weighted diagonal
 * A_ii of the rule (which needs r_i = sum_{j != i} |A_ij|, formed here by a
 * compensated sum in index order).  Not defined for the uniform rule. */
static double svm_row(const float *XT, const float *X, const float *y, int64_t N,
                      int64_t m, double gamma, double C, double lam,
                      int diag_mode, double delta, int64_t i, double *row)
{
    const float *xi = X + (size_t)i * m;
    for (int64_t j = 0; j < N; ++j) row[j] = 0.0;
    for (int64_t k = 0; k < m; ++k) {
        const double xk = (double)xi[k];
        const float *col = XT + (size_t)k * N;
        for (int64_t j = 0; j < N; ++j) {
            double d = xk - (double)col[j];
            row[j] += d * d;
        }
    }
    for (int64_t j = 0; j < N; ++j)
        row[j] = (exp(-gamma * row[j]) + lam * lam) * ((double)y[i] * (double)y[j]);
    nsum_t r = {0.0, 0.0};
    for (int64_t j = 0; j < N; ++j)
        if (j != i) nsum_add(&r, fabs(row[j]));
    const double aii = diag_rule(diag_mode, row[i], nsum_get(&r), C, delta);
    row[i] = aii;
    return aii;
}

/* out = A v without forming A (each row rebuilt from the features and
 * summed with compensation in index order); adiag (optional) receives the
 * weighted diagonal.  O(N^2 m) work, O(N) memory per thread. */
int oracle_svm_matvec(const float *X, const float *y, int64_t N, int64_t m,
                      double gamma, double C, double lam, int diag_mode,
                      double delta, const double *v, double *out,
                      double *adiag)
{
    if (N < 1 || m < 1 || diag_mode == OR_DIAG_DOMINANT_UNIFORM) return OR_INVALID;
    float *XT = transpose_features(X, N, m);
    if (!XT) return OR_NOMEM;
    int err = 0;
#pragma omp parallel reduction(| : err)
    {
        double *row = malloc((size_t)N * sizeof(double));
        if (!row) err = 1;
        else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t i = 0; i < N; ++i) {
                const double aii = svm_row(XT, X, y, N, m, gamma, C, lam, diag_mode,
                                           delta, i, row);
                nsum_t acc = {0.0, 0.0};
                for (int64_t j = 0; j < N; ++j) nsum_add(&acc, row[j] * v[j]);
                out[i] = nsum_get(&acc);
                if (adiag) adiag[i] = aii;
            }
            free(row);
        }
    }
    free(XT);
    return err ? OR_NOMEM : OR_CONVERGED;
}

/* Aggregates of target node j after sweep t of the stateless form, from the
 * aggregate history hP[s], hS[s] (sweeps s = 0 .. t-1, every node) and row j
 * of A (arow[i] = A_ij).  The message i -> j of sweep t depends on stored
 * state only through the reverse message j -> i of sweep t-1, which depends
 * on i -> j of sweep t-2, and so on: the chain is unrolled from sweep
 * lo = max(1, t - depth + 1), whose reverse message is taken as zero (exact
 * while t <= depth, since the messages of sweep 0 are zero).  Level s is the
 * message of sweep s, sent by i when t - s is even and by j otherwise:
 * P = -a^2 / (P~_src^(s-1) - P_rev), E = -a (S_src^(s-1) - E_rev) / (same).
 * Returns nonzero if some cavity precision is <= 0 or not finite. */
static int stateless_target(const double *arow, int64_t N, int64_t j, double ajj,
                            double bj, const double *const *hP,
                            const double *const *hS, int t, int depth,
                            double *Pt_out, double *S_out)
{
    int lo = t - depth + 1;
    if (lo < 1) lo = 1;
    int bad = 0;
    nsum_t sp = {0.0, 0.0}, se = {0.0, 0.0};
    nsum_add(&sp, ajj);
    nsum_add(&se, bj);
    for (int64_t i = 0; i < N; ++i) {
        if (i == j) continue;
        const double a = arow[i];
        double P = 0.0, E = 0.0;
        for (int s = lo; s <= t; ++s) {
            const int64_t src = ((t - s) % 2 == 0) ? i : j;
            const double q = hP[s - 1][src] - P;
            if (!(q > 0.0) || !isfinite(q)) bad = 1;
            const double Pn = -a * a / q;
            const double En = -a * (hS[s - 1][src] - E) / q;
            P = Pn;
            E = En;
        }
        nsum_add(&sp, P);
        nsum_add(&se, E);
    }
    *Pt_out = nsum_get(&sp);
    *S_out = nsum_get(&se);
    return bad;
}

/* Synchronous GaBP with stateless messages on an explicit matrix A (N*N,
 * row-major, symmetric): `sweeps` sweeps at unroll depth `depth`.  alpha_traj
 * receives alpha^1 .. alpha^sweeps (sweeps*N), ptilde the last P~.  For
 * t <= depth the trajectory equals the stored-state sweep (oracle_matrix_solve)
 * bit for bit.  Returns OR_CONVERGED (all sweeps done), OR_DIVERGED or
 * OR_NOMEM. */
int oracle_stateless_matrix(const double *A, const double *b, int64_t N, int depth,
                            int sweeps, double *alpha_traj, double *ptilde)
{
    if (N < 1 || depth < 1 || sweeps < 1) return OR_INVALID;
    double *hist = malloc((size_t)2 * (size_t)(sweeps + 1) * (size_t)N * sizeof(double));
    const double **hP = malloc((size_t)(sweeps + 1) * sizeof(double *));
    const double **hS = malloc((size_t)(sweeps + 1) * sizeof(double *));
    if (!hist || !hP || !hS) { free(hist); free(hP); free(hS); return OR_NOMEM; }
    for (int s = 0; s <= sweeps; ++s) {
        hP[s] = hist + (size_t)(2 * s) * N;
        hS[s] = hist + (size_t)(2 * s + 1) * N;
    }
    for (int64_t i = 0; i < N; ++i) {
        ((double *)hP[0])[i] = A[(size_t)i * N + i];
        ((double *)hS[0])[i] = b[i];
    }
    int status = OR_CONVERGED;
    for (int t = 1; t <= sweeps && status == OR_CONVERGED; ++t) {
        double *nP = (double *)hP[t], *nS = (double *)hS[t];
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (int64_t j = 0; j < N; ++j) {
            bad |= stateless_target(A + (size_t)j * N, N, j, A[(size_t)j * N + j], b[j],
                                    hP, hS, t, depth, &nP[j], &nS[j]);
            if (!(nP[j] > 0.0) || !isfinite(nP[j]) || !isfinite(nS[j])) bad = 1;
        }
        for (int64_t j = 0; j < N; ++j) alpha_traj[(size_t)(t - 1) * N + j] = nS[j] / nP[j];
        if (bad) status = OR_DIVERGED;
        if (ptilde) for (int64_t j = 0; j < N; ++j) ptilde[j] = nP[j];
    }
    free(hist); free(hP); free(hS);
    return status;
}

/* One stateless sweep t (unroll depth `depth`) of the SVM system for the
 * listed target rows only, every row of A rebuilt from the features: the
 * per-node work of a sweep at the full N.  hist_P / hist_S hold the
 * aggregates of sweeps 0 .. t-1 for every node ([t][N]); adiag is the
 * weighted diagonal (the sweep-0 precisions).  outP / outS receive P~^t and
 * S^t of the listed rows; *secs the wall time of the row loop (the features
 * are transposed before it).  Returns OR_DIVERGED if a cavity precision is
 * <= 0, else OR_CONVERGED. */
int oracle_stateless_rows(const float *X, const float *y, int64_t N, int64_t m,
                          double gamma, double lam, const double *adiag,
                          const double *hist_P, const double *hist_S, int t,
                          int depth, const int64_t *rows, int64_t nrows,
                          double *outP, double *outS, double *secs)
{
    if (N < 1 || m < 1 || t < 1 || depth < 1) return OR_INVALID;
    float *XT = transpose_features(X, N, m);
    const double **hP = malloc((size_t)t * sizeof(double *));
    const double **hS = malloc((size_t)t * sizeof(double *));
    if (!XT || !hP || !hS) { free(XT); free(hP); free(hS); return OR_NOMEM; }
    for (int s = 0; s < t; ++s) {
        hP[s] = hist_P + (size_t)s * N;
        hS[s] = hist_S + (size_t)s * N;
    }
    int bad = 0, err = 0;
    const double t0 = omp_get_wtime();
#pragma omp parallel reduction(| : bad, err)
    {
        double *row = malloc((size_t)N * sizeof(double));
        if (!row) err = 1;
        else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t r = 0; r < nrows; ++r) {
                const int64_t j = rows[r];
                const float *xj = X + (size_t)j * m;
                for (int64_t i = 0; i < N; ++i) row[i] = 0.0;
                for (int64_t k = 0; k < m; ++k) {
                    const double xk = (double)xj[k];
                    const float *col = XT + (size_t)k * N;
                    for (int64_t i = 0; i < N; ++i) {
                        double d = xk - (double)col[i];
                        row[i] += d * d;
                    }
                }
                for (int64_t i = 0; i < N; ++i)
                    row[i] = (exp(-gamma * row[i]) + lam * lam) * ((double)y[j] * (double)y[i]);
                bad |= stateless_target(row, N, j, adiag[j], 1.0, hP, hS, t, depth,
                                        &outP[r], &outS[r]);
            }
            free(row);
        }
    }
    if (secs) *secs = omp_get_wtime() - t0;
    free(XT); free(hP); free(hS);
    if (err) return OR_NOMEM;
    return bad ? OR_DIVERGED : OR_CONVERGED;
}

/* Sets the OpenMP thread count of later calls (timing at 1 thread and at all
 * threads). */
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
