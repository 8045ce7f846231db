/*
 * Plain binary64 CPU reference for the dense Krylov solvers.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * Everything is written for a reader to check against the paper by eye:
 * straight loops in the order the algorithms state, no blocking, no fusion.
 * The only concession to speed is an OpenMP "parallel for" over the rows of
 * the dense matrix-vector product; each row's sum is still the plain
 * left-to-right loop, so the result does not depend on the thread count.
 *
 * Matrices are row-major: element (i, j) of A is A[i * lda + j].
 *
 * Status codes: 0 converged, 1 iteration limit, 2 breakdown, 3 stagnation,
 * 4 non-finite value met, -1 invalid argument.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KO_OK 0
#define KO_MAXITER 1
#define KO_BREAKDOWN 2
#define KO_STAGNATED 3
#define KO_NONFINITE 4
#define KO_EINVAL (-1)

/* CG is restarted from its current iterate when the recursive residual says
 * "converged" but the true residual b - A x does not; after this many
 * restarts without meeting the tolerance the solve reports stagnation. */
#define KO_CG_MAX_RESTARTS 16

/* GMRES happy breakdown: h(k+1,k) <= this factor times ||A v(k)||. */
#define KO_HAPPY 1e-14

void ko_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int ko_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- BLAS-like */

/* inner product x'y, summed left to right */
double ko_dot(int n, const double *x, const double *y) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

double ko_nrm2(int n, const double *x) { return sqrt(ko_dot(n, x, x)); }

/* y = A x, one row at a time (the matrix-vector product of every Krylov step) */
void ko_matvec(int n, const double *A, long lda, const double *x, double *y) {
#pragma omp parallel for schedule(static) if (n >= 256)
    for (int i = 0; i < n; ++i) {
        const double *a = A + (long)i * lda;
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += a[j] * x[j];
        y[i] = s;
    }
}

/* y[k] = row rows[k] of A times x, k < m (sampled outputs of the product, for
 * checks at sizes where the whole product is too slow on the CPU) */
void ko_matvec_rows(int n, const double *A, long lda, const int *rows, int m, const double *x,
                    double *y) {
    for (int k = 0; k < m; ++k) {
        const double *a = A + (long)rows[k] * lda;
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += a[j] * x[j];
        y[k] = s;
    }
}

/* r = b - A x */
void ko_residual(int n, const double *A, long lda, const double *b, const double *x,
                 double *r) {
#pragma omp parallel for schedule(static) if (n >= 256)
    for (int i = 0; i < n; ++i) {
        const double *a = A + (long)i * lda;
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += a[j] * x[j];
        r[i] = b[i] - s;
    }
}

/* ||A||_inf = max over rows of the row's absolute sum */
double ko_norm_inf_mat(int n, const double *A, long lda) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += fabs(A[(long)i * lda + j]);
        if (s > m) m = s;
    }
    return m;
}

static double norm_inf_vec(int n, const double *x) {
    double m = 0.0;
    for (int i = 0; i < n; ++i)
        if (fabs(x[i]) > m) m = fabs(x[i]);
    return m;
}

/* out[0] = ||b - A x||_2 / ||b||_2
 * out[1] = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)   (normwise
 *          backward error in the infinity norm, Rigal and Gaches)
 * out[2] = ||b - A x||_2
 * Returns 0, or -1 on bad arguments. */
int ko_metrics(int n, const double *A, long lda, const double *b, const double *x,
               double *out) {
    if (n <= 0 || !A || !b || !x || !out || lda < n) return KO_EINVAL;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r) return KO_EINVAL;
    ko_residual(n, A, lda, b, x, r);
    double rn = ko_nrm2(n, r), bn = ko_nrm2(n, b);
    out[0] = bn > 0.0 ? rn / bn : rn;
    double den = ko_norm_inf_mat(n, A, lda) * norm_inf_vec(n, x) + norm_inf_vec(n, b);
    double rinf = norm_inf_vec(n, r);
    out[1] = den > 0.0 ? rinf / den : rinf;
    out[2] = rn;
    free(r);
    return 0;
}

/* ------------------------------------------------------------ conjugate gradient
 *
 * Conjugate gradient for SPD A, Hestenes-Stiefel form (the method the paper
 * describes in prose in its Krylov section: one matrix-vector product per
 * iteration, A-orthogonal search directions, at most n steps in exact
 * arithmetic; full statement in Golub and Van Loan).
 *
 *   r = b - A x, p = r, rho = r'r
 *   repeat:  q = A p;  sigma = p'q  (sigma <= 0 means A is not SPD)
 *            alpha = rho / sigma;  x = x + alpha p;  r = r - alpha q
 *            rho' = r'r;  stop when sqrt(rho') <= tol ||b||
 *            p = r + (rho'/rho) p;  rho = rho'
 *
 * When the recursive residual meets the tolerance the true residual b - A x
 * is recomputed; if it does not meet it, CG starts again from the current x.
 * max_iter bounds the number of products q = A p.  hist (optional) receives
 * sqrt(rho') after every iteration.
 */
int ko_cg(int n, const double *A, long lda, const double *b, double *x, double tol,
          int max_iter, int *iters_out, int *restarts_out, double *rel_res_out,
          double *hist, int hist_cap) {
    if (n <= 0 || !A || !b || !x || lda < n || !(tol > 0.0) || max_iter < 0)
        return KO_EINVAL;
    int iters = 0, restarts = 0, status = KO_MAXITER;
    double bnorm = ko_nrm2(n, b), res = 0.0;
    if (!isfinite(bnorm)) {
        status = KO_NONFINITE;
        goto done_noalloc;
    }
    if (bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        status = KO_OK;
        goto done_noalloc;
    }
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !p || !q) {
        free(r); free(p); free(q);
        return KO_EINVAL;
    }
    int first = 1;
    for (;;) {
        ko_residual(n, A, lda, b, x, r);
        double rho = ko_dot(n, r, r);
        res = sqrt(rho);
        if (!isfinite(res)) { status = KO_NONFINITE; break; }
        if (res <= tol * bnorm) { status = KO_OK; break; }
        if (iters >= max_iter) { status = KO_MAXITER; break; }
        if (!first) {
            if (restarts >= KO_CG_MAX_RESTARTS) { status = KO_STAGNATED; break; }
            ++restarts;
        }
        first = 0;
        for (int i = 0; i < n; ++i) p[i] = r[i];
        int stop = 0;
        while (!stop) {
            ko_matvec(n, A, lda, p, q);
            ++iters;
            double sigma = ko_dot(n, p, q);
            if (!isfinite(sigma)) { status = KO_NONFINITE; stop = 2; break; }
            if (sigma <= 0.0) { status = KO_BREAKDOWN; stop = 2; break; }
            double alpha = rho / sigma;
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
            double rho_new = ko_dot(n, r, r);
            if (hist && iters <= hist_cap) hist[iters - 1] = sqrt(rho_new);
            if (!isfinite(rho_new)) { status = KO_NONFINITE; stop = 2; break; }
            if (sqrt(rho_new) <= tol * bnorm) stop = 1;
            else if (iters >= max_iter) stop = 1;
            else {
                double beta = rho_new / rho;
                for (int i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
                rho = rho_new;
            }
        }
        if (stop == 2) {
            /* breakdown / non-finite: report the true residual of the last x */
            ko_residual(n, A, lda, b, x, r);
            res = ko_nrm2(n, r);
            break;
        }
    }
    free(r); free(p); free(q);
done_noalloc:
    if (iters_out) *iters_out = iters;
    if (restarts_out) *restarts_out = restarts;
    if (rel_res_out) *rel_res_out = (bnorm > 0.0 && isfinite(bnorm)) ? res / bnorm : 0.0;
    return status;
}

/* ---------------------------------------------------------------- BiCGSTAB
 *
 * BiConjugate gradient stabilised (Krylov section, BiCGSTAB paragraph).  The
 * residual after k steps is r_k = psi_k(A) phi_k(A) r0, where phi_k is the
 * residual polynomial of BiCG (degree k, phi_k(0) = 1, phi_k(A) r0 orthogonal
 * to the shadow space spanned by r0h, A' r0h, ..., here with r0h = r0) and
 * psi_k(t) = (1 - omega_1 t) ... (1 - omega_k t) a product of local
 * minimal-residual factors.  The short recurrences that carry this, with
 * rho = r0h' r and p the BiCG direction multiplied by psi:
 *   v = A p;  alpha = rho / (r0h' v);  s = r - alpha v       (the BiCG step)
 *   t = A s;  omega = (t' s) / (t' t)                         (minimises ||s - omega t||)
 *   x = x + alpha p + omega s;  r = s - omega t
 *   rho' = r0h' r;  beta = (rho' / rho)(alpha / omega);  p = r + beta (p - omega v)
 * starting from p = r = b - A x.  The paper's ω line reads as the quotient
 * above (it prints a product), and it omits the r and rho updates, which are
 * restored.  If ||s|| already meets the tolerance, or the product budget
 * ends after v = A p, the half step x = x + alpha p ends the pass.  Stop on
 * ||r||_2 <= tol ||b||_2 (recursive), confirmed on the true residual (a new
 * pass from x, with r0h the new residual, if it fails).  max_iter bounds the
 * number of products with A (two per step).  Breakdown: rho, r0h'v or t't
 * equal to 0, or omega = 0.
 */
int ko_bicgstab(int n, const double *A, long lda, const double *b, double *x, double tol,
                int max_iter, int *iters_out, int *restarts_out, double *rel_res_out) {
    if (n <= 0 || !A || !b || !x || lda < n || !(tol > 0.0) || max_iter < 0) return KO_EINVAL;
    int prods = 0, restarts = 0, status = KO_MAXITER, first = 1;
    double bnorm = ko_nrm2(n, b), res = 0.0;
    if (!isfinite(bnorm)) {
        if (iters_out) *iters_out = 0;
        if (restarts_out) *restarts_out = 0;
        if (rel_res_out) *rel_res_out = 0.0;
        return KO_NONFINITE;
    }
    if (bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        if (iters_out) *iters_out = 0;
        if (restarts_out) *restarts_out = 0;
        if (rel_res_out) *rel_res_out = 0.0;
        return KO_OK;
    }
    size_t nn = (size_t)n;
    double *r = (double *)malloc(sizeof(double) * nn), *r0h = (double *)malloc(sizeof(double) * nn);
    double *p = (double *)malloc(sizeof(double) * nn), *v = (double *)malloc(sizeof(double) * nn);
    double *sv = (double *)malloc(sizeof(double) * nn), *t = (double *)malloc(sizeof(double) * nn);
    if (!r || !r0h || !p || !v || !sv || !t) {
        status = KO_EINVAL;
        goto out;
    }
    for (;;) {
        ko_residual(n, A, lda, b, x, r);
        res = ko_nrm2(n, r);
        if (!isfinite(res)) { status = KO_NONFINITE; break; }
        if (res <= tol * bnorm) { status = KO_OK; break; }
        if (prods >= max_iter) { status = KO_MAXITER; break; }
        if (!first) {
            if (restarts >= KO_CG_MAX_RESTARTS) { status = KO_STAGNATED; break; }
            ++restarts;
        }
        first = 0;
        for (int i = 0; i < n; ++i) { r0h[i] = r[i]; p[i] = r[i]; }
        double rho = ko_dot(n, r0h, r);
        int stop = 0;
        while (!stop) {
            if (rho == 0.0 || !isfinite(rho)) { status = isfinite(rho) ? KO_BREAKDOWN : KO_NONFINITE; stop = 2; break; }
            /* BiCG step */
            ko_matvec(n, A, lda, p, v);
            ++prods;
            double r0v = ko_dot(n, r0h, v);
            if (r0v == 0.0 || !isfinite(r0v)) { status = isfinite(r0v) ? KO_BREAKDOWN : KO_NONFINITE; stop = 2; break; }
            double alpha = rho / r0v;
            for (int i = 0; i < n; ++i) sv[i] = r[i] - alpha * v[i];
            if (ko_nrm2(n, sv) <= tol * bnorm || prods >= max_iter) {
                /* half step: s already small enough, or no product left for A s */
                for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
                stop = 1;
                break;
            }
            /* minimal-residual step along t = A s */
            ko_matvec(n, A, lda, sv, t);
            ++prods;
            double tt = ko_dot(n, t, t);
            if (tt == 0.0 || !isfinite(tt)) { status = isfinite(tt) ? KO_BREAKDOWN : KO_NONFINITE; stop = 2; break; }
            double omega = ko_dot(n, t, sv) / tt;
            for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i] + omega * sv[i];
            for (int i = 0; i < n; ++i) r[i] = sv[i] - omega * t[i];
            if (ko_nrm2(n, r) <= tol * bnorm || prods >= max_iter) { stop = 1; break; }
            if (omega == 0.0) { status = KO_BREAKDOWN; stop = 2; break; }
            /* next direction */
            double rho_new = ko_dot(n, r0h, r);
            double beta = (rho_new / rho) * (alpha / omega);
            for (int i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
            rho = rho_new;
        }
        if (stop == 2) {
            ko_residual(n, A, lda, b, x, r);
            res = ko_nrm2(n, r);
            break;
        }
    }
out:
    free(r); free(r0h); free(p); free(v); free(sv); free(t);
    if (iters_out) *iters_out = prods;
    if (restarts_out) *restarts_out = restarts;
    if (rel_res_out) *rel_res_out = res / bnorm;
    return status;
}

/* ------------------------------------------------------- stationary methods
 *
 * Jacobi and Gauss-Seidel, the classical stationary iterations the paper
 * lists in its library beside the Krylov methods (introductory section and
 * the parallel-implementation section; timed in Tables 1-2).  The paper
 * defers their definition to the textbooks, so these are the textbook forms
 * with the splitting A = L + D + U (strictly lower, diagonal, strictly upper):
 *   Jacobi        D x(k+1) = b - (L + U) x(k)
 *   Gauss-Seidel  (D + L) x(k+1) = b - U x(k)   (one forward sweep, new values
 *                                                used as soon as computed)
 * Both test the true residual of x(k) before forming x(k+1):
 * ||b - A x(k)|| <= tol ||b|| stops with x(k); `iters` counts the updates
 * made.  A zero on the diagonal is a breakdown before any update.
 */

/* shared front end: ||b||, the b = 0 and zero-diagonal cases.  Returns -2 to
 * go on iterating, else the final status (x, counters set). */
static int stationary_start(int n, const double *A, long lda, const double *b, double *x,
                            double *bnorm, int *iters_out, double *rel_res_out) {
    *bnorm = ko_nrm2(n, b);
    if (iters_out) *iters_out = 0;
    if (rel_res_out) *rel_res_out = 0.0;
    if (!isfinite(*bnorm)) return KO_NONFINITE;
    if (*bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        return KO_OK;
    }
    for (int i = 0; i < n; ++i)
        if (A[(long)i * lda + i] == 0.0) return KO_BREAKDOWN;
    return -2;
}

int ko_jacobi(int n, const double *A, long lda, const double *b, double *x, double tol,
              int max_iter, int *iters_out, double *rel_res_out) {
    if (n <= 0 || !A || !b || !x || lda < n || !(tol > 0.0) || max_iter < 0) return KO_EINVAL;
    double bnorm;
    int status = stationary_start(n, A, lda, b, x, &bnorm, iters_out, rel_res_out);
    if (status != -2) return status;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *xn = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !xn) {
        free(r);
        free(xn);
        return KO_EINVAL;
    }
    int k = 0;
    double res = 0.0;
    for (;;) {
        ko_residual(n, A, lda, b, x, r);
        res = ko_nrm2(n, r);
        if (!isfinite(res)) { status = KO_NONFINITE; break; }
        if (res <= tol * bnorm) { status = KO_OK; break; }
        if (k >= max_iter) { status = KO_MAXITER; break; }
        /* x(k+1)_i = (b_i - sum_{j != i} a_ij x(k)_j) / a_ii, all from x(k) */
#pragma omp parallel for schedule(static) if (n >= 256)
        for (int i = 0; i < n; ++i) {
            const double *a = A + (long)i * lda;
            double s = b[i];
            for (int j = 0; j < n; ++j)
                if (j != i) s -= a[j] * x[j];
            xn[i] = s / a[i];
        }
        memcpy(x, xn, sizeof(double) * (size_t)n);
        ++k;
    }
    free(r);
    free(xn);
    if (iters_out) *iters_out = k;
    if (rel_res_out) *rel_res_out = res / bnorm;
    return status;
}

int ko_gauss_seidel(int n, const double *A, long lda, const double *b, double *x, double tol,
                    int max_iter, int *iters_out, double *rel_res_out) {
    if (n <= 0 || !A || !b || !x || lda < n || !(tol > 0.0) || max_iter < 0) return KO_EINVAL;
    double bnorm;
    int status = stationary_start(n, A, lda, b, x, &bnorm, iters_out, rel_res_out);
    if (status != -2) return status;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r) return KO_EINVAL;
    int k = 0;
    double res = 0.0;
    for (;;) {
        ko_residual(n, A, lda, b, x, r);
        res = ko_nrm2(n, r);
        if (!isfinite(res)) { status = KO_NONFINITE; break; }
        if (res <= tol * bnorm) { status = KO_OK; break; }
        if (k >= max_iter) { status = KO_MAXITER; break; }
        /* one forward sweep in place: x_j for j < i already holds x(k+1)_j */
        for (int i = 0; i < n; ++i) {
            const double *a = A + (long)i * lda;
            double s = b[i];
            for (int j = 0; j < n; ++j)
                if (j != i) s -= a[j] * x[j];
            x[i] = s / a[i];
        }
        ++k;
    }
    free(r);
    if (iters_out) *iters_out = k;
    if (rel_res_out) *rel_res_out = res / bnorm;
    return status;
}


/* ---------------------------------------------------------------- GMRES(m)
 *
 * Arnoldi step as the paper prints it: project A v(k) on every v(j), j <= k,
 * subtract, normalise by h(k+1,k) (the printed "v(k+1,k)" is read as
 * v(k+1)).  The oracle does the projection as modified Gram-Schmidt, twice
 * (every h(j,k) accumulates both passes); in exact arithmetic this is the
 * same H and V as the printed classical form.
 *
 * Least squares: the paper stops at the basis; the minimal-residual update
 * (Saad) is used: Givens rotations G_i = [c s; -s c] reduce H to upper
 * triangular R, with rho = hypot(a, b) >= 0, c = a/rho, s = b/rho, applied to
 * g = beta e1; |g(k+1)| is the residual estimate; at the end of a cycle
 * R y = g is back-substituted and x = x0 + V y.
 *
 * Restart after m steps from the current x (the paper's "intermediate
 * results as a new starting point"): r = b - A x is recomputed.  max_iter
 * bounds the total number of Arnoldi steps over all cycles.  est (optional)
 * receives |g(k+1)| after every step; cres (optional) the true residual norm
 * at the start of every cycle and at exit.
 */
int ko_gmres(int n, const double *A, long lda, const double *b, double *x, double tol,
             int max_iter, int m, int *iters_out, int *cycles_out, double *rel_res_out,
             double *est, int est_cap, double *cres, int cres_cap) {
    if (n <= 0 || !A || !b || !x || lda < n || !(tol > 0.0) || max_iter < 0 || m < 1)
        return KO_EINVAL;
    int steps = 0, cycles = 0, status = KO_MAXITER, ncres = 0;
    double bnorm = ko_nrm2(n, b), res = 0.0;
    if (!isfinite(bnorm)) {
        if (iters_out) *iters_out = 0;
        if (cycles_out) *cycles_out = 0;
        if (rel_res_out) *rel_res_out = 0.0;
        return KO_NONFINITE;
    }
    if (bnorm == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        if (iters_out) *iters_out = 0;
        if (cycles_out) *cycles_out = 0;
        if (rel_res_out) *rel_res_out = 0.0;
        return KO_OK;
    }
    size_t nn = (size_t)n;
    double *V = (double *)calloc(nn * (size_t)(m + 1), sizeof(double));
    double *w = (double *)malloc(sizeof(double) * nn);
    double *r = (double *)malloc(sizeof(double) * nn);
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double *R = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    double *sn = (double *)calloc((size_t)m, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *y = (double *)calloc((size_t)m, sizeof(double));
    if (!V || !w || !r || !H || !R || !cs || !sn || !g || !y) {
        status = KO_EINVAL;
        goto out;
    }
#define HH(i, j) H[(size_t)(i) * (size_t)m + (size_t)(j)]
#define RR(i, j) R[(size_t)(i) * (size_t)m + (size_t)(j)]
    for (;;) {
        ko_residual(n, A, lda, b, x, r);
        double beta = ko_nrm2(n, r);
        res = beta;
        if (cres && ncres < cres_cap) cres[ncres++] = beta;
        if (!isfinite(beta)) { status = KO_NONFINITE; break; }
        if (beta <= tol * bnorm) { status = KO_OK; break; }
        if (steps >= max_iter) { status = KO_MAXITER; break; }
        for (int i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int kd = 0, fail = 0;
        for (int k = 0; k < m; ++k) {
            const double *vk = V + (size_t)k * nn;
            ko_matvec(n, A, lda, vk, w);
            ++steps;
            double avk = ko_nrm2(n, w);
            for (int j = 0; j <= k; ++j) HH(j, k) = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int j = 0; j <= k; ++j) {
                    const double *vj = V + (size_t)j * nn;
                    double t = ko_dot(n, vj, w);
                    HH(j, k) += t;
                    for (int i = 0; i < n; ++i) w[i] = w[i] - t * vj[i];
                }
            }
            double hk1 = ko_nrm2(n, w);
            HH(k + 1, k) = hk1;
            for (int j = 0; j <= k + 1; ++j) RR(j, k) = HH(j, k);
            for (int i = 0; i < k; ++i) {
                double a = RR(i, k), bb = RR(i + 1, k);
                RR(i, k) = cs[i] * a + sn[i] * bb;
                RR(i + 1, k) = -sn[i] * a + cs[i] * bb;
            }
            double rho = hypot(RR(k, k), RR(k + 1, k));
            if (!isfinite(rho) || !isfinite(avk)) { status = KO_NONFINITE; fail = 1; break; }
            if (rho == 0.0) { status = KO_BREAKDOWN; fail = 1; break; }
            cs[k] = RR(k, k) / rho;
            sn[k] = RR(k + 1, k) / rho;
            RR(k, k) = rho;
            RR(k + 1, k) = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            kd = k + 1;
            if (est && steps <= est_cap) est[steps - 1] = fabs(g[k + 1]);
            if (hk1 <= KO_HAPPY * avk) break;                 /* happy breakdown */
            double *vn = V + (size_t)(k + 1) * nn;
            for (int i = 0; i < n; ++i) vn[i] = w[i] / hk1;
            if (fabs(g[k + 1]) <= tol * bnorm || steps >= max_iter) break;
        }
        if (kd > 0) {
            for (int i = kd - 1; i >= 0; --i) {
                double s = g[i];
                for (int j = i + 1; j < kd; ++j) s -= RR(i, j) * y[j];
                y[i] = s / RR(i, i);
            }
            for (int j = 0; j < kd; ++j) {
                const double *vj = V + (size_t)j * nn;
                for (int i = 0; i < n; ++i) x[i] = x[i] + y[j] * vj[i];
            }
        }
        ++cycles;
        if (fail) {
            ko_residual(n, A, lda, b, x, r);
            res = ko_nrm2(n, r);
            break;
        }
    }
#undef HH
#undef RR
out:
    free(V); free(w); free(r); free(H); free(R); free(cs); free(sn); free(g); free(y);
    if (iters_out) *iters_out = steps;
    if (cycles_out) *cycles_out = cycles;
    if (rel_res_out) *rel_res_out = res / bnorm;
    return status;
}

/* k Arnoldi steps from v0 (normalised first), modified Gram-Schmidt twice.
 * V: n x (k+1), vector j stored contiguously at V + j*n.  H: (k+1) x k
 * row-major, the unrotated Hessenberg matrix.  Returns the number of steps
 * completed (fewer than k after a happy breakdown), or -1. */
int ko_arnoldi(int n, const double *A, long lda, const double *v0, int k, double *V,
               double *H) {
    if (n <= 0 || !A || !v0 || !V || !H || lda < n || k < 1) return KO_EINVAL;
    size_t nn = (size_t)n;
    double nv = ko_nrm2(n, v0);
    if (!(nv > 0.0)) return KO_EINVAL;
    memset(H, 0, sizeof(double) * (size_t)(k + 1) * (size_t)k);
    for (int i = 0; i < n; ++i) V[i] = v0[i] / nv;
    double *w = (double *)malloc(sizeof(double) * nn);
    if (!w) return KO_EINVAL;
    int done = 0;
    for (int c = 0; c < k; ++c) {
        ko_matvec(n, A, lda, V + (size_t)c * nn, w);
        double avk = ko_nrm2(n, w);
        for (int pass = 0; pass < 2; ++pass)
            for (int j = 0; j <= c; ++j) {
                const double *vj = V + (size_t)j * nn;
                double t = ko_dot(n, vj, w);
                H[(size_t)j * (size_t)k + (size_t)c] += t;
                for (int i = 0; i < n; ++i) w[i] = w[i] - t * vj[i];
            }
        double h = ko_nrm2(n, w);
        H[(size_t)(c + 1) * (size_t)k + (size_t)c] = h;
        done = c + 1;
        if (h <= KO_HAPPY * avk) break;
        for (int i = 0; i < n; ++i) V[(size_t)(c + 1) * nn + i] = w[i] / h;
    }
    free(w);
    return done;
}

/* ------------------------------------------------- Gaussian elimination (GEPP)
 *
 * Right-looking LU with partial pivoting as the paper lists it in its direct
 * methods section: at step k pick the row v >= k with the largest |A(v,k)|,
 * swap A(k,k:n) with A(v,k:n), record p(k) = v, divide the column below the
 * pivot by it and apply the rank-1 update to the trailing block.  Only the
 * columns k:n are swapped, so the forward substitution applies the
 * interchanges step by step.  A is overwritten by L (unit, below the
 * diagonal) and U.  Returns 0, or k+1 if U(k,k) == 0 (singular). */
int ko_lu_factor(int n, double *A, long lda, int *piv) {
    if (n <= 0 || !A || !piv || lda < n) return KO_EINVAL;
    int sing = 0;
    for (int k = 0; k < n - 1; ++k) {
        int v = k;
        double best = fabs(A[(long)k * lda + k]);
        for (int i = k + 1; i < n; ++i) {
            double a = fabs(A[(long)i * lda + k]);
            if (a > best) { best = a; v = i; }
        }
        if (v != k)
            for (int j = k; j < n; ++j) {
                double t = A[(long)k * lda + j];
                A[(long)k * lda + j] = A[(long)v * lda + j];
                A[(long)v * lda + j] = t;
            }
        piv[k] = v;
        double akk = A[(long)k * lda + k];
        if (akk != 0.0) {
            for (int i = k + 1; i < n; ++i) A[(long)i * lda + k] /= akk;
            for (int i = k + 1; i < n; ++i) {
                double lik = A[(long)i * lda + k];
                for (int j = k + 1; j < n; ++j)
                    A[(long)i * lda + j] -= lik * A[(long)k * lda + j];
            }
        } else if (!sing) {
            sing = k + 1;
        }
    }
    piv[n - 1] = n - 1;
    if (!sing && A[(long)(n - 1) * lda + (n - 1)] == 0.0) sing = n;
    return sing;
}

/* Solve with the factors of ko_lu_factor: L y = P b (interchanges applied in
 * step order), then U x = y by back substitution. */
int ko_lu_solve(int n, const double *LU, long lda, const int *piv, const double *b,
                double *x) {
    if (n <= 0 || !LU || !piv || !b || !x || lda < n) return KO_EINVAL;
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!y) return KO_EINVAL;
    for (int i = 0; i < n; ++i) y[i] = b[i];
    for (int k = 0; k < n - 1; ++k) {
        int v = piv[k];
        if (v != k) { double t = y[k]; y[k] = y[v]; y[v] = t; }
        for (int i = k + 1; i < n; ++i) y[i] -= LU[(long)i * lda + k] * y[k];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int j = i + 1; j < n; ++j) s -= LU[(long)i * lda + j] * x[j];
        x[i] = s / LU[(long)i * lda + i];
    }
    free(y);
    return 0;
}

/* ------------------------------------------- binary32 block LU, GMRES-IR
 *
 * Block LU with partial pivoting (direct-methods section, Figure 1 and
 * equations (1)-(4)), in binary32 arithmetic on the binary32 rounding of A.
 * With the leading b columns split off, P A = L U reads
 *   [A11 A12]   [L11  0] [U11 U12]
 *   [A21 A22] = [L21  I] [ 0   S ]
 * so (i) the panel [A11; A21] is factored column by column (the unblocked
 * right-looking elimination, pivot = the first row of largest magnitude in
 * the column, whole rows interchanged) into L11, L21 and U11; (ii) U12 solves
 * L11 U12 = A12 (unit lower triangle); (iii) S = A22 - L21 U12 is the delayed
 * rank-b update; and the same is repeated on S.  b >= n is the unblocked
 * algorithm.  L (unit, below the diagonal) and U overwrite LU; piv[k] is the
 * row swapped with row k at step k.  Returns 0, or 1 + the first column
 * whose pivot is zero (that column is left as it is and the factorization
 * goes on).
 *
 * The factors then precondition GMRES inside binary64 iterative refinement
 * (GMRES-IR): r = b - A x in binary64; the correction solves
 * M^-1 A d = M^-1 r by restarted GMRES(m) in binary64 with
 * M^-1 v = U^-1 L^-1 P v applied with the binary32 factors widened to
 * binary64; x += d; until the normwise backward error
 * ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) <= tol.
 */
int ko_lu32_block(int n, const double *A, long lda, float *LU, long ldl, int *piv, int b) {
    if (n <= 0 || !A || !LU || !piv || lda < n || ldl < n || b < 1) return KO_EINVAL;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) LU[(long)i * ldl + j] = (float)A[(long)i * lda + j];
#define F(i, j) LU[(long)(i) * ldl + (j)]
    int sing = 0;
    for (int kb = 0; kb < n; kb += b) {
        const int bf = kb + b < n ? kb + b : n; /* the panel's columns kb .. bf-1 */
        /* (i) the panel, column by column: pivot, interchange, multipliers */
        for (int i = kb; i < bf; ++i) {
            int p = i;
            float best = fabsf(F(i, i));
            for (int r = i + 1; r < n; ++r)
                if (fabsf(F(r, i)) > best) { best = fabsf(F(r, i)); p = r; }
            if (p != i)
                for (int j = 0; j < n; ++j) { float t = F(i, j); F(i, j) = F(p, j); F(p, j) = t; }
            piv[i] = p;
            const float d = F(i, i);
            if (d == 0.0f) {
                if (!sing) sing = i + 1;
                continue;
            }
            for (int r = i + 1; r < n; ++r) F(r, i) = F(r, i) / d;
            for (int r = i + 1; r < n; ++r) {
                const float l = F(r, i);
                for (int j = i + 1; j < bf; ++j) F(r, j) = F(r, j) - l * F(i, j);
            }
        }
        /* (ii) the block row of U: L11 U12 = A12 */
        for (int c = bf; c < n; ++c)
            for (int i = kb; i < bf; ++i) {
                float s = F(i, c);
                for (int j = kb; j < i; ++j) s = s - F(i, j) * F(j, c);
                F(i, c) = s;
            }
        /* (iii) S = A22 - L21 U12, the delayed rank-(bf - kb) update */
        for (int r = bf; r < n; ++r)
            for (int c = bf; c < n; ++c) {
                float s = F(r, c);
                for (int j = kb; j < bf; ++j) s = s - F(r, j) * F(j, c);
                F(r, c) = s;
            }
    }
#undef F
    return sing;
}

/* z = U^-1 L^-1 P v in binary64 with the binary32 factors of ko_lu32_block */
void ko_lu32_apply(int n, const float *LU, long ldl, const int *piv, const double *v, double *z) {
    for (int i = 0; i < n; ++i) z[i] = v[i];
    for (int k = 0; k < n; ++k) {
        const int p = piv[k];
        if (p != k) { double t = z[k]; z[k] = z[p]; z[p] = t; }
    }
    for (int i = 0; i < n; ++i) {
        double s = z[i];
        for (int j = 0; j < i; ++j) s -= (double)LU[(long)i * ldl + j] * z[j];
        z[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int j = i + 1; j < n; ++j) s -= (double)LU[(long)i * ldl + j] * z[j];
        z[i] = s / (double)LU[(long)i * ldl + i];
    }
}

/* Left-preconditioned restarted GMRES(m), MGS twice + Givens as ko_gmres,
 * on M^-1 A d = M^-1 r from d = 0; stops when the preconditioned residual
 * estimate is <= tol ||M^-1 r||, or after max_steps products.  *steps
 * counts products. */
static int gmres_lu_inner(int n, const double *A, long lda, const float *LU, long ldl,
                          const int *piv, const double *r, double *d, double tol, int m,
                          int max_steps, int *steps_out) {
    size_t nn = (size_t)n;
    int steps = 0, status = KO_MAXITER;
    double *V = (double *)calloc(nn * (size_t)(m + 1), sizeof(double));
    double *w = (double *)malloc(sizeof(double) * nn);
    double *t = (double *)malloc(sizeof(double) * nn);
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double *cs = (double *)calloc((size_t)m, sizeof(double));
    double *sn = (double *)calloc((size_t)m, sizeof(double));
    double *g = (double *)calloc((size_t)m + 1, sizeof(double));
    double *y = (double *)calloc((size_t)m, sizeof(double));
    if (!V || !w || !t || !H || !cs || !sn || !g || !y) {
        status = KO_EINVAL;
        goto out;
    }
#define HH(i, j) H[(size_t)(i) * (size_t)m + (size_t)(j)]
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    ko_lu32_apply(n, LU, ldl, piv, r, t);
    const double pnorm = ko_nrm2(n, t);
    if (!isfinite(pnorm)) { status = KO_NONFINITE; goto out; }
    if (pnorm == 0.0) { status = KO_OK; goto out; }
    for (;;) {
        /* preconditioned residual M^-1 (r - A d) */
        ko_residual(n, A, lda, r, d, w);
        ko_lu32_apply(n, LU, ldl, piv, w, t);
        const double beta = ko_nrm2(n, t);
        if (!isfinite(beta)) { status = KO_NONFINITE; break; }
        if (beta <= tol * pnorm) { status = KO_OK; break; }
        if (steps >= max_steps) { status = KO_MAXITER; break; }
        for (int i = 0; i < n; ++i) V[i] = t[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int kd = 0, fail = 0;
        for (int k = 0; k < m; ++k) {
            ko_matvec(n, A, lda, V + (size_t)k * nn, t);
            ko_lu32_apply(n, LU, ldl, piv, t, w);
            ++steps;
            const double avk = ko_nrm2(n, w);
            for (int j = 0; j <= k + 1; ++j) HH(j, k) = 0.0;
            for (int pass = 0; pass < 2; ++pass)
                for (int j = 0; j <= k; ++j) {
                    const double *vj = V + (size_t)j * nn;
                    const double h = ko_dot(n, vj, w);
                    HH(j, k) += h;
                    for (int i = 0; i < n; ++i) w[i] = w[i] - h * vj[i];
                }
            const double hk1 = ko_nrm2(n, w);
            HH(k + 1, k) = hk1;
            for (int i = 0; i < k; ++i) {
                const double a = HH(i, k), bb = HH(i + 1, k);
                HH(i, k) = cs[i] * a + sn[i] * bb;
                HH(i + 1, k) = -sn[i] * a + cs[i] * bb;
            }
            const double rho = hypot(HH(k, k), HH(k + 1, k));
            if (!isfinite(rho) || !isfinite(avk)) { status = KO_NONFINITE; fail = 1; break; }
            if (rho == 0.0) { status = KO_BREAKDOWN; fail = 1; break; }
            cs[k] = HH(k, k) / rho;
            sn[k] = HH(k + 1, k) / rho;
            HH(k, k) = rho;
            HH(k + 1, k) = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            kd = k + 1;
            if (hk1 <= KO_HAPPY * avk) break;
            double *vn = V + (size_t)(k + 1) * nn;
            for (int i = 0; i < n; ++i) vn[i] = w[i] / hk1;
            if (fabs(g[k + 1]) <= tol * pnorm || steps >= max_steps) break;
        }
        for (int i = kd - 1; i >= 0; --i) {
            double s2 = g[i];
            for (int j = i + 1; j < kd; ++j) s2 -= HH(i, j) * y[j];
            y[i] = s2 / HH(i, i);
        }
        for (int j = 0; j < kd; ++j) {
            const double *vj = V + (size_t)j * nn;
            for (int i = 0; i < n; ++i) d[i] = d[i] + y[j] * vj[i];
        }
        if (fail) break;
    }
#undef HH
out:
    free(V); free(w); free(t); free(H); free(cs); free(sn); free(g); free(y);
    if (steps_out) *steps_out = steps;
    return status;
}

int ko_gmres_ir_lu(int n, const double *A, long lda, const double *b, double *x, double tol,
                   int m, double inner_tol, int max_inner, int max_outer, int nb, int *outer_out,
                   int *inner_out, double *eta_out) {
    if (n <= 0 || !A || !b || !x || lda < n || !(tol > 0.0) || m < 1 || !(inner_tol > 0.0) ||
        max_inner < 1 || max_outer < 0 || nb < 1)
        return KO_EINVAL;
    size_t nn = (size_t)n;
    float *LU = (float *)malloc(sizeof(float) * nn * nn);
    int *piv = (int *)malloc(sizeof(int) * nn);
    double *r = (double *)malloc(sizeof(double) * nn);
    double *d = (double *)malloc(sizeof(double) * nn);
    int status = KO_STAGNATED, outer = 0, inner = 0;
    double eta = 0.0;
    if (!LU || !piv || !r || !d) {
        status = KO_EINVAL;
        goto out;
    }
    const double anorm = ko_norm_inf_mat(n, A, lda);
    const double binf = norm_inf_vec(n, b);
    if (!isfinite(binf)) { status = KO_NONFINITE; goto out; }
    if (binf == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        status = KO_OK;
        goto out;
    }
    if (ko_lu32_block(n, A, lda, LU, (long)n, piv, nb)) { status = KO_BREAKDOWN; goto out; }
    for (;;) {
        ko_residual(n, A, lda, b, x, r);
        const double rinf = norm_inf_vec(n, r), xinf = norm_inf_vec(n, x);
        const double den = anorm * xinf + binf;
        eta = den > 0.0 ? rinf / den : rinf;
        if (!isfinite(eta)) { status = KO_NONFINITE; break; }
        if (eta <= tol) { status = KO_OK; break; }
        if (outer >= max_outer) { status = KO_STAGNATED; break; }
        int steps = 0;
        const int st = gmres_lu_inner(n, A, lda, LU, (long)n, piv, r, d, inner_tol, m, max_inner,
                                      &steps);
        inner += steps;
        ++outer;
        if (st == KO_NONFINITE || st == KO_BREAKDOWN || st == KO_EINVAL) { status = st; break; }
        for (int i = 0; i < n; ++i) x[i] = x[i] + d[i];
    }
out:
    free(LU); free(piv); free(r); free(d);
    if (outer_out) *outer_out = outer;
    if (inner_out) *inner_out = inner;
    if (eta_out) *eta_out = eta;
    return status;
}

/* ------------------------------------------ binary32 block Cholesky, CG-IR
 *
 * Block Cholesky (direct-methods section, the Cholesky relations that follow
 * the block LU), in binary32 arithmetic on the binary32 rounding of a
 * symmetric A (only its lower triangle is read).  With the leading b columns
 * split off, A = L L^T reads
 *   [A11 A21^T]   [L11  0 ] [L11^T L21^T]
 *   [A21 A22  ] = [L21 L22] [ 0    L22^T]
 * so (i) A11 = L11 L11^T is factored column by column,
 *   l_jj = sqrt(a_jj - sum_{k<j} l_jk^2),  l_ij = (a_ij - sum_{k<j} l_ik l_jk) / l_jj;
 * (ii) L21 = A21 L11^-T, each row of A21 solved against L11^T by the same
 * formula; (iii) S = A22 - L21 L21^T (lower triangle), and the same on S.
 * Every sum subtracts its terms one at a time in increasing k, in whichever
 * step they arrive, so the result does not depend on b (b >= n is the
 * unblocked algorithm).  L (lower triangle, diagonal included) is written to
 * L; entries above the diagonal are set to 0.  Returns 0, or 1 + the first
 * column whose pivot a_jj - sum l_jk^2 is not positive (A is not positive
 * definite in binary32); the factorization stops there.
 *
 * The factor then preconditions CG inside binary64 iterative refinement
 * (CG-IR): r = b - A x in binary64; the correction solves A d = r by CG in
 * binary64 preconditioned with M = L L^T (M^-1 v = L^-T L^-1 v with the
 * binary32 factor widened to binary64), from d = 0 to ||r - A d||_2 <=
 * inner_tol ||r||_2; x += d; until the normwise backward error
 * ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf) <= tol.
 */
int ko_chol32_block(int n, const double *A, long lda, float *L, long ldl, int b) {
    if (n <= 0 || !A || !L || lda < n || ldl < n || b < 1) return KO_EINVAL;
#define F(i, j) L[(long)(i) * ldl + (j)]
    int notpd = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) F(i, j) = (j <= i) ? (float)A[(long)i * lda + j] : 0.0f;
    for (int kb = 0; kb < n; kb += b) {
        const int bf = kb + b < n ? kb + b : n; /* the block's columns kb .. bf-1 */
        /* (i) the diagonal block: its entries already hold the updates of
         * the columns before kb; subtract the block's own columns, in order */
        for (int j = kb; j < bf; ++j) {
            float d = F(j, j);
            for (int k = kb; k < j; ++k) d = d - F(j, k) * F(j, k);
            if (!(d > 0.0f)) {
                notpd = j + 1;
                goto done;
            }
            const float ljj = sqrtf(d);
            F(j, j) = ljj;
            for (int i = j + 1; i < bf; ++i) {
                float s = F(i, j);
                for (int k = kb; k < j; ++k) s = s - F(i, k) * F(j, k);
                F(i, j) = s / ljj;
            }
        }
        /* (ii) L21 = A21 L11^-T: row i of the panel below the block */
        for (int i = bf; i < n; ++i)
            for (int j = kb; j < bf; ++j) {
                float s = F(i, j);
                for (int k = kb; k < j; ++k) s = s - F(i, k) * F(j, k);
                F(i, j) = s / F(j, j);
            }
        /* (iii) S = A22 - L21 L21^T on the lower triangle */
        for (int i = bf; i < n; ++i)
            for (int j = bf; j <= i; ++j) {
                float s = F(i, j);
                for (int k = kb; k < bf; ++k) s = s - F(i, k) * F(j, k);
                F(i, j) = s;
            }
    }
done:
#undef F
    return notpd;
}

/* z = L^-T L^-1 v in binary64 with the binary32 factor of ko_chol32_block */
void ko_chol32_apply(int n, const float *L, long ldl, const double *v, double *z) {
    for (int i = 0; i < n; ++i) {
        double s = v[i];
        for (int j = 0; j < i; ++j) s -= (double)L[(long)i * ldl + j] * z[j];
        z[i] = s / (double)L[(long)i * ldl + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int j = i + 1; j < n; ++j) s -= (double)L[(long)j * ldl + i] * z[j];
        z[i] = s / (double)L[(long)i * ldl + i];
    }
}

/* Preconditioned CG in binary64 on A d = r from d = 0 with M = L L^T:
 * stops when ||r - A d||_2 <= tol ||r||_2 (recursive residual) or after
 * max_steps products.  *steps counts products. */
static int pcg_chol_inner(int n, const double *A, long lda, const float *L, long ldl,
                          const double *r, double *d, double tol, int max_steps,
                          int *steps_out) {
    size_t nn = (size_t)n;
    int steps = 0, status = KO_MAXITER;
    double *res = (double *)malloc(sizeof(double) * nn), *z = (double *)malloc(sizeof(double) * nn);
    double *p = (double *)malloc(sizeof(double) * nn), *q = (double *)malloc(sizeof(double) * nn);
    if (!res || !z || !p || !q) {
        status = KO_EINVAL;
        goto out;
    }
    for (int i = 0; i < n; ++i) { d[i] = 0.0; res[i] = r[i]; }
    const double rnorm = ko_nrm2(n, r);
    if (!isfinite(rnorm)) { status = KO_NONFINITE; goto out; }
    if (rnorm == 0.0) { status = KO_OK; goto out; }
    ko_chol32_apply(n, L, ldl, res, z);
    for (int i = 0; i < n; ++i) p[i] = z[i];
    double rz = ko_dot(n, res, z);
    for (;;) {
        const double rn = ko_nrm2(n, res);
        if (!isfinite(rn) || !isfinite(rz)) { status = KO_NONFINITE; break; }
        if (rn <= tol * rnorm) { status = KO_OK; break; }
        if (steps >= max_steps) { status = KO_MAXITER; break; }
        ko_matvec(n, A, lda, p, q);
        ++steps;
        const double sigma = ko_dot(n, p, q);
        if (!isfinite(sigma)) { status = KO_NONFINITE; break; }
        if (sigma <= 0.0 || rz <= 0.0) { status = KO_BREAKDOWN; break; }
        const double alpha = rz / sigma;
        for (int i = 0; i < n; ++i) d[i] = d[i] + alpha * p[i];
        for (int i = 0; i < n; ++i) res[i] = res[i] - alpha * q[i];
        ko_chol32_apply(n, L, ldl, res, z);
        const double rz_new = ko_dot(n, res, z);
        const double beta = rz_new / rz;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rz = rz_new;
    }
out:
    free(res); free(z); free(p); free(q);
    if (steps_out) *steps_out = steps;
    return status;
}

int ko_cg_ir_chol(int n, const double *A, long lda, const double *b, double *x, double tol,
                  double inner_tol, int max_inner, int max_outer, int nb, int *outer_out,
                  int *inner_out, double *eta_out) {
    if (n <= 0 || !A || !b || !x || lda < n || !(tol > 0.0) || !(inner_tol > 0.0) ||
        max_inner < 1 || max_outer < 0 || nb < 1)
        return KO_EINVAL;
    size_t nn = (size_t)n;
    float *L = (float *)malloc(sizeof(float) * nn * nn);
    double *r = (double *)malloc(sizeof(double) * nn);
    double *d = (double *)malloc(sizeof(double) * nn);
    int status = KO_STAGNATED, outer = 0, inner = 0;
    double eta = 0.0;
    if (!L || !r || !d) {
        status = KO_EINVAL;
        goto out;
    }
    const double anorm = ko_norm_inf_mat(n, A, lda);
    const double binf = norm_inf_vec(n, b);
    if (!isfinite(binf)) { status = KO_NONFINITE; goto out; }
    if (binf == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        status = KO_OK;
        goto out;
    }
    if (ko_chol32_block(n, A, lda, L, (long)n, nb)) { status = KO_BREAKDOWN; goto out; }
    for (;;) {
        ko_residual(n, A, lda, b, x, r);
        const double rinf = norm_inf_vec(n, r), xinf = norm_inf_vec(n, x);
        const double den = anorm * xinf + binf;
        eta = den > 0.0 ? rinf / den : rinf;
        if (!isfinite(eta)) { status = KO_NONFINITE; break; }
        if (eta <= tol) { status = KO_OK; break; }
        if (outer >= max_outer) { status = KO_STAGNATED; break; }
        int steps = 0;
        const int st = pcg_chol_inner(n, A, lda, L, (long)n, r, d, inner_tol, max_inner, &steps);
        inner += steps;
        ++outer;
        if (st == KO_NONFINITE || st == KO_BREAKDOWN || st == KO_EINVAL) { status = st; break; }
        for (int i = 0; i < n; ++i) x[i] = x[i] + d[i];
    }
out:
    free(L); free(r); free(d);
    if (outer_out) *outer_out = outer;
    if (inner_out) *inner_out = inner;
    if (eta_out) *eta_out = eta;
    return status;
}
