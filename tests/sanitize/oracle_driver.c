/*
 * Drives every function of the CPU oracle on small and degenerate inputs so
 * that an AddressSanitizer / UndefinedBehaviorSanitizer build of it can
 * report out-of-bounds accesses, leaks, uninitialised reads turned into UB,
 * signed overflow and the like.  Host only; the oracle is included as one
 * translation unit.  Exit status 0 when every call returned a plausible
 * status; the sanitizers abort on the first error they find.
 */
#include "../../oracle/ks_oracle.c"

#include <stdio.h>

static unsigned long long lcg = 88172645463325252ULL;
static double urand(void) {
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

/* diagonally dominant nonsymmetric (kind 0) or SPD (kind 1) n x n, row-major, ld lda */
static void make(int n, long lda, int kind, double *A) {
    for (int i = 0; i < n; ++i)
        for (long j = 0; j < lda; ++j) A[i * lda + j] = (j < n) ? (urand() - 0.5) / n : 1e300;
    if (kind == 1)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < i; ++j) A[i * lda + j] = A[j * lda + i];
    for (int i = 0; i < n; ++i) A[i * lda + i] += 2.0 + urand();
}

static int fails = 0;
static void check(int ok, const char *what, int n) {
    if (!ok) {
        fprintf(stderr, "FAIL %s n=%d\n", what, n);
        ++fails;
    }
}

int main(void) {
    const int sizes[] = {1, 2, 7, 33, 100};
    for (size_t si = 0; si < sizeof(sizes) / sizeof(sizes[0]); ++si) {
        const int n = sizes[si];
        const long lda = n + 3;
        double *A = malloc(sizeof(double) * n * lda), *S = malloc(sizeof(double) * n * lda);
        double *b = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n);
        double *V = malloc(sizeof(double) * n * (n + 1)), *H = malloc(sizeof(double) * (n + 1) * n);
        double *hist = malloc(sizeof(double) * 4 * n), *z = malloc(sizeof(double) * n);
        float *LU = malloc(sizeof(float) * n * lda);
        int *piv = malloc(sizeof(int) * n), *rows = malloc(sizeof(int) * n);
        make(n, lda, 0, A);
        make(n, lda, 1, S);
        for (int i = 0; i < n; ++i) b[i] = urand() - 0.5;
        int it = 0, rs = 0, cy = 0, o = 0, in = 0;
        double rr = 0.0, eta = 0.0, met[3];
        /* Krylov solvers */
        memset(x, 0, sizeof(double) * n);
        check(ko_cg(n, S, lda, b, x, 1e-12, 10 * n, &it, &rs, &rr, hist, 4 * n) == 0, "cg", n);
        check(ko_metrics(n, S, lda, b, x, met) == 0 && met[0] <= 1e-10, "metrics", n);
        memset(x, 0, sizeof(double) * n);
        check(ko_gmres(n, A, lda, b, x, 1e-12, 10 * n, 5, &it, &cy, &rr, hist, 4 * n, hist, 4 * n) == 0,
              "gmres", n);
        memset(x, 0, sizeof(double) * n);
        check(ko_bicgstab(n, A, lda, b, x, 1e-12, 20 * n, &it, &rs, &rr) == 0, "bicgstab", n);
        memset(x, 0, sizeof(double) * n);
        check(ko_jacobi(n, A, lda, b, x, 1e-12, 200 * n, &it, &rr) == 0, "jacobi", n);
        memset(x, 0, sizeof(double) * n);
        check(ko_gauss_seidel(n, A, lda, b, x, 1e-12, 200 * n, &it, &rr) == 0, "gauss-seidel", n);
        check(ko_arnoldi(n, A, lda, b, n, V, H) >= 1, "arnoldi", n);
        /* direct methods */
        double *F = malloc(sizeof(double) * n * lda);
        memcpy(F, A, sizeof(double) * n * lda);
        check(ko_lu_factor(n, F, lda, piv) == 0, "gepp factor", n);
        check(ko_lu_solve(n, F, lda, piv, b, x) == 0, "gepp solve", n);
        for (int nb = 1; nb <= n + 1; nb = 2 * nb + 1)
            check(ko_lu32_block(n, A, lda, LU, lda, piv, nb) == 0, "lu32 block", n);
        ko_lu32_apply(n, LU, lda, piv, b, z);
        memset(x, 0, sizeof(double) * n);
        check(ko_gmres_ir_lu(n, A, lda, b, x, 1e-12, 5, 1e-4, 10 * n, 20, 4, &o, &in, &eta) == 0,
              "gmres-ir lu", n);
        for (int i = 0; i < n; ++i) rows[i] = n - 1 - i;
        ko_matvec_rows(n, A, lda, rows, n, b, z);
        (void)ko_norm_inf_mat(n, A, lda);
        /* special inputs: b = 0, a NaN, a zero diagonal, tiny budgets */
        double *zb = calloc(n, sizeof(double));
        for (int i = 0; i < n; ++i) x[i] = 1.0;
        check(ko_cg(n, S, lda, zb, x, 1e-10, n, &it, &rs, &rr, NULL, 0) == 0, "cg b=0", n);
        b[n / 2] = NAN;
        memset(x, 0, sizeof(double) * n);
        check(ko_gmres(n, A, lda, b, x, 1e-10, n, 3, &it, &cy, &rr, NULL, 0, NULL, 0) == 4, "gmres nan", n);
        memset(x, 0, sizeof(double) * n);
        check(ko_bicgstab(n, A, lda, b, x, 1e-10, n, &it, &rs, &rr) == 4, "bicgstab nan", n);
        b[n / 2] = 0.25;
        memset(x, 0, sizeof(double) * n);
        (void)ko_cg(n, S, lda, b, x, 1e-14, 1, &it, &rs, &rr, NULL, 0);
        A[0] = 0.0;
        memset(x, 0, sizeof(double) * n);
        check(ko_jacobi(n, A, lda, b, x, 1e-10, n, &it, &rr) == 2, "jacobi zero diagonal", n);
        free(A); free(S); free(b); free(x); free(V); free(H); free(hist); free(z); free(LU);
        free(piv); free(rows); free(F); free(zb);
    }
    if (fails) return 1;
    printf("oracle driver: all calls returned\n");
    return 0;
}
