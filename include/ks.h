/*
 * ks.h - dense Krylov solvers for MI355X (gfx950), C ABI.
 *
 * Solves A x = b for a dense n x n matrix A (the linear system of the paper's
 * Krylov section) with
 *   - conjugate gradient (CG) when A is symmetric positive definite,
 *   - restarted GMRES(m) otherwise (Arnoldi step of the paper's GMRES
 *     pseudo-code, restart after m steps from the current iterate), or
 *   - BiCGSTAB (the paper's BiCGSTAB listing: two products with A per
 *     iteration, short recurrences, no basis kept) for any nonsingular A,
 * in binary64, or with an inner solve on a binary32 / bfloat16 copy of A and
 * binary64 iterative refinement around it; and with the two classical
 * stationary iterations the paper's library lists beside them (introductory
 * section, timed in Tables 1-2), in binary64:
 *   - Jacobi, D x(k+1) = b - (L + U) x(k), and
 *   - Gauss-Seidel, (D + L) x(k+1) = b - U x(k) (forward sweeps),
 * with A = L + D + U (strictly lower, diagonal, strictly upper).  They
 * converge for strictly diagonally dominant A (Gauss-Seidel also for SPD A).
 *
 * The call sequence follows the host flow of the paper's "parallel
 * implementation" section (allocate device memory, copy, pick the launch
 * grid, run the kernels, copy back, clean up), reduced to
 *     ks_workspace_bytes -> ks_create -> ks_solve ... -> ks_free.
 *
 * Memory model
 *   - Every pointer argument named d_* is a device pointer (hipMalloc or a
 *     torch tensor's data_ptr) on the current HIP device.  A, b, x and the
 *     workspace are owned by the caller; the library never frees them.
 *   - A is row-major: element (i, j) is dA[i * lda + j], lda >= n.  When A is
 *     16-byte aligned and lda * 8 is a multiple of 16 the solver reads A in
 *     place ("borrowed"; it must stay valid and unmodified until ks_free);
 *     otherwise ks_create copies it into the workspace with a padded lda.
 *   - All work is enqueued on the HIP stream given to ks_create (NULL = the
 *     null stream).  ks_solve returns after the solve has finished on that
 *     stream, with x and *info final.
 *   - A solver is not re-entrant: one ks_solve at a time per solver.
 *     Distinct solvers may run concurrently on distinct streams.
 *
 * Errors: every int-returning call returns KS_OK (0), a positive numerical
 * outcome (x then holds the last iterate) or a negative usage / system error
 * (outputs untouched).  No C++ exception crosses this interface.
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define KS_OK 0
#define KS_MAXITER 1     /* iteration limit reached before the tolerance        */
#define KS_BREAKDOWN 2   /* CG: p'Ap <= 0 (A not SPD); GMRES: singular H;
                            BiCGSTAB: r0'r, r0'v or t't became 0, or omega = 0;
                            Jacobi / Gauss-Seidel: a zero on the diagonal      */
#define KS_STAGNATED 3   /* refinement / restarts stopped making progress       */
#define KS_NONFINITE 4   /* a NaN or Inf appeared (in b, x0, A or an iterate)    */
#define KS_EINVAL (-1)   /* bad argument (n <= 0, lda < n, NULL, tol <= 0, ...) */
#define KS_ENOMEM (-2)   /* workspace too small, or allocation failed           */
#define KS_EHIP (-3)     /* a HIP runtime call failed                            */
#define KS_EDEVICE (-4)  /* current device is not gfx950                         */
#define KS_ETOOLARGE (-5) /* server: request larger than the memory budget       */

/* ---- method / precision ---------------------------------------------- */
#define KS_CG 0
#define KS_GMRES 1
#define KS_BICGSTAB 2
/* Stationary methods (binary64 only, nrhs 1).  max_iter counts updates of x;
 * each update is one product with A: Jacobi the full A (x += D^-1 (b - A x)),
 * Gauss-Seidel its strict upper triangle plus a forward substitution with
 * the lower one.  The stop test is made on the residual of the current
 * iterate, as for the Krylov methods. */
#define KS_JACOBI 3
#define KS_GAUSS_SEIDEL 4

#define KS_FP64 0        /* everything in binary64                               */
#define KS_IR_FP32 1     /* inner solve on binary32 A, binary64 refinement       */
#define KS_IR_BF16 2     /* inner solve on bfloat16 A (fp32 accumulation)        */
#define KS_IR_LU32 3     /* GMRES-IR: binary64 refinement around GMRES(m) in
                            binary64, left-preconditioned by a binary32 block LU
                            with partial pivoting (the direct-methods section's
                            block algorithm) computed in ks_create; method
                            KS_GMRES, nrhs 1, n <= 32768.  A factorization with a
                            zero pivot makes ks_solve return KS_BREAKDOWN     */
#define KS_IR_CHOL32 4   /* CG-IR: binary64 refinement around preconditioned CG
                            in binary64 with M = L L^T, L the binary32 block
                            Cholesky factor of A (the direct-methods section's
                            Cholesky relations, computed in ks_create with the
                            trailing updates on the matrix cores); method
                            KS_CG, nrhs 1, no KS_FLAG_SYMMETRIC.  Each inner
                            solve starts from d = 0 and stops at relative
                            residual inner_tol or max_iter products; a
                            non-positive pivot makes ks_solve return
                            KS_BREAKDOWN                                        */

/* element types for the kernel-level entry points */
#define KS_DT_F64 0
#define KS_DT_F32 1
#define KS_DT_BF16 2

/* ks_params.flags */
#define KS_FLAG_TIMING 1 /* time the A*v launches with HIP events (info->gemv_ms;
                            all of them, or a sample: timing_every) */
#define KS_FLAG_STOP_BACKWARD 2 /* binary64 solves: tol bounds the normwise backward
                                   error eta_inf = ||r||_inf / (||A||_inf ||x||_inf +
                                   ||b||_inf) instead of ||r||_2 / ||b||_2.  CG and
                                   BiCGSTAB stop when eta_inf of the recursive
                                   residual and the current iterate meets tol;
                                   GMRES when its 2-norm estimate does, scaled by
                                   ||r||_2 / ||r||_inf of the cycle's starting
                                   residual; every stop is confirmed on eta_inf of
                                   the true residual */
#define KS_FLAG_SYMMETRIC 4 /* CG, nrhs = 1: the binary64 products of the Krylov
                               loop, and the binary32 products of KS_IR_FP32's
                               inner solves, read only the lower triangle of A
                               (i >= j; of its binary32 copy), half the bytes of
                               the general product (KS_IR_BF16 inner solves keep
                               the general one).  A must still hold the whole
                               symmetric matrix: the true residual and
                               ||A||_inf read both triangles */
#define KS_FLAG_NO_PERSIST 8 /* binary64 CG at n <= 1024 (not stopping on the
                                backward error) normally runs every iteration
                                of a polling interval in one cooperative
                                launch with a grid barrier between iterations,
                                and the substitutions of the LU and Cholesky
                                preconditioners (KS_IR_LU32, KS_IR_CHOL32) one
                                cooperative launch per sweep; this flag runs
                                one launch per iteration and one per 64-row
                                step instead (the same results bit for bit) */

typedef struct ks_solver ks_solver; /* opaque, library-owned handle */

typedef struct {
    int32_t n;          /* order of A, >= 1                                       */
    int32_t method;     /* KS_CG, KS_GMRES, KS_BICGSTAB, KS_JACOBI or
                           KS_GAUSS_SEIDEL                                       */
    int64_t lda;        /* leading dimension of A in elements, >= n               */
    int32_t precision;  /* KS_FP64, KS_IR_FP32, KS_IR_BF16 or KS_IR_LU32           */
    int32_t max_iter;   /* FP64: A*v products in the Krylov loop over the whole
                           solve; IR: per inner solve                              */
    double tol;         /* FP64: stop at ||b - A x||_2 <= tol ||b||_2 (checked on
                           the true residual); IR: stop at the normwise backward
                           error ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf)      */
    int32_t restart;    /* m of GMRES(m), 1..KS_MAX_RESTART; ignored by CG        */
    int32_t max_outer;  /* IR: refinement steps (default 30)                     */
    double inner_tol;   /* IR: relative tolerance of each inner solve (1e-4)     */
    int32_t poll_every; /* host checks the device's stop flag every this many
                           iterations (0 = chosen from n)                          */
    int32_t flags;      /* KS_FLAG_*                                              */
    int32_t nrhs;       /* right-hand sides solved together (CG only): 1, or up to
                           KS_MAX_NRHS for lockstep CG with A*P on the matrix
                           cores; precision KS_FP64 or KS_IR_FP32               */
    int32_t timing_every; /* with KS_FLAG_TIMING: time one A*v launch in every
                           this many, counted over the solve (0 or 1: all of
                           them).  Each timed launch records two HIP events,
                           which cost the stream a few microseconds; sampling
                           keeps that out of a timed solve's wall time */
} ks_params;

#define KS_MAX_RESTART 128
#define KS_MAX_NRHS 64

typedef struct {
    int32_t status;        /* KS_OK or a positive outcome                           */
    int32_t iters;         /* A*v products inside the Krylov loops (all levels;
                              BiCGSTAB makes two per iteration)                     */
    int32_t outer_iters;   /* IR refinement steps (0 for KS_FP64)                   */
    int32_t restarts;      /* GMRES cycles beyond the first / CG restarts            */
    double rel_res;        /* ||b - A x||_2 / ||b||_2 of the returned x (binary64)  */
    double backward_err;   /* ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)    */
    double elapsed_ms;     /* device time of the solve (HIP events on the stream)   */
    double gemv_ms;        /* with KS_FLAG_TIMING: summed time of the A*v launches  */
    int32_t gemv_calls;    /* with KS_FLAG_TIMING: number of timed A*v launches     */
    int32_t precision_used;/* IR: precision of the last inner solve after fallback  */
} ks_info;

/* Fill *p with defaults for an n x n system (lda = n, tol 1e-10, max_iter
 * 10 n, restart 30, KS_FP64, inner_tol 1e-4, max_outer 30).  KS_EINVAL if
 * p is NULL, n < 1 or method unknown. */
int ks_params_init(ks_params *p, int32_t n, int32_t method);

/* Bytes of device workspace ks_create needs for these parameters (including
 * room for a padded copy of A in case it cannot be borrowed, and the binary32 /
 * bfloat16 copy for the IR precisions).  *bytes is written on KS_OK. */
int ks_workspace_bytes(const ks_params *p, size_t *bytes);

/* Bytes needed when A is borrowed (aligned, see above): smaller than
 * ks_workspace_bytes by the size of the binary64 copy. */
int ks_workspace_bytes_borrowed(const ks_params *p, size_t *bytes);

/* Create a solver for A.  d_ws must be 256-byte aligned and ws_bytes at least
 * what ks_workspace_bytes (or ks_workspace_bytes_borrowed, when A can be
 * borrowed) returned; d_ws == NULL with ws_bytes == 0 makes the library
 * allocate (and later free) its own workspace.  Enqueues the set-up work
 * (padding copy, ||A||_inf, low-precision copy) on `stream` and returns
 * without waiting.  Errors: KS_EINVAL, KS_ENOMEM, KS_EHIP, KS_EDEVICE. */
int ks_create(ks_solver **out, const ks_params *p, const double *d_A, void *d_ws,
              size_t ws_bytes, void *stream);

/* Solve A x = b.  d_b: n binary64 values; d_x: n binary64 values, x0 on
 * entry, the solution on return (the last iterate for a positive status).
 * Both must be 16-byte aligned (KS_EINVAL otherwise).
 * With nrhs = s > 1, d_b and d_x are n x s column-major (right-hand side j
 * at d_b + j * n): s independent CG solves advanced in lockstep, each column
 * with its own scalars and stopping test (equal to the one-column solve in
 * exact arithmetic); *info then summarises them (worst status, largest
 * residual and backward error, lockstep iterations) and ks_column_info gives
 * each column.
 * Returns the status (also in info->status); info may be NULL. */
int ks_solve(ks_solver *s, const double *d_b, double *d_x, ks_info *info);

/* Result of column j (0 <= j < nrhs) of the last ks_solve: status, iters
 * (products in which the column took part), restarts, rel_res and
 * backward_err of that column.  KS_EINVAL if j is out of range. */
int ks_column_info(const ks_solver *s, int32_t j, ks_info *info);

/* Run k Arnoldi steps (classical Gram-Schmidt applied twice) from d_v0,
 * which is normalised first.  d_V receives the basis, vector j at
 * d_V + j * n (n x (k+1)); d_H the unrotated (k+1) x k Hessenberg matrix,
 * row-major; *k_done the number of steps completed (< k after a happy
 * breakdown).  Uses the solver's workspace; the solver must have been
 * created with method KS_GMRES, precision KS_FP64 and restart >= k. */
int ks_arnoldi(ks_solver *s, const double *d_v0, int32_t k, double *d_V, double *d_H,
               int32_t *k_done);

/* Release the handle and any memory the library allocated itself.  NULL-safe.
 * Waits for the solver's stream. */
void ks_free(ks_solver *s);

/* Static English text for a status code. */
const char *ks_strerror(int status);

/* ---- request server (continuous batching) ------------------------------
 * Many CG / GMRES(m) solves of different sizes, binary64 or mixed precision
 * (KS_IR_FP32 / KS_IR_BF16 inner solves with binary64 refinement), submitted
 * as they arrive.  Each ks_server_step admits queued requests first come first served
 * while the memory budget (8 n lda bytes of the request's A plus its solve
 * workspace) and the in-flight slot count allow, then advances every
 * in-flight solve by `chunk` iterations with one batched launch per phase (a
 * launch covers all solves at once), and retires the finished ones.  A
 * request's x is the same, bit for bit, whatever else is in flight with it
 * and equal to what ks_solve computes for it alone.  The caller keeps A, b, x
 * valid and unmodified until the ticket is returned by ks_server_poll (an A
 * that is not 16-byte aligned with lda * 8 a multiple of 16 is copied into
 * the server's workspace at admission, like ks_create does).  b and x must be
 * 16-byte aligned.  One thread drives a server; all work runs on its stream. */
typedef struct ks_server ks_server;

/* Create a server with a device-memory admission budget (bytes), at most
 * max_inflight concurrent solves and `chunk` iterations per step (0 = 16).
 * The solves' workspaces come from device segments the server allocates as
 * admission needs them (at least 1 GiB each, never more than the budget in
 * all), so the budget alone decides admission; they are freed by
 * ks_server_free. */
int ks_server_create(ks_server **out, size_t mem_budget_bytes, int32_t max_inflight, int32_t chunk,
                     void *stream);

/* Queue a solve (method KS_CG or KS_GMRES, nrhs 1, precision KS_FP64,
 * KS_IR_FP32 or KS_IR_BF16; KS_FLAG_SYMMETRIC for CG as in ks_solve;
 * otherwise KS_EINVAL).  d_x holds x0 and receives x.  *ticket identifies it
 * in ks_server_poll.  KS_ETOOLARGE if it can never fit the budget. */
int ks_server_submit(ks_server *sv, const ks_params *p, const double *d_A, const double *d_b,
                     double *d_x, uint64_t *ticket);

/* One scheduling tick (admit, advance all in-flight solves, retire); waits
 * for the tick's device work.  Within a tick a solve's set-up, start and
 * steps run back to back, and a refinement request's check of the backward
 * error is taken on the device, which starts its next inner solve in the same
 * tick (precision promotions are left to the host's next tick).  Every
 * request's arithmetic is that of ks_solve with the same parameters.
 * Optional outputs: solves in flight and queued. */
int ks_server_step(ks_server *sv, int32_t *n_inflight, int32_t *n_queued);

/* Up to cap finished requests: their tickets and infos (elapsed_ms = time
 * from submission to completion on the host clock).  *n_done = count. */
int ks_server_poll(ks_server *sv, uint64_t *tickets, ks_info *infos, int32_t cap, int32_t *n_done);

/* Budget bytes charged to admitted requests, in-flight and queued counts. */
int ks_server_stats(const ks_server *sv, size_t *bytes_in_use, int32_t *n_inflight,
                    int32_t *n_queued);

/* Free the server (waits for its stream; unfinished requests are dropped). */
void ks_server_free(ks_server *sv);

/* ---- kernel-level entry points ------------------------------------------
 * The solvers' own kernels, exposed for tests and measurement.  All enqueue
 * on `stream` and return without waiting. */

/* y = A v with A n x n row-major of element type a_dtype (KS_DT_*).  For
 * KS_DT_F64 v and y are binary64 with binary64 accumulation; for KS_DT_F32 and
 * KS_DT_BF16 they are binary32 with binary32 accumulation.  d_A must be
 * 16-byte aligned and lda * sizeof(element) a multiple of 16 (else KS_EINVAL);
 * d_v and d_y 16-byte aligned. */
int ks_gemv(int32_t n, int64_t lda, int32_t a_dtype, const void *d_A, const void *d_v,
            void *d_y, void *stream);

/* Q = A P for s <= KS_MAX_NRHS columns: the product that the lockstep CG for
 * many right-hand sides (the Krylov section's CG, one recurrence per column)
 * shares each iteration, on the matrix cores.  A: n x n row-major, element
 * type a_dtype: KS_DT_F64 (P, Q binary64, binary64 MFMA) or KS_DT_F32 (P, Q
 * binary32, binary32 MFMA with binary32 accumulation).  P and Q: column-major
 * n x s with leading dimension ldv >= n (column j at j * ldv), caller-owned,
 * Q not overlapping P; only columns 0 .. s-1 and rows 0 .. n-1 of them are
 * touched.  d_ws: caller-owned device workspace of at least
 * ks_gemm_mr_workspace_bytes(n, s, a_dtype) bytes (a padded copy of P and the
 * K-split partial products; overwritten), KS_ENOMEM below that.  d_A and d_ws
 * 16-byte aligned and lda * sizeof(element) a multiple of 16, else KS_EINVAL
 * (also for s outside 1 .. KS_MAX_NRHS or another a_dtype).  The sums over K
 * run in a fixed order: the same inputs give the same Q bit for bit.
 * Enqueued on `stream`. */
int ks_gemm_mr_workspace_bytes(int32_t n, int32_t s, int32_t a_dtype, size_t *bytes);
int ks_gemm_mr(int32_t n, int64_t lda, int32_t a_dtype, const void *d_A, int32_t s,
               const void *d_P, int64_t ldv, void *d_Q, void *d_ws, size_t ws_bytes,
               void *stream);

/* Symmetric product y = A x for a symmetric binary64 A, reading only the
 * lower triangle (elements (i, j) with i >= j; the values above the diagonal
 * never affect y).  d_ws: device workspace of at least
 * ks_symv_workspace_bytes(n) bytes, 16-byte aligned, owned by the caller
 * (tile partials, overwritten).  d_A 16-byte aligned with lda * 8 a multiple
 * of 16; d_x, d_y 16-byte aligned, not overlapping.  Enqueued on `stream`. */
int ks_symv_workspace_bytes(int32_t n, size_t *bytes);
int ks_symv(int32_t n, int64_t lda, const double *d_A, const double *d_x, double *d_y,
            void *d_ws, size_t ws_bytes, void *stream);

/* The same product for a symmetric binary32 A with binary32 x, y and binary32
 * accumulation (the product of CG's binary32 inner solves under
 * KS_FLAG_SYMMETRIC).  d_ws: at least ks_symv_workspace_bytes(n) / 2 bytes
 * (KS_ENOMEM below that).  d_A 16-byte aligned with lda * 4 a multiple of 16;
 * d_x, d_y, d_ws 16-byte aligned (else KS_EINVAL).  Enqueued on `stream`. */
int ks_symv_f32(int32_t n, int64_t lda, const float *d_A, const float *d_x, float *d_y,
                void *d_ws, size_t ws_bytes, void *stream);

/* ks_symv without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): it calls no allocating routine.  The tile partials
 * go to a fixed device array the library holds on every GPU it runs on until
 * the process ends (sized for n <= KS_SYMV_NOALLOC_MAX_N: 33.8 MB); a larger
 * n returns KS_ETOOLARGE before any device call.  Same kernels as ks_symv, so
 * the same y bit for bit.  All calls on one GPU share that array: calls that
 * overlap in time on one GPU (other streams, other host threads) race and must
 * be serialized by the caller.  Argument rules and errors otherwise as
 * ks_symv.  Enqueued on `stream`. */
#define KS_SYMV_NOALLOC_MAX_N 32768
int ks_symv_noalloc(int32_t n, int64_t lda, const double *d_A, const double *d_x, double *d_y,
                    void *stream);

/* Binary32 block LU with partial pivoting (the direct-methods section's block
 * algorithm, panels of 16 columns inside column blocks of 256 whose trailing
 * update runs on the matrix cores; the factorization GMRES-IR uses): d_LU
 * (n x lda_lu floats, row-major, lda_lu >= n) receives the binary32 rounding
 * of A factored in place, L (unit diagonal implied) below the diagonal and U
 * on and above it; d_piv[k] (n int32) is the row interchanged with row k at
 * step k, 0-based (whole rows, so P A = L U).  1 <= n <= 32768, else
 * KS_EINVAL.  *info = 0, or 1 + the first column whose pivot is zero (the
 * factorization goes on past it).  Allocates and frees a 16 KiB device work
 * area; returns after the factorization has finished on `stream` (KS_EHIP if
 * a panel's bounded wait for its other blocks gave up). */
int ks_lu32_factor(int32_t n, int64_t lda, const double *d_A, int64_t lda_lu, float *d_LU,
                   int32_t *d_piv, int32_t *info, void *stream);

/* Binary32 block Cholesky (the direct-methods section's Cholesky relations,
 * column blocks of 64, trailing updates on the matrix cores; the
 * factorization KS_IR_CHOL32 uses): d_L (n x ldl floats, row-major,
 * ldl >= n, ldl a multiple of 4, 16-byte aligned) receives the binary32
 * rounding of the symmetric A factored as L L^T, L on and below the diagonal
 * and L^T strictly above it.  *info = 0, or 1 + the first column whose pivot
 * is not positive (the factorization stops there; d_L is then partly
 * factored).  Allocates and frees one device word; returns after the
 * factorization has finished on `stream`. */
int ks_chol32_factor(int32_t n, int64_t lda, const double *d_A, int64_t ldl, float *d_L,
                     int32_t *info, void *stream);

/* Convert an n x n binary64 matrix (lda_src) into dst_dtype (KS_DT_F32:
 * round to nearest even; KS_DT_BF16: round to binary32, then to bfloat16,
 * both nearest even) with leading dimension lda_dst. */
int ks_convert(int32_t n, int64_t lda_src, const double *d_src, int32_t dst_dtype,
               int64_t lda_dst, void *d_dst, void *stream);

/* Streaming read of `bytes` bytes (multiple of 16) from d_src, with a
 * checksum written to d_sink[0]: the read ceiling of the memory system that
 * the GEMV is measured against. */
int ks_read_ceiling(const void *d_src, size_t bytes, double *d_sink, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */
