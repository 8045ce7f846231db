// Internal declarations of the dense Krylov library: the device-resident
// solver state, the workspace regions and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ks.h"

namespace ks {

constexpr int WAVE = 64;

// Flags word of State (device-resident; the host reads it after a sync).
enum : int32_t {
    F_STOP = 1,         // the inner Krylov loop is over: its kernels return at once
    F_CONV = 2,         // recursive residual / GMRES estimate met the tolerance
    F_MAXIT = 4,        // iteration limit
    F_BREAK = 8,        // CG p'Ap <= 0, or a zero Givens norm in GMRES
    F_NONFIN = 16,      // non-finite scalar inside the Krylov loop
    F_HAPPY = 32,       // GMRES happy breakdown (exact solution in the space)
    F_TRUE_OK = 64,     // last true residual met the tolerance
    F_TRUE_NONFIN = 128,// last true residual (or ||b||) not finite
    F_HALF = 256,       // BiCGSTAB ends on the half step x += alpha p (with
                        // F_CONV or F_MAXIT; F_STOP follows one kernel later)
    F_SETUP_END = 512   // server: the set-up ended the solve before its first
                        // step (b = 0, a non-finite or already small residual,
                        // no iterations allowed); no Krylov kernel ran
};
constexpr int32_t INNER_FLAGS = F_STOP | F_CONV | F_MAXIT | F_BREAK | F_NONFIN | F_HAPPY | F_HALF;

// Scalars of one solve, kept on the device so that no iteration needs the host.
// Within one kernel a field is either read by every block or written by
// block 0, never both (the next kernel sees the write at the kernel boundary).
struct alignas(256) State {
    double bnorm, binf;        // ||b||_2, ||b||_inf
    double thresh;             // tol * ||b||_2 (absolute residual threshold)
    double rho, rho_prev;      // CG r'r: current, and the value before the update
    double sigma, alpha, beta; // CG scalars
    double res, resinf, xinf;  // last true residual: ||r||_2, ||r||_inf, ||x||_inf
    double avk, hk1;           // GMRES: ||A v_k||, h(k+1,k)
    double anorm_inf;          // ||A||_inf
    double eta_tol;            // > 0: stop on the backward error eta_inf <= eta_tol
    double xinf_it;            // ||x||_inf of the CG iterate (backward-error stopping)
    double omega;              // BiCGSTAB stabilisation scalar
    int32_t iters;             // A*v products in the Krylov loop
    int32_t flags;
    int32_t k_done;            // GMRES: steps in the current cycle
    int32_t kcur;              // GMRES step counter of batched launches
    int32_t kcur_odd;          // the same counter for odd steps of a server tick
                               // (step c reads kcur / kcur_odd by parity, its
                               // Givens stage writes the other one)
    // fused small-n CG: per-launch copies of rho, iters and flags, alternating
    // between two slots so that no block reads a value another block of the
    // same launch writes
    double fz_rho[2];
    int32_t fz_iters[2];
    int32_t fz_flags[2];
    int32_t sync_fail;  // persistent kernels: a bounded grid-barrier wait gave up
    int32_t ir_next;    // server: the device's refinement check of this outer State (IR_*)
};
static_assert(sizeof(State) == 256, "one 256-byte State per solve");

// Per-column scalars of lockstep multi-right-hand-side CG (same rule as State).
struct ColState {
    double bnorm, binf, thresh;
    double rho, rho_prev, sigma;
    double res, resinf, xinf;
    int32_t iters, flags, restarts, pad;
};

// Per-block partial results, one region per producing kernel kind.
struct Partials {
    double *g;    // GEMV-shaped kernels: 3 per block
    double *v;    // vector kernels: 3 per block (r'r, ||x||_inf, ||r||_inf)
    double *h1;   // Gram-Schmidt pass 1: (m+1) per block
    double *h2;   // Gram-Schmidt pass 2: (m+1) per block
    double *nrm;  // ||w||^2 after pass 2: 1 per block
    double *w;    // BiCGSTAB x/r update: 4 per vector block (r'r, r0'r, ||x||_inf,
                  // ||r||_inf)
};

// Tuning of the dense matrix-vector product: a block of GEMV_NT threads owns
// GemvShape<TA>::ROWS rows and its threads split each row's columns in 16-byte
// chunks, UNR chunks in flight per lane (values from a sweep on MI355X: rows
// in {1,2,4,8,16}, threads in {128,256,512}, unroll in {1,2,4,8}).
constexpr int GEMV_NT = 256;
// Vector kernels: threads per block, elements per thread.
constexpr int VEC_NT = 256;
constexpr int VEC_EPT = 4;
// Gram-Schmidt kernels: one row per thread.
constexpr int CGS_NT = 256;
// Single-block reductions (||b||, finishing kernels).
constexpr int ONE_NT = 1024;

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
__host__ __device__ inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

__host__ __device__ inline int vec_blocks(int n) { return div_up(n, VEC_NT * VEC_EPT); }
__host__ __device__ inline int cgs_blocks(int n) { return div_up(n, CGS_NT); }

struct bf16_t {
    uint16_t bits;
};

template <typename TA>
struct GemvShape;
template <>
struct GemvShape<double> {
    static constexpr int ROWS = 2, UNR = 4;
};
template <>
struct GemvShape<float> {
    static constexpr int ROWS = 2, UNR = 4;
};
template <>
struct GemvShape<bf16_t> {
    // two 16-byte loads per row in flight per thread (not four): 62 VGPRs and
    // eight waves per SIMD instead of 80 and six; measured at n = 32768
    // 305 us against 349 us per product (the same sums in the same order)
    static constexpr int ROWS = 4, UNR = 2;
};
// blocks (= partials) of a GEMV-shaped launch on element type TA
template <typename TA>
__host__ __device__ inline int gemv_blocks(int n) {
    return div_up(n, GemvShape<TA>::ROWS);
}
// the largest of them, for sizing the partial region
__host__ __device__ inline int gemv_blocks_max(int n) { return div_up(n, 2); }

// Symmetric product (lower triangle only): SY_T x SY_T tiles, one block of
// SY_NT threads per tile; the workspace holds two SY_T-vectors per tile.
constexpr int SY_T = 256;
constexpr int SY_NT = 512;
__host__ __device__ inline int sy_tiles(int n) {
    const int t = div_up(n, SY_T);
    return t * (t + 1) / 2;
}
__host__ __device__ inline size_t sy_ws_doubles(int n) { return (size_t)sy_tiles(n) * 2 * SY_T; }
constexpr int SY_FIN = 64;  // elements per block of the finishing kernel
// CG with the symmetric product keeps, after W, one p'Ap share per tile and
// the r'r, ||x||_inf and ||r||_inf partials of the finishing blocks.
__host__ __device__ inline size_t sy_cg_doubles(int n) {
    return (size_t)round_up(sy_tiles(n), 32) + 3 * (size_t)div_up(n, SY_FIN);
}

// GMRES small dense arrays (binary64 always).
struct GmArrays {
    double *H;   // (m+1) x m unrotated Hessenberg, row-major, ld m
    double *R;   // (m+1) x m rotated copy (upper triangular after rotations)
    double *cs, *sn;  // m rotations
    double *g;   // m+1
    double *y;   // m
    double *h1;  // m+1: first Gram-Schmidt coefficients
    int m;
};

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.

// y = A v  (a_dtype: KS_DT_*)
hipError_t launch_gemv(int n, int64_t lda, int a_dtype, const void *A, const void *v, void *y,
                       hipStream_t s);

// ||b||_2, ||b||_inf into st; thresh = tol * ||b||_2; flags, iters, k_done
// reset; eta_tol = eta ? tol : 0 (stop on the normwise backward error).
template <typename T>
hipError_t launch_vec_stats(int n, const T *b, double tol, State *st, hipStream_t s, int eta = 0);

// r = b - A x, then st->rho = r'r, res, resinf, xinf and F_TRUE_OK /
// F_TRUE_NONFIN.  gate 1: only when the inner loop has stopped (F_STOP).
template <typename TA, typename T>
hipError_t launch_residual(int n, int64_t lda, const TA *A, const T *b, const T *x, T *r,
                           State *st, Partials P, int gate, hipStream_t s);

// the product kernel of launch_residual alone (3 partials per block into
// `partial`); gate 2: skipped once the loop has stopped
template <typename TA, typename T>
hipError_t launch_residual_rows(int n, int64_t lda, const TA *A, const T *b, const T *x, T *r,
                                const State *st, double *partial, int gate, hipStream_t s);

// Stationary methods (binary64).  d = diag(A), F_BREAK on a zero element;
// decide: residual metrics of the current iterate from `nblocks` residual
// partials, then stop or count one more update; begin: inner flags cleared.
hipError_t launch_st_diag(int n, int64_t lda, const double *A, double *d, State *st,
                          hipStream_t s);
hipError_t launch_st_decide(int nblocks, State *st, const double *partial, int max_iter,
                            hipStream_t s);
hipError_t launch_st_begin(State *st, hipStream_t s);
// Jacobi: x += r / d
hipError_t launch_jacobi_update(int n, double *x, const double *r, const double *d,
                                const State *st, hipStream_t s);
// Gauss-Seidel: u = U x, c = b - u (+ residual partials u_prev - u when
// with_res, gs_upper_blocks(n) blocks of 3); then the forward substitution
// (D + L) x = c, ceil(n / 64) launches, overwriting x and c.
int gs_upper_blocks(int n);
hipError_t launch_gs_upper(int n, int64_t lda, const double *A, const double *b, const double *x,
                           const double *u_prev, double *u, double *c, const State *st,
                           double *partial, int with_res, hipStream_t s);
hipError_t launch_gs_sweep(int n, int64_t lda, const double *A, double *x, double *c,
                           const State *st, hipStream_t s);

// Binary32 block LU with partial pivoting (GMRES-IR preconditioner): outer
// column blocks of 256, panels of LU_NB columns, n <= LU_MAX_N (a panel is
// held in the registers of at most LU_PANEL_MAX_BLOCKS blocks of
// LU_PANEL_ROWS rows).  factor: LU holds A in binary32 on entry, L (unit,
// below the diagonal) and U on return, piv[k] the row swapped with row k.
// work: LU_WORK_BYTES of device memory (4-byte aligned), owned by the call
// while it runs; on return its word 0 is 1 + the first zero pivot's column
// (0 if none) and word 1 is nonzero if a panel's bounded wait gave up.
constexpr int LU_NB = 16;
constexpr int LU_MAX_N = 32768;
constexpr int LU_PANEL_ROWS = 1024;
constexpr int LU_PANEL_MAX_BLOCKS = LU_MAX_N / LU_PANEL_ROWS;
constexpr size_t LU_WORK_BYTES = 16384;
hipError_t launch_lu_factor(int n, int64_t ldl, float *LU, int *piv, void *work, hipStream_t s);
// dst = U^-1 L^-1 P src (perm: (P v)_i = v[perm[i]]), t scratch; dst may be
// src; the squares of dst left in `partial` as the GMRES product leaves them
// xw: ts_persist_words(n) words of device memory for the persistent sweeps
// (one cooperative launch per substitution; the per-launch form, n/64
// launches per substitution, when xw is null), fail: set nonzero if one of
// their bounded waits gave up (cleared by each application)
size_t ts_persist_words(int n);
hipError_t launch_lu_apply(int n, int64_t ldl, const float *LU, const int *perm, const double *src,
                           double *dst, double *t, double *partial, uint64_t *xw, int *fail, hipStream_t s);
// ||w||_2 from launch_lu_apply's partials into st->rho / res, with the
// true-residual flags against st->thresh
hipError_t launch_lu_res_finish(int n, State *st, const double *partial, hipStream_t s);
// x += d
hipError_t launch_lu_xupdate(int n, double *x, const double *d, hipStream_t s);

// Binary32 block Cholesky (CG-IR preconditioner): column blocks of CH_NB,
// the trailing update on the matrix cores.  factor: L holds the binary32 A
// on entry (both triangles), L in the lower triangle and L^T in the strict
// upper one on return; info[0] = 1 + the first column with a non-positive
// pivot (0 if none; must be 0 on entry).
constexpr int CH_NB = 64;
hipError_t launch_chol_factor(int n, int64_t ldl, float *L, int *info, hipStream_t s);
// dst = L^-T L^-1 src (binary64 vectors, the factor widened); dst may be src
hipError_t launch_chol_apply(int n, int64_t ldl, const float *L, const double *src, double *dst,
                             uint64_t *xw, int *fail, hipStream_t s);
// preconditioned CG pieces: r'z partials (one per vector block), p = z with
// rho = r'z, and the stop test with p = z + beta p
hipError_t launch_pcg_dot(int n, const double *r, const double *z, const State *st, double *partial,
                          hipStream_t s);
hipError_t launch_pcg_begin(int n, const double *z, double *p, State *st, const double *rz_part,
                            hipStream_t s);
hipError_t launch_pcg_pupdate(int n, const double *z, double *p, State *st, const double *rr_part,
                              const double *rz_part, int max_iter, hipStream_t s);

// CG iteration, three kernels:
//   q = A p (sigma partials);  x += alpha p, r -= alpha q (rho' partials);
//   convergence / limit checks, p = r + beta p.
template <typename TA, typename T>
hipError_t launch_cg_matvec(int n, int64_t lda, const TA *A, const T *p, T *q, State *st,
                            Partials P, hipStream_t s);
// nsigma: number of partials the matrix-vector product left (gemv_blocks<TA>)
template <typename T>
hipError_t launch_cg_update(int n, T *x, T *r, const T *p, const T *q, State *st, Partials P,
                            int nsigma, hipStream_t s);
template <typename T>
hipError_t launch_cg_pupdate(int n, const T *r, T *p, State *st, Partials P, int max_iter,
                             hipStream_t s);
// the same with the r'r and ||x||_inf partials at prho ([nrho] each)
template <typename T>
hipError_t launch_cg_pupdate_from(int n, const T *r, T *p, State *st, const double *prho, int nrho,
                                  int max_iter, hipStream_t s);
// p = r, inner flags cleared (rho comes from the residual kernel).
template <typename T>
hipError_t launch_cg_begin(int n, const T *r, T *p, State *st, hipStream_t s);

// GMRES: cycle start, one Arnoldi step (matrix-vector product, two Gram-Schmidt
// passes, Givens update and normalisation), cycle end.  ev_before / ev_after
// (may be null) are recorded around the matrix-vector product.
template <typename T>
hipError_t launch_gm_begin(int n, const T *r, T *V, State *st, GmArrays ga, hipStream_t s);
// The Arnoldi step after the product w = A v_k: the two Gram-Schmidt passes,
// ||w||, the Givens rotation and v_{k+1} (launch_gm_step = product + this).
// ngemv: the number of ||w||^2 partials the product left in P.g.
template <typename T>
hipError_t launch_gm_ortho(int n, int ldv, T *V, T *w, int k, State *st, GmArrays ga, Partials P,
                           int ngemv, int max_iter, hipStream_t s);
template <typename TA, typename T>
hipError_t launch_gm_step(int n, int64_t lda, const TA *A, int ldv, T *V, T *w, int k,
                          State *st, GmArrays ga, Partials P, int max_iter, hipStream_t s,
                          hipEvent_t ev_before, hipEvent_t ev_after);
// w = A v_k with ||w||^2 partials (first kernel of the step)
template <typename TA, typename T>
hipError_t launch_gm_matvec(int n, int64_t lda, const TA *A, const T *vk, T *w, State *st,
                            Partials P, hipStream_t s);
template <typename T>
hipError_t launch_gm_finish(int n, int ldv, const T *V, T *x, State *st, GmArrays ga,
                            hipStream_t s);

// BiCGSTAB iteration, five kernels (two products with A):
//   begin: r0 = p = r, inner flags cleared (rho = r'r from the residual kernel)
//   v = A p (r0'v partials);  alpha, s = r - alpha v (s's partials);
//   t = A s (t's, t't partials; skipped on the half-step exit);
//   omega, x += alpha p + omega s, r = s - omega t (r'r, r0'r partials);
//   stop tests, beta, p = r + beta (p - omega v).
// vec = {r, r0, p, v, s, t}; ev_* (may be null) bracket the two products.
// the two products of the iteration (first and third kernels)
template <typename TA, typename T>
hipError_t launch_bs_vmatvec(int n, int64_t lda, const TA *A, const T *p, const T *r0, T *v,
                             State *st, Partials P, hipStream_t s);
template <typename TA, typename T>
hipError_t launch_bs_tmatvec(int n, int64_t lda, const TA *A, const T *sv, T *t, State *st,
                             Partials P, int max_iter, hipStream_t s);
template <typename T>
hipError_t launch_bs_begin(int n, const T *r, T *r0, T *p, State *st, hipStream_t s);
template <typename TA, typename T>
hipError_t launch_bs_iteration(int n, int64_t lda, const TA *A, T *x, T *const vec[6], State *st,
                               Partials P, int max_iter, hipStream_t s, hipEvent_t ev_v0,
                               hipEvent_t ev_v1, hipEvent_t ev_t0, hipEvent_t ev_t1);

// y = A x from the lower triangle of A (binary64).  W: sy_ws_doubles(n).
// st != nullptr: return at once when st has F_STOP (CG loop).  p != nullptr:
// partial[b] = sum of p_j y_j over finishing block b (symv_finish_blocks(n)).
int symv_finish_blocks(int n);
hipError_t launch_symv(int n, int64_t lda, const double *A, const double *x, double *y,
                       double *W, const State *st, const double *p, double *partial,
                       hipStream_t s);

// The product and update of one binary64 CG iteration with the symmetric
// product, in two launches.  The tile blocks also leave their share of p'Ap,
// p_I'(row part) + p_J'(column part), in sig[tile]; the finishing blocks sum
// q = A p as launch_symv does, reduce sigma = p'q from the shares (the same
// fixed order in every block), and apply alpha = rho / sigma: x += alpha p,
// r -= alpha q on their elements (q is not stored), recording the iteration in
// st as launch_cg_update does.  rho_part: [r'r partials][||x||_inf partials],
// symv_finish_blocks(n) each, for launch_cg_pupdate_f64.  W, sig and rho_part
// lie in one region of sy_ws_doubles(n) + sy_cg_doubles(n) doubles.
hipError_t launch_symv_cg(int n, int64_t lda, const double *A, const double *p, double *x,
                          double *r, double *region, State *st, hipStream_t s);
// where the r'r partials of launch_symv_cg lie in that region
__host__ __device__ inline double *symv_cg_rho_part(int n, double *region) {
    return region + sy_ws_doubles(n) + round_up(sy_tiles(n), 32);
}

// The same two products for binary32 A and vectors with binary32
// accumulation (the inner solves of refinement): y = A x from the lower
// triangle (W: at least sy_ws_doubles(n) doubles, used as floats), and CG's
// product and update in two launches (region as for launch_symv_cg, W as
// floats; the shares of p'Ap and the partials binary64).
hipError_t launch_symv32(int n, int64_t lda, const float *A, const float *x, float *y, float *W,
                         hipStream_t s);
hipError_t launch_symv32_cg(int n, int64_t lda, const float *A, const float *p, float *x, float *r,
                            double *region, State *st, hipStream_t s);

// Fused small-n CG (n <= FZ_MAX_N, binary64, no backward-error stopping): one
// launch per iteration instead of three, bitwise the same arithmetic.
//   fz_start: q0 = A p0 with the p'q partials into pg[0]; slot 0 = (rho, iters, flags)
//   fz_step:  launch k (cur = k % 2) turns the partials of q_k = A p_k into
//             alpha, x += alpha p_k, r_{k+1}, rho', the stop test, beta,
//             p_{k+1} and q_{k+1} = A p_{k+1}; slot[1 - cur] for the next launch
//   fz_publish: slot `which` -> st->rho, iters, flags
// vec = {r0, r1, p0, p1, q0, q1}, pg = {partials 0, partials 1}
constexpr int FZ_MAX_N = 4096;
hipError_t launch_fz_start(int n, int64_t lda, const double *A, const double *p0, double *q0,
                           State *st, double *pg0, hipStream_t s);
hipError_t launch_fz_step(int n, int64_t lda, const double *A, double *x, double *const vec[6],
                          State *st, double *const pg[2], int cur, int max_iter, hipStream_t s);
hipError_t launch_fz_publish(State *st, int which, hipStream_t s);
// The same iterations in one cooperative launch for n <= fz_persist_max_n():
// up to nsteps iterations from slot `cur`, the blocks exchanging each
// iteration's q and p'q partials as tagged words (the blocks' rows of A read
// once per launch).  bar: fz_bar_words(n) 32-bit words for that exchange
// (reset by the launcher, with st->sync_fail).  Slot (cur + nsteps) % 2 holds
// the result, as after nsteps fz_step launches.  A bounded wait that gives up
// sets st->sync_fail.
constexpr int FZ_BAR_STRIDE = 1;       // words between two blocks' flags of grid_barrier
constexpr int FZ_BAR_MAX_WORDS = 256 * 48;
int fz_persist_max_n();
size_t fz_bar_words(int n);
hipError_t launch_fz_persist(int n, int64_t lda, const double *A, double *x, double *const vec[6],
                             State *st, double *const pg[2], int cur, int nsteps, int max_iter,
                             uint32_t *bar, uint32_t spin_limit, hipStream_t s);

// ||A||_inf into st->anorm_inf
hipError_t launch_norm_inf(int n, int64_t lda, const double *A, State *st, Partials P,
                           hipStream_t s);
// dst = convert(src), padding columns zeroed
hipError_t launch_convert(int n, int64_t lda_src, const double *src, int dst_dtype,
                          int64_t lda_dst, void *dst, hipStream_t s);
hipError_t launch_copy_pad(int n, int64_t lda_src, const double *src, int64_t lda_dst,
                           double *dst, hipStream_t s);

// IR helpers
// r32 = (float)(r / st->res)
hipError_t launch_ir_scale_cast(int n, const double *r, float *r32, const State *st,
                                hipStream_t s);
// x += (*scale) * (double)d32
hipError_t launch_ir_update(int n, double *x, const float *d32, const double *scale,
                            hipStream_t s);
template <typename T>
hipError_t launch_fill(int n, T *x, T value, hipStream_t s);

hipError_t launch_read_ceiling(const void *src, size_t bytes, double *sink, hipStream_t s);

// ------------------------------------------------------- batched launches
// One in-flight solve of the request server: A in TA, vectors in T (binary64
// solves and refinement outer steps: double/double; inner solves of the
// mixed-precision requests: float/float or bf16_t/float).
template <typename TA, typename T>
struct BatchItemT {
    const TA *A;
    int64_t lda;
    int n, ldv, m, max_iter;
    double tol;
    int eta;            // stop on the backward error
    int pad;
    const T *b;
    T *x;
    T *resid;           // r (CG) or w (GMRES): the residual kernel's output
    T *p, *q, *V;       // CG search direction and product; GMRES basis
    State *st;
    Partials P;
    GmArrays ga;
    // server: an inner solve whose refinement check ran on the device in
    // this tick (the outer State); its kernels run only if that check said
    // IR_GO.  nullptr otherwise.
    const State *outer;
    // CG with the symmetric product (KS_FLAG_SYMMETRIC): the region of its
    // tile partials, shares of p'Ap and r'r partials (binary32 solves keep
    // their tile partials as floats in it); nullptr for the general product
    double *sy;
};
using BatchItem = BatchItemT<double, double>;
// A subset of items for one launch: offs[i] = first block of idx[i]'s grid.
template <typename Item>
struct BatchSetT {
    const Item *items;
    const int *idx;
    const int *offs;
    int count;
};
using BatchSet = BatchSetT<BatchItem>;
enum BatchKernel {
    BK_VEC_STATS, BK_NORM_INF, BK_NORM_INF_FINISH, BK_RESIDUAL, BK_RESIDUAL_FINISH,
    BK_CG_BEGIN, BK_GM_BEGIN, BK_GM_FINISH, BK_GATHER
};
// blocks = offs[count]; gate for the residual / finish kernels.  BK_NORM_INF
// and BK_NORM_INF_FINISH exist for binary64 items only.
template <typename TA, typename T>
hipError_t batch_launch(BatchKernel kind, const BatchSetT<BatchItemT<TA, T>> &bs, int blocks,
                        int gate, hipStream_t s, State *staging);

// One stage of a server tick: the same position of one Krylov step for the
// CG and GMRES items of every storage type, in one launch (blocks of 256
// threads; each entry = one item's grid for its kernel kind).
//   stage 1: CG q = A p            | GMRES w = A v_k
//   stage 2: CG x, r update        | GMRES Gram-Schmidt pass 0
//   stage 3: CG p update           | GMRES pass 1
//   stage 4:                       | GMRES pass 2
//   stage 5:                       | GMRES Givens rotation (and the step counter)
//   (CG with the symmetric product: its tiles and finishing sum with the
//   update run as the batched launches below, between stages 1 and 2 and
//   between stages 2 and 3; its p update in stage 3)
enum StageKind : int32_t {
    SK_CG_MATVEC, SK_CG_UPDATE, SK_CG_PUPDATE, SK_GM_MATVEC, SK_GM_CGS0, SK_GM_CGS1, SK_GM_CGS2,
    SK_GM_GIVENS, SK_SY_PUPDATE
};
struct StageSet {
    const BatchItemT<double, double> *i64;  // the items' binary64 views (index = slot)
    const BatchItemT<float, float> *i32;    // binary32 inner solves
    const BatchItemT<bf16_t, float> *i16;   // bfloat16 inner solves
    const int *idx;    // slot of entry e
    const int *kind;   // StageKind | (storage << 8), storage 0 binary64, 1 binary32, 2 bfloat16
    const int *offs;   // first block of entry e (offs[count] = blocks)
    int count;
};
// stage 2..5, or 10 + storage for the product stage (one launch per
// storage); step: the step's index in the tick (its parity selects the
// GMRES step counter); blocks = offs[count]
hipError_t stage_launch(const StageSet &ss, int stage, int blocks, int step, hipStream_t s);

// The symmetric CG product of a set of solves (items with sy != nullptr):
// the tiles (which = 0; blocks = sum of sy_tiles(n)) or the finishing sum with
// the x, r update (which = 1; blocks = sum of symv_finish_blocks(n)), binary64
// or, for binary32 inner solves, binary32.
hipError_t batch_symv(int which, const BatchSetT<BatchItemT<double, double>> &bs, int blocks,
                      hipStream_t s);
hipError_t batch_symv32(int which, const BatchSetT<BatchItemT<float, float>> &bs, int blocks,
                        hipStream_t s);

// One refinement step of a mixed-precision request (the vector work between
// its binary64 outer residual and its inner solve), and the inputs of its
// refinement check on the device: the host's counters as of the tick.
struct IrItem {
    int n;
    const double *r64;  // outer residual
    float *rhs;         // inner right-hand side r / ||r||
    float *d;           // inner solution (correction)
    double *x;          // the request's iterate
    State *st;          // outer State (st->res = ||r||)
    State *inner;       // the inner solve's State
    double tol;         // backward-error target
    double eta_prev;    // backward error of the previous check (inf at first)
    int outer_steps, max_outer, bad, prec;
    int first;          // the first check (after the set-up of b and r0)
    int gated;          // the check ran on the device in this tick: the inner
                        // set-up runs only if it said IR_GO
};
using IrSet = BatchSetT<IrItem>;
enum IrKernel { IK_SCALE, IK_ZERO_D, IK_UPDATE, IK_DECIDE };
// Outcomes of the device refinement check (State::ir_next), the host's
// check in the same arithmetic: go on with an inner solve; stop (backward
// error met, b = 0, the step limit, non-finite); or a precision promotion,
// which the host carries out.
enum IrNext : int32_t { IR_NONE = 0, IR_GO, IR_DONE, IR_ZERO, IR_STAG, IR_NONFIN, IR_PROMOTE };
hipError_t ir_batch_launch(IrKernel kind, const IrSet &bs, int blocks, hipStream_t s);
// staging[i] = *d_ptrs[i] (device array of State pointers)
hipError_t gather_states(const State *const *d_ptrs, int count, State *staging, hipStream_t s);

// ------------------------------------------------ multi-right-hand-side CG
// n x s column-major blocks with leading dimension ldv; s <= KS_MAX_NRHS.
int mr_splits(int n, int elem_bytes);  // K splits of the contraction (8: binary64, 4: binary32)
int mr_blocks(int n);          // blocks of the per-column kernels
template <typename T>
hipError_t launch_mr_gemm(int n, int64_t lda, const T *A, const T *P, int ldp, T *Qpart, int ldq,
                          int s, const State *st, int gate, hipStream_t strm);
template <typename T>
hipError_t launch_mr_stats(int n, int s, const T *B, int ldb, double tol, ColState *cols,
                           State *st, hipStream_t strm);
// R = B - A X with per-column norms (gate 1: only when every column stopped)
template <typename T>
hipError_t launch_mr_residual(int n, int64_t lda, const T *A, int s, const T *B, int ldb,
                              const T *X, T *Qpart, T *R, int ldv, double *part, ColState *cols,
                              State *st, int gate, hipStream_t strm);
template <typename T>
hipError_t launch_mr_begin(int n, int s, const T *R, T *P, int ldv, ColState *cols, State *st,
                           uint64_t mask, hipStream_t strm);
// one lockstep iteration: Q = A P (MFMA), alpha, x/r update, stop tests, p update
template <typename T>
hipError_t launch_mr_iteration(int n, int64_t lda, const T *A, int s, T *X, T *R, T *P, T *Q,
                               T *Qpart, int ldv, double *part_a, double *part_b, ColState *cols,
                               State *st, int max_iter, hipStream_t strm, hipEvent_t e0,
                               hipEvent_t e1);
template <typename T>
hipError_t launch_mr_copy(int n, int s, const T *src, int lds, T *dst, int ldd, hipStream_t strm);
size_t mr_product_ws_bytes(int n, int s, int elem_bytes);
template <typename T>
hipError_t launch_mr_product(int n, int64_t lda, const T *A, int s, const T *P, int64_t ldv, T *Q,
                             void *ws, hipStream_t strm);
hipError_t launch_mr_ir_scale(int n, int s, const double *R, int ldv, float *rhs,
                              const ColState *cols, uint64_t mask, hipStream_t strm);
hipError_t launch_mr_ir_update(int n, int s, double *X, const float *D, int ldv,
                               const ColState *cols, uint64_t mask, hipStream_t strm);

}  // namespace ks
