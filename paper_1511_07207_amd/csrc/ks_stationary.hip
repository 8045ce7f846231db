// Jacobi and Gauss-Seidel, the classical stationary iterations that the
// paper's library offers beside CG, GMRES and BiCGSTAB (introductory section
// and the parallel-implementation section; timed in Tables 1-2).  binary64,
// one right-hand side.  With A = L + D + U (strictly lower, diagonal,
// strictly upper):
//
//   Jacobi        x(k+1) = x(k) + D^-1 (b - A x(k))
//                 one full product per update; the product is the true
//                 residual of x(k), so the stop test costs nothing extra.
//
//   Gauss-Seidel  (D + L) x(k+1) = b - U x(k)
//                 one product with the strict upper triangle, u(k) = U x(k),
//                 then a forward substitution with D + L.  Since
//                 (D + L) x(k) = b - u(k-1), the residual of x(k) is
//                 b - A x(k) = u(k-1) - u(k): the upper product also yields
//                 the residual of the current iterate, and the sweep reads the
//                 lower triangle once, so an update reads A once in all.
//
// Forward substitution (the one sequential part).  The rows are taken in
// blocks of GS_SB = 64, two per launch: launch J
//   - in its first block: subtracts from c = b - U x(k) the contribution of
//     the two column blocks solved by launch J - 1 to rows of blocks 2J and
//     2J + 1, solves block 2J's 64 x 64 lower-triangular diagonal tile by
//     substitution in one wave (lane i holds row i; x_j is broadcast from
//     lane j with readlane, one fused multiply-add per lane and step),
//     subtracts its x from block 2J + 1's rows and solves that block too;
//   - in its other blocks: subtracts the contribution of the previous two
//     column blocks from the rows below (one wave instruction per row).
// So every row has all the columns to its left subtracted before its own
// solve.  No block of a launch waits on another (no spin-waits); the
// launches are ordered by the stream.  Two blocks per launch halve the
// launches, whose fixed cost (one memory round trip, start and end) was most
// of a 64-row step.
// The substitution multiplies by the reciprocal of the diagonal element (one
// rounding more than a division; the division would sit on the sequential
// path 64 times per step).
#include "ks_gemv_body.h"

namespace ks {

constexpr int GS_SB = 64;                     // rows per substitution step
constexpr int GS_PW = 8;                      // rows per wave per pass in the row updates
constexpr int GS_LDT = GS_SB + 1;             // LDS row stride of the diagonal tile (padded)
constexpr int GS_ROWS = GemvShape<double>::ROWS;  // rows per block of the upper product
constexpr int GS_UNR = GemvShape<double>::UNR;    // column chunks in flight per thread
static_assert(GS_SB == WAVE, "one lane per row of the diagonal tile, one per panel column");

// --------------------------------------------------------------- common
// d = diag(A); F_BREAK | F_STOP when an element is zero (one block)
__global__ __launch_bounds__(ONE_NT) void st_diag_kernel(int n, int64_t lda,
                                                         const double *__restrict__ A,
                                                         double *__restrict__ d, State *st) {
    int zero = 0;
    for (int i = threadIdx.x; i < n; i += ONE_NT) {
        const double a = A[(int64_t)i * lda + i];
        d[i] = a;
        zero |= (a == 0.0);
    }
    zero = __syncthreads_or(zero);
    if (threadIdx.x == 0 && zero) st->flags |= F_BREAK | F_STOP;
}

// After a residual's partials: the true-residual metrics and flags of the
// current iterate (as the residual's finishing kernel), then the decision:
// stop (converged, non-finite, iteration limit) or count one more update.
// One block, so that no other block reads `iters` while it changes.
__global__ __launch_bounds__(ONE_NT) void st_decide_kernel(int nblocks, State *st,
                                                           const double *partial, int max_iter) {
    if (st->flags & F_STOP) return;
    residual_finish_body(nblocks, st, partial, 0);
    __syncthreads();
    if (threadIdx.x == 0) {
        int f = st->flags;
        if (f & F_TRUE_NONFIN)
            f |= F_NONFIN | F_STOP;
        else if (f & F_TRUE_OK)
            f |= F_CONV | F_STOP;
        else if (st->iters >= max_iter)
            f |= F_MAXIT | F_STOP;
        else
            st->iters += 1;
        st->flags = f;
    }
}

// start of a cycle: inner flags cleared (the true residual's are kept)
__global__ void st_begin_kernel(State *st) {
    if (threadIdx.x == 0) st->flags &= ~INNER_FLAGS;
}

// --------------------------------------------------------------- Jacobi
// x += r / d for every element (r = b - A x from the product just made)
__global__ __launch_bounds__(VEC_NT) void jacobi_update_kernel(int n, double *__restrict__ x,
                                                               const double *__restrict__ r,
                                                               const double *__restrict__ d,
                                                               const State *st) {
    const int base = blockIdx.x * VEC_NT * VEC_EPT + threadIdx.x;
    double xv[VEC_EPT], rv[VEC_EPT], dv[VEC_EPT];
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = min(base + e * VEC_NT, n - 1);
        xv[e] = x[i];
        rv[e] = r[i];
        dv[e] = d[i];
    }
    if (st->flags & F_STOP) return;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) x[i] = xv[e] + rv[e] / dv[e];
    }
}

// --------------------------------------------------------- Gauss-Seidel
// u = U x (columns j > i of each row), c = b - u; with_res: the residual of
// x, u_prev - u, reduced into 3 partials per block as the residual kernel
// leaves them (r'r, max |r_i|, max |x_i|).  GS_ROWS rows per block, each
// thread two adjacent columns per 2 * GEMV_NT-column chunk, starting at the
// chunk that holds the first column right of the block's first row.
__global__ __launch_bounds__(GEMV_NT) void gs_upper_kernel(int n, int64_t lda,
                                                           const double *__restrict__ A,
                                                           const double *__restrict__ b,
                                                           const double *__restrict__ x,
                                                           const double *__restrict__ u_prev,
                                                           double *__restrict__ u,
                                                           double *__restrict__ c, const State *st,
                                                           double *partial, int with_res) {
    if (st->flags & F_STOP) return;
    constexpr int STEP = 2 * GEMV_NT;
    const int row0 = blockIdx.x * GS_ROWS;
    const double *rp[GS_ROWS];
    double acc[GS_ROWS];
#pragma unroll
    for (int r = 0; r < GS_ROWS; ++r) {
        rp[r] = A + (int64_t)min(row0 + r, n - 1) * lda;
        acc[r] = 0.0;
    }
    const int nfull = n / STEP;
    int s = (row0 + 1) / STEP;
    // GS_UNR chunks in flight per thread, then one at a time
    for (; s + GS_UNR <= nfull; s += GS_UNR) {
        d2v xv[GS_UNR], a[GS_UNR][GS_ROWS];
#pragma unroll
        for (int q = 0; q < GS_UNR; ++q) {
            const int col = (s + q) * STEP + 2 * threadIdx.x;
            xv[q] = *reinterpret_cast<const d2v *>(x + col);
#pragma unroll
            for (int r = 0; r < GS_ROWS; ++r) a[q][r] = load_a<double>(rp[r] + col);
        }
#pragma unroll
        for (int q = 0; q < GS_UNR; ++q) {
            const int col = (s + q) * STEP + 2 * threadIdx.x;
#pragma unroll
            for (int r = 0; r < GS_ROWS; ++r) {
                const int row = row0 + r;
                acc[r] = fma(col > row ? a[q][r].x : 0.0, xv[q].x, acc[r]);
                acc[r] = fma(col + 1 > row ? a[q][r].y : 0.0, xv[q].y, acc[r]);
            }
        }
    }
    for (; s < nfull; ++s) {
        const int col = s * STEP + 2 * threadIdx.x;
        const d2v xv = *reinterpret_cast<const d2v *>(x + col);
#pragma unroll
        for (int r = 0; r < GS_ROWS; ++r) {
            const d2v a = load_a<double>(rp[r] + col);
            const int row = row0 + r;
            acc[r] = fma(col > row ? a.x : 0.0, xv.x, acc[r]);
            acc[r] = fma(col + 1 > row ? a.y : 0.0, xv.y, acc[r]);
        }
    }
    {
        const int col = nfull * STEP + 2 * threadIdx.x;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int j = col + e;
            if (j < n) {
                const double xj = x[j];
#pragma unroll
                for (int r = 0; r < GS_ROWS; ++r)
                    if (j > row0 + r) acc[r] = fma(rp[r][j], xj, acc[r]);
            }
        }
    }
    const double out = reduce_rows<double, GS_ROWS, GEMV_NT>(acc);
    const int row = row0 + threadIdx.x;
    double s2 = 0.0, rmax = 0.0, xmax = 0.0;
    if (threadIdx.x < GS_ROWS && row < n) {
        u[row] = out;
        c[row] = b[row] - out;
        if (with_res) {
            const double ri = u_prev[row] - out;
            s2 = ri * ri;
            rmax = fabs(ri);
            xmax = fabs(x[row]);
            if (!finite_d(rmax)) rmax = INFINITY;
            if (!finite_d(xmax)) xmax = INFINITY;
        }
    }
    if (with_res && threadIdx.x < WAVE) {
        const double t0 = wave_sum(s2);
        const double t1 = wave_max(rmax);
        const double t2 = wave_max(xmax);
        if (threadIdx.x == 0) {
            partial[3 * blockIdx.x + 0] = t0;
            partial[3 * blockIdx.x + 1] = t1;
            partial[3 * blockIdx.x + 2] = t2;
        }
    }
}

__device__ __forceinline__ double gs_readlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Launch J of a sweep solves the two 64-row blocks B0 = 2J and B1 = 2J + 1
// (rows r0 = 128 J ..).  Block 0 (GS_SWT waves) issues every load first:
// both diagonal tiles (to LDS), the 64 x 64 tile coupling B1 to B0's columns,
// and the rows of B0 and B1 over the 128 columns solved by the launch before
// (cb = r0 - 128 ..).  Then wave 0 solves B0, all waves apply x_B0 to B1's
// rows through the coupling tile, and wave 0 solves B1.  The launch's other
// blocks subtract the 128 columns cb .. from the rows below B1, GS_SWT * 8
// rows per block, two columns per lane.
constexpr int GS_SWT = 8;                       // waves per block
constexpr int GS_SNT = GS_SWT * WAVE;
constexpr int GS_SPR = GS_SWT * GS_PW;          // rows per row-update block (64)
constexpr int GS_TQ = GS_SB * 2 / GS_SWT;       // rows of the two diagonal tiles per wave (16)
constexpr int GS_UQ = GS_SB / GS_SWT;           // rows of B0 (and of B1) per wave (8)

typedef double gs_d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void gs_solve_tile(const double *T, double acc, double dinv, int lane,
                                              double &xi) {
    // forward substitution in one wave: lane i holds row i
#pragma unroll
    for (int j = 0; j < GS_SB; ++j) {
        const double xc = acc * dinv;
        const double xj = gs_readlane(xc, j);
        xi = (lane == j) ? xc : xi;
        acc = fma(-T[lane * GS_LDT + j], xj, acc);
    }
}

__global__ __launch_bounds__(GS_SNT) void gs_sweep_kernel(int n, int64_t lda,
                                                          const double *__restrict__ A,
                                                          double *__restrict__ x,
                                                          double *__restrict__ c, const State *st,
                                                          int J) {
    __shared__ double T0[GS_SB * GS_LDT], T1[GS_SB * GS_LDT];
    __shared__ double s0[GS_SB], s1[GS_SB], s1b[GS_SB], xb0[GS_SB];
    if (st->flags & F_STOP) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int r0 = 2 * J * GS_SB;
    const int cb = r0 - 2 * GS_SB;  // the 128 columns solved in launch J - 1 (J >= 1)
    gs_d2 xl = {0.0, 0.0};
    if (J >= 1) xl = *reinterpret_cast<const gs_d2 *>(x + cb + 2 * lane);
    if (blockIdx.x > 0) {
        const int rs = r0 + 2 * GS_SB + (blockIdx.x - 1) * GS_SPR + w * GS_PW;
        gs_d2 v[GS_PW];
#pragma unroll
        for (int k = 0; k < GS_PW; ++k)
            v[k] = load_a<double>(A + (int64_t)min(rs + k, n - 1) * lda + cb + 2 * lane);
        double pv[GS_PW];
#pragma unroll
        for (int k = 0; k < GS_PW; ++k) pv[k] = fma(v[k].y, xl.y, v[k].x * xl.x);
        const double sm = rows_reduce<GS_PW>(pv, lane);
        constexpr int PLR = WAVE / GS_PW;
        if (lane % PLR == 0 && rs + lane / PLR < n) c[rs + lane / PLR] -= sm;
        return;
    }
    const int m0 = min(GS_SB, n - r0);
    const int r1 = r0 + GS_SB;
    const bool has1 = r1 < n;
    const int m1 = has1 ? min(GS_SB, n - r1) : 0;
    // ---- all loads: diagonal tiles (rows k = w + GS_SWT q: q < 8 for B0, 8.. for B1),
    // B0 / B1 rows over the previous columns, the coupling tile
    double tl[GS_TQ], tc[GS_UQ];
    gs_d2 u0[GS_UQ], u1[GS_UQ];
#pragma unroll
    for (int q = 0; q < GS_TQ; ++q) {
        const int k = w + GS_SWT * q;  // 0 .. 127
        if (k < GS_SB)
            tl[q] = A[(int64_t)(r0 + min(k, m0 - 1)) * lda + r0 + min(lane, m0 - 1)];
        else if (has1)
            tl[q] = A[(int64_t)(r1 + min(k - GS_SB, m1 - 1)) * lda + r1 + min(lane, m1 - 1)];
        else
            tl[q] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < GS_UQ; ++q) {
        const int k = w * GS_UQ + q;  // row of the block
        if (J >= 1) {
            u0[q] = load_a<double>(A + (int64_t)(r0 + min(k, m0 - 1)) * lda + cb + 2 * lane);
            if (has1) u1[q] = load_a<double>(A + (int64_t)(r1 + min(k, m1 - 1)) * lda + cb + 2 * lane);
        }
        tc[q] = has1 ? A[(int64_t)(r1 + min(k, m1 - 1)) * lda + r0 + min(lane, m0 - 1)] : 0.0;
    }
    const double c0 = (w == 0 && lane < m0) ? c[r0 + lane] : 0.0;
    const double c1 = (w == 0 && lane < m1) ? c[r1 + lane] : 0.0;
    // ---- the diagonal tiles into LDS, lower part; rows past n get a unit diagonal
#pragma unroll
    for (int q = 0; q < GS_TQ; ++q) {
        const int k = w + GS_SWT * q;
        if (k < GS_SB) {
            T0[k * GS_LDT + lane] = (k < m0 && lane < m0) ? (lane <= k ? tl[q] : 0.0) : (lane == k ? 1.0 : 0.0);
        } else {
            const int kk = k - GS_SB;
            T1[kk * GS_LDT + lane] = (kk < m1 && lane < m1) ? (lane <= kk ? tl[q] : 0.0) : (lane == kk ? 1.0 : 0.0);
        }
    }
    // ---- sums over the previous columns, the wave's 8 rows of each block at
    // once (halving butterfly: lane group g = lane / 8 ends with row g)
    constexpr int LPR = WAVE / GS_UQ;
    {
        double v0[GS_UQ], v1[GS_UQ];
#pragma unroll
        for (int q = 0; q < GS_UQ; ++q) {
            v0[q] = J >= 1 ? fma(u0[q].y, xl.y, u0[q].x * xl.x) : 0.0;
            v1[q] = (J >= 1 && has1) ? fma(u1[q].y, xl.y, u1[q].x * xl.x) : 0.0;
        }
        const double a0 = rows_reduce<GS_UQ>(v0, lane);
        const double a1 = rows_reduce<GS_UQ>(v1, lane);
        if (lane % LPR == 0) {
            s0[w * GS_UQ + lane / LPR] = a0;
            s1[w * GS_UQ + lane / LPR] = a1;
        }
    }
    __syncthreads();
    // ---- B0
    if (w == 0) {
        double xi = 0.0;
        gs_solve_tile(T0, lane < m0 ? c0 - s0[lane] : 0.0, 1.0 / T0[lane * GS_LDT + lane], lane, xi);
        xb0[lane] = lane < m0 ? xi : 0.0;
        if (lane < m0) x[r0 + lane] = xi;
    }
    __syncthreads();
    if (!has1) return;
    // ---- B1's rows less the coupling tile times x_B0
    const double xv = xb0[lane];
    {
        double v[GS_UQ];
#pragma unroll
        for (int q = 0; q < GS_UQ; ++q) v[q] = (lane < m0 ? tc[q] : 0.0) * xv;
        const double sm = rows_reduce<GS_UQ>(v, lane);
        if (lane % LPR == 0) s1b[w * GS_UQ + lane / LPR] = sm;
    }
    __syncthreads();
    if (w == 0) {
        double xi = 0.0;
        gs_solve_tile(T1, lane < m1 ? (c1 - s1[lane]) - s1b[lane] : 0.0,
                      1.0 / T1[lane * GS_LDT + lane], lane, xi);
        if (lane < m1) x[r1 + lane] = xi;
    }
}

// ------------------------------------------------------------- launchers
hipError_t launch_st_diag(int n, int64_t lda, const double *A, double *d, State *st,
                          hipStream_t s) {
    st_diag_kernel<<<1, ONE_NT, 0, s>>>(n, lda, A, d, st);
    return hipGetLastError();
}

hipError_t launch_st_decide(int nblocks, State *st, const double *partial, int max_iter,
                            hipStream_t s) {
    st_decide_kernel<<<1, ONE_NT, 0, s>>>(nblocks, st, partial, max_iter);
    return hipGetLastError();
}

hipError_t launch_st_begin(State *st, hipStream_t s) {
    st_begin_kernel<<<1, WAVE, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_jacobi_update(int n, double *x, const double *r, const double *d,
                                const State *st, hipStream_t s) {
    jacobi_update_kernel<<<vec_blocks(n), VEC_NT, 0, s>>>(n, x, r, d, st);
    return hipGetLastError();
}

int gs_upper_blocks(int n) { return div_up(n, GS_ROWS); }

hipError_t launch_gs_upper(int n, int64_t lda, const double *A, const double *b, const double *x,
                           const double *u_prev, double *u, double *c, const State *st,
                           double *partial, int with_res, hipStream_t s) {
    gs_upper_kernel<<<gs_upper_blocks(n), GEMV_NT, 0, s>>>(n, lda, A, b, x, u_prev, u, c, st,
                                                          partial, with_res);
    return hipGetLastError();
}

hipError_t launch_gs_sweep(int n, int64_t lda, const double *A, double *x, double *c,
                           const State *st, hipStream_t s) {
    const int nl = div_up(n, 2 * GS_SB);
    for (int J = 0; J < nl; ++J) {
        const int below = n - (J + 1) * 2 * GS_SB;
        const int blocks = 1 + ((J >= 1 && below > 0) ? div_up(below, GS_SPR) : 0);
        gs_sweep_kernel<<<blocks, GS_SNT, 0, s>>>(n, lda, A, x, c, st, J);
    }
    return hipGetLastError();
}

}  // namespace ks
