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
// steps of GS_SB = 64; launch I of a sweep
//   - in its first block: subtracts from c = b - U x(k) the contribution of
//     column block I - 1 (just solved) to rows of block I, then solves the
//     64 x 64 lower-triangular diagonal tile of block I by substitution in
//     one wave (lane i holds row i; x_j is broadcast from lane j with
//     readlane, one fused multiply-add per lane and step), and writes x_I;
//   - in its other blocks: subtracts the contribution of column block I - 1
//     from the rows below block I (the panel, one wave instruction per row).
// So column block J reaches the rows below block J + 1 in launch J + 1, and
// block J + 1 itself in launch J + 1's first block: every row has all the
// columns to its left subtracted before its own step.  No block of a launch
// waits on another (no spin-waits); the steps are ordered by the stream.
// The substitution multiplies by the reciprocal of the diagonal element (one
// rounding more than a division; the division would sit on the sequential
// path 64 times per step).
#include "ks_gemv_body.h"

namespace ks {

constexpr int GS_SB = 64;                     // rows per substitution step
constexpr int GS_PW = 8;                      // rows per wave per pass in the row updates
constexpr int GS_WAVES = GEMV_NT / WAVE;      // waves per block
constexpr int GS_PR = GS_WAVES * GS_PW;       // rows per panel block (32)
constexpr int GS_LDT = GS_SB + 1;             // LDS row stride of the diagonal tile (padded)
constexpr int GS_ROWS = GemvShape<double>::ROWS;  // rows per block of the upper product
constexpr int GS_UNR = GemvShape<double>::UNR;    // column chunks in flight per thread
static_assert(GS_SB == WAVE, "one lane per row of the diagonal tile, one per panel column");
static_assert(GS_SB % GS_WAVES == 0, "the block's waves share its rows evenly");

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

// One wave: the sums over column block cb (64 columns, lane l takes column
// cb + l) of GS_PW rows from rs on, row k's sum returned in out[k] (lane 0's
// copy is the one used).
__device__ __forceinline__ void gs_row_sums(int n, int64_t lda, const double *__restrict__ A,
                                            double xl, int rs, int cb, int lane,
                                            double (&out)[GS_PW]) {
    double v[GS_PW];
#pragma unroll
    for (int k = 0; k < GS_PW; ++k) v[k] = A[(int64_t)min(rs + k, n - 1) * lda + cb + lane];
#pragma unroll
    for (int k = 0; k < GS_PW; ++k) out[k] = wave_sum(v[k] * xl);
}

// Launch I of a sweep (see the head of the file).  Block 0: rows of block I;
// blocks 1..: the rows below, GS_PR per block.
__global__ __launch_bounds__(GEMV_NT) void gs_sweep_kernel(int n, int64_t lda,
                                                           const double *__restrict__ A,
                                                           double *__restrict__ x,
                                                           double *__restrict__ c, const State *st,
                                                           int I) {
    __shared__ double T[GS_SB * GS_LDT];
    __shared__ double cI[GS_SB];  // the block's row sums over column block I - 1
    if (st->flags & F_STOP) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int cb = (I - 1) * GS_SB;  // column block just solved (I >= 1)
    const double xl = I >= 1 ? x[cb + lane] : 0.0;
    if (blockIdx.x > 0) {
        // panel: rows below block I
        const int rs = (I + 1) * GS_SB + (blockIdx.x - 1) * GS_PR + w * GS_PW;
        double sums[GS_PW];
        gs_row_sums(n, lda, A, xl, rs, cb, lane, sums);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < GS_PW; ++k)
                if (rs + k < n) c[rs + k] -= sums[k];
        }
        return;
    }
    const int r0 = I * GS_SB;
    const int m = min(GS_SB, n - r0);
    // every global load of the step first (one memory round trip): the
    // wave's rows of the diagonal tile (k = w + GS_WAVES q), its rows of the
    // block's update by column block I - 1, and c of the block's rows
    constexpr int TQ = GS_SB / GS_WAVES;   // tile rows per wave
    constexpr int PQ = GS_SB / GS_WAVES;   // update rows per wave
    double tl[TQ], pv[PQ];
    const int cc = min(lane, m - 1);
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
        const int k = w + GS_WAVES * q;
        tl[q] = A[(int64_t)(r0 + min(k, m - 1)) * lda + r0 + cc];
    }
    if (I >= 1) {
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int k = w * PQ + q;
            pv[q] = A[(int64_t)(r0 + min(k, m - 1)) * lda + cb + lane];
        }
    }
    const double cval = (w == 0 && lane < m) ? c[r0 + lane] : 0.0;
    // the diagonal tile into LDS, lower part only; rows past n get a unit
    // diagonal (their x is 0 and never written)
#pragma unroll
    for (int q = 0; q < TQ; ++q) {
        const int k = w + GS_WAVES * q;
        T[k * GS_LDT + lane] =
            (k < m && lane < m) ? (lane <= k ? tl[q] : 0.0) : (lane == k ? 1.0 : 0.0);
    }
    // sums of the block's rows over column block I - 1
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const double sq = I >= 1 ? wave_sum(pv[q] * xl) : 0.0;
        if (lane == 0) cI[w * PQ + q] = sq;
    }
    __syncthreads();
    if (w != 0) return;
    // forward substitution in wave 0: lane i holds row i
    double acc = lane < m ? cval - cI[lane] : 0.0;
    const double dinv = 1.0 / T[lane * GS_LDT + lane];
    double xi = 0.0;
#pragma unroll
    for (int j = 0; j < GS_SB; ++j) {
        const double xc = acc * dinv;
        const double xj = gs_readlane(xc, j);
        xi = (lane == j) ? xc : xi;
        acc = fma(-T[lane * GS_LDT + j], xj, acc);
    }
    if (lane < m) x[r0 + lane] = xi;
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
    const int nb = div_up(n, GS_SB);
    for (int I = 0; I < nb; ++I) {
        const int below = n - (I + 1) * GS_SB;
        const int blocks = 1 + ((I >= 1 && below > 0) ? div_up(below, GS_PR) : 0);
        gs_sweep_kernel<<<blocks, GEMV_NT, 0, s>>>(n, lda, A, x, c, st, I);
    }
    return hipGetLastError();
}

}  // namespace ks
