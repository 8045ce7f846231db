// Binary32 block LU with partial pivoting, and its application as the
// preconditioner M^-1 v = U^-1 L^-1 P v of GMRES inside binary64 iterative
// refinement (GMRES-IR).
//
// Factorization: the block algorithm of the paper's direct-methods section
// (Figure 1, equations (1)-(4)), column blocks of LU_NB = 16:
//   lu_panel_kernel   the panel A(k0:n, k0:k0+16) factored column by column
//                     with partial pivoting (largest magnitude, first row on
//                     ties), in one block of 1024 threads that keeps the panel
//                     in registers (4 rows of 16 per thread: n <= 4096);
//   lu_swap_kernel    the panel's row interchanges applied to the other columns;
//   lu_trsm_kernel    the block row of U: unit-lower panel triangle \ A(k0:k0+16, k0+16:n);
//   lu_update_kernel  the delayed rank-16 update of the trailing matrix.
// The update has 16 multiply-adds per element read and written (8 bytes),
// so it is bound by memory traffic, not by arithmetic: a tiled vector-ALU
// kernel rather than matrix cores.
//
// Application (binary64 vectors, binary32 factors widened): a gather by the
// permutation, then the forward (unit lower) and backward (upper)
// substitutions as sequences of 64-row launches, each solving one diagonal
// tile in a wave (lane i holds row i, x_j broadcast by readlane) after
// subtracting the column block solved in the launch before, while the
// launch's other blocks subtract that column block from the remaining rows.
#include <utility>

#include "ks_gemv_body.h"

namespace ks {

constexpr int LU_NT = 1024;              // threads of the panel block
constexpr int LU_R = LU_MAX_N / LU_NT;   // panel rows per thread
constexpr int LU_TILE = 64;              // trailing-update tile (rows and columns)
constexpr int TS_SB = 64;                // rows per substitution step
constexpr int TS_PW = 8;                 // rows per wave in the row updates
constexpr int TS_WAVES = GEMV_NT / WAVE;
constexpr int TS_PR = TS_WAVES * TS_PW;  // rows per row-update block
constexpr int TS_LDT = TS_SB + 1;        // padded LDS row stride of a diagonal tile
static_assert(LU_R * LU_NT == LU_MAX_N, "the panel fits the block's registers");
static_assert(LU_NB <= WAVE && LU_NB * LU_NB <= GEMV_NT, "panel width");

// ------------------------------------------------------------ factorization
struct LuPanelShared {
    float rowA[LU_NB], rowB[LU_NB];
    float red_v[LU_NT / WAVE];
    int red_i[LU_NT / WAVE];
    int piv;
};

// Column J of the panel (J a template parameter, so that the panel stays in
// registers: every index into p is a compile-time constant).
template <int J>
__device__ __forceinline__ void lu_panel_col(int n, int k0, int b, float (&p)[LU_R][LU_NB],
                                             LuPanelShared &sh, int *__restrict__ piv,
                                             int *__restrict__ info) {
    if (J >= b) return;  // uniform: the last panel may be narrower
    const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
    const int rj = k0 + J;
    // pivot: largest |a(r, J)| over rows r >= rj, the first such row; the
    // search starts from row rj, so the pivot is a row of the panel even when
    // no magnitude compares greater (a column of NaNs)
    float bv = -1.0f;
    int bi = rj;
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
        const int r = k0 + t + LU_NT * q;
        const float a = fabsf(p[q][J]);
        if (r >= rj && r < n && a > bv) {
            bv = a;
            bi = r;
        }
    }
#pragma unroll
    for (int off = WAVE / 2; off >= 1; off >>= 1) {
        const float ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) {
        sh.red_v[wv] = bv;
        sh.red_i[wv] = bi;
    }
    __syncthreads();
    // the waves' candidates reduced by wave 0 with the same rule (the largest
    // magnitude, the lowest row on ties: a total order, so any reduction
    // order picks the same row)
    if (wv == 0) {
        constexpr int NW = LU_NT / WAVE;
        static_assert(NW <= WAVE && (NW & (NW - 1)) == 0, "one candidate per lane");
        float v = lane < NW ? sh.red_v[lane] : -2.0f;
        int i = lane < NW ? sh.red_i[lane] : rj;
#pragma unroll
        for (int off = NW / 2; off >= 1; off >>= 1) {
            const float ov = __shfl_xor(v, off);
            const int oi = __shfl_xor(i, off);
            if (ov > v || (ov == v && oi < i)) {
                v = ov;
                i = oi;
            }
        }
        if (lane == 0) {
            sh.piv = i;
            piv[rj] = i;
        }
    }
    __syncthreads();
    const int pr = sh.piv;
    // interchange rows rj and pr through LDS, each register row matched by
    // its row index
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
        const int r = k0 + t + LU_NT * q;
        if (r == rj) {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c) sh.rowA[c] = p[q][c];
        }
        if (r == pr) {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c) sh.rowB[c] = p[q][c];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
        const int r = k0 + t + LU_NT * q;
        if (pr != rj && r == rj) {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c) p[q][c] = sh.rowB[c];
        } else if (pr != rj && r == pr) {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c) p[q][c] = sh.rowA[c];
        }
    }
    // eliminate below the pivot (the pivot row is now rowB)
    const float d = sh.rowB[J];
    if (d != 0.0f) {
#pragma unroll
        for (int q = 0; q < LU_R; ++q) {
            const int r = k0 + t + LU_NT * q;
            if (r > rj && r < n) {
                const float l = p[q][J] / d;
                p[q][J] = l;
#pragma unroll
                for (int c = J + 1; c < LU_NB; ++c) p[q][c] = p[q][c] - l * sh.rowB[c];
            }
        }
    } else if (t == 0 && info[0] == 0) {
        info[0] = rj + 1;
    }
    __syncthreads();
}

template <int... J>
__device__ __forceinline__ void lu_panel_cols(int n, int k0, int b, float (&p)[LU_R][LU_NB],
                                              LuPanelShared &sh, int *__restrict__ piv,
                                              int *__restrict__ info,
                                              std::integer_sequence<int, J...>) {
    (lu_panel_col<J>(n, k0, b, p, sh, piv, info), ...);
}

__global__ __launch_bounds__(LU_NT) void lu_panel_kernel(int n, int64_t ldl, float *__restrict__ LU,
                                                         int k0, int *__restrict__ piv,
                                                         int *__restrict__ info) {
    __shared__ LuPanelShared sh;
    const int t = threadIdx.x;
    const int b = min(LU_NB, n - k0);
    float p[LU_R][LU_NB];
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
        const int r = k0 + t + LU_NT * q;
#pragma unroll
        for (int c = 0; c < LU_NB; ++c)
            p[q][c] = (r < n && c < b) ? LU[(int64_t)r * ldl + k0 + c] : 0.0f;
    }
    lu_panel_cols(n, k0, b, p, sh, piv, info, std::make_integer_sequence<int, LU_NB>{});
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
        const int r = k0 + t + LU_NT * q;
        if (r < n) {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c)
                if (c < b) LU[(int64_t)r * ldl + k0 + c] = p[q][c];
        }
    }
}

// the panel's interchanges, in order, on every column outside the panel
__global__ __launch_bounds__(GEMV_NT) void lu_swap_kernel(int n, int64_t ldl, float *__restrict__ LU,
                                                          int k0, int b,
                                                          const int *__restrict__ piv) {
    const int c = blockIdx.x * GEMV_NT + threadIdx.x;
    if (c >= n || (c >= k0 && c < k0 + b)) return;
    for (int j = 0; j < b; ++j) {
        const int pr = piv[k0 + j], rj = k0 + j;
        if (pr != rj) {
            const float a = LU[(int64_t)rj * ldl + c], e = LU[(int64_t)pr * ldl + c];
            LU[(int64_t)rj * ldl + c] = e;
            LU[(int64_t)pr * ldl + c] = a;
        }
    }
}

// the block row of U: z = L00^-1 A(k0:k0+b, c), one column per thread
__global__ __launch_bounds__(GEMV_NT) void lu_trsm_kernel(int n, int64_t ldl, float *__restrict__ LU,
                                                          int k0, int b) {
    __shared__ float L00[LU_NB][LU_NB];
    {
        const int i = threadIdx.x / LU_NB, j = threadIdx.x % LU_NB;
        if (i < LU_NB) L00[i][j] = (i < b && j < b) ? LU[(int64_t)(k0 + i) * ldl + k0 + j] : 0.0f;
    }
    __syncthreads();
    const int c = k0 + b + blockIdx.x * GEMV_NT + threadIdx.x;
    if (c >= n) return;
    float z[LU_NB];
#pragma unroll
    for (int i = 0; i < LU_NB; ++i) z[i] = (i < b) ? LU[(int64_t)(k0 + i) * ldl + c] : 0.0f;
#pragma unroll
    for (int i = 1; i < LU_NB; ++i) {
        float s = z[i];
#pragma unroll
        for (int j = 0; j < i; ++j) s = s - L00[i][j] * z[j];
        z[i] = s;
    }
#pragma unroll
    for (int i = 0; i < LU_NB; ++i)
        if (i < b) LU[(int64_t)(k0 + i) * ldl + c] = z[i];
}

// A(k1:n, k1:n) -= A(k1:n, k0:k1) A(k0:k1, k1:n), k1 = k0 + b; 64 x 64 tiles,
// each thread 4 x 4 (rows tr + 16 i, columns tc + 16 j)
__global__ __launch_bounds__(GEMV_NT) void lu_update_kernel(int n, int64_t ldl, float *__restrict__ LU,
                                                            int k0, int b) {
    __shared__ float Ls[LU_TILE][LU_NB + 1];
    __shared__ float Us[LU_NB][LU_TILE];
    const int k1 = k0 + b;
    const int r0 = k1 + blockIdx.y * LU_TILE, c0 = k1 + blockIdx.x * LU_TILE;
#pragma unroll
    for (int e = 0; e < LU_TILE * LU_NB / GEMV_NT; ++e) {
        const int idx = threadIdx.x + GEMV_NT * e;
        const int rr = idx / LU_NB, jj = idx % LU_NB;
        const int r = r0 + rr;
        Ls[rr][jj] = (r < n && jj < b) ? LU[(int64_t)r * ldl + k0 + jj] : 0.0f;
        const int j2 = idx / LU_TILE, cc = idx % LU_TILE;
        const int c = c0 + cc;
        Us[j2][cc] = (c < n && j2 < b) ? LU[(int64_t)(k0 + j2) * ldl + c] : 0.0f;
    }
    __syncthreads();
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = tr + 16 * i, r = r0 + rr;
        if (r >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cc = tc + 16 * j, c = c0 + cc;
            if (c >= n) continue;
            float s = LU[(int64_t)r * ldl + c];
#pragma unroll
            for (int jj = 0; jj < LU_NB; ++jj) s = s - Ls[rr][jj] * Us[jj][cc];
            LU[(int64_t)r * ldl + c] = s;
        }
    }
}

// ------------------------------------------------------------- application
__global__ __launch_bounds__(VEC_NT) void lu_gather_kernel(int n, const int *__restrict__ perm,
                                                           const double *__restrict__ v,
                                                           double *__restrict__ t) {
    const int i = blockIdx.x * VEC_NT + threadIdx.x;
    if (i < n) t[i] = v[perm[i]];
}

__device__ __forceinline__ double ts_readlane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// out[q] = sum over the wave of pv[q] * xl for the wave's Q = TS_SB / TS_WAVES
// rows, eight rows at a time by the halving butterfly (lane group g = lane / 8
// ends with row q0 + g), instead of one wave sum per row.
template <int Q>
__device__ __forceinline__ void ts_rows_sums(const double (&pv)[Q], double xl, int lane, double *out) {
    static_assert(Q % 8 == 0, "rows in groups of eight");
#pragma unroll
    for (int q0 = 0; q0 < Q; q0 += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pv[q0 + u] * xl;
        const double s = rows_reduce<8>(v, lane);
        if (lane % 8 == 0) out[q0 + lane / 8] = s;
    }
}

// Step I of the forward substitution L y = t in place: L unit lower (the LU
// factor, UNIT) or lower with its diagonal (the Cholesky factor).
template <bool UNIT>
__global__ __launch_bounds__(GEMV_NT) void lu_fwd_kernel(int n, int64_t ldl,
                                                         const float *__restrict__ LU,
                                                         double *__restrict__ t, int I) {
    __shared__ double T[TS_SB * TS_LDT];
    __shared__ double sI[TS_SB];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int cb = (I - 1) * TS_SB;  // column block solved in step I - 1
    const double xl = I >= 1 ? t[cb + lane] : 0.0;
    if (blockIdx.x > 0) {
        const int rs = (I + 1) * TS_SB + (blockIdx.x - 1) * TS_PR + w * TS_PW;
        double v[TS_PW];
#pragma unroll
        for (int k = 0; k < TS_PW; ++k)
            v[k] = (double)LU[(int64_t)min(rs + k, n - 1) * ldl + cb + lane] * xl;
        // the wave's rows summed together (lane group lane / 8 ends with row rs + g)
        const double s = rows_reduce<TS_PW>(v, lane);
        if (lane % (WAVE / TS_PW) == 0 && rs + lane / (WAVE / TS_PW) < n) t[rs + lane / (WAVE / TS_PW)] -= s;
        return;
    }
    const int r0 = I * TS_SB, m = min(TS_SB, n - r0);
    constexpr int Q = TS_SB / TS_WAVES;
    double tl[Q], pv[Q];
    const int cc = min(lane, m - 1);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = w + TS_WAVES * q;
        tl[q] = (double)LU[(int64_t)(r0 + min(k, m - 1)) * ldl + r0 + cc];
        pv[q] = I >= 1 ? (double)LU[(int64_t)(r0 + min(w * Q + q, m - 1)) * ldl + cb + lane] : 0.0;
    }
    const double cval = (w == 0 && lane < m) ? t[r0 + lane] : 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = w + TS_WAVES * q;
        if constexpr (UNIT) {
            // strictly lower part (the unit diagonal is implicit)
            T[k * TS_LDT + lane] = (k < m && lane < k) ? tl[q] : 0.0;
        } else {
            // lower part with the diagonal; rows past n get a unit diagonal
            T[k * TS_LDT + lane] = (k < m && lane < m) ? (lane <= k ? tl[q] : 0.0) : (lane == k ? 1.0 : 0.0);
        }
    }
    ts_rows_sums(pv, I >= 1 ? xl : 0.0, lane, sI + w * Q);
    __syncthreads();
    if (w != 0) return;
    double acc = lane < m ? cval - sI[lane] : 0.0;
    double xi = 0.0;
    if constexpr (UNIT) {
#pragma unroll
        for (int j = 0; j < TS_SB; ++j) {
            const double xj = ts_readlane(acc, j);
            xi = (lane == j) ? acc : xi;
            acc = fma(-T[lane * TS_LDT + j], xj, acc);
        }
    } else {
        const double dinv = 1.0 / T[lane * TS_LDT + lane];
#pragma unroll
        for (int j = 0; j < TS_SB; ++j) {
            const double xc = acc * dinv;
            const double xj = ts_readlane(xc, j);
            xi = (lane == j) ? xc : xi;
            // rows i > j take L(i, j) x_j; the diagonal and above are zero here
            acc = fma(lane > j ? -T[lane * TS_LDT + j] : 0.0, xj, acc);
        }
    }
    if (lane < m) t[r0 + lane] = xi;
}

// Step J (from the last block up) of the backward substitution U z = t in place.
__global__ __launch_bounds__(GEMV_NT) void lu_bwd_kernel(int n, int64_t ldl,
                                                         const float *__restrict__ LU,
                                                         double *__restrict__ t, int J, int nb) {
    __shared__ double T[TS_SB * TS_LDT];
    __shared__ double sI[TS_SB];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const bool has = J + 1 < nb;      // a column block solved in the step before
    const int cb = (J + 1) * TS_SB;
    const bool lin = has && cb + lane < n;
    const int cl = lin ? cb + lane : 0;
    const double xl = lin ? t[cl] : 0.0;
    if (blockIdx.x > 0) {
        // rows above block J
        const int rs = (blockIdx.x - 1) * TS_PR + w * TS_PW;
        const int rend = J * TS_SB;
        double v[TS_PW];
#pragma unroll
        for (int k = 0; k < TS_PW; ++k)
            v[k] = (lin ? (double)LU[(int64_t)min(rs + k, rend - 1) * ldl + cl] : 0.0) * xl;
        const double s = rows_reduce<TS_PW>(v, lane);
        if (lane % (WAVE / TS_PW) == 0 && rs + lane / (WAVE / TS_PW) < rend) t[rs + lane / (WAVE / TS_PW)] -= s;
        return;
    }
    const int r0 = J * TS_SB, m = min(TS_SB, n - r0);
    constexpr int Q = TS_SB / TS_WAVES;
    double tl[Q], pv[Q];
    const int cc = min(lane, m - 1);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = w + TS_WAVES * q;
        tl[q] = (double)LU[(int64_t)(r0 + min(k, m - 1)) * ldl + r0 + cc];
        pv[q] = lin ? (double)LU[(int64_t)(r0 + min(w * Q + q, m - 1)) * ldl + cl] : 0.0;
    }
    const double cval = (w == 0 && lane < m) ? t[r0 + lane] : 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = w + TS_WAVES * q;
        // upper part with the diagonal; rows past n get a unit diagonal
        T[k * TS_LDT + lane] = (k < m && lane < m) ? (lane >= k ? tl[q] : 0.0) : (lane == k ? 1.0 : 0.0);
    }
    ts_rows_sums(pv, xl, lane, sI + w * Q);
    __syncthreads();
    if (w != 0) return;
    double acc = lane < m ? cval - sI[lane] : 0.0;
    const double dinv = 1.0 / T[lane * TS_LDT + lane];
    double xi = 0.0;
#pragma unroll
    for (int j = TS_SB - 1; j >= 0; --j) {
        const double xc = acc * dinv;
        const double xj = ts_readlane(xc, j);
        xi = (lane == j) ? xc : xi;
        // rows i < j take U(i, j) x_j; the diagonal and below are zero here
        acc = fma(lane < j ? -T[lane * TS_LDT + j] : 0.0, xj, acc);
    }
    if (lane < m) t[r0 + lane] = xi;
}

// w = t, and the squares of w in the partials the GMRES product leaves (one
// per pair of rows), so that the Arnoldi step sees ||M^-1 A v||
__global__ __launch_bounds__(WAVE) void lu_pc_copy_kernel(int n, const double *__restrict__ t,
                                                          double *__restrict__ w,
                                                          double *__restrict__ partial) {
    constexpr int R = GemvShape<double>::ROWS;
    const int row = blockIdx.x * R + threadIdx.x;
    double s = 0.0;
    if (threadIdx.x < R && row < n) {
        const double v = t[row];
        w[row] = v;
        s = v * v;
    }
    s = wave_sum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// ||w||_2 from those partials into the State, with the true-residual flags
__global__ __launch_bounds__(ONE_NT) void lu_res_finish_kernel(int nblocks, State *st,
                                                               const double *partial) {
    const double rho = reduce_partials_all<ONE_NT>(partial, nblocks, 1);
    if (threadIdx.x == 0) {
        const double res = sqrt(rho);
        st->rho = rho;
        st->res = res;
        int f = st->flags & ~(F_TRUE_OK | F_TRUE_NONFIN);
        if (!finite_d(res))
            f |= F_TRUE_NONFIN;
        else if (res <= st->thresh)
            f |= F_TRUE_OK;
        st->flags = f;
    }
}

__global__ __launch_bounds__(VEC_NT) void lu_xupdate_kernel(int n, double *__restrict__ x,
                                                            const double *__restrict__ d) {
    const int i = blockIdx.x * VEC_NT + threadIdx.x;
    if (i < n) x[i] += d[i];
}

// ---------------------------------------------------------------- launchers
hipError_t launch_lu_factor(int n, int64_t ldl, float *LU, int *piv, int *info, hipStream_t s) {
    for (int k0 = 0; k0 < n; k0 += LU_NB) {
        const int b = min(LU_NB, n - k0);
        lu_panel_kernel<<<1, LU_NT, 0, s>>>(n, ldl, LU, k0, piv, info);
        lu_swap_kernel<<<div_up(n, GEMV_NT), GEMV_NT, 0, s>>>(n, ldl, LU, k0, b, piv);
        const int rest = n - k0 - b;
        if (rest > 0) {
            lu_trsm_kernel<<<div_up(rest, GEMV_NT), GEMV_NT, 0, s>>>(n, ldl, LU, k0, b);
            const dim3 grid(div_up(rest, LU_TILE), div_up(rest, LU_TILE));
            lu_update_kernel<<<grid, GEMV_NT, 0, s>>>(n, ldl, LU, k0, b);
        }
    }
    return hipGetLastError();
}

hipError_t launch_lu_apply(int n, int64_t ldl, const float *LU, const int *perm, const double *src,
                           double *dst, double *t, double *partial, hipStream_t s) {
    lu_gather_kernel<<<div_up(n, VEC_NT), VEC_NT, 0, s>>>(n, perm, src, t);
    const int nb = div_up(n, TS_SB);
    for (int I = 0; I < nb; ++I) {
        const int below = n - (I + 1) * TS_SB;
        const int blocks = 1 + ((I >= 1 && below > 0) ? div_up(below, TS_PR) : 0);
        lu_fwd_kernel<true><<<blocks, GEMV_NT, 0, s>>>(n, ldl, LU, t, I);
    }
    for (int J = nb - 1; J >= 0; --J) {
        const int above = J * TS_SB;
        const int blocks = 1 + ((J + 1 < nb && above > 0) ? div_up(above, TS_PR) : 0);
        lu_bwd_kernel<<<blocks, GEMV_NT, 0, s>>>(n, ldl, LU, t, J, nb);
    }
    lu_pc_copy_kernel<<<gemv_blocks<double>(n), WAVE, 0, s>>>(n, t, dst, partial);
    return hipGetLastError();
}

__global__ __launch_bounds__(VEC_NT) void ch_copy_kernel(int n, const double *__restrict__ v,
                                                         double *__restrict__ z) {
    const int i = blockIdx.x * VEC_NT + threadIdx.x;
    if (i < n) z[i] = v[i];
}

hipError_t launch_chol_apply(int n, int64_t ldl, const float *L, const double *src, double *dst,
                             hipStream_t s) {
    if (dst != src) ch_copy_kernel<<<div_up(n, VEC_NT), VEC_NT, 0, s>>>(n, src, dst);
    const int nb = div_up(n, TS_SB);
    for (int I = 0; I < nb; ++I) {
        const int below = n - (I + 1) * TS_SB;
        const int blocks = 1 + ((I >= 1 && below > 0) ? div_up(below, TS_PR) : 0);
        lu_fwd_kernel<false><<<blocks, GEMV_NT, 0, s>>>(n, ldl, L, dst, I);
    }
    // L^T is held in the strict upper triangle (and the shared diagonal)
    for (int J = nb - 1; J >= 0; --J) {
        const int above = J * TS_SB;
        const int blocks = 1 + ((J + 1 < nb && above > 0) ? div_up(above, TS_PR) : 0);
        lu_bwd_kernel<<<blocks, GEMV_NT, 0, s>>>(n, ldl, L, dst, J, nb);
    }
    return hipGetLastError();
}

hipError_t launch_lu_xupdate(int n, double *x, const double *d, hipStream_t s) {
    lu_xupdate_kernel<<<div_up(n, VEC_NT), VEC_NT, 0, s>>>(n, x, d);
    return hipGetLastError();
}

hipError_t launch_lu_res_finish(int n, State *st, const double *partial, hipStream_t s) {
    lu_res_finish_kernel<<<1, ONE_NT, 0, s>>>(gemv_blocks<double>(n), st, partial);
    return hipGetLastError();
}

}  // namespace ks
