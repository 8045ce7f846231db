// Binary32 block Cholesky factorization A = L L^T of the binary32 copy of a
// symmetric positive definite A, the preconditioner of CG-IR (binary64
// refinement around preconditioned CG, M = L L^T).
//
// The direct-methods section's block relations for the symmetric case, right
// looking, in two levels: outer column blocks of CH_NBO = 256 columns, inside
// each block columns of CH_NB = 64:
//   ch_diag_kernel    the diagonal block A11 = L11 L11^T, factored column by
//                     column in LDS by one block (the block's entries already
//                     carry the updates of the columns before it);
//   ch_panel_kernel   the block column below it, L21 = A21 L11^-T: one row
//                     per thread, forward substitution against L11 in LDS;
//   ch_update_kernel  the block column's rank-64 update of the rest of the
//                     outer block's columns (all rows below), which the next
//                     block columns read: 64 x 64 tiles on the matrix cores,
//                     each wave a 32 x 32 quarter as 2 x 2 MFMA tiles, K = 64
//                     in steps of 16;
//   ch_syrk_kernel    once the outer block K0:K1 is factored, the rank-256
//                     update of the trailing lower triangle A(K1:n, K1:n) -=
//                     L21 L21^T (L21 = L(K1:n, K0:K1)), 128 x 128 tiles on
//                     and below the diagonal, K = 256 through LDS.
// Each element of the trailing triangle is read and written once per outer
// block with 256 multiply-adds (64 flops per byte): a contraction for the
// matrix cores (v_mfma_f32_16x16x4f32).  The grouping changes only the order
// in which each element's sum is rounded.
//
// After the last block, ch_mirror_kernel copies L^T into the strict upper
// triangle, so that the backward substitution L^T z = y reads rows (the
// substitution kernels of the LU preconditioner read U by rows).
//
// A non-positive (or non-finite) pivot: the first such column + 1 is stored
// in *info and every later kernel of the factorization returns at once.
#include "ks_vec_body.h"

namespace ks {

constexpr int CH_TILE = 64;           // trailing-update tile (rows and columns)
constexpr int CH_LDT = CH_NB + 1;     // padded LDS row stride
constexpr int CH_PANEL_ROWS = 64;     // rows of the panel per block (one per thread)
static_assert(CH_NB == 64, "one wave holds a block column's row; the update's K is 4 x 16");

typedef float ch_f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ diagonal block
// One block of 256 threads: the b x b diagonal block at (k0, k0) in LDS, then
// for each column j: l_jj = sqrt(a_jj), l_ij = a_ij / l_jj (i > j), and the
// update a_ic -= l_ij l_cj of the block's remaining lower triangle.
__global__ __launch_bounds__(256) void ch_diag_kernel(int n, int64_t ldl, float *__restrict__ L, int k0,
                                                      int *__restrict__ info) {
    __shared__ float T[CH_NB * CH_LDT];
    __shared__ int bad;
    if (*info) return;
    const int b = min(CH_NB, n - k0);
    for (int e = threadIdx.x; e < CH_NB * CH_NB; e += 256) {
        const int i = e / CH_NB, j = e % CH_NB;
        T[i * CH_LDT + j] = (i < b && j <= i) ? L[(int64_t)(k0 + i) * ldl + k0 + j] : 0.0f;
    }
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < b; ++j) {
        const float d = T[j * CH_LDT + j];
        if (!(d > 0.0f) || !(d < INFINITY)) {
            if (threadIdx.x == 0) bad = k0 + j + 1;
            break;  // uniform: every thread read the same d
        }
        const float ljj = sqrtf(d);
        __syncthreads();  // every thread has read d before it is overwritten
        if (threadIdx.x == 0) T[j * CH_LDT + j] = ljj;
        for (int i = j + 1 + threadIdx.x; i < b; i += 256) T[i * CH_LDT + j] = T[i * CH_LDT + j] / ljj;
        __syncthreads();
        // remaining lower triangle of the block: rows i > j, columns j < c <= i
        const int m = b - j - 1;
        for (int e = threadIdx.x; e < m * m; e += 256) {
            const int i = j + 1 + e / m, c = j + 1 + e % m;
            if (c <= i) T[i * CH_LDT + c] = fmaf(-T[i * CH_LDT + j], T[c * CH_LDT + j], T[i * CH_LDT + c]);
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) *info = bad;
        return;
    }
    for (int e = threadIdx.x; e < b * CH_NB; e += 256) {
        const int i = e / CH_NB, j = e % CH_NB;
        if (j <= i) L[(int64_t)(k0 + i) * ldl + k0 + j] = T[i * CH_LDT + j];
    }
}

// ------------------------------------------------------------------- panel
// Rows r >= k0 + b of the block column: l_rj = (a_rj - sum_{k<j} l_rk l_jk) / l_jj,
// one row per thread (its b values in LDS), L11 in LDS.
__global__ __launch_bounds__(CH_PANEL_ROWS) void ch_panel_kernel(int n, int64_t ldl, float *__restrict__ L,
                                                                 int k0, const int *__restrict__ info) {
    __shared__ float L11[CH_NB * CH_LDT];
    __shared__ float R[CH_PANEL_ROWS * CH_LDT];
    if (*info) return;
    const int b = min(CH_NB, n - k0);
    const int r0 = k0 + b + blockIdx.x * CH_PANEL_ROWS;
    const int t = threadIdx.x;
    for (int i = 0; i < CH_NB; ++i) L11[i * CH_LDT + t] = (i < b && t <= i) ? L[(int64_t)(k0 + i) * ldl + k0 + t] : 0.0f;
    for (int i = 0; i < CH_PANEL_ROWS; ++i) {
        const int r = r0 + i;
        R[i * CH_LDT + t] = (r < n && t < b) ? L[(int64_t)r * ldl + k0 + t] : 0.0f;
    }
    __syncthreads();
    float *row = R + t * CH_LDT;
    for (int j = 0; j < b; ++j) {
        float s = row[j];
        for (int k = 0; k < j; ++k) s = fmaf(-row[k], L11[j * CH_LDT + k], s);
        row[j] = s / L11[j * CH_LDT + j];
    }
    __syncthreads();
    for (int i = 0; i < CH_PANEL_ROWS; ++i) {
        const int r = r0 + i;
        if (r < n && t < b) L[(int64_t)r * ldl + k0 + t] = R[i * CH_LDT + t];
    }
}

// ---------------------------------------------------------- trailing update
// Tile (I, J), I >= J, J < tj, of the trailing triangle A(k1:n, k1:n), k1 =
// k0 + b (block bx takes I = bx / tj, J = bx % tj; blocks with I < J leave):
// C -= L21(I rows) L21(J rows)^T.  Lane l of a wave (g = l / 16, c = l % 16)
// feeds the MFMA's A operand with row c of a row tile and its B operand with
// row c of a column tile, taking k = 16 s + 4 g + u in MFMA u of step s (the
// sum over k is the same, in the matrix core's order); accumulator item v of
// lane l holds C[4 g + v][c].
__global__ __launch_bounds__(256) void ch_update_kernel(int n, int64_t ldl, float *__restrict__ L, int k0,
                                                        int tj, const int *__restrict__ info) {
    if (*info) return;
    const int b = min(CH_NB, n - k0);
    const int k1 = k0 + b;
    const int I = blockIdx.x / tj, J = blockIdx.x % tj;
    if (I < J) return;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int g = lane >> 4, c = lane & 15;
    const int rbase = k1 + I * CH_TILE + (w >> 1) * 32;  // the wave's 32 rows
    const int cbase = k1 + J * CH_TILE + (w & 1) * 32;   // and 32 columns
    // operands: 2 row tiles and 2 column tiles, 16 values of k each (4 steps x 4)
    float av[2][16], bv[2][16];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const float *ra = L + (int64_t)min(rbase + 16 * rt + c, n - 1) * ldl + k0;
        const float *rb = L + (int64_t)min(cbase + 16 * rt + c, n - 1) * ldl + k0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int kk = 16 * s + 4 * g;
            if (kk + 3 < b) {
                const ch_f4 x = *reinterpret_cast<const ch_f4 *>(ra + kk);
                const ch_f4 y = *reinterpret_cast<const ch_f4 *>(rb + kk);
                av[rt][4 * s] = x.x, av[rt][4 * s + 1] = x.y, av[rt][4 * s + 2] = x.z, av[rt][4 * s + 3] = x.w;
                bv[rt][4 * s] = y.x, bv[rt][4 * s + 1] = y.y, bv[rt][4 * s + 2] = y.z, bv[rt][4 * s + 3] = y.w;
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    av[rt][4 * s + u] = kk + u < b ? ra[kk + u] : 0.0f;
                    bv[rt][4 * s + u] = kk + u < b ? rb[kk + u] : 0.0f;
                }
            }
        }
    }
    ch_f4 acc[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = ch_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rt][4 * s + u], bv[ct][4 * s + u],
                                                                       acc[rt][ct], 0, 0, 0);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            const int col = cbase + 16 * ct + c;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rbase + 16 * rt + 4 * g + v;
                if (row < n && col < n && col <= row) {
                    float *pc = L + (int64_t)row * ldl + col;
                    *pc = *pc - acc[rt][ct][v];
                }
            }
        }
}

// ------------------------------------------------------------ rank-256 update
// Tile (I, J), I >= J, of A(K1:n, K1:n) -= L(K1:n, K0:K1) L(K1:n, K0:K1)^T:
// a block of four waves per 128 x 128 tile, each wave a 64 x 64 quarter as
// 4 x 4 MFMA tiles; K in LDS chunks of 32 (double-buffered, the next chunk's
// loads in flight while the matrix cores work).  Both operands are rows of
// L21 with k contiguous, staged alike; lane (g, c) takes k = 8 g + s in step
// s, so each fragment is two 16-byte LDS reads.  Blocks are numbered
// round-robin over the eight XCDs: block b takes logical tile (b % 8) q + b /
// 8 of the T (T + 1) / 2 lower tiles in row order (q per XCD), so the tiles
// in flight on one XCD share rows of L21 in its L2.  Only elements on and
// below the diagonal are written.
constexpr int CH_NBO = 256;           // outer column block: K of this update
constexpr int CS_T = 128, CS_BK = 32, CS_LD = CS_BK + 4, CS_XCD = 8;
static_assert(CH_NBO % CH_NB == 0 && CH_NBO % CS_BK == 0, "outer blocks of whole block columns and chunks");

__global__ __launch_bounds__(256) void ch_syrk_kernel(int n, int64_t ldl, float *__restrict__ L, int K0, int K1,
                                                      int T, const int *__restrict__ info) {
    __shared__ __attribute__((aligned(16))) float As[2][CS_T * CS_LD];
    __shared__ __attribute__((aligned(16))) float Bs[2][CS_T * CS_LD];
    if (*info) return;
    const int total = T * (T + 1) / 2;
    const int per_xcd = div_up(total, CS_XCD);
    const int lt = (blockIdx.x % CS_XCD) * per_xcd + blockIdx.x / CS_XCD;
    if (lt >= total) return;
    int I, J;
    tri_ij(lt, I, J);
    const int r0 = K1 + I * CS_T, c0 = K1 + J * CS_T;
    const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
    const int g = lane >> 4, c = lane & 15;
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    const int nch = (K1 - K0) / CS_BK;
    // staging: rows t / 8 + 32 i of both row tiles, k = 4 (t % 8)
    const int ar = t / 8, ak = 4 * (t % 8);
    ch_f4 ra[4], rb[4];
    auto gload = [&](int ch) {
        const int kb = K0 + ch * CS_BK + ak;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + ar + 32 * i, q = c0 + ar + 32 * i;
            ra[i] = r < n ? *reinterpret_cast<const ch_f4 *>(L + (int64_t)r * ldl + kb) : ch_f4{0.f, 0.f, 0.f, 0.f};
            rb[i] = q < n ? *reinterpret_cast<const ch_f4 *>(L + (int64_t)q * ldl + kb) : ch_f4{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            *reinterpret_cast<ch_f4 *>(&As[buf][(ar + 32 * i) * CS_LD + ak]) = ra[i];
            *reinterpret_cast<ch_f4 *>(&Bs[buf][(ar + 32 * i) * CS_LD + ak]) = rb[i];
        }
    };
    ch_f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = ch_f4{0.f, 0.f, 0.f, 0.f};
    gload(0);
    sstore(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) gload(ch + 1);
        ch_f4 a[4][2], bq[4][2];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const ch_f4 *pa = reinterpret_cast<const ch_f4 *>(&As[buf][(wr + 16 * rt + c) * CS_LD + 8 * g]);
            const ch_f4 *pb = reinterpret_cast<const ch_f4 *>(&Bs[buf][(wc + 16 * rt + c) * CS_LD + 8 * g]);
            a[rt][0] = pa[0], a[rt][1] = pa[1];
            bq[rt][0] = pb[0], bq[rt][1] = pb[1];
        }
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][s / 4][s % 4], bq[ct][s / 4][s % 4],
                                                                       acc[rt][ct], 0, 0, 0);
        if (ch + 1 < nch) sstore(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int col = c0 + wc + 16 * ct + c;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = r0 + wr + 16 * rt + 4 * g + v;
                if (row < n && col <= row) {
                    float *pc = L + (int64_t)row * ldl + col;
                    *pc = *pc - acc[rt][ct][v];
                }
            }
        }
}

// ------------------------------------------------------------------ mirror
// upper(i, j) = L(j, i) for j > i, through a 64 x 64 LDS tile per block pair
// (tile (I, J) of the lower triangle, I >= J, written transposed to (J, I)).
__global__ __launch_bounds__(256) void ch_mirror_kernel(int n, int64_t ldl, float *__restrict__ L) {
    __shared__ float T[CH_TILE * (CH_TILE + 1)];
    int I, J;
    tri_ij(blockIdx.x, I, J);
    const int r0 = I * CH_TILE, c0 = J * CH_TILE;
    for (int e = threadIdx.x; e < CH_TILE * CH_TILE; e += 256) {
        const int i = e / CH_TILE, j = e % CH_TILE;
        const int r = r0 + i, cc = c0 + j;
        T[i * (CH_TILE + 1) + j] = (r < n && cc < n && cc < r) ? L[(int64_t)r * ldl + cc] : 0.0f;
    }
    __syncthreads();
    // element (r, cc) of the lower triangle goes to (cc, r)
    for (int e = threadIdx.x; e < CH_TILE * CH_TILE; e += 256) {
        const int j = e / CH_TILE, i = e % CH_TILE;  // consecutive threads: consecutive columns r
        const int r = r0 + i, cc = c0 + j;
        if (r < n && cc < n && cc < r) L[(int64_t)cc * ldl + r] = T[i * (CH_TILE + 1) + j];
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_chol_factor(int n, int64_t ldl, float *L, int *info, hipStream_t s) {
    for (int K0 = 0; K0 < n; K0 += CH_NBO) {
        const int K1 = min(K0 + CH_NBO, n);
        for (int k0 = K0; k0 < K1; k0 += CH_NB) {
            const int b = min(CH_NB, n - k0), k1 = k0 + b;
            ch_diag_kernel<<<1, 256, 0, s>>>(n, ldl, L, k0, info);
            const int rest = n - k1;
            if (rest > 0) {
                ch_panel_kernel<<<div_up(rest, CH_PANEL_ROWS), CH_PANEL_ROWS, 0, s>>>(n, ldl, L, k0, info);
                if (k1 < K1) {
                    const int tj = div_up(K1 - k1, CH_TILE), ti = div_up(rest, CH_TILE);
                    ch_update_kernel<<<tj * ti, 256, 0, s>>>(n, ldl, L, k0, tj, info);
                }
            }
        }
        if (K1 < n) {
            const int T = div_up(n - K1, CS_T);
            const int grid = CS_XCD * div_up(T * (T + 1) / 2, CS_XCD);
            ch_syrk_kernel<<<grid, 256, 0, s>>>(n, ldl, L, K0, K1, T, info);
        }
    }
    const int T = div_up(n, CH_TILE);
    ch_mirror_kernel<<<T * (T + 1) / 2, 256, 0, s>>>(n, ldl, L);
    return hipGetLastError();
}

// ------------------------------------------------- preconditioned CG (binary64)
// Preconditioned CG on A d = rhs from d = 0 with M = L L^T: the plain CG
// kernels form q = A p with the p'q partials and d += alpha p, r -= alpha q
// with the r'r partials (alpha = rho / sigma, rho = r'z); z = M^-1 r is the
// two substitutions; then the kernels below reduce r'z and r'r, test the
// stop (||r||_2 against tol ||rhs||_2, the iteration limit, a non-positive
// r'z) and form p = z + beta p, beta = (r'z)_new / (r'z).

// partial[b] = sum of r_i z_i over vector block b (element i = base + e * 256
// of thread t, summed in order of e, then over the block)
__global__ __launch_bounds__(VEC_NT) void pcg_dot_kernel(int n, const double *__restrict__ r,
                                                         const double *__restrict__ z,
                                                         const State *st, double *__restrict__ partial) {
    __shared__ double sm[VEC_NT / WAVE];
    if (st->flags & F_STOP) return;
    const int base = blockIdx.x * VEC_NT * VEC_EPT + threadIdx.x;
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) s += r[i] * z[i];
    }
    const double t = block_sum<VEC_NT>(s, sm);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// start of the iteration: p = z, rho = r'z (> 0 for SPD A and M)
__global__ __launch_bounds__(VEC_NT) void pcg_begin_kernel(int n, const double *__restrict__ z,
                                                           double *__restrict__ p, State *st,
                                                           const double *__restrict__ rz_part, int nvb) {
    const double rz = reduce_partials_all<VEC_NT>(rz_part, nvb, 1);
    if (st->flags & F_STOP) return;
    const int base = blockIdx.x * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) p[i] = z[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->rho = rz;
        if (!finite_d(rz))
            st->flags |= F_NONFIN | F_STOP;
        else if (!(rz > 0.0))
            st->flags |= F_BREAK | F_STOP;
    }
}

__global__ __launch_bounds__(VEC_NT) void pcg_pupdate_kernel(int n, const double *__restrict__ z,
                                                             double *__restrict__ p, State *st,
                                                             const double *__restrict__ rr_part,
                                                             const double *__restrict__ rz_part, int nvb,
                                                             int max_iter) {
    const int base = blockIdx.x * VEC_NT * VEC_EPT + threadIdx.x;
    double zv[VEC_EPT], pv[VEC_EPT];
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = min(base + e * VEC_NT, n - 1);
        zv[e] = z[i];
        pv[e] = p[i];
    }
    const double thresh = st->thresh, rz_prev = st->rho;
    const int iters = st->iters;
    const double rr = reduce_partials_all<VEC_NT>(rr_part, nvb, 1);
    const double rz = reduce_partials_all<VEC_NT>(rz_part, nvb, 1);
    if (st->flags & F_STOP) return;
    int stop = 0;
    if (!finite_d(rr) || !finite_d(rz))
        stop = F_NONFIN | F_STOP;
    else if (sqrt(rr) <= thresh)
        stop = F_CONV | F_STOP;
    else if (iters >= max_iter)
        stop = F_MAXIT | F_STOP;
    else if (!(rz > 0.0))
        stop = F_BREAK | F_STOP;
    const double beta = rz / rz_prev;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (stop) {
            st->flags |= stop;
        } else {
            st->beta = beta;
            st->rho = rz;
        }
    }
    if (stop) return;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) p[i] = fma(beta, pv[e], zv[e]);
    }
}

hipError_t launch_pcg_dot(int n, const double *r, const double *z, const State *st, double *partial,
                          hipStream_t s) {
    pcg_dot_kernel<<<vec_blocks(n), VEC_NT, 0, s>>>(n, r, z, st, partial);
    return hipGetLastError();
}

hipError_t launch_pcg_begin(int n, const double *z, double *p, State *st, const double *rz_part,
                            hipStream_t s) {
    pcg_begin_kernel<<<vec_blocks(n), VEC_NT, 0, s>>>(n, z, p, st, rz_part, vec_blocks(n));
    return hipGetLastError();
}

hipError_t launch_pcg_pupdate(int n, const double *z, double *p, State *st, const double *rr_part,
                              const double *rz_part, int max_iter, hipStream_t s) {
    pcg_pupdate_kernel<<<vec_blocks(n), VEC_NT, 0, s>>>(n, z, p, st, rr_part, rz_part, vec_blocks(n),
                                                        max_iter);
    return hipGetLastError();
}

}  // namespace ks
