// Binary32 block LU with partial pivoting, and its application as the
// preconditioner M^-1 v = U^-1 L^-1 P v of GMRES inside binary64 iterative
// refinement (GMRES-IR).
//
// Factorization: the block algorithm of the paper's direct-methods section
// (Figure 1, equations (1)-(4)) in two levels.  Outer column blocks of
// LU_NBO = 256 columns; inside one, panels of LU_NB = 16 columns:
//   lu_panel_kernel   the panel A(k0:n, k0:k0+16) factored column by column
//                     with partial pivoting (largest magnitude, first row on
//                     ties), the panel in registers: one block of 1024
//                     threads when it has at most 4096 rows, else a
//                     cooperative grid of up to 32 blocks of 1024 rows; per
//                     column the blocks exchange their candidates (magnitude,
//                     row, the row's 16 values) in one device-scope round
//                     trip, then every block picks the same pivot and
//                     eliminates its rows;
//   lu_swap_kernel    the panel's row interchanges applied to every other
//                     column (so every row of A(K0:n, K1:n) stays in the same
//                     state: none of the outer block's updates applied yet);
//   lu_trsm_kernel    rows k0:k0+16 of U in the outer block's columns: the
//                     unit-lower panel triangle \ A(k0:k0+16, k0+16:K1);
//   lu_update_kernel  the panel's rank-16 update of the rest of the outer
//                     block's columns, A(k0+16:n, k0+16:K1), which the next
//                     panels read;
// and once the outer block K0:K1 is factored:
//   U12 = L11^-1 A(K0:K1, K1:n), row block by row block: lu_trsm_kernel on
//                     the block's 16 rows, then lu_update_kernel's rank-16
//                     update of the rows below it in the outer block;
//   lu_gemm_kernel    the rank-256 update of the trailing matrix
//                     A(K1:n, K1:n) -= L21 U12 on the matrix cores
//                     (v_mfma_f32_16x16x4f32).
// The rank-16 updates have 16 multiply-adds per element read and written (8
// bytes), bound by memory traffic: a tiled vector-ALU kernel.  The rank-256
// update has 256 per element, 64 flops per byte of the trailing matrix: a
// contraction for the matrix cores.  The grouping of the delayed updates
// changes only the order in which each element's sum is rounded.
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

constexpr int LU_NBO = 256;              // outer column block: K of the trailing update
constexpr int LU_TILE = 64;              // rank-16 update tile (rows and columns)
constexpr int TS_SB = 64;                // rows per substitution step
constexpr int TS_PW = 8;                 // rows per wave in the row updates
constexpr int TS_WAVES = GEMV_NT / WAVE;
constexpr int TS_PR = TS_WAVES * TS_PW;  // rows per row-update block
constexpr int TS_LDT = TS_SB + 1;        // padded LDS row stride of a diagonal tile
static_assert(LU_NB <= WAVE && LU_NB * LU_NB <= GEMV_NT, "panel width");
static_assert(LU_NBO % LU_NB == 0, "outer blocks hold whole panels");

typedef float lg_f4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------- panel
// Per column the blocks of a panel exchange packets: block g publishes its
// candidate (|a|, row, the row's 16 values) and block 0 also row rj, as
// 64-bit words whose high half is the column's tag rj + 1 and whose low half
// is the value, with agent-scope relaxed (device-coherent) atomic stores.
// Every block loads every packet word the same way until each shows the
// tag: so one device-scope round trip both synchronizes the blocks and
// carries the data (a word is written and read whole, so a matching tag
// means its value is that column's).  The packets of odd and even columns
// alternate: a block writes column J + 2's packet only after reading every
// block's packet of J + 1, which each block writes only after reading all of
// column J's, so no packet is overwritten before every block has read it.
// Tags grow through the factorization (the work area starts zeroed), so a
// word left from an earlier column never matches.  Every wait is bounded.
// A panel block of NT threads holds 4 NT rows: NT = 1024 when one block
// holds the whole panel (n - k0 <= 4096; the exchange goes through LDS and
// the launch is an ordinary one), NT = 256 for the cooperative grid of up to
// LU_PANEL_MAX_BLOCKS blocks of LU_PANEL_ROWS rows (more, smaller blocks:
// measured faster per column than fewer large ones)
constexpr int LP_R = 4;                          // panel rows per thread
constexpr int LP_NT_ONE = 1024, LP_NT_GRID = LU_PANEL_ROWS / LP_R;
constexpr int LP_SLOT = LU_NB + 2;               // a candidate: |a|, row, the row's values
constexpr uint32_t LP_SPIN_LIMIT = 1u << 20;     // polls before a wait gives up
constexpr int LP_WORDS = LU_PANEL_MAX_BLOCKS * LP_SLOT + LU_NB;  // packet words per column
static_assert(LP_R * LP_NT_GRID == LU_PANEL_ROWS, "rows per block");
static_assert(LU_PANEL_MAX_BLOCKS <= WAVE, "one candidate per lane");
// the work area (LU_WORK_BYTES): 32-bit words [0] info, [1] timeout; from
// byte 512 the packet words (64-bit) of the two column parities, each
// LU_PANEL_MAX_BLOCKS candidate slots then row rj
constexpr int LW_PACKETS = 512 / 8;  // in 64-bit words
static_assert((LW_PACKETS + 2 * LP_WORDS) * 8 <= (int)LU_WORK_BYTES, "work area");

template <int NT>
struct LpShared {
    float red_v[NT / WAVE];
    int red_i[NT / WAVE];
    float cand[LP_WORDS];  // every block's candidate slot, then row rj
};

__device__ __forceinline__ uint64_t lp_word(uint32_t tag, float v) {
    return ((uint64_t)tag << 32) | (uint32_t)__float_as_uint(v);
}

// the better of two candidates: larger magnitude, then lower row (a total
// order, so any reduction order picks the same row)
__device__ __forceinline__ bool lp_better(float ov, int oi, float v, int i) {
    return ov > v || (ov == v && oi < i);
}

// the packet exchange of column J between the blocks of a panel; false when
// a wait timed out
template <int J, int NT>
__device__ __forceinline__ bool lu_panel_exchange(int n, int row0, float (&p)[LP_R][LU_NB], LpShared<NT> &sh,
                                                  uint32_t *work, uint32_t tag, uint64_t *pk, float cv,
                                                  int ci, int rj) {
    const int t = threadIdx.x;
    // publish: |a| and row (thread 0), the row's values (the thread holding
    // it, or zeros from thread 0 when the candidate is row rj held by block
    // 0), row rj (the thread of block 0 holding it)
    uint64_t *slot = pk + blockIdx.x * LP_SLOT;
    if (t == 0) {
        coh_store(slot, lp_word(tag, cv));
        coh_store(slot + 1, lp_word(tag, __int_as_float(ci)));
    }
    const bool held = ci >= row0 && ci < row0 + (LP_R * NT) && ci < n;
    if (!held && t == 0) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) coh_store(slot + 2 + c, lp_word(tag, 0.0f));
    }
#pragma unroll
    for (int q = 0; q < LP_R; ++q) {
        const int r = row0 + t + NT * q;
        if (held && r == ci) {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c) coh_store(slot + 2 + c, lp_word(tag, p[q][c]));
        }
        if (r == rj) {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c)
                coh_store(pk + LU_PANEL_MAX_BLOCKS * LP_SLOT + c, lp_word(tag, p[q][c]));
        }
    }
    // every block's packet (G slots, then row rj): the thread's words are
    // loaded together and those without this column's tag loaded again,
    // together, until all carry it
    const int G = gridDim.x;
    const int nw = G * LP_SLOT;
    int late = 0;
    constexpr int WPT = (LP_WORDS + NT - 1) / NT;  // words loaded per thread
    uint64_t wv8[WPT];
    const uint64_t *src[WPT];
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
        const int e = t + NT * u;
        src[u] = e < nw ? pk + e : (e < nw + LU_NB ? pk + LU_PANEL_MAX_BLOCKS * LP_SLOT + (e - nw) : nullptr);
        wv8[u] = src[u] ? coh_load(src[u]) : lp_word(tag, 0.0f);
    }
    for (uint32_t polls = 0;; ++polls) {
        bool all = true;
#pragma unroll
        for (int u = 0; u < WPT; ++u) all = all && (uint32_t)(wv8[u] >> 32) == tag;
        if (all) break;
        if (polls >= LP_SPIN_LIMIT) {
            late = 1;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int u = 0; u < WPT; ++u)
            if ((uint32_t)(wv8[u] >> 32) != tag) wv8[u] = coh_load(src[u]);
    }
#pragma unroll
    for (int u = 0; u < WPT; ++u) {
        const int e = t + NT * u;
        if (src[u]) sh.cand[e < nw ? e : LU_PANEL_MAX_BLOCKS * LP_SLOT + (e - nw)] = __uint_as_float((uint32_t)wv8[u]);
    }
    return __syncthreads_or(late) == 0;
}

// pivot choice (every wave reduces the G candidates the same way), the
// interchange and the elimination of column J
template <int J, int NT>
__device__ __forceinline__ bool lu_panel_eliminate(int n, int k0, int row0, float (&p)[LP_R][LU_NB],
                                                   LpShared<NT> &sh, int *__restrict__ piv, uint32_t *work,
                                                   int rj) {
    const int t = threadIdx.x, lane = t & (WAVE - 1);
    const int G = gridDim.x;
    // every wave reduces the G candidates the same way
    float v = lane < G ? sh.cand[lane * LP_SLOT] : -2.0f;
    int i = lane < G ? __float_as_int(sh.cand[lane * LP_SLOT + 1]) : rj;
    int gw = lane < G ? lane : 0;
#pragma unroll
    for (int off = WAVE / 2; off >= 1; off >>= 1) {
        const float ov = __shfl_xor(v, off);
        const int oi = __shfl_xor(i, off);
        const int og = __shfl_xor(gw, off);
        if (ov > v || (ov == v && (oi < i || (oi == i && og < gw)))) {
            v = ov;
            i = oi;
            gw = og;
        }
    }
    const int pr = __shfl(i, 0);
    gw = __shfl(gw, 0);
    if (blockIdx.x == 0 && t == 0) piv[rj] = pr;
    // the pivot row: published by the block that holds it (row rj itself
    // when no other row won)
    const float *rowA = sh.cand + LU_PANEL_MAX_BLOCKS * LP_SLOT;
    const float *rowB = pr == rj ? rowA : sh.cand + gw * LP_SLOT + 2;
    if (pr != rj) {
#pragma unroll
        for (int q = 0; q < LP_R; ++q) {
            const int r = row0 + t + NT * q;
            if (r == rj) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) p[q][c] = rowB[c];
            } else if (r == pr) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) p[q][c] = rowA[c];
            }
        }
    }
    // eliminate below the pivot
    const float d = rowB[J];
    if (d != 0.0f) {
#pragma unroll
        for (int q = 0; q < LP_R; ++q) {
            const int r = row0 + t + NT * q;
            if (r > rj && r < n) {
                const float l = p[q][J] / d;
                p[q][J] = l;
#pragma unroll
                for (int c = J + 1; c < LU_NB; ++c) p[q][c] = p[q][c] - l * rowB[c];
            }
        }
    } else if (blockIdx.x == 0 && t == 0 && work[0] == 0) {
        work[0] = rj + 1;  // the first zero pivot (block 0 alone writes the info word)
    }
    return true;
}

// Column J of the panel (J a template parameter, so that the panel stays in
// registers: every index into p is a compile-time constant).  False when a
// wait timed out.
template <int J, int NT>
__device__ __forceinline__ bool lu_panel_col(int n, int k0, int b, int row0, float (&p)[LP_R][LU_NB],
                                             LpShared<NT> &sh, int *__restrict__ piv, uint32_t *work) {
    if (J >= b) return true;  // uniform: the last panel may be narrower
    const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
    const int rj = k0 + J;
    const uint32_t tag = (uint32_t)(rj + 1);
    uint64_t *pk = reinterpret_cast<uint64_t *>(work) + LW_PACKETS + (J & 1) * LP_WORDS;
    // the block's candidate: largest |a(r, J)| over its rows r >= rj, the
    // first such row; the search starts from row rj, so the pivot is a row of
    // the panel even when no magnitude compares greater (a column of NaNs)
    float bv = -1.0f;
    int bi = rj;
#pragma unroll
    for (int q = 0; q < LP_R; ++q) {
        const int r = row0 + t + NT * q;
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
        if (lp_better(ov, oi, bv, bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) {
        sh.red_v[wv] = bv;
        sh.red_i[wv] = bi;
    }
    __syncthreads();
    // every thread reduces the waves' candidates (the same order everywhere)
    float cv = sh.red_v[0];
    int ci = sh.red_i[0];
#pragma unroll
    for (int w2 = 1; w2 < NT / WAVE; ++w2) {
        if (lp_better(sh.red_v[w2], sh.red_i[w2], cv, ci)) {
            cv = sh.red_v[w2];
            ci = sh.red_i[w2];
        }
    }
    const int G = gridDim.x;
    if (G == 1) {
        // one block holds the whole panel: its candidate and row rj through LDS
#pragma unroll
        for (int q = 0; q < LP_R; ++q) {
            const int r = row0 + t + NT * q;
            if (r == ci) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) sh.cand[2 + c] = p[q][c];
            }
            if (r == rj) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) sh.cand[LU_PANEL_MAX_BLOCKS * LP_SLOT + c] = p[q][c];
            }
        }
        if (t == 0) {
            sh.cand[0] = cv;
            sh.cand[1] = __int_as_float(ci);
        }
        __syncthreads();
    } else if (!lu_panel_exchange<J, NT>(n, row0, p, sh, work, tag, pk, cv, ci, rj)) {
        return false;
    }
    return lu_panel_eliminate<J, NT>(n, k0, row0, p, sh, piv, work, rj);
}

template <int NT, int... J>
__device__ __forceinline__ bool lu_panel_cols(int n, int k0, int b, int row0, float (&p)[LP_R][LU_NB],
                                              LpShared<NT> &sh, int *__restrict__ piv, uint32_t *work,
                                              std::integer_sequence<int, J...>) {
    return (lu_panel_col<J, NT>(n, k0, b, row0, p, sh, piv, work) && ...);
}

// Block g holds rows k0 + 4 NT g + t + NT q (q < 4) of the panel.
template <int NT>
__global__ __launch_bounds__(NT) void lu_panel_kernel(int n, int64_t ldl, float *__restrict__ LU,
                                                         int k0, int *__restrict__ piv,
                                                         uint32_t *__restrict__ work) {
    __shared__ LpShared<NT> sh;
    const int t = threadIdx.x;
    const int b = min(LU_NB, n - k0);
    const int row0 = k0 + blockIdx.x * (LP_R * NT);
    float p[LP_R][LU_NB];
    // whole 16-byte pieces of full panels when aligned (vec), else element by element
    const bool vec = b == LU_NB && ldl % 4 == 0 && reinterpret_cast<uintptr_t>(LU) % 16 == 0;
#pragma unroll
    for (int q = 0; q < LP_R; ++q) {
        const int r = row0 + t + NT * q;
        const float *src = LU + (int64_t)min(r, n - 1) * ldl + k0;
        if (vec) {
#pragma unroll
            for (int c4 = 0; c4 < LU_NB / 4; ++c4) {
                const lg_f4 v = r < n ? reinterpret_cast<const lg_f4 *>(src)[c4] : lg_f4{0.f, 0.f, 0.f, 0.f};
                p[q][4 * c4] = v.x, p[q][4 * c4 + 1] = v.y, p[q][4 * c4 + 2] = v.z, p[q][4 * c4 + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int c = 0; c < LU_NB; ++c) p[q][c] = (r < n && c < b) ? src[c] : 0.0f;
        }
    }
    if (!lu_panel_cols<NT>(n, k0, b, row0, p, sh, piv, work, std::make_integer_sequence<int, LU_NB>{})) {
        if (t == 0) coh_store(work + 1, 1u);
        return;
    }
#pragma unroll
    for (int q = 0; q < LP_R; ++q) {
        const int r = row0 + t + NT * q;
        if (r < n) {
            float *dst = LU + (int64_t)r * ldl + k0;
            if (vec) {
#pragma unroll
                for (int c4 = 0; c4 < LU_NB / 4; ++c4)
                    reinterpret_cast<lg_f4 *>(dst)[c4] = lg_f4{p[q][4 * c4], p[q][4 * c4 + 1], p[q][4 * c4 + 2], p[q][4 * c4 + 3]};
            } else {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c)
                    if (c < b) dst[c] = p[q][c];
            }
        }
    }
}

// the whole work area starts at zero: info, the timeout word, every packet tag
__global__ __launch_bounds__(WAVE * 4) void lu_work_reset_kernel(uint32_t *work) {
    for (int i = threadIdx.x; i < (int)(LU_WORK_BYTES / 4); i += WAVE * 4) work[i] = 0u;
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

// rows k0:k0+b of U in columns [cs, ce): z = L00^-1 A(k0:k0+b, c), one column per thread
__global__ __launch_bounds__(GEMV_NT) void lu_trsm_kernel(int n, int64_t ldl, float *__restrict__ LU,
                                                          int k0, int b, int cs, int ce) {
    __shared__ float L00[LU_NB][LU_NB];
    {
        const int i = threadIdx.x / LU_NB, j = threadIdx.x % LU_NB;
        if (i < LU_NB) L00[i][j] = (i < b && j < b) ? LU[(int64_t)(k0 + i) * ldl + k0 + j] : 0.0f;
    }
    __syncthreads();
    const int c = cs + blockIdx.x * GEMV_NT + threadIdx.x;
    if (c >= ce) return;
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

// A(r, c) -= sum_{j < b} A(r, k0 + j) A(k0 + j, c), k1 = k0 + b, on two
// regions: rows [k1, n) x columns [k1, kend) (the rest of the outer block's
// columns) and rows [k1, kend) x columns [kend, n) (the rest of its rows).
// 64 x 64 tiles, each thread 4 x 4 (rows tr + 16 i, columns tc + 16 j); the
// first t1r x t1c blocks take region one, the others region two (t2c tile
// columns).
__global__ __launch_bounds__(GEMV_NT) void lu_update_kernel(int n, int64_t ldl, float *__restrict__ LU,
                                                            int k0, int b, int kend, int t1r, int t1c,
                                                            int t2c) {
    __shared__ float Ls[LU_TILE][LU_NB + 1];
    __shared__ float Us[LU_NB][LU_TILE];
    const int k1 = k0 + b;
    int r0, c0, rlim, clim;
    const int bx = blockIdx.x;
    if (bx < t1r * t1c) {
        r0 = k1 + (bx / t1c) * LU_TILE, c0 = k1 + (bx % t1c) * LU_TILE;
        rlim = n, clim = kend;
    } else {
        const int e = bx - t1r * t1c;
        r0 = k1 + (e / t2c) * LU_TILE, c0 = kend + (e % t2c) * LU_TILE;
        rlim = kend, clim = n;
    }
#pragma unroll
    for (int e = 0; e < LU_TILE * LU_NB / GEMV_NT; ++e) {
        const int idx = threadIdx.x + GEMV_NT * e;
        const int rr = idx / LU_NB, jj = idx % LU_NB;
        const int r = r0 + rr;
        Ls[rr][jj] = (r < rlim && jj < b) ? LU[(int64_t)r * ldl + k0 + jj] : 0.0f;
        const int j2 = idx / LU_TILE, cc = idx % LU_TILE;
        const int c = c0 + cc;
        Us[j2][cc] = (c < clim && j2 < b) ? LU[(int64_t)(k0 + j2) * ldl + c] : 0.0f;
    }
    __syncthreads();
    const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = tr + 16 * i, r = r0 + rr;
        if (r >= rlim) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int cc = tc + 16 * j, c = c0 + cc;
            if (c >= clim) continue;
            float s = LU[(int64_t)r * ldl + c];
#pragma unroll
            for (int jj = 0; jj < LU_NB; ++jj) s = s - Ls[rr][jj] * Us[jj][cc];
            LU[(int64_t)r * ldl + c] = s;
        }
    }
}

// ------------------------------------------------- trailing update (MFMA)
// A(K1:n, K1:n) -= A(K1:n, K0:K1) A(K0:K1, K1:n), K = K1 - K0 a multiple of
// LG_BK.  A block of four waves owns a 128 x 128 tile, each wave a 64 x 64
// quarter as 4 x 4 tiles of v_mfma_f32_16x16x4f32.  K streams through LDS in
// chunks of 32 (double-buffered: the next chunk's global loads are in flight
// while the matrix cores work on the current one).  Lane l of a wave (g = l /
// 16, c = l % 16) feeds step s of a chunk with k = 8 g + s: A operand row c
// of a row tile, B operand column c of a column tile (the sum over k is the
// same, in the matrix core's order); accumulator item v of lane l is
// C[4 g + v][c].  Blocks are numbered round-robin over the eight XCDs, so
// block b takes logical tile (b % 8) q + b / 8 (q tiles per XCD), and the
// logical tiles run down groups of 8 tile rows: the tiles in flight on one
// XCD share rows of L21 and columns of U12 in its L2.
constexpr int LG_BM = 128, LG_BN = 128, LG_BK = 32, LG_NT = 256;
constexpr int LG_LDA = LG_BK + 4;  // LDS row stride of the L21 chunk (16-byte aligned rows)
constexpr int LG_LDB = LG_BN + 4;  // LDS row stride of the U12 chunk
constexpr int LG_GROUP = 8;
constexpr int LG_XCD = 8;
static_assert(LU_NBO % LG_BK == 0, "K in whole chunks");

template <bool VEC>
__device__ __forceinline__ lg_f4 lg_load4(const float *p, int valid) {
    if (VEC && valid >= 4) return *reinterpret_cast<const lg_f4 *>(p);
    lg_f4 v;
    v.x = valid > 0 ? p[0] : 0.0f;
    v.y = valid > 1 ? p[1] : 0.0f;
    v.z = valid > 2 ? p[2] : 0.0f;
    v.w = valid > 3 ? p[3] : 0.0f;
    return v;
}

__device__ __forceinline__ bool lg_tile(int bid, int tiles_r, int tiles_c, int &tr, int &tc) {
    const int total = tiles_r * tiles_c;
    const int per_xcd = div_up(total, LG_XCD);
    const int L = (bid % LG_XCD) * per_xcd + bid / LG_XCD;
    if (L >= total) return false;
    const int per_group = LG_GROUP * tiles_c;
    const int first = (L / per_group) * LG_GROUP;
    const int gm = min(tiles_r - first, LG_GROUP);
    const int l = L % per_group;
    tr = first + l % gm;
    tc = l / gm;
    return true;
}

// VEC: 16-byte loads (LU 16-byte aligned, ldl a multiple of 4)
template <bool VEC>
__global__ __launch_bounds__(LG_NT) void lu_gemm_kernel(int n, int64_t ldl, float *__restrict__ LU, int K0,
                                                        int K1, int tiles_r, int tiles_c) {
    __shared__ __attribute__((aligned(16))) float As[2][LG_BM * LG_LDA];
    __shared__ __attribute__((aligned(16))) float Bs[2][LG_BK * LG_LDB];
    int tr, tc;
    if (!lg_tile(blockIdx.x, tiles_r, tiles_c, tr, tc)) return;
    const int r0 = K1 + tr * LG_BM, c0 = K1 + tc * LG_BN;
    const int t = threadIdx.x, lane = t & (WAVE - 1), w = t / WAVE;
    const int g = lane >> 4, c = lane & 15;
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    const int nch = (K1 - K0) / LG_BK;
    // staging: L21 rows t / 8 + 32 i, k = 4 (t % 8); U12 rows t / 32 + 8 i, columns 4 (t % 32)
    const int ar = t / 8, ak = 4 * (t % 8);
    const int bk = t / 32, bc = 4 * (t % 32);
    lg_f4 ra[4], rb[4];
    auto gload = [&](int ch) {
        const int kb = K0 + ch * LG_BK;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + ar + 32 * i;
            ra[i] = lg_load4<VEC>(LU + (int64_t)min(r, n - 1) * ldl + kb + ak, r < n ? 4 : 0);
            rb[i] = lg_load4<VEC>(LU + (int64_t)(kb + bk + 8 * i) * ldl + c0 + bc, n - (c0 + bc));
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            *reinterpret_cast<lg_f4 *>(&As[buf][(ar + 32 * i) * LG_LDA + ak]) = ra[i];
            *reinterpret_cast<lg_f4 *>(&Bs[buf][(bk + 8 * i) * LG_LDB + bc]) = rb[i];
        }
    };
    lg_f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = lg_f4{0.f, 0.f, 0.f, 0.f};
    gload(0);
    sstore(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nch) gload(ch + 1);
        const float *as = As[buf];
        const float *bs = Bs[buf];
        float a[4][8], bq[4][8];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const lg_f4 *pa = reinterpret_cast<const lg_f4 *>(as + (wr + 16 * rt + c) * LG_LDA + 8 * g);
            const lg_f4 x = pa[0], y = pa[1];
            a[rt][0] = x.x, a[rt][1] = x.y, a[rt][2] = x.z, a[rt][3] = x.w;
            a[rt][4] = y.x, a[rt][5] = y.y, a[rt][6] = y.z, a[rt][7] = y.w;
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int s = 0; s < 8; ++s) bq[ct][s] = bs[(8 * g + s) * LG_LDB + wc + 16 * ct + c];
#pragma unroll
        for (int s = 0; s < 8; ++s)
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rt][s], bq[ct][s], acc[rt][ct], 0, 0, 0);
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
                if (row < n && col < n) {
                    float *pc = LU + (int64_t)row * ldl + col;
                    *pc = *pc - acc[rt][ct][v];
                }
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

// ------------------------------------------- persistent substitutions
// One cooperative launch per substitution (instead of n/64): row block J of
// 64 rows belongs to block J mod G of the grid, which applies every solved
// column block to it and solves its diagonal tile when its turn comes.  In
// sweep order (forward: row block 0 first; backward: the last first), at
// position s with row block I solved: the block owning the next position
// applies x_I to that row block first and solves it at once (the critical
// path), then every block applies x_I to its other row blocks still ahead.
// The owner of a row block publishes its x (64 words) with agent-scope
// relaxed stores, waits for them to complete (vmcnt(0)) and then stores the
// row block's flag word; in every other block one thread polls that flag
// (agent-scope relaxed loads, backing off between polls: a flag polled by
// every thread of every block measured slower than the launches it
// replaces), and then the block loads x the same way.  The flags start at
// zero (tp_reset_kernel); the forward sweep sets 1, the backward sweep 2, so
// a flag left by the other sweep never matches.  The owner of the
// next position loads that row block's tile of the solved column and its
// diagonal tile before it waits, so the wait overlaps those loads.  Each
// column block's contribution to a row is the same butterfly sum as in the
// per-launch kernels (rows_reduce over eight rows), applied in the same
// order, so the results are the same bit for bit.  Every wait is bounded;
// a block that gives up sets *fail and leaves (the other blocks' waits then
// give up too).
//
// Measured per solve (GMRES-IR with the LU, 2 refinement steps): n = 2000
// 3.09 ms against 3.85 with a launch per step, 4096 6.59 / 8.07, 8192
// 13.3 / 15.6, 16384 38.8 / 40.8, but 32768 122 / 87.5 (a block per row
// block, 512 blocks): each step's chain of device-scope round trips (x,
// its flag, the reads of x and t) costs about as much as a launch does, and
// at 512 row blocks more.  So the sweeps run persistent up to TP_MAX_NB row
// blocks and as launches per step beyond.
constexpr int TP_NT = GEMV_NT;             // threads of a block (4 waves)
constexpr int TP_MAX_BLOCKS = 256;
constexpr int TP_MAX_NB = 256;             // row blocks up to which the sweeps are persistent
constexpr uint32_t TP_SPIN_LIMIT = 1u << 21;
constexpr int TP_WORDS = 2 * TS_SB;        // words per row block: x (64), the flag (word 64)
constexpr int TP_BACKOFF = 4;              // s_sleep units between polls of a flag
static_assert(TP_NT == TS_WAVES * WAVE, "four waves of 16 rows");

size_t ts_persist_words(int n) { return (size_t)div_up(n, TS_SB) * TP_WORDS; }

__global__ __launch_bounds__(VEC_NT) void tp_reset_kernel(uint64_t *xw, size_t count, int *fail) {
    const size_t i = (size_t)blockIdx.x * VEC_NT + threadIdx.x;
    if (i < count) xw[i] = 0u;
    if (i == 0) *fail = 0;
}

// The diagonal tile of row block J (rows r0 .. r0 + m) into T, widened, with
// the mask of the sweep: forward unit-lower (strict lower part), forward
// lower with its diagonal, backward upper with its diagonal; rows past n get
// a unit diagonal.
template <bool FWD, bool UNIT>
__device__ __forceinline__ void tp_load_diag(int n, int64_t ldl, const float *__restrict__ F, int r0, int m,
                                             double *T) {
    constexpr int Q = TS_SB / TS_WAVES;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int cc = min(lane, m - 1);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int k = w + TS_WAVES * q;
        const double tl = (double)F[(int64_t)(r0 + min(k, m - 1)) * ldl + r0 + cc];
        double v;
        if constexpr (FWD && UNIT)
            v = (k < m && lane < k) ? tl : 0.0;
        else if constexpr (FWD)
            v = (k < m && lane < m) ? (lane <= k ? tl : 0.0) : (lane == k ? 1.0 : 0.0);
        else
            v = (k < m && lane < m) ? (lane >= k ? tl : 0.0) : (lane == k ? 1.0 : 0.0);
        T[k * TS_LDT + lane] = v;
    }
}

// Wave 0: x of the diagonal tile from acc (the row's right-hand side with
// every earlier column block applied), as in the per-launch kernels.
template <bool FWD, bool UNIT>
__device__ __forceinline__ double tp_diag_solve(const double *T, double acc, int lane) {
    double xi = 0.0;
    if constexpr (FWD && UNIT) {
#pragma unroll
        for (int j = 0; j < TS_SB; ++j) {
            const double xj = ts_readlane(acc, j);
            xi = (lane == j) ? acc : xi;
            acc = fma(-T[lane * TS_LDT + j], xj, acc);
        }
    } else if constexpr (FWD) {
        const double dinv = 1.0 / T[lane * TS_LDT + lane];
#pragma unroll
        for (int j = 0; j < TS_SB; ++j) {
            const double xc = acc * dinv;
            const double xj = ts_readlane(xc, j);
            xi = (lane == j) ? xc : xi;
            acc = fma(lane > j ? -T[lane * TS_LDT + j] : 0.0, xj, acc);
        }
    } else {
        const double dinv = 1.0 / T[lane * TS_LDT + lane];
#pragma unroll
        for (int j = TS_SB - 1; j >= 0; --j) {
            const double xc = acc * dinv;
            const double xj = ts_readlane(xc, j);
            xi = (lane == j) ? xc : xi;
            acc = fma(lane < j ? -T[lane * TS_LDT + j] : 0.0, xj, acc);
        }
    }
    return xi;
}

template <bool FWD, bool UNIT>
__global__ __launch_bounds__(TP_NT) void tp_sweep_kernel(int n, int64_t ldl, const float *__restrict__ F,
                                                         double *__restrict__ t, uint64_t *__restrict__ xw,
                                                         int *__restrict__ fail, uint32_t spin_limit) {
    constexpr int Q = TS_SB / TS_WAVES;  // rows of a tile per wave
    __shared__ double T[TS_SB * TS_LDT];
    __shared__ double xs[2][TS_SB];
    __shared__ double sI[TS_SB];
    const int nb = div_up(n, TS_SB), G = gridDim.x, b = blockIdx.x;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const uint32_t tag = FWD ? 1u : 2u;
    auto blk = [&](int s) { return FWD ? s : nb - 1 - s; };
    // the block's last sweep position
    int last = -1;
    for (int s = nb - 1; s >= 0; --s)
        if (blk(s) % G == b) {
            last = s;
            break;
        }
    if (last < 0) return;
    // t_J -= F(J rows, I columns) x_I for the rows of row block J, with the
    // tile's values already in pv (wave w rows w Q .. w Q + Q - 1)
    auto apply = [&](int J, const double (&pv)[Q], const double *x) {
        const double xl = x[lane];
        ts_rows_sums(pv, xl, lane, sI + w * Q);
        __syncthreads();
        const int rj = J * TS_SB + threadIdx.x;
        if (threadIdx.x < TS_SB && rj < n) t[rj] -= sI[threadIdx.x];
        __syncthreads();
    };
    auto load_tile = [&](int J, int I, double (&pv)[Q]) {
        const int r0 = J * TS_SB, m = min(TS_SB, n - r0);
        const int c = I * TS_SB + lane;
        const bool cin = c < n;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            pv[q] = cin ? (double)F[(int64_t)(r0 + min(w * Q + q, m - 1)) * ldl + c] : 0.0;
    };
    // solve row block J (its t has every earlier column applied), keep x in
    // xs[buf], write it to t and publish it
    auto solve = [&](int J, int buf) {
        const int r0 = J * TS_SB, m = min(TS_SB, n - r0);
        __syncthreads();
        if (w == 0) {
            const double acc = lane < m ? t[r0 + lane] : 0.0;
            const double xi = tp_diag_solve<FWD, UNIT>(T, acc, lane);
            const double xv = lane < m ? xi : 0.0;
            if (lane < m) t[r0 + lane] = xi;
            xs[buf][lane] = xv;
            uint64_t *dst = xw + (size_t)J * TP_WORDS;
            coh_store(dst + lane, __builtin_bit_cast(uint64_t, xv));
            __builtin_amdgcn_s_waitcnt(WAIT_VMEM);  // x stored before the flag
            if (lane == 0) coh_store(dst + TS_SB, (uint64_t)tag);
        }
        __syncthreads();
    };
    // position 0
    if (blk(0) % G == b) {
        const int J = blk(0);
        tp_load_diag<FWD, UNIT>(n, ldl, F, J * TS_SB, min(TS_SB, n - J * TS_SB), T);
        solve(J, 0);
    }
    for (int s = 0; s < last; ++s) {
        const int I = blk(s), buf = s & 1;
        const bool mine = I % G == b;
        const int nx = blk(s + 1);
        const bool next_mine = nx % G == b;
        double pv[Q];
        if (next_mine) {
            // the critical row block's tile and diagonal tile, before the wait
            load_tile(nx, I, pv);
            tp_load_diag<FWD, UNIT>(n, ldl, F, nx * TS_SB, min(TS_SB, n - nx * TS_SB), T);
        }
        if (!mine) {
            // x_I from its owner: thread 0 waits for the flag, then x
            int late = 0;
            const uint64_t *src = xw + (size_t)I * TP_WORDS;
            if (threadIdx.x == 0) {
                uint32_t polls = 0;
                while (coh_load(src + TS_SB) != (uint64_t)tag) {
                    if (++polls > spin_limit) {
                        late = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(TP_BACKOFF);
                }
            }
            if (__syncthreads_or(late)) {
                if (threadIdx.x == 0) coh_store(fail, 1);
                return;
            }
            if (threadIdx.x < TS_SB) xs[buf][threadIdx.x] = __builtin_bit_cast(double, coh_load(src + threadIdx.x));
            __syncthreads();
        }
        if (next_mine) {
            apply(nx, pv, xs[buf]);
            solve(nx, buf ^ 1);
        }
        // the block's other row blocks still ahead of the sweep
        for (int p = s + 2; p <= last; ++p) {
            const int J = blk(p);
            if (J % G != b) continue;
            load_tile(J, I, pv);
            apply(J, pv, xs[buf]);
        }
    }
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
hipError_t launch_lu_factor(int n, int64_t ldl, float *LU, int *piv, void *work, hipStream_t s) {
    if (n < 1 || n > LU_MAX_N) return hipErrorInvalidValue;
    uint32_t *w = static_cast<uint32_t *>(work);
    lu_work_reset_kernel<<<1, WAVE * 4, 0, s>>>(w);
    const bool vec = ldl % 4 == 0 && reinterpret_cast<uintptr_t>(LU) % 16 == 0;
    for (int K0 = 0; K0 < n; K0 += LU_NBO) {
        const int K1 = min(K0 + LU_NBO, n);
        for (int k0 = K0; k0 < K1; k0 += LU_NB) {
            const int b = min(LU_NB, n - k0), k1 = k0 + b;
            if (n - k0 <= LP_R * LP_NT_ONE) {
                // one block holds the panel: nothing to be co-resident with
                lu_panel_kernel<LP_NT_ONE><<<1, LP_NT_ONE, 0, s>>>(n, ldl, LU, k0, piv, w);
            } else {
                const int G = div_up(n - k0, LU_PANEL_ROWS);
                int an = n, ak0 = k0;
                int64_t aldl = ldl;
                float *aLU = LU;
                int *apiv = piv;
                void *args[] = {&an, &aldl, &aLU, &ak0, &apiv, &w};
                const hipError_t e = hipLaunchCooperativeKernel(
                    reinterpret_cast<const void *>(lu_panel_kernel<LP_NT_GRID>), dim3(G), dim3(LP_NT_GRID),
                    args, 0, s);
                if (e != hipSuccess) return e;
            }
            lu_swap_kernel<<<div_up(n, GEMV_NT), GEMV_NT, 0, s>>>(n, ldl, LU, k0, b, piv);
            if (k1 < K1) {
                lu_trsm_kernel<<<div_up(K1 - k1, GEMV_NT), GEMV_NT, 0, s>>>(n, ldl, LU, k0, b, k1, K1);
                const int t1r = div_up(n - k1, LU_TILE), t1c = div_up(K1 - k1, LU_TILE);
                lu_update_kernel<<<t1r * t1c, GEMV_NT, 0, s>>>(n, ldl, LU, k0, b, K1, t1r, t1c, 1);
            }
        }
        if (K1 < n) {
            // U12, row block by row block (region two of lu_update_kernel only)
            for (int k0 = K0; k0 < K1; k0 += LU_NB) {
                const int k1 = k0 + LU_NB;
                lu_trsm_kernel<<<div_up(n - K1, GEMV_NT), GEMV_NT, 0, s>>>(n, ldl, LU, k0, LU_NB, K1, n);
                if (k1 < K1) {
                    const int t2r = div_up(K1 - k1, LU_TILE), t2c = div_up(n - K1, LU_TILE);
                    lu_update_kernel<<<t2r * t2c, GEMV_NT, 0, s>>>(n, ldl, LU, k0, LU_NB, K1, 0, 1, t2c);
                }
            }
            const int tr = div_up(n - K1, LG_BM), tc = div_up(n - K1, LG_BN);
            const int grid = LG_XCD * div_up(tr * tc, LG_XCD);
            if (vec)
                lu_gemm_kernel<true><<<grid, LG_NT, 0, s>>>(n, ldl, LU, K0, K1, tr, tc);
            else
                lu_gemm_kernel<false><<<grid, LG_NT, 0, s>>>(n, ldl, LU, K0, K1, tr, tc);
        }
    }
    return hipGetLastError();
}

// the two persistent sweeps on t: forward (unit lower or lower with its
// diagonal), then backward (upper with its diagonal)
template <bool UNIT>
static hipError_t launch_tp_sweeps(int n, int64_t ldl, const float *F, double *t, uint64_t *xw, int *fail,
                                   hipStream_t s) {
    const int nb = div_up(n, TS_SB);
    const size_t words = ts_persist_words(n);
    tp_reset_kernel<<<(unsigned)div_up((int)words, VEC_NT), VEC_NT, 0, s>>>(xw, words, fail);
    int an = n;
    int64_t aldl = ldl;
    const float *aF = F;
    double *at = t;
    uint64_t *axw = xw;
    int *afail = fail;
    uint32_t spin = TP_SPIN_LIMIT;
    void *args[] = {&an, &aldl, &aF, &at, &axw, &afail, &spin};
    const int G = min(nb, TP_MAX_BLOCKS);
    hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(tp_sweep_kernel<true, UNIT>), dim3(G),
                                              dim3(TP_NT), args, 0, s);
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(tp_sweep_kernel<false, false>), dim3(G),
                                      dim3(TP_NT), args, 0, s);
}

hipError_t launch_lu_apply(int n, int64_t ldl, const float *LU, const int *perm, const double *src,
                           double *dst, double *t, double *partial, uint64_t *xw, int *fail, hipStream_t s) {
    lu_gather_kernel<<<div_up(n, VEC_NT), VEC_NT, 0, s>>>(n, perm, src, t);
    if (xw && div_up(n, TS_SB) <= TP_MAX_NB) {
        const hipError_t e = launch_tp_sweeps<true>(n, ldl, LU, t, xw, fail, s);
        if (e != hipSuccess) return e;
        lu_pc_copy_kernel<<<gemv_blocks<double>(n), WAVE, 0, s>>>(n, t, dst, partial);
        return hipGetLastError();
    }
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
                             uint64_t *xw, int *fail, hipStream_t s) {
    if (dst != src) ch_copy_kernel<<<div_up(n, VEC_NT), VEC_NT, 0, s>>>(n, src, dst);
    if (xw && div_up(n, TS_SB) <= TP_MAX_NB) return launch_tp_sweeps<false>(n, ldl, L, dst, xw, fail, s);
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
