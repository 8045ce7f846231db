// Multi-right-hand-side conjugate gradient in lockstep: s independent CG
// recurrences (one per column of B) that share each iteration's product
// Q = A P, an n x n times n x s dense contraction computed on the matrix
// cores (MFMA).  Each column keeps its own alpha, beta, rho and stopping test,
// exactly as a single-right-hand-side solve would (the Krylov section's CG,
// column by column); columns that have converged are frozen.
//
// Layout: P, Q, R, X (working copy) and B are column-major n x s with leading
// dimension ldv (each right-hand side contiguous); s is padded to a multiple
// of 16 (the MFMA tile width), up to KS_MAX_NRHS.
//
// The contraction (binary64: v_mfma_f64_16x16x4f64; binary32 for the refined
// inner solve: v_mfma_f32_16x16x4f32): a wave owns 32 rows of Q and all s
// columns (2 x (s/16) accumulator tiles).  In one MFMA the four lane groups g
// supply four values of K; which four is free, since the sum over K is the
// same whatever the order, so K is permuted to make each lane's loads
// contiguous: binary64 walks K in steps of 16 with lane group g on
// k = 4g + t (4 doubles = 32 bytes per lane, a whole 128-byte line per row),
// binary32 in steps of 32 with g on k = 8g + t (8 floats: again a whole line
// per row in each pair of 16-byte loads).  K is split S ways for parallelism
// (partials summed in fixed order by the next kernel), and blocks are mapped
// to XCDs so that all blocks of one split run on the same XCDs and that
// split's slice of P stays in their L2.  Each block stages P's chunks of 64
// values of K in LDS (double buffered), shared by its waves (four in
// binary64, eight in binary32): measured on
// MI355X at n = 16384, s = 64, binary64 0.84 -> 0.66 ms (0.52 -> 0.67 of the
// matrix-core peak), the same sums bit for bit.  A streams from HBM a few
// steps ahead of its use: binary64 three steps of 16 ahead through a ring of
// four register sets, binary32 four steps of 32 ahead through a queue of
// five (measured faster, each, than the other's scheme for that precision).
// The binary32 kernel keeps one block of eight waves per CU (S = 4 at
// n = 16384) and relies on that queue for its loads in flight: measured
// 0.39 ms (one step of 16 ahead, four-wave blocks, S = 8) -> 0.30-0.31 ms
// (0.70-0.72 of the peak); binary64 is fastest at two four-wave blocks per
// CU (S = 4: 0.60 -> 0.57 ms, 0.77 of the peak).
#include <algorithm>

#include "ks_device.h"

namespace ks {

typedef double mr_d4 __attribute__((ext_vector_type(4)));
typedef float mr_f4 __attribute__((ext_vector_type(4)));
typedef double mr_d2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    using Acc = mr_d4;
    // lane l, accumulator item v holds D[4v + l/16][l%16]
    static __device__ __forceinline__ int row_of(int v, int g) { return 4 * v + g; }
    static __device__ __forceinline__ Acc mma(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // 4 consecutive values at p (16-byte aligned)
    static __device__ __forceinline__ void load4(const double *p, double (&o)[4]) {
        const mr_d2 x = *reinterpret_cast<const mr_d2 *>(p);
        const mr_d2 y = *reinterpret_cast<const mr_d2 *>(p + 2);
        o[0] = x.x;
        o[1] = x.y;
        o[2] = y.x;
        o[3] = y.y;
    }
    static __device__ __forceinline__ void load4_nt(const double *p, double (&o)[4]) {
        const mr_d2 x = __builtin_nontemporal_load(reinterpret_cast<const mr_d2 *>(p));
        const mr_d2 y = __builtin_nontemporal_load(reinterpret_cast<const mr_d2 *>(p + 2));
        o[0] = x.x;
        o[1] = x.y;
        o[2] = y.x;
        o[3] = y.y;
    }
};
template <>
struct Mfma<float> {
    using Acc = mr_f4;
    // lane l, accumulator item v holds D[4(l/16) + v][l%16]
    static __device__ __forceinline__ int row_of(int v, int g) { return 4 * g + v; }
    static __device__ __forceinline__ Acc mma(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ void load4(const float *p, float (&o)[4]) {
        const mr_f4 x = *reinterpret_cast<const mr_f4 *>(p);
        o[0] = x.x;
        o[1] = x.y;
        o[2] = x.z;
        o[3] = x.w;
    }
    static __device__ __forceinline__ void load4_nt(const float *p, float (&o)[4]) {
        const mr_f4 x = __builtin_nontemporal_load(reinterpret_cast<const mr_f4 *>(p));
        o[0] = x.x;
        o[1] = x.y;
        o[2] = x.z;
        o[3] = x.w;
    }
};

constexpr int MR_KC = 64;        // values of K per LDS-staged chunk of P
constexpr int MR_KPAD = MR_KC + 2;  // padded column stride of the staged chunk (bank spread)
constexpr int MR_STEPS = MR_KC / 16;  // MFMA steps of 16 per chunk
constexpr int MR_AHEAD = 3;      // binary64: steps of 16 of A in flight ahead of the one multiplied
constexpr int MR_AHEAD32 = 4;    // binary32: steps of 32 of A in flight ahead
static_assert(MR_AHEAD < MR_STEPS, "a ring of MR_STEPS register sets for A");
static_assert(MR_KC % 32 == 0, "binary32 steps of 32 inside a chunk");

// Row tiles (of 16 rows) per wave: two (each value of P read from LDS feeds
// two MFMAs); one row tile per wave measured no faster for either precision
// on MI355X at n = 16384, s = 64.
template <typename T>
constexpr int mr_row_tiles() {
    return 2;
}
// Waves per block: binary64 four; binary32 eight (two per SIMD at one block
// per CU, sharing each staged chunk of P: measured 7% faster than four at
// n = 16384, s = 64, with the same number of blocks).
template <typename T>
constexpr int mr_waves() {
    return sizeof(T) == 4 ? 8 : 4;
}
template <typename T>
constexpr int mr_nthr() {
    return mr_waves<T>() * WAVE;
}
template <typename T>
constexpr int mr_block_rows() {
    return mr_waves<T>() * 16 * mr_row_tiles<T>();
}

// Block -> (row block, split).  Work-groups are dispatched round-robin over
// the 8 XCDs; give each split a fixed group of 8/S XCDs when the counts allow.
__device__ __forceinline__ void mr_block_map(int nrb, int S, int &rb, int &sp) {
    const int b = blockIdx.x;
    if (S <= 8 && 8 % S == 0 && nrb % (8 / S) == 0) {
        const int xpg = 8 / S;        // XCDs per split
        const int xcd = b % 8, idx = b / 8;
        sp = xcd / xpg;
        rb = (xcd % xpg) + xpg * idx;
    } else {
        sp = b / nrb;
        rb = b % nrb;
    }
}

// Qpart[sp] = A[:, K_sp] * P[K_sp, :] for the split's K range.
template <typename T, int CT>
__global__ __launch_bounds__(mr_nthr<T>()) __attribute__((amdgpu_waves_per_eu(2, 8))) void mr_gemm_kernel(int n, int64_t lda,
                                                                  const T *__restrict__ A,
                                                                  const T *__restrict__ P, int ldp,
                                                                  T *__restrict__ Qpart, int ldq,
                                                                  int S, int kchunk,
                                                                  const State *st, int gate) {
    using M = Mfma<T>;
    using Acc = typename M::Acc;
    constexpr int RT = mr_row_tiles<T>();
    constexpr int BROWS = mr_block_rows<T>();
    if (gate == 2 && (st->flags & F_STOP)) return;       // iteration: skip when all stopped
    if (gate == 1 && !(st->flags & F_STOP)) return;      // residual: only when all stopped
    const int nrb = (n + BROWS - 1) / BROWS;
    int rb, sp;
    mr_block_map(nrb, S, rb, sp);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int g = lane >> 4, c16 = lane & 15;
    const int row0 = rb * BROWS + w * 16 * RT;
    const int kb = sp * kchunk, ke = min(n, kb + kchunk);
    Acc acc[RT][CT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = Acc{0, 0, 0, 0};
    const T *arow[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) arow[rt] = A + (int64_t)min(row0 + 16 * rt + c16, n - 1) * lda;
    const T *pcol[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) pcol[ct] = P + (size_t)(16 * ct + c16) * ldp;
    // Whole chunks of MR_KC values of K: the block stages P's chunk (all s
    // columns) in LDS once, double-buffered, instead of every wave fetching
    // its own copy from L2; the next chunk is loaded into registers while the
    // current one is multiplied.  A streams from HBM MR_AHEAD steps of 16
    // ahead through a ring of MR_STEPS register sets (step j in set j % 4).
    // Every lane still takes k = k0 + 4g .. k0 + 4g + 3 per step of 16, in
    // order, so the sums are those of the unstaged loop.
    constexpr int NC = 16 * CT;
    // column stride of the staged chunk: binary64 padded by 2 (bank spread),
    // binary32 by 4 (16-byte aligned columns for 16-byte LDS reads)
    constexpr int KPAD = sizeof(T) == 8 ? MR_KPAD : MR_KC + 4;
    __shared__ __attribute__((aligned(16))) T lp[2][NC * KPAD];
    const int nch = (ke - kb) / MR_KC;
    const int ks_end = kb + nch * MR_KC;
    const int ns = nch * MR_STEPS;  // steps inside whole chunks
    T a[RT][4], p[CT][4];
    if (nch > 0) {
        // staging: the chunk's NG value groups of 4 consecutive k, group
        // gi = tid + NTHR j of thread tid
        constexpr int NTHR = mr_nthr<T>();
        constexpr int NG = NC * (MR_KC / 4);
        constexpr int GPT = (NG + NTHR - 1) / NTHR;
        const int tid = threadIdx.x;
        T stg[GPT][4];
        auto gload = [&](int c) {
#pragma unroll
            for (int j = 0; j < GPT; ++j) {
                const int gi = tid + NTHR * j;
                if (NG % NTHR != 0 && gi >= NG) continue;
                const int col = gi / (MR_KC / 4), k4 = (gi % (MR_KC / 4)) * 4;
                M::load4(P + (size_t)col * ldp + kb + c * MR_KC + k4, stg[j]);
            }
        };
        auto lstore = [&](int buf) {
#pragma unroll
            for (int j = 0; j < GPT; ++j) {
                const int gi = tid + NTHR * j;
                if (NG % NTHR != 0 && gi >= NG) continue;
                const int col = gi / (MR_KC / 4), k4 = (gi % (MR_KC / 4)) * 4;
                if constexpr (sizeof(T) == 4) {
                    *reinterpret_cast<mr_f4 *>(&lp[buf][col * KPAD + k4]) =
                        mr_f4{stg[j][0], stg[j][1], stg[j][2], stg[j][3]};
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t) lp[buf][col * KPAD + k4 + t] = stg[j][t];
                }
            }
        };
        gload(0);
        lstore(0);
        __syncthreads();
        if constexpr (sizeof(T) == 8) {
            // binary64: A MR_AHEAD steps ahead, P one value of t at a time
            T ar[MR_STEPS][RT][4];
#pragma unroll
            for (int d = 0; d < MR_AHEAD; ++d)
                if (d < ns) {
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) M::load4_nt(arow[rt] + kb + 16 * d + 4 * g, ar[d][rt]);
                }
            for (int c = 0; c < nch; ++c) {
                const int buf = c & 1;
                if (c + 1 < nch) gload(c + 1);
#pragma unroll
                for (int st16 = 0; st16 < MR_STEPS; ++st16) {
                    const int j = MR_STEPS * c + st16;
                    if (j + MR_AHEAD < ns) {
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
                            M::load4_nt(arow[rt] + kb + 16 * (j + MR_AHEAD) + 4 * g,
                                        ar[(st16 + MR_AHEAD) % MR_STEPS][rt]);
                    }
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        T pt[CT];
#pragma unroll
                        for (int ct = 0; ct < CT; ++ct)
                            pt[ct] = lp[buf][(16 * ct + c16) * KPAD + st16 * 16 + 4 * g + t];
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                            for (int ct = 0; ct < CT; ++ct)
                                acc[rt][ct] = M::mma(ar[st16][rt][t], pt[ct], acc[rt][ct]);
                    }
                }
                if (c + 1 < nch) lstore(buf ^ 1);
                __syncthreads();
            }
        } else {
            // binary32: steps of 32 values of K, lane group g on k = 8g + t;
            // A MR_AHEAD32 steps ahead through a queue of register sets
            // (a[0] is multiplied, a[MR_AHEAD32] receives the newest load)
            constexpr int SPC = MR_KC / 32;  // steps per chunk
            const int nsteps = nch * SPC;
            auto aload = [&](int j, mr_f4 (&dst)[RT][2]) {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        dst[rt][h] = __builtin_nontemporal_load(
                            reinterpret_cast<const mr_f4 *>(arow[rt] + kb + 32 * j + 8 * g + 4 * h));
            };
            mr_f4 aq[MR_AHEAD32 + 1][RT][2];
#pragma unroll
            for (int d = 0; d < MR_AHEAD32; ++d)
                if (d < nsteps) aload(d, aq[d]);
            for (int c = 0; c < nch; ++c) {
                const int buf = c & 1;
                if (c + 1 < nch) gload(c + 1);
#pragma unroll
                for (int hs = 0; hs < SPC; ++hs) {
                    const int j = c * SPC + hs;
                    if (j + MR_AHEAD32 < nsteps) aload(j + MR_AHEAD32, aq[MR_AHEAD32]);
                    mr_f4 pq[CT][2];
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            pq[ct][h] = *reinterpret_cast<const mr_f4 *>(
                                &lp[buf][(16 * ct + c16) * KPAD + 32 * hs + 8 * g + 4 * h]);
#pragma unroll
                    for (int t = 0; t < 8; ++t)
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                            for (int ct = 0; ct < CT; ++ct)
                                acc[rt][ct] = M::mma(aq[0][rt][t / 4][t % 4], pq[ct][t / 4][t % 4], acc[rt][ct]);
#pragma unroll
                    for (int d = 0; d < MR_AHEAD32; ++d)
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                            for (int h = 0; h < 2; ++h) aq[d][rt][h] = aq[d + 1][rt][h];
                }
                if (c + 1 < nch) lstore(buf ^ 1);
                __syncthreads();
            }
        }
    }
    // the rest of the range: full steps of 16 straight from P, then the tail
    int k0 = ks_end;
    const int kfull = k0 + ((ke - k0) / 16) * 16;
    for (; k0 < kfull; k0 += 16) {
        const int kk = k0 + 4 * g;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) M::load4_nt(arow[rt] + kk, a[rt]);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) M::load4(pcol[ct] + kk, p[ct]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = M::mma(a[rt][t], p[ct][t], acc[rt][ct]);
    }
    if (k0 < ke) {  // ragged tail of the K range, element by element
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = k0 + 4 * g + t;
            const bool ok = k < ke;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) a[rt][t] = ok ? arow[rt][k] : T(0);
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) p[ct][t] = ok ? pcol[ct][k] : T(0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = M::mma(a[rt][t], p[ct][t], acc[rt][ct]);
    }
    T *qs = Qpart + (size_t)sp * (size_t)(16 * CT) * ldq;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + 16 * rt + M::row_of(v, g);
                if (row < n) qs[(size_t)(16 * ct + c16) * ldq + row] = acc[rt][ct][v];
            }
}

// ------------------------------------------------------- per-column kernels
// A block takes MR_NT rows and a group of MR_CG columns (grid rows x column
// groups): at n = 16384, s = 64 that is 64 x 16 blocks instead of 64 blocks
// that each walk all s columns.  Each thread handles one row of the group's
// columns; per-column block partials [row block][KS_MAX_NRHS] are reduced by
// the next kernel.  A column's partial is the same sum, in the same order,
// whatever the grouping: the sums do not depend on MR_CG.
constexpr int MR_NT = 256;
constexpr int MR_CG = 4;  // columns per block

__device__ __forceinline__ int mr_j0() { return blockIdx.y * MR_CG; }
__device__ __forceinline__ int mr_j1(int s) { return min(s, (int)(blockIdx.y + 1) * MR_CG); }

// per-column sums of `val` over the block's rows: one wave sum per wave into red[wave][j]
__device__ __forceinline__ void mr_col_partial(double val, int j, double (*red)[KS_MAX_NRHS],
                                               bool is_max) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const double t = is_max ? wave_max(val) : wave_sum(val);
    if (lane == 0) red[w][j] = t;
}

// the waves' sums of columns [j0, j1), in wave order, to part[blockIdx.x][j]
__device__ __forceinline__ void mr_col_flush(int j0, int j1, double (*red)[KS_MAX_NRHS],
                                             double *part, bool is_max) {
    __syncthreads();
    for (int j = j0 + threadIdx.x; j < j1; j += MR_NT) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < MR_NT / WAVE; ++q) acc = is_max ? fmax(acc, red[q][j]) : acc + red[q][j];
        part[(size_t)blockIdx.x * KS_MAX_NRHS + j] = acc;
    }
    __syncthreads();
}

// totals over the nblk row blocks of columns [j0, j1), into LDS (all threads)
__device__ __forceinline__ void mr_col_reduce(int j0, int j1, const double *part, int nblk,
                                              double *out, bool is_max) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    for (int j = j0 + w; j < j1; j += MR_NT / WAVE) {
        double acc = 0.0;
        for (int b = lane; b < nblk; b += WAVE) {
            const double v = part[(size_t)b * KS_MAX_NRHS + j];
            acc = is_max ? fmax(acc, v) : acc + v;
        }
        acc = is_max ? wave_max(acc) : wave_sum(acc);
        if (lane == 0) out[j] = acc;
    }
    __syncthreads();
}

// ||b_j||_2, ||b_j||_inf, thresh_j: one block per column
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_stats_kernel(int n, const T *__restrict__ B, int ldb,
                                                         double tol, ColState *cols, State *st) {
    __shared__ double sm[MR_NT / WAVE];
    const int j = blockIdx.x;
    double s2 = 0.0, mx = 0.0;
    for (int i = threadIdx.x; i < n; i += MR_NT) {
        const double v = (double)B[(size_t)j * ldb + i];
        s2 += v * v;
        mx = fmax(mx, finite_d(v) ? fabs(v) : INFINITY);
    }
    const double ss = block_sum<MR_NT>(s2, sm);
    __syncthreads();
    const double bm = block_max<MR_NT>(mx, sm);
    if (threadIdx.x == 0) {
        ColState &c = cols[j];
        c.bnorm = sqrt(ss);
        c.binf = bm;
        c.thresh = tol * c.bnorm;
        c.iters = 0;
        c.restarts = 0;
        c.flags = F_STOP;
        if (j == 0) {
            st->flags = F_STOP;
            st->iters = 0;
        }
    }
}

// R = B - sum_sp Qpart[sp]; per column ||r||^2, ||r||_inf, ||x||_inf partials.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_resid_kernel(int n, int s, const T *__restrict__ B,
                                                         int ldb, const T *__restrict__ X,
                                                         const T *__restrict__ Qpart, int S,
                                                         int ldv, T *__restrict__ R, double *part,
                                                         const State *st, int gate) {
    __shared__ double red[MR_NT / WAVE][KS_MAX_NRHS];
    if (gate == 1 && !(st->flags & F_STOP)) return;
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    const bool valid = i < n;
    const int sp16 = (s + 15) / 16 * 16;
    const int j0 = mr_j0(), j1 = mr_j1(s);
    for (int pass = 0; pass < 3; ++pass) {
        for (int j = j0; j < j1; ++j) {
            double val = 0.0;
            if (valid) {
                if (pass == 2) {
                    const double xv = (double)X[(size_t)j * ldv + i];
                    val = finite_d(xv) ? fabs(xv) : INFINITY;
                } else {
                    T q = 0;
                    for (int k = 0; k < S; ++k) q += Qpart[((size_t)k * sp16 + j) * ldv + i];
                    const T r = B[(size_t)j * ldb + i] - q;
                    if (pass == 0) R[(size_t)j * ldv + i] = r;
                    val = (pass == 0) ? (double)r * (double)r
                                      : (finite_d((double)r) ? fabs((double)r) : INFINITY);
                }
            }
            mr_col_partial(val, j, red, pass != 0);
        }
        mr_col_flush(j0, j1, red, part + (size_t)pass * gridDim.x * KS_MAX_NRHS, pass != 0);
    }
}

// one block: per-column residual norms and true-residual flags
__global__ __launch_bounds__(MR_NT) void mr_resid_finish_kernel(int s, const double *part, int nblk,
                                                                ColState *cols, const State *st,
                                                                int gate) {
    __shared__ double v2[KS_MAX_NRHS], vr[KS_MAX_NRHS], vx[KS_MAX_NRHS];
    if (gate == 1 && !(st->flags & F_STOP)) return;
    mr_col_reduce(0, s, part, nblk, v2, false);
    mr_col_reduce(0, s, part + (size_t)nblk * KS_MAX_NRHS, nblk, vr, true);
    mr_col_reduce(0, s, part + (size_t)2 * nblk * KS_MAX_NRHS, nblk, vx, true);
    for (int j = threadIdx.x; j < s; j += MR_NT) {
        ColState &c = cols[j];
        const double res = sqrt(v2[j]);
        c.rho = v2[j];
        c.res = res;
        c.resinf = vr[j];
        c.xinf = vx[j];
        int f = c.flags & ~(F_TRUE_OK | F_TRUE_NONFIN);
        if (!finite_d(res) || !finite_d(vx[j]))
            f |= F_TRUE_NONFIN;
        else if (res <= c.thresh)
            f |= F_TRUE_OK;
        c.flags = f;
    }
}

// (Re)start the columns in `mask`: p_j = r_j, inner flags cleared.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_begin_kernel(int n, int s, const T *__restrict__ R,
                                                         T *__restrict__ P, int ldv,
                                                         ColState *cols, State *st,
                                                         uint64_t mask) {
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    const int j1 = mr_j1(s);
    if (i < n)
        for (int j = mr_j0(); j < j1; ++j)
            if ((mask >> j) & 1ull) P[(size_t)j * ldv + i] = R[(size_t)j * ldv + i];
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        for (int j = 0; j < s; ++j)
            if ((mask >> j) & 1ull) cols[j].flags &= ~INNER_FLAGS;
        st->flags = mask ? 0 : F_STOP;
    }
}

// Q = sum_sp Qpart[sp]; sigma_j partials of p_j' q_j.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_sigma_kernel(int n, int s, const T *__restrict__ P,
                                                         const T *__restrict__ Qpart, int S,
                                                         int ldv, T *__restrict__ Q, double *part,
                                                         const State *st) {
    __shared__ double red[MR_NT / WAVE][KS_MAX_NRHS];
    if (st->flags & F_STOP) return;
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    const bool valid = i < n;
    const int sp16 = (s + 15) / 16 * 16;
    const int j0 = mr_j0(), j1 = mr_j1(s);
    for (int j = j0; j < j1; ++j) {
        double val = 0.0;
        if (valid) {
            T q = 0;
            for (int k = 0; k < S; ++k) q += Qpart[((size_t)k * sp16 + j) * ldv + i];
            Q[(size_t)j * ldv + i] = q;
            val = (double)P[(size_t)j * ldv + i] * (double)q;
        }
        mr_col_partial(val, j, red, false);
    }
    mr_col_flush(j0, j1, red, part, false);
}

// sigma_j from the partials, alpha_j = rho_j / sigma_j; x_j += alpha_j p_j,
// r_j -= alpha_j q_j for the active columns; r_j' r_j partials.  The blocks of
// row block 0 write their columns' state (rho_prev and sigma, which no block
// of this kernel reads, and stop flags only where every block finds the
// column stopped anyway).
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_update_kernel(int n, int s, T *__restrict__ X,
                                                          T *__restrict__ R,
                                                          const T *__restrict__ P,
                                                          const T *__restrict__ Q, int ldv,
                                                          ColState *cols, State *st,
                                                          const double *psig, int nblk,
                                                          double *prho) {
    __shared__ double red[MR_NT / WAVE][KS_MAX_NRHS];
    __shared__ double sig[KS_MAX_NRHS], alpha[KS_MAX_NRHS];
    __shared__ int act[KS_MAX_NRHS];
    if (st->flags & F_STOP) return;
    const int j0 = mr_j0(), j1 = mr_j1(s);
    mr_col_reduce(j0, j1, psig, nblk, sig, false);
    for (int j = j0 + threadIdx.x; j < j1; j += MR_NT) {
        const ColState &c = cols[j];
        const bool active = !(c.flags & F_STOP);
        const bool ok = finite_d(sig[j]) && sig[j] > 0.0;
        act[j] = active && ok;
        alpha[j] = ok ? c.rho / sig[j] : 0.0;
        if (blockIdx.x == 0 && active) {
            ColState &cw = cols[j];
            cw.iters += 1;
            cw.sigma = sig[j];
            cw.rho_prev = c.rho;
            if (!finite_d(sig[j]))
                cw.flags |= F_NONFIN | F_STOP;
            else if (sig[j] <= 0.0)
                cw.flags |= F_BREAK | F_STOP;
        }
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) st->iters += 1;
    __syncthreads();
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    const bool valid = i < n;
    for (int j = j0; j < j1; ++j) {
        double val = 0.0;
        if (valid && act[j]) {
            const T a = (T)alpha[j];
            const size_t o = (size_t)j * ldv + i;
            X[o] = fma(a, P[o], X[o]);
            const T r = fma(-a, Q[o], R[o]);
            R[o] = r;
            val = (double)r * (double)r;
        }
        mr_col_partial(val, j, red, false);
    }
    mr_col_flush(j0, j1, red, prho, false);
}

// rho'_j; per-column stop tests; beta_j and p_j = r_j + beta_j p_j.  Block
// (0, 0) also tests every other column, to set the solve's stop flag when no
// column is left; the blocks of row block 0 write their own columns' state.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_pupdate_kernel(int n, int s, const T *__restrict__ R,
                                                           T *__restrict__ P, int ldv,
                                                           ColState *cols, State *st,
                                                           const double *prho, int nblk,
                                                           int max_iter) {
    __shared__ double rn[KS_MAX_NRHS], beta[KS_MAX_NRHS];
    __shared__ int act[KS_MAX_NRHS];
    if (st->flags & F_STOP) return;
    const int j0 = mr_j0(), j1 = mr_j1(s);
    const bool lead = blockIdx.x == 0 && blockIdx.y == 0;
    const int c0 = lead ? 0 : j0, c1 = lead ? s : j1;
    mr_col_reduce(c0, c1, prho, nblk, rn, false);
    int mine = 0;
    for (int j = c0 + threadIdx.x; j < c1; j += MR_NT) {
        const ColState &c = cols[j];
        int stop = 0;
        const bool active = !(c.flags & F_STOP);
        if (active) {
            if (!finite_d(rn[j]))
                stop = F_NONFIN | F_STOP;
            else if (sqrt(rn[j]) <= c.thresh)
                stop = F_CONV | F_STOP;
            else if (c.iters >= max_iter)
                stop = F_MAXIT | F_STOP;
        }
        act[j] = active && !stop;
        beta[j] = rn[j] / c.rho_prev;
        mine |= act[j];
        if (blockIdx.x == 0 && active && j >= j0 && j < j1) {
            ColState &cw = cols[j];
            if (stop)
                cw.flags |= stop;
            else
                cw.rho = rn[j];
        }
    }
    const int any_active = __syncthreads_or(mine);
    if (lead && threadIdx.x == 0 && !any_active) st->flags |= F_STOP;
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    if (i < n)
        for (int j = j0; j < j1; ++j)
            if (act[j]) {
                const size_t o = (size_t)j * ldv + i;
                P[o] = fma((T)beta[j], P[o], R[o]);
            }
}

// copy n x s between leading dimensions (column-major)
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_copy_kernel(int n, int s, const T *__restrict__ src,
                                                        int lds, T *__restrict__ dst, int ldd) {
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    const int j1 = mr_j1(s);
    if (i < n)
        for (int j = mr_j0(); j < j1; ++j) dst[(size_t)j * ldd + i] = src[(size_t)j * lds + i];
}

// Refinement: inner right-hand sides r_j / ||r_j|| in binary32 (masked
// columns; others zero), and the binary64 update x_j += ||r_j|| d_j.
__global__ __launch_bounds__(MR_NT) void mr_ir_scale_kernel(int n, int s, const double *__restrict__ R,
                                                            int ldv, float *__restrict__ rhs,
                                                            const ColState *cols, uint64_t mask) {
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    if (i >= n) return;
    const int j1 = mr_j1(s);
    for (int j = mr_j0(); j < j1; ++j) {
        const size_t o = (size_t)j * ldv + i;
        rhs[o] = ((mask >> j) & 1ull) ? (float)(R[o] / cols[j].res) : 0.0f;
    }
}

__global__ __launch_bounds__(MR_NT) void mr_ir_update_kernel(int n, int s, double *__restrict__ X,
                                                             const float *__restrict__ D, int ldv,
                                                             const ColState *cols, uint64_t mask) {
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    if (i >= n) return;
    const int j1 = mr_j1(s);
    for (int j = mr_j0(); j < j1; ++j)
        if ((mask >> j) & 1ull) {
            const size_t o = (size_t)j * ldv + i;
            X[o] = fma(cols[j].res, (double)D[o], X[o]);
        }
}

// The contraction on its own (ks_gemm_mr): the caller's P (s columns,
// leading dimension ldv) copied to a zero-padded block of sp16 columns with
// leading dimension ldw, and Q summed from the K-split partials.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_stage_kernel(int n, int s, int sp16, const T *__restrict__ P,
                                                         int64_t ldv, T *__restrict__ Pw, int ldw) {
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    const int j = blockIdx.y;
    if (i < n && j < sp16) Pw[(size_t)j * ldw + i] = j < s ? P[(size_t)j * ldv + i] : T(0);
}

template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_qsum_kernel(int n, int s, int sp16, int S,
                                                        const T *__restrict__ Qpart, int ldw,
                                                        T *__restrict__ Q, int64_t ldv) {
    const int i = blockIdx.x * MR_NT + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= n || j >= s) return;
    T q = 0;
    for (int k = 0; k < S; ++k) q += Qpart[((size_t)k * sp16 + j) * ldw + i];
    Q[(size_t)j * ldv + i] = q;
}

// ------------------------------------------------------------- launchers
// row blocks x column groups of the per-column kernels
static dim3 mr_grid(int n, int s) { return dim3(div_up(n, MR_NT), div_up(s, MR_CG)); }

hipError_t launch_mr_ir_scale(int n, int s, const double *R, int ldv, float *rhs,
                              const ColState *cols, uint64_t mask, hipStream_t strm) {
    mr_ir_scale_kernel<<<mr_grid(n, s), MR_NT, 0, strm>>>(n, s, R, ldv, rhs, cols, mask);
    return hipGetLastError();
}

hipError_t launch_mr_ir_update(int n, int s, double *X, const float *D, int ldv,
                               const ColState *cols, uint64_t mask, hipStream_t strm) {
    mr_ir_update_kernel<<<mr_grid(n, s), MR_NT, 0, strm>>>(n, s, X, D, ldv, cols, mask);
    return hipGetLastError();
}

int mr_splits(int n, int elem_bytes) {
    // Work-groups per CU of the contraction: binary64 two (1024 blocks at
    // n = 16384 measured slower than 512), binary32 one, its loads in flight
    // coming from the queue of A steps instead; each split's slice of K is kept
    // at least 512 long.
    const int target = elem_bytes == 8 ? 512 : 256;
    const int brows = elem_bytes == 8 ? mr_block_rows<double>() : mr_block_rows<float>();
    const int nrb = (n + brows - 1) / brows;
    int S = 1;
    while (S < 8 && nrb * S * 2 <= target && n / (2 * S) >= 512) S *= 2;
    return S;
}

int mr_kchunk(int n, int S) { return (int)round_up(div_up(n, S), 16); }

int mr_blocks(int n) { return div_up(n, MR_NT); }

template <typename T>
hipError_t launch_mr_gemm(int n, int64_t lda, const T *A, const T *P, int ldp, T *Qpart, int ldq,
                          int s, const State *st, int gate, hipStream_t strm) {
    const int S = mr_splits(n, (int)sizeof(T)), kc = mr_kchunk(n, S);
    const int nrb = div_up(n, mr_block_rows<T>());
    const int grid = nrb * S;
    switch ((s + 15) / 16) {
        case 1:
            mr_gemm_kernel<T, 1><<<grid, mr_nthr<T>(), 0, strm>>>(n, lda, A, P, ldp, Qpart, ldq, S, kc, st, gate);
            break;
        case 2:
            mr_gemm_kernel<T, 2><<<grid, mr_nthr<T>(), 0, strm>>>(n, lda, A, P, ldp, Qpart, ldq, S, kc, st, gate);
            break;
        case 3:
            mr_gemm_kernel<T, 3><<<grid, mr_nthr<T>(), 0, strm>>>(n, lda, A, P, ldp, Qpart, ldq, S, kc, st, gate);
            break;
        case 4:
            mr_gemm_kernel<T, 4><<<grid, mr_nthr<T>(), 0, strm>>>(n, lda, A, P, ldp, Qpart, ldq, S, kc, st, gate);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mr_stats(int n, int s, const T *B, int ldb, double tol, ColState *cols,
                           State *st, hipStream_t strm) {
    mr_stats_kernel<T><<<s, MR_NT, 0, strm>>>(n, B, ldb, tol, cols, st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mr_residual(int n, int64_t lda, const T *A, int s, const T *B, int ldb,
                              const T *X, T *Qpart, T *R, int ldv, double *part, ColState *cols,
                              State *st, int gate, hipStream_t strm) {
    hipError_t e = launch_mr_gemm<T>(n, lda, A, X, ldv, Qpart, ldv, s, st, gate, strm);
    if (e != hipSuccess) return e;
    const int nb = mr_blocks(n);
    mr_resid_kernel<T><<<mr_grid(n, s), MR_NT, 0, strm>>>(n, s, B, ldb, X, Qpart, mr_splits(n, (int)sizeof(T)), ldv, R, part,
                                               st, gate);
    mr_resid_finish_kernel<<<1, MR_NT, 0, strm>>>(s, part, nb, cols, st, gate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mr_begin(int n, int s, const T *R, T *P, int ldv, ColState *cols, State *st,
                           uint64_t mask, hipStream_t strm) {
    mr_begin_kernel<T><<<mr_grid(n, s), MR_NT, 0, strm>>>(n, s, R, P, ldv, cols, st, mask);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mr_iteration(int n, int64_t lda, const T *A, int s, T *X, T *R, T *P, T *Q,
                               T *Qpart, int ldv, double *part_a, double *part_b, ColState *cols,
                               State *st, int max_iter, hipStream_t strm, hipEvent_t e0,
                               hipEvent_t e1) {
    hipError_t e;
    if (e0 && (e = hipEventRecord(e0, strm)) != hipSuccess) return e;
    if ((e = launch_mr_gemm<T>(n, lda, A, P, ldv, Qpart, ldv, s, st, 2, strm)) != hipSuccess) return e;
    if (e1 && (e = hipEventRecord(e1, strm)) != hipSuccess) return e;
    const int nb = mr_blocks(n), S = mr_splits(n, (int)sizeof(T));
    mr_sigma_kernel<T><<<mr_grid(n, s), MR_NT, 0, strm>>>(n, s, P, Qpart, S, ldv, Q, part_a, st);
    mr_update_kernel<T><<<mr_grid(n, s), MR_NT, 0, strm>>>(n, s, X, R, P, Q, ldv, cols, st, part_a, nb, part_b);
    mr_pupdate_kernel<T><<<mr_grid(n, s), MR_NT, 0, strm>>>(n, s, R, P, ldv, cols, st, part_b, nb, max_iter);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mr_copy(int n, int s, const T *src, int lds, T *dst, int ldd, hipStream_t strm) {
    mr_copy_kernel<T><<<mr_grid(n, s), MR_NT, 0, strm>>>(n, s, src, lds, dst, ldd);
    return hipGetLastError();
}

// ks_gemm_mr's workspace: the padded P block and the S partial products
size_t mr_product_ws_bytes(int n, int s, int elem_bytes) {
    const size_t ldw = round_up(n, 64), sp16 = round_up(s, 16);
    return (1 + (size_t)mr_splits(n, elem_bytes)) * sp16 * ldw * (size_t)elem_bytes;
}

template <typename T>
hipError_t launch_mr_product(int n, int64_t lda, const T *A, int s, const T *P, int64_t ldv, T *Q,
                             void *ws, hipStream_t strm) {
    const int ldw = (int)round_up(n, 64), sp16 = (int)round_up(s, 16);
    const int S = mr_splits(n, (int)sizeof(T));
    T *Pw = (T *)ws;
    T *Qpart = Pw + (size_t)sp16 * ldw;
    mr_stage_kernel<T><<<dim3(div_up(n, MR_NT), sp16), MR_NT, 0, strm>>>(n, s, sp16, P, ldv, Pw, ldw);
    hipError_t e = launch_mr_gemm<T>(n, lda, A, Pw, ldw, Qpart, ldw, s, nullptr, 0, strm);
    if (e != hipSuccess) return e;
    mr_qsum_kernel<T><<<dim3(div_up(n, MR_NT), s), MR_NT, 0, strm>>>(n, s, sp16, S, Qpart, ldw, Q, ldv);
    return hipGetLastError();
}

#define KS_INST_MR(T)                                                                           \
    template hipError_t launch_mr_gemm<T>(int, int64_t, const T *, const T *, int, T *, int, int, \
                                          const State *, int, hipStream_t);                      \
    template hipError_t launch_mr_stats<T>(int, int, const T *, int, double, ColState *, State *, \
                                           hipStream_t);                                         \
    template hipError_t launch_mr_residual<T>(int, int64_t, const T *, int, const T *, int,      \
                                              const T *, T *, T *, int, double *, ColState *,    \
                                              State *, int, hipStream_t);                        \
    template hipError_t launch_mr_begin<T>(int, int, const T *, T *, int, ColState *, State *,   \
                                           uint64_t, hipStream_t);                               \
    template hipError_t launch_mr_iteration<T>(int, int64_t, const T *, int, T *, T *, T *, T *,  \
                                               T *, int, double *, double *, ColState *, State *, \
                                               int, hipStream_t, hipEvent_t, hipEvent_t);        \
    template hipError_t launch_mr_copy<T>(int, int, const T *, int, T *, int, hipStream_t);      \
    template hipError_t launch_mr_product<T>(int, int64_t, const T *, int, const T *, int64_t, T *, \
                                             void *, hipStream_t);

KS_INST_MR(double)
KS_INST_MR(float)

}  // namespace ks
