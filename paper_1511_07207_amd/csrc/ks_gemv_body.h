// Dense row-major matrix-vector product y = A v and its fused epilogues
// (device bodies; the single-solve kernels and the batched kernels of the
// server both call them with an explicit block index).
//
// The product is the one matrix-vector multiplication per Krylov iteration
// (CG) or per Arnoldi step (GMRES) that the paper's Krylov section counts as
// the Theta(n^2) part of each iteration.  It is bound by HBM bandwidth: every
// element of A is read once per call, so the design goal is to stream A at
// the chip's read ceiling.
//
// Layout: a block of GEMV_NT = 256 threads (4 wave64s) owns ROWS rows (2 for
// binary64 and binary32, 4 for bfloat16).  All of its threads walk the columns
// together in 16-byte chunks (2 binary64, 4 binary32 or 8 bfloat16 elements
// per lane), so each wave's load of one row is a contiguous 1 KiB transaction,
// and each chunk of v is loaded once per block and used for ROWS rows (v is
// held in registers: each element is used by one lane only, so staging it in
// LDS would add traffic without reuse).  UNR = 4 chunks per row are loaded
// before use to keep enough bytes in flight per CU.  A is read with
// nontemporal loads: it is streamed once per call, and keeping it out of the
// caches leaves them to v (measured: +12-14% bandwidth on MI355X).  Per-thread
// partial sums are reduced with DPP inside each wave and across the 4 waves
// through LDS.
#pragma once
#include "ks_device.h"

namespace ks {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

template <typename TA>
struct ATraits;
template <>
struct ATraits<double> {
    using V = d2v;
    using TV = double;
    static constexpr int EPL = 2;
};
template <>
struct ATraits<float> {
    using V = f4v;
    using TV = float;
    static constexpr int EPL = 4;
};
template <>
struct ATraits<bf16_t> {
    using V = u4v;
    using TV = float;
    static constexpr int EPL = 8;
};

// 16 bytes of a row of A, nontemporal (global_load_dwordx4 ... nt)
template <typename TA>
__device__ __forceinline__ typename ATraits<TA>::V load_a(const TA *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const typename ATraits<TA>::V *>(p));
}

__device__ __forceinline__ void unpack(const d2v &a, double (&o)[2]) {
    o[0] = a.x;
    o[1] = a.y;
}
__device__ __forceinline__ void unpack(const f4v &a, float (&o)[4]) {
    o[0] = a.x;
    o[1] = a.y;
    o[2] = a.z;
    o[3] = a.w;
}
__device__ __forceinline__ void unpack(const u4v &a, float (&o)[8]) {
    o[0] = bf16_lo(a.x);
    o[1] = bf16_hi(a.x);
    o[2] = bf16_lo(a.y);
    o[3] = bf16_hi(a.y);
    o[4] = bf16_lo(a.z);
    o[5] = bf16_hi(a.z);
    o[6] = bf16_lo(a.w);
    o[7] = bf16_hi(a.w);
}

__device__ __forceinline__ double scalar_a(const double *p) { return *p; }
__device__ __forceinline__ float scalar_a(const float *p) { return *p; }
__device__ __forceinline__ float scalar_a(const bf16_t *p) { return bf16_to_f32(p->bits); }

// v chunk of EPL elements starting at column c (16-byte aligned).
template <typename TV, int EPL>
__device__ __forceinline__ void load_v(const TV *__restrict__ v, int c, TV (&o)[EPL]) {
    if constexpr (sizeof(TV) == 8) {
        static_assert(EPL == 2, "");
        double2 t = *reinterpret_cast<const double2 *>(v + c);
        o[0] = t.x;
        o[1] = t.y;
    } else {
#pragma unroll
        for (int q = 0; q < EPL / 4; ++q) {
            float4 t = *reinterpret_cast<const float4 *>(v + c + 4 * q);
            o[4 * q + 0] = t.x;
            o[4 * q + 1] = t.y;
            o[4 * q + 2] = t.z;
            o[4 * q + 3] = t.w;
        }
    }
}

// Partial dot products of ROWS consecutive rows starting at row0 with v,
// accumulated per thread (acc), columns split over the block's NT threads.
// Rows at or beyond n are clamped to row n-1 (loads stay in bounds; callers
// discard those results).  ABS: accumulate |a| instead of a * v.
template <typename TA, int ROWS, int NT, int UNR, bool ABS = false>
__device__ __forceinline__ void rows_dot(const TA *__restrict__ A, int64_t lda, int n, int row0,
                                         const typename ATraits<TA>::TV *__restrict__ v,
                                         typename ATraits<TA>::TV (&acc)[ROWS]) {
    using AV = typename ATraits<TA>::V;
    using TV = typename ATraits<TA>::TV;
    constexpr int EPL = ATraits<TA>::EPL;
    constexpr int STEP = NT * EPL;
    const TA *rp[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int row = min(row0 + r, n - 1);
        rp[r] = A + (int64_t)row * lda;
        acc[r] = 0;
    }
    const int nfull = n / STEP;
    int c = threadIdx.x * EPL;
    int s = 0;
    for (; s + UNR <= nfull; s += UNR) {
        AV a[UNR][ROWS];
        TV vv[UNR][EPL];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            if constexpr (!ABS) load_v<TV, EPL>(v, c + u * STEP, vv[u]);
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
                a[u][r] = load_a<TA>(rp[r] + c + u * STEP);
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                TV ae[EPL];
                unpack(a[u][r], ae);
#pragma unroll
                for (int e = 0; e < EPL; ++e) {
                    if constexpr (ABS)
                        acc[r] += fabs(ae[e]);
                    else
                        acc[r] = fma(ae[e], vv[u][e], acc[r]);
                }
            }
        c += UNR * STEP;
    }
    for (; s < nfull; ++s) {
        TV vv[EPL];
        if constexpr (!ABS) load_v<TV, EPL>(v, c, vv);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            AV a = load_a<TA>(rp[r] + c);
            TV ae[EPL];
            unpack(a, ae);
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                if constexpr (ABS)
                    acc[r] += fabs(ae[e]);
                else
                    acc[r] = fma(ae[e], vv[e], acc[r]);
            }
        }
        c += STEP;
    }
    // ragged tail: the last n - nfull*STEP columns, element by element
    if (c < n) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            if (c + e < n) {
                TV ve = ABS ? TV(0) : v[c + e];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    TV ae = scalar_a(rp[r] + c + e);
                    if constexpr (ABS)
                        acc[r] += fabs(ae);
                    else
                        acc[r] = fma(ae, ve, acc[r]);
                }
            }
        }
    }
}

// Reduce acc[ROWS] over the block; thread r < ROWS returns row r's value.
template <typename TV, int ROWS, int NT>
__device__ __forceinline__ TV reduce_rows(TV (&acc)[ROWS]) {
    constexpr int NW = NT / WAVE;
    __shared__ TV red[NW][ROWS];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        TV t = wave_sum(acc[r]);
        if (lane == 0) red[w][r] = t;
    }
    __syncthreads();
    TV out = 0;
    if (threadIdx.x < ROWS) {
#pragma unroll
        for (int i = 0; i < NW; ++i) out += red[i][threadIdx.x];
    }
    return out;
}

// ------------------------------------------------------------ plain y = A v
template <typename TA>
__device__ __forceinline__ void gemv_plain_body(int n, int64_t lda, const TA *__restrict__ A,
                                                const typename ATraits<TA>::TV *__restrict__ v,
                                                typename ATraits<TA>::TV *__restrict__ y, int bid) {
    using TV = typename ATraits<TA>::TV;
    const int row0 = bid * GemvShape<TA>::ROWS;
    TV acc[GemvShape<TA>::ROWS];
    rows_dot<TA, GemvShape<TA>::ROWS, GEMV_NT, GemvShape<TA>::UNR>(A, lda, n, row0, v, acc);
    TV out = reduce_rows<TV, GemvShape<TA>::ROWS, GEMV_NT>(acc);
    const int row = row0 + threadIdx.x;
    if (threadIdx.x < GemvShape<TA>::ROWS && row < n) y[row] = out;
}

// -------------------------------------------------- CG: q = A p, p'q partial
template <typename TA>
__device__ __forceinline__ void cg_matvec_body(int n, int64_t lda, const TA *__restrict__ A,
                                               const typename ATraits<TA>::TV *__restrict__ p,
                                               typename ATraits<TA>::TV *__restrict__ q,
                                               const State *st, double *partial, int bid) {
    using TV = typename ATraits<TA>::TV;
    if (st->flags & F_STOP) return;
    const int row0 = bid * GemvShape<TA>::ROWS;
    TV acc[GemvShape<TA>::ROWS];
    rows_dot<TA, GemvShape<TA>::ROWS, GEMV_NT, GemvShape<TA>::UNR>(A, lda, n, row0, p, acc);
    TV out = reduce_rows<TV, GemvShape<TA>::ROWS, GEMV_NT>(acc);
    const int row = row0 + threadIdx.x;
    double contrib = 0.0;
    if (threadIdx.x < GemvShape<TA>::ROWS && row < n) {
        q[row] = out;
        contrib = (double)p[row] * (double)out;
    }
    // the rows' values live in lanes 0..ROWS-1 of wave 0
    if (threadIdx.x < WAVE) {
        double t = wave_sum(contrib);
        if (threadIdx.x == 0) partial[bid] = t;
    }
}

// ---------------------------------------------- GMRES: w = A v_k, w'w partial
template <typename TA>
__device__ __forceinline__ void gm_matvec_body(int n, int64_t lda, const TA *__restrict__ A,
                                               const typename ATraits<TA>::TV *__restrict__ vk,
                                               typename ATraits<TA>::TV *__restrict__ w,
                                               const State *st, double *partial, int bid) {
    using TV = typename ATraits<TA>::TV;
    if (st->flags & F_STOP) return;
    const int row0 = bid * GemvShape<TA>::ROWS;
    TV acc[GemvShape<TA>::ROWS];
    rows_dot<TA, GemvShape<TA>::ROWS, GEMV_NT, GemvShape<TA>::UNR>(A, lda, n, row0, vk, acc);
    TV out = reduce_rows<TV, GemvShape<TA>::ROWS, GEMV_NT>(acc);
    const int row = row0 + threadIdx.x;
    double contrib = 0.0;
    if (threadIdx.x < GemvShape<TA>::ROWS && row < n) {
        w[row] = out;
        contrib = (double)out * (double)out;
    }
    if (threadIdx.x < WAVE) {
        double t = wave_sum(contrib);
        if (threadIdx.x == 0) partial[bid] = t;
    }
}

// ------------------------------------- BiCGSTAB: v = A p, r0'v partial
template <typename TA>
__device__ __forceinline__ void bs_vmatvec_body(int n, int64_t lda, const TA *__restrict__ A,
                                                const typename ATraits<TA>::TV *__restrict__ p,
                                                const typename ATraits<TA>::TV *__restrict__ r0,
                                                typename ATraits<TA>::TV *__restrict__ v,
                                                const State *st, double *partial, int bid) {
    using TV = typename ATraits<TA>::TV;
    if (st->flags & F_STOP) return;
    const int row0 = bid * GemvShape<TA>::ROWS;
    TV acc[GemvShape<TA>::ROWS];
    rows_dot<TA, GemvShape<TA>::ROWS, GEMV_NT, GemvShape<TA>::UNR>(A, lda, n, row0, p, acc);
    TV out = reduce_rows<TV, GemvShape<TA>::ROWS, GEMV_NT>(acc);
    const int row = row0 + threadIdx.x;
    double contrib = 0.0;
    if (threadIdx.x < GemvShape<TA>::ROWS && row < n) {
        v[row] = out;
        contrib = (double)r0[row] * (double)out;
    }
    if (threadIdx.x < WAVE) {
        double t = wave_sum(contrib);
        if (threadIdx.x == 0) partial[bid] = t;
    }
}

// ------------------------------ BiCGSTAB: t = A s, t's and t't partials
// Every block first reduces ||s||^2 from the previous kernel's partials and
// takes the same decision: if ||s|| already meets the threshold (or the
// product budget is spent) the iteration ends on the half step, the product
// is skipped and block 0 marks F_HALF (with F_CONV or F_MAXIT) for the next
// kernels.  No block tests F_HALF here, so the mark cannot race.
template <typename TA>
__device__ __forceinline__ void bs_tmatvec_body(int n, int64_t lda, const TA *__restrict__ A,
                                                const typename ATraits<TA>::TV *__restrict__ s,
                                                typename ATraits<TA>::TV *__restrict__ t,
                                                State *st, const double *__restrict__ pss, int nss,
                                                int max_iter, double *partial, int bid) {
    using TV = typename ATraits<TA>::TV;
    if (st->flags & F_STOP) return;
    const double ss = reduce_partials_all<GEMV_NT>(pss, nss, 1);
    const bool conv = sqrt(ss) <= stop_threshold(st, st->xinf_it);
    if (conv || st->iters >= max_iter) {
        if (bid == 0 && threadIdx.x == 0) st->flags |= F_HALF | (conv ? F_CONV : F_MAXIT);
        return;
    }
    const int row0 = bid * GemvShape<TA>::ROWS;
    TV acc[GemvShape<TA>::ROWS];
    rows_dot<TA, GemvShape<TA>::ROWS, GEMV_NT, GemvShape<TA>::UNR>(A, lda, n, row0, s, acc);
    TV out = reduce_rows<TV, GemvShape<TA>::ROWS, GEMV_NT>(acc);
    const int row = row0 + threadIdx.x;
    double ts = 0.0, tt = 0.0;
    if (threadIdx.x < GemvShape<TA>::ROWS && row < n) {
        t[row] = out;
        ts = (double)out * (double)s[row];
        tt = (double)out * (double)out;
    }
    if (threadIdx.x < WAVE) {
        double a = wave_sum(ts);
        double b = wave_sum(tt);
        if (threadIdx.x == 0) {
            partial[2 * bid] = a;
            partial[2 * bid + 1] = b;
        }
    }
}

// --------------------------------------------- true residual r = b - A x
// gate 1: run only when the inner loop has stopped (F_STOP set).
template <typename TA>
__device__ __forceinline__ void residual_body(int n, int64_t lda, const TA *__restrict__ A,
                                              const typename ATraits<TA>::TV *__restrict__ b,
                                              const typename ATraits<TA>::TV *__restrict__ x,
                                              typename ATraits<TA>::TV *__restrict__ r,
                                              const State *st, double *partial, int gate, int bid) {
    using TV = typename ATraits<TA>::TV;
    // gate 0: always; 1: only once the loop has stopped; 2: only while it runs
    if (gate == 1 && !(st->flags & F_STOP)) return;
    if (gate == 2 && (st->flags & F_STOP)) return;
    const int row0 = bid * GemvShape<TA>::ROWS;
    TV acc[GemvShape<TA>::ROWS];
    rows_dot<TA, GemvShape<TA>::ROWS, GEMV_NT, GemvShape<TA>::UNR>(A, lda, n, row0, x, acc);
    TV out = reduce_rows<TV, GemvShape<TA>::ROWS, GEMV_NT>(acc);
    const int row = row0 + threadIdx.x;
    double s2 = 0.0, rmax = 0.0, xmax = 0.0;
    if (threadIdx.x < GemvShape<TA>::ROWS && row < n) {
        TV ri = b[row] - out;
        r[row] = ri;
        s2 = (double)ri * (double)ri;
        rmax = fabs((double)ri);
        xmax = fabs((double)x[row]);
        // a NaN must survive the max reductions below
        if (!finite_d(rmax)) rmax = INFINITY;
        if (!finite_d(xmax)) xmax = INFINITY;
    }
    if (threadIdx.x < WAVE) {
        double t0 = wave_sum(s2);
        double t1 = wave_max(rmax);
        double t2 = wave_max(xmax);
        if (threadIdx.x == 0) {
            partial[3 * bid + 0] = t0;
            partial[3 * bid + 1] = t1;
            partial[3 * bid + 2] = t2;
        }
    }
}

// One block: reduce the residual partials into the State.
__device__ __forceinline__ void residual_finish_body(int nblocks, State *st, const double *partial,
                                                     int gate) {
    if (gate == 1 && !(st->flags & F_STOP)) return;
    const double rho = reduce_partials_all<ONE_NT>(partial, nblocks, 3);
    const double rinf = reduce_partials_max_all<ONE_NT>(partial + 1, nblocks, 3);
    const double xinf = reduce_partials_max_all<ONE_NT>(partial + 2, nblocks, 3);
    if (threadIdx.x == 0) {
        const double res = sqrt(rho);
        st->rho = rho;
        st->res = res;
        st->resinf = rinf;
        st->xinf = xinf;
        int f = st->flags & ~(F_TRUE_OK | F_TRUE_NONFIN);
        const bool ok = st->eta_tol > 0.0
                            ? rinf <= st->eta_tol * (st->anorm_inf * xinf + st->binf)
                            : res <= st->thresh;
        if (!finite_d(res) || !finite_d(xinf))
            f |= F_TRUE_NONFIN;
        else if (ok)
            f |= F_TRUE_OK;
        st->flags = f;
    }
}

// -------------------------------------------------------------- ||A||_inf
__device__ __forceinline__ void norm_inf_body(int n, int64_t lda, const double *__restrict__ A,
                                              double *partial, int bid) {
    constexpr int R = GemvShape<double>::ROWS;
    const int row0 = bid * R;
    double acc[R];
    rows_dot<double, R, GEMV_NT, GemvShape<double>::UNR, true>(A, lda, n, row0, nullptr, acc);
    double out = reduce_rows<double, R, GEMV_NT>(acc);
    const int row = row0 + threadIdx.x;
    double m = 0.0;
    if (threadIdx.x < R && row < n) m = finite_d(out) ? out : INFINITY;
    if (threadIdx.x < WAVE) {
        double t = wave_max(m);
        if (threadIdx.x == 0) partial[bid] = t;
    }
}

__device__ __forceinline__ void norm_inf_finish_body(int nblocks, State *st, const double *partial) {
    const double mx = reduce_partials_max_all<ONE_NT>(partial, nblocks, 1);
    if (threadIdx.x == 0) st->anorm_inf = mx;
}


}  // namespace ks
