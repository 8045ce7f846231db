// Fused conjugate gradient for small n: one launch per iteration.
//
// At small n an iteration of the three-kernel CG (product, x/r update,
// p update) costs three dependent launches of a few microseconds each while
// moving little data.  Here each launch does a whole iteration: every block
// forms, redundantly, the O(n) vector quantities it needs -- alpha from the
// previous product's partials, r_{k+1}, rho', the stop test, beta and
// p_{k+1} -- writes its own slice of x, r and p, and computes its 8 rows of
// the next product q = A p with their p'q partials.  The vectors are tiny
// next to A at these sizes (4 n doubles read per block against 8 n per row).
//
// Bitwise the same as the three-kernel path: the product uses the same
// per-row column order and reduction tree (rows_dot), the p'q partials are
// formed per pair of rows exactly as the product kernel forms them, and the
// r'r sum is rebuilt from the same per-1024-element partials in the same
// order as the update kernels form and reduce them; every update is the
// same fma.  So ks_solve at small n and the server's batched kernels give
// identical results.
//
// Races: within a launch no block may read what another block writes.  The
// vectors r, p, q and the partials alternate between two copies (launch k
// reads copy k % 2 and writes the other), and so do the scalars rho, iters
// and flags (State::fz_*).  A launch after the stop copies its slot forward
// so that the last slot is always current.
#include "ks_gemv_body.h"

namespace ks {

constexpr int FZ_NT = 256;   // threads per block
constexpr int FZ_ROWS = 8;   // rows of the product per block (4 pairs)
constexpr int FZ_PAIRS = FZ_ROWS / GemvShape<double>::ROWS;
static_assert(GemvShape<double>::ROWS == 2, "the p'q partials are formed per pair of rows");
static_assert(FZ_NT == VEC_NT && FZ_NT == GEMV_NT, "same block shape as the three-kernel path");

// rows row0 .. row0 + FZ_ROWS - 1 of q = A v (v in LDS or global), written to
// q, and the p'q partial of each pair of rows into pg[row / 2]
__device__ __forceinline__ void fz_product(int n, int64_t lda, const double *__restrict__ A,
                                           const double *v, double *__restrict__ q,
                                           double *__restrict__ pg, int row0) {
    double acc[FZ_ROWS];
    rows_dot<double, FZ_ROWS, FZ_NT, 2>(A, lda, n, row0, v, acc);
    const double out = reduce_rows<double, FZ_ROWS, FZ_NT>(acc);
    // lanes 0 .. FZ_ROWS - 1 of wave 0 hold the rows
    if (threadIdx.x < WAVE) {
        const int lane = threadIdx.x;
        const int row = row0 + lane;
        double contrib = 0.0;
        if (lane < FZ_ROWS && row < n) {
            q[row] = out;
            contrib = v[row] * out;
        }
#pragma unroll
        for (int j = 0; j < FZ_PAIRS; ++j) {
            // the pair's two rows sit in lanes 2j, 2j + 1: summed as the
            // product kernel sums its pair (lanes 0 and 1) over the wave
            const bool mine = (lane >> 1) == j;
            const double t = wave_sum(mine ? contrib : 0.0);
            const int gb = row0 / 2 + j;
            if (lane == 0 && 2 * gb < n) pg[gb] = t;
        }
    }
}

__global__ __launch_bounds__(FZ_NT) void fz_start_kernel(int n, int64_t lda, const double *__restrict__ A,
                                                         const double *__restrict__ p0,
                                                         double *__restrict__ q0, State *st,
                                                         double *__restrict__ pg0) {
    if (st->flags & F_STOP) return;
    fz_product(n, lda, A, p0, q0, pg0, blockIdx.x * FZ_ROWS);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->fz_rho[0] = st->rho;
        st->fz_iters[0] = st->iters;
        st->fz_flags[0] = st->flags;
    }
}

__global__ __launch_bounds__(FZ_NT) void fz_step_kernel(int n, int64_t lda, const double *__restrict__ A,
                                                        double *__restrict__ x,
                                                        const double *__restrict__ rc,
                                                        double *__restrict__ rn,
                                                        const double *__restrict__ pc,
                                                        double *__restrict__ pn,
                                                        const double *__restrict__ qc,
                                                        double *__restrict__ qn, State *st,
                                                        const double *__restrict__ pgc,
                                                        double *__restrict__ pgn, int cur,
                                                        int max_iter) {
    __shared__ double pnew[FZ_MAX_N];
    __shared__ double vpart[FZ_MAX_N / (VEC_NT * VEC_EPT)];
    __shared__ double sm[FZ_NT / WAVE];
    const int nxt = 1 - cur;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const double rho = st->fz_rho[cur];
    const int iters = st->fz_iters[cur] + 1;
    const int flags = st->fz_flags[cur];
    if (flags & F_STOP) {
        if (lead) {
            st->fz_rho[nxt] = rho;
            st->fz_iters[nxt] = iters - 1;
            st->fz_flags[nxt] = flags;
        }
        return;
    }
    // sigma = p'q from the product's partials, as the update kernel reduces them
    const int ngemv = gemv_blocks<double>(n);
    const double sigma = reduce_partials_all<FZ_NT>(pgc, ngemv, 1);
    if (!(finite_d(sigma) && sigma > 0.0)) {
        if (lead) {
            st->fz_rho[nxt] = rho;
            st->fz_iters[nxt] = iters;
            st->fz_flags[nxt] = flags | F_STOP | (finite_d(sigma) ? F_BREAK : F_NONFIN);
        }
        return;
    }
    const double a = rho / sigma;
    const int row0 = blockIdx.x * FZ_ROWS;
    // x += alpha p and r -= alpha q for the block's own rows
    if (threadIdx.x < FZ_ROWS) {
        const int i = row0 + threadIdx.x;
        if (i < n) {
            x[i] = fma(a, pc[i], x[i]);
            rn[i] = fma(-a, qc[i], rc[i]);
        }
    }
    // rho' = r'r over the whole vector, as the update kernel's blocks form
    // their partials (element base + e * VEC_NT of thread t) and the p-update
    // kernel sums them
    const int nvb = vec_blocks(n);
    for (int vb = 0; vb < nvb; ++vb) {
        const int base = vb * VEC_NT * VEC_EPT + threadIdx.x;
        double s2 = 0.0;
#pragma unroll
        for (int e = 0; e < VEC_EPT; ++e) {
            const int i = base + e * VEC_NT;
            if (i < n) {
                const double ri = fma(-a, qc[i], rc[i]);
                s2 += ri * ri;
            }
        }
        const double t = block_sum<FZ_NT>(s2, sm);
        if (threadIdx.x == 0) vpart[vb] = t;
        __syncthreads();
    }
    const double rho_new = reduce_partials_all<FZ_NT>(vpart, nvb, 1);
    int stop = 0;
    if (!finite_d(rho_new))
        stop = F_NONFIN | F_STOP;
    else if (sqrt(rho_new) <= st->thresh)
        stop = F_CONV | F_STOP;
    else if (iters >= max_iter)
        stop = F_MAXIT | F_STOP;
    if (stop) {
        if (lead) {
            st->fz_rho[nxt] = rho;
            st->fz_iters[nxt] = iters;
            st->fz_flags[nxt] = flags | stop;
        }
        return;
    }
    const double beta = rho_new / rho;
    // p' = r' + beta p for the whole vector (the product needs all of it)
    for (int i = threadIdx.x; i < n; i += FZ_NT) {
        const double ri = fma(-a, qc[i], rc[i]);
        pnew[i] = fma(beta, pc[i], ri);
    }
    __syncthreads();
    if (threadIdx.x < FZ_ROWS) {
        const int i = row0 + threadIdx.x;
        if (i < n) pn[i] = pnew[i];
    }
    fz_product(n, lda, A, pnew, qn, pgn, row0);
    if (lead) {
        st->fz_rho[nxt] = rho_new;
        st->fz_iters[nxt] = iters;
        st->fz_flags[nxt] = flags;
    }
}

// The same iteration for n <= FZ_SMALL_N, written for latency: every global
// load a thread needs (its p'q partials, its elements of r, q and p, the
// block's own rows of x, p, q, r, and its columns of the block's 8 rows of A)
// is issued at entry, unconditionally at clamped indices, so one memory round
// trip precedes the arithmetic instead of four.  The arithmetic and its order
// are those of fz_step_kernel (and so of the three-kernel path): thread t owns
// vector elements t + 256 m, and of each row the columns 2t, 2t + 1,
// 2t + 512, 2t + 513 -- those rows_dot gives it, in the same order (at
// n <= 1024 there are at most two 512-column chunks, the last possibly
// ragged).
// block_sum's sum handed to every thread: the same wave sums added in the
// same order, each thread adding them itself after the one barrier instead
// of thread 0 adding them and broadcasting through a second barrier.
// smem: FZ_NT / 64 entries, not reused by a later sum of the same launch.
__device__ __forceinline__ double fz_sum_all(double v, double *smem) {
    constexpr int NW = FZ_NT / WAVE;
    v = wave_sum(v);
    if ((threadIdx.x & (WAVE - 1)) == 0) smem[threadIdx.x / WAVE] = v;
    __syncthreads();
    double s = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += smem[i];
    return s;
}

constexpr int FZ_SMALL_N = 1024;
constexpr int FZ_SM_ELEM = FZ_SMALL_N / FZ_NT;       // vector elements per thread (4)
constexpr int FZ_SM_CH = FZ_SMALL_N / (2 * FZ_NT);   // 512-column chunks (2)
static_assert(VEC_NT * VEC_EPT >= FZ_SMALL_N, "one r'r partial covers the whole vector");
static_assert(FZ_SMALL_N / GemvShape<double>::ROWS <= 2 * FZ_NT, "two p'q partials per thread");

// A rows of the block (rows row0 .. row0 + 7), the columns rows_dot gives
// thread t: 2t, 2t + 1, 2t + 512, 2t + 513, clamped into the matrix.
typedef double fz_rows_t[FZ_ROWS][FZ_SM_CH][2];

__device__ __forceinline__ void fz_load_rows(int n, int64_t lda, const double *__restrict__ A, int row0,
                                             fz_rows_t &av) {
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < FZ_ROWS; ++r) {
        const double *rowp = A + (int64_t)min(row0 + r, n - 1) * lda;
#pragma unroll
        for (int ch = 0; ch < FZ_SM_CH; ++ch)
#pragma unroll
            for (int e = 0; e < 2; ++e) av[r][ch][e] = rowp[min(2 * t + ch * 2 * FZ_NT + e, n - 1)];
    }
}

// Loads and stores of what other blocks read or wrote: plain (COH = false,
// across a launch boundary) or agent-scope relaxed atomics (COH = true: the
// persistent launch, whose barrier has no cache writeback or invalidate).
template <bool COH, typename T>
__device__ __forceinline__ T fz_ld(const T *p) {
    if constexpr (COH)
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}
template <bool COH, typename T>
__device__ __forceinline__ void fz_st(T *p, T v) {
    if constexpr (COH)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// One iteration k (slot cur = k % 2) of the small-n fused CG on the block's
// rows of A held in registers.  Returns true when the solve has stopped
// (in this iteration or before): the block then wrote slot 1 - cur and,
// from a live iteration, x and r of its rows, but no p, q or partials.
template <bool COH>
__device__ __forceinline__ bool fz_small_iteration(
    int n, const fz_rows_t &av, double *__restrict__ x, const double *__restrict__ rc,
    double *__restrict__ rn, const double *__restrict__ pc, double *__restrict__ pn,
    const double *__restrict__ qc, double *__restrict__ qn, State *st, const double *__restrict__ pgc,
    double *__restrict__ pgn, int cur, int max_iter, double *pnew, double *sm_sigma, double *sm_rho) {
    const int nxt = 1 - cur;
    const int t = threadIdx.x;
    const bool lead = blockIdx.x == 0 && t == 0;
    const int row0 = blockIdx.x * FZ_ROWS;
    const int ngemv = gemv_blocks<double>(n);
    // ---- all loads first
    const double pg0 = fz_ld<COH>(&pgc[min(t, ngemv - 1)]);
    const double pg1 = fz_ld<COH>(&pgc[min(t + FZ_NT, ngemv - 1)]);
    double qv[FZ_SM_ELEM], rv[FZ_SM_ELEM], pv[FZ_SM_ELEM];
#pragma unroll
    for (int m = 0; m < FZ_SM_ELEM; ++m) {
        const int i = min(t + m * FZ_NT, n - 1);
        qv[m] = fz_ld<COH>(&qc[i]);
        rv[m] = fz_ld<COH>(&rc[i]);
        pv[m] = fz_ld<COH>(&pc[i]);
    }
    const int io = min(row0 + (t & (FZ_ROWS - 1)), n - 1);  // own row of threads t < FZ_ROWS
    const double xo = fz_ld<COH>(&x[io]), po = fz_ld<COH>(&pc[io]), qo = fz_ld<COH>(&qc[io]),
                 ro = fz_ld<COH>(&rc[io]);
    // this iteration's slot was written by the iteration before (this one
    // writes the other), so it is read with the other loads, not after the barrier
    const double rho = fz_ld<COH>(&st->fz_rho[cur]);
    const int iters = fz_ld<COH>(&st->fz_iters[cur]) + 1;
    const int flags = fz_ld<COH>(&st->fz_flags[cur]);
    const double thresh = st->thresh;  // fixed for the solve, written before the launch
    // ---- sigma, summed as reduce_partials_all sums the partials
    double sg = 0.0;
    if (t < ngemv) sg += pg0;
    if (t + FZ_NT < ngemv) sg += pg1;
    const double sigma = fz_sum_all(sg, sm_sigma);
    // the stop test comes after the barrier so that no load above is deferred
    // behind it; an iteration after the stop only copies its slot forward
    if (flags & F_STOP) {
        if (lead) {
            fz_st<COH>(&st->fz_rho[nxt], rho);
            fz_st<COH>(&st->fz_iters[nxt], iters - 1);
            fz_st<COH>(&st->fz_flags[nxt], flags);
        }
        return true;
    }
    if (!(finite_d(sigma) && sigma > 0.0)) {
        if (lead) {
            fz_st<COH>(&st->fz_rho[nxt], rho);
            fz_st<COH>(&st->fz_iters[nxt], iters);
            fz_st<COH>(&st->fz_flags[nxt], flags | F_STOP | (finite_d(sigma) ? F_BREAK : F_NONFIN));
        }
        return true;
    }
    const double a = rho / sigma;
    // ---- r' and r'r (one update-kernel partial holds the whole vector, its
    // thread t summing elements t + 256 e in order of e)
    double rr[FZ_SM_ELEM];
    double s2 = 0.0;
#pragma unroll
    for (int m = 0; m < FZ_SM_ELEM; ++m) {
        rr[m] = fma(-a, qv[m], rv[m]);
        if (t + m * FZ_NT < n) s2 += rr[m] * rr[m];
    }
    if (t < FZ_ROWS && row0 + t < n) {
        fz_st<COH>(&x[io], fma(a, po, xo));
        fz_st<COH>(&rn[io], fma(-a, qo, ro));
    }
    // the unfused path sums this block sum as its single partial, which
    // returns it unchanged (r'r >= 0)
    const double rho_new = fz_sum_all(s2, sm_rho);
    int stop = 0;
    if (!finite_d(rho_new))
        stop = F_NONFIN | F_STOP;
    else if (sqrt(rho_new) <= thresh)
        stop = F_CONV | F_STOP;
    else if (iters >= max_iter)
        stop = F_MAXIT | F_STOP;
    if (stop) {
        if (lead) {
            fz_st<COH>(&st->fz_rho[nxt], rho);
            fz_st<COH>(&st->fz_iters[nxt], iters);
            fz_st<COH>(&st->fz_flags[nxt], flags | stop);
        }
        return true;
    }
    const double beta = rho_new / rho;
#pragma unroll
    for (int m = 0; m < FZ_SM_ELEM; ++m) {
        const int i = t + m * FZ_NT;
        if (i < n) pnew[i] = fma(beta, pv[m], rr[m]);
    }
    __syncthreads();
    if (t < FZ_ROWS && row0 + t < n) fz_st<COH>(&pn[io], pnew[io]);
    // ---- q' = A p' for the block's rows, each row's columns in rows_dot's order
    double acc[FZ_ROWS];
#pragma unroll
    for (int r = 0; r < FZ_ROWS; ++r) acc[r] = 0.0;
#pragma unroll
    for (int ch = 0; ch < FZ_SM_CH; ++ch)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = 2 * t + ch * 2 * FZ_NT + e;
            if (c < n) {
                const double ve = pnew[c];
#pragma unroll
                for (int r = 0; r < FZ_ROWS; ++r) acc[r] = fma(av[r][ch][e], ve, acc[r]);
            }
        }
    const double out = reduce_rows<double, FZ_ROWS, FZ_NT>(acc);
    if (t < WAVE) {
        const int row = row0 + t;
        double contrib = 0.0;
        if (t < FZ_ROWS && row < n) {
            fz_st<COH>(&qn[row], out);
            contrib = pnew[row] * out;
        }
#pragma unroll
        for (int j = 0; j < FZ_PAIRS; ++j) {
            const bool mine = (t >> 1) == j;
            const double ts = wave_sum(mine ? contrib : 0.0);
            const int gb = row0 / 2 + j;
            if (t == 0 && 2 * gb < n) fz_st<COH>(&pgn[gb], ts);
        }
    }
    if (lead) {
        fz_st<COH>(&st->fz_rho[nxt], rho_new);
        fz_st<COH>(&st->fz_iters[nxt], iters);
        fz_st<COH>(&st->fz_flags[nxt], flags);
    }
    return false;
}

__global__ __launch_bounds__(FZ_NT) void fz_step_small_kernel(
    int n, int64_t lda, const double *__restrict__ A, double *__restrict__ x,
    const double *__restrict__ rc, double *__restrict__ rn, const double *__restrict__ pc,
    double *__restrict__ pn, const double *__restrict__ qc, double *__restrict__ qn, State *st,
    const double *__restrict__ pgc, double *__restrict__ pgn, int cur, int max_iter) {
    __shared__ double pnew[FZ_SMALL_N];
    __shared__ double sm_sigma[FZ_NT / WAVE], sm_rho[FZ_NT / WAVE];
    fz_rows_t av;
    fz_load_rows(n, lda, A, blockIdx.x * FZ_ROWS, av);
    (void)fz_small_iteration<false>(n, av, x, rc, rn, pc, pn, qc, qn, st, pgc, pgn, cur, max_iter, pnew,
                             sm_sigma, sm_rho);
}

// ---------------------------------------------------------------------------
// Persistent form (n <= FZ_SMALL_N): one cooperative launch runs up to
// `nsteps` iterations, with the arithmetic of fz_small_iteration in the same
// order, so the iterates, the slots and the vectors are bit for bit those of
// the per-launch path after the same number of iterations.  The block's
// eight rows of A are read once per launch and stay in registers.
//
// Between iterations the blocks depend on each other only through q = A p
// (each block forms its 8 rows) and the p'q partials (its 4 pairs of rows):
// r, p, alpha, beta, rho and the stop decision every block forms itself from
// the same values in the same order, so after the first iteration (whose
// inputs earlier launches wrote) a block keeps its elements of r and p, and
// x at its rows, in registers.  q and the partials cross between blocks as
// tagged 64-bit words, the tag (the iteration) in the high half and one half
// of the double in the low half, stored and loaded with agent-scope relaxed
// atomics: a block loads every word it needs until each carries the
// iteration's tag, so one device-scope round trip both synchronizes the
// blocks and carries the data (a barrier followed by the loads would take
// two).  The words of odd and even iterations alternate: a block writes
// iteration k + 2's words only after reading every block's words of k + 1,
// which each block writes only after reading all of k's, so none is
// overwritten before it has been read; the launcher zeroes them, and tags
// start at 1, so a word of an earlier launch never matches.  The block's
// rows of x, r, p, q, its partials and block 0's slot are still written every
// iteration, for whatever reads them after the launch.  All blocks take the
// same stop decision in the same iteration, so none waits for a block that
// has left.  A wait past `spin_limit` polls records FZ_SYNC_TIMEOUT in
// st->sync_fail and the blocks leave (the host reports an error);
// co-residency of the grid is guaranteed by the cooperative launch.
constexpr int FZ_SYNC_TIMEOUT = 1;

__device__ __forceinline__ uint64_t fz_word(uint32_t tag, uint32_t half) {
    return ((uint64_t)tag << 32) | half;
}

// a double as its two tagged words (low half first)
__device__ __forceinline__ void fz_publish(uint64_t *dst, uint32_t tag, double v) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    coh_store(dst, fz_word(tag, (uint32_t)bits));
    coh_store(dst + 1, fz_word(tag, (uint32_t)(bits >> 32)));
}

__global__ __launch_bounds__(FZ_NT) void fz_persist_kernel(
    int n, int64_t lda, const double *__restrict__ A, double *__restrict__ x, double *r0, double *r1,
    double *p0, double *p1, double *q0, double *q1, State *st, double *pg0, double *pg1, int cur0,
    int nsteps, int max_iter, uint32_t *xwords, uint32_t spin_limit) {
    constexpr int E = FZ_SM_ELEM;
    __shared__ double pnew[FZ_SMALL_N];
    __shared__ double sm_sigma[FZ_NT / WAVE], sm_rho[FZ_NT / WAVE];
    __shared__ int sm_late[FZ_NT / WAVE];  // a wave's wait gave up (read after sigma's barrier)
    const int t = threadIdx.x;
    const bool lead = blockIdx.x == 0 && t == 0;
    const int row0 = blockIdx.x * FZ_ROWS;
    const int ngemv = gemv_blocks<double>(n);
    const int nd = n + ngemv;  // doubles exchanged per iteration: q, then the partials
    if ((t & (WAVE - 1)) == 0) sm_late[t / WAVE] = 0;
    uint64_t *xw = reinterpret_cast<uint64_t *>(xwords);
    fz_rows_t av;
    fz_load_rows(n, lda, A, row0, av);
    int cur = cur0;
    // the first iteration's inputs, written by earlier launches
    double rv[E], pv[E], qv[E], xv[E];
    double pga, pgb;
    {
        const double *rc = cur ? r1 : r0, *pc = cur ? p1 : p0, *qc = cur ? q1 : q0;
        const double *pgc = cur ? pg1 : pg0;
        pga = fz_ld<true>(&pgc[min(t, ngemv - 1)]);
        pgb = fz_ld<true>(&pgc[min(t + FZ_NT, ngemv - 1)]);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = min(t + m * FZ_NT, n - 1);
            rv[m] = fz_ld<true>(&rc[i]);
            pv[m] = fz_ld<true>(&pc[i]);
            qv[m] = fz_ld<true>(&qc[i]);
            xv[m] = fz_ld<true>(&x[i]);
        }
    }
    double rho = fz_ld<true>(&st->fz_rho[cur]);
    int iters = fz_ld<true>(&st->fz_iters[cur]);
    const int flags = fz_ld<true>(&st->fz_flags[cur]);
    const double thresh = st->thresh;
    bool stopped = false;
    for (int k = 0; k < nsteps; ++k) {
        const int nxt = 1 - cur;
        double *rn = nxt ? r1 : r0, *pn = nxt ? p1 : p0, *qn = nxt ? q1 : q0;
        double *pgn = nxt ? pg1 : pg0;
        if (k > 0) {
            // q and the partials of iteration k - 1: the thread's elements
            // t + 256 m of q and partials t, t + 256, until all carry tag k
            const uint64_t *src = xw + (size_t)(k & 1) * 2 * nd;
            const uint32_t tag = (uint32_t)k;
            constexpr int D = E + 2;
            const uint64_t *wp[D];
#pragma unroll
            for (int m = 0; m < E; ++m) wp[m] = t + m * FZ_NT < n ? src + 2 * (t + m * FZ_NT) : nullptr;
            wp[E] = t < ngemv ? src + 2 * (n + t) : nullptr;
            wp[E + 1] = t + FZ_NT < ngemv ? src + 2 * (n + t + FZ_NT) : nullptr;
            uint64_t wv[D][2];
#pragma unroll
            for (int d = 0; d < D; ++d)
#pragma unroll
                for (int h = 0; h < 2; ++h) wv[d][h] = wp[d] ? coh_load(wp[d] + h) : fz_word(tag, 0u);
            int late = 0;
            for (uint32_t polls = 0;; ++polls) {
                bool all = true;
#pragma unroll
                for (int d = 0; d < D; ++d)
#pragma unroll
                    for (int h = 0; h < 2; ++h) all = all && (uint32_t)(wv[d][h] >> 32) == tag;
                if (all) break;
                if (polls >= spin_limit) {
                    late = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int d = 0; d < D; ++d)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
                        if ((uint32_t)(wv[d][h] >> 32) != tag) wv[d][h] = coh_load(wp[d] + h);
            }
            // the wave's timeout flag, read by every thread after the barrier of
            // sigma's sum below (no barrier of its own)
            const int wlate = __any(late);
            if ((t & (WAVE - 1)) == 0) sm_late[t / WAVE] = wlate;
            double dv[D];
#pragma unroll
            for (int d = 0; d < D; ++d)
                dv[d] = __longlong_as_double((long long)(((wv[d][1] & 0xffffffffull) << 32) |
                                                         (wv[d][0] & 0xffffffffull)));
#pragma unroll
            for (int m = 0; m < E; ++m) qv[m] = dv[m];
            pga = dv[E];
            pgb = dv[E + 1];
        }
        const int it = iters + 1;
        // ---- sigma, summed as reduce_partials_all sums the partials
        double sg = 0.0;
        if (t < ngemv) sg += pga;
        if (t + FZ_NT < ngemv) sg += pgb;
        const double sigma = fz_sum_all(sg, sm_sigma);
        {
            int any_late = 0;
#pragma unroll
            for (int w2 = 0; w2 < FZ_NT / WAVE; ++w2) any_late |= sm_late[w2];
            if (any_late) {
                if (t == 0)
                    __hip_atomic_store(&st->sync_fail, FZ_SYNC_TIMEOUT, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        }
        if (flags & F_STOP) {
            if (lead) {
                fz_st<true>(&st->fz_rho[nxt], rho);
                fz_st<true>(&st->fz_iters[nxt], iters);
                fz_st<true>(&st->fz_flags[nxt], flags);
            }
            stopped = true;
            cur = nxt;
            break;
        }
        if (!(finite_d(sigma) && sigma > 0.0)) {
            if (lead) {
                fz_st<true>(&st->fz_rho[nxt], rho);
                fz_st<true>(&st->fz_iters[nxt], it);
                fz_st<true>(&st->fz_flags[nxt], flags | F_STOP | (finite_d(sigma) ? F_BREAK : F_NONFIN));
            }
            stopped = true;
            cur = nxt;
            break;
        }
        const double a = rho / sigma;
        // ---- r' and r'r; x and r' at the block's rows
        double rr[E];
        double s2 = 0.0;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = t + m * FZ_NT;
            rr[m] = fma(-a, qv[m], rv[m]);
            if (i < n) s2 += rr[m] * rr[m];
            if (i >= row0 && i < row0 + FZ_ROWS && i < n) {
                xv[m] = fma(a, pv[m], xv[m]);
                fz_st<true>(&x[i], xv[m]);
                fz_st<true>(&rn[i], rr[m]);
            }
        }
        const double rho_new = fz_sum_all(s2, sm_rho);
        int stop = 0;
        if (!finite_d(rho_new))
            stop = F_NONFIN | F_STOP;
        else if (sqrt(rho_new) <= thresh)
            stop = F_CONV | F_STOP;
        else if (it >= max_iter)
            stop = F_MAXIT | F_STOP;
        if (stop) {
            if (lead) {
                fz_st<true>(&st->fz_rho[nxt], rho);
                fz_st<true>(&st->fz_iters[nxt], it);
                fz_st<true>(&st->fz_flags[nxt], flags | stop);
            }
            stopped = true;
            cur = nxt;
            break;
        }
        const double beta = rho_new / rho;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = t + m * FZ_NT;
            pv[m] = fma(beta, pv[m], rr[m]);
            rv[m] = rr[m];
            if (i < n) pnew[i] = pv[m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = t + m * FZ_NT;
            if (i >= row0 && i < row0 + FZ_ROWS && i < n) fz_st<true>(&pn[i], pv[m]);
        }
        // ---- q' = A p' for the block's rows, each row's columns in rows_dot's order
        double acc[FZ_ROWS];
#pragma unroll
        for (int r = 0; r < FZ_ROWS; ++r) acc[r] = 0.0;
#pragma unroll
        for (int ch = 0; ch < FZ_SM_CH; ++ch)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int c = 2 * t + ch * 2 * FZ_NT + e;
                if (c < n) {
                    const double ve = pnew[c];
#pragma unroll
                    for (int r = 0; r < FZ_ROWS; ++r) acc[r] = fma(av[r][ch][e], ve, acc[r]);
                }
            }
        const double out = reduce_rows<double, FZ_ROWS, FZ_NT>(acc);
        uint64_t *dst = xw + (size_t)((k + 1) & 1) * 2 * nd;
        const uint32_t tag = (uint32_t)(k + 1);
        if (t < WAVE) {
            const int row = row0 + t;
            double contrib = 0.0;
            if (t < FZ_ROWS && row < n) {
                fz_st<true>(&qn[row], out);
                fz_publish(dst + 2 * row, tag, out);
                contrib = pnew[row] * out;
            }
#pragma unroll
            for (int j = 0; j < FZ_PAIRS; ++j) {
                const bool mine = (t >> 1) == j;
                const double ts = wave_sum(mine ? contrib : 0.0);
                const int gb = row0 / 2 + j;
                if (t == 0 && 2 * gb < n) {
                    fz_st<true>(&pgn[gb], ts);
                    fz_publish(dst + 2 * (n + gb), tag, ts);
                }
            }
        }
        if (lead) {
            fz_st<true>(&st->fz_rho[nxt], rho_new);
            fz_st<true>(&st->fz_iters[nxt], it);
            fz_st<true>(&st->fz_flags[nxt], flags);
        }
        rho = rho_new;
        iters = it;
        cur = nxt;
    }
    // the per-launch path would copy the final slot forward in the launches
    // after a stop: the host publishes slot (cur0 + nsteps) % 2, so both
    // slots hold the final values (block 0 wrote the one read here)
    if (stopped && lead) {
        st->fz_rho[1 - cur] = st->fz_rho[cur];
        st->fz_iters[1 - cur] = st->fz_iters[cur];
        st->fz_flags[1 - cur] = st->fz_flags[cur];
    }
}

__global__ void fz_bar_reset_kernel(uint32_t *bar, int count, State *st) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) bar[i] = 0u;
    if (threadIdx.x == 0) st->sync_fail = 0;
}

__global__ void fz_publish_kernel(State *st, int which) {
    if (threadIdx.x == 0) {
        st->rho = st->fz_rho[which];
        st->iters = st->fz_iters[which];
        st->flags = st->fz_flags[which];
    }
}

static inline int fz_blocks(int n) { return div_up(n, FZ_ROWS); }

hipError_t launch_fz_start(int n, int64_t lda, const double *A, const double *p0, double *q0,
                           State *st, double *pg0, hipStream_t s) {
    if (n > FZ_MAX_N) return hipErrorInvalidValue;
    fz_start_kernel<<<fz_blocks(n), FZ_NT, 0, s>>>(n, lda, A, p0, q0, st, pg0);
    return hipGetLastError();
}

hipError_t launch_fz_step(int n, int64_t lda, const double *A, double *x, double *const vec[6],
                          State *st, double *const pg[2], int cur, int max_iter, hipStream_t s) {
    if (n > FZ_MAX_N || (cur != 0 && cur != 1)) return hipErrorInvalidValue;
    const int nxt = 1 - cur;
    if (n <= FZ_SMALL_N)
        fz_step_small_kernel<<<fz_blocks(n), FZ_NT, 0, s>>>(n, lda, A, x, vec[cur], vec[nxt],
                                                            vec[2 + cur], vec[2 + nxt], vec[4 + cur],
                                                            vec[4 + nxt], st, pg[cur], pg[nxt], cur,
                                                            max_iter);
    else
        fz_step_kernel<<<fz_blocks(n), FZ_NT, 0, s>>>(n, lda, A, x, vec[cur], vec[nxt], vec[2 + cur],
                                                      vec[2 + nxt], vec[4 + cur], vec[4 + nxt], st,
                                                      pg[cur], pg[nxt], cur, max_iter);
    return hipGetLastError();
}

int fz_persist_max_n() { return FZ_SMALL_N; }

// the exchange words: two parities of 2 (n + ngemv) 64-bit words
size_t fz_bar_words(int n) { return (size_t)8 * (n + gemv_blocks<double>(n)); }

hipError_t launch_fz_persist(int n, int64_t lda, const double *A, double *x, double *const vec[6],
                             State *st, double *const pg[2], int cur, int nsteps, int max_iter,
                             uint32_t *bar, uint32_t spin_limit, hipStream_t s) {
    if (n > FZ_SMALL_N || (cur != 0 && cur != 1) || nsteps < 1) return hipErrorInvalidValue;
    const int G = fz_blocks(n);
    const int words = (int)fz_bar_words(n);
    if (words > FZ_BAR_MAX_WORDS) return hipErrorInvalidValue;
    fz_bar_reset_kernel<<<1, 256, 0, s>>>(bar, words, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double *r0 = vec[0], *r1 = vec[1], *p0 = vec[2], *p1 = vec[3], *q0 = vec[4], *q1 = vec[5];
    double *pg0 = pg[0], *pg1 = pg[1];
    void *args[] = {&n, &lda, &A, &x, &r0, &r1, &p0, &p1, &q0, &q1, &st, &pg0, &pg1, &cur, &nsteps,
                    &max_iter, &bar, &spin_limit};
    return hipLaunchCooperativeKernel((const void *)fz_persist_kernel, dim3(G), dim3(FZ_NT), args, 0, s);
}

hipError_t launch_fz_publish(State *st, int which, hipStream_t s) {
    fz_publish_kernel<<<1, 64, 0, s>>>(st, which);
    return hipGetLastError();
}

}  // namespace ks
