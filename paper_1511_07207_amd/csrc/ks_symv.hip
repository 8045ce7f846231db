// Symmetric matrix-vector product y = A x that reads only the lower triangle
// of A (elements i >= j): half the bytes of the general product, which is the
// whole cost of a CG iteration on a dense SPD matrix (the Krylov section
// counts one matrix-vector product per CG iteration as its Theta(n^2) part).
//
// Tiling.  The lower triangle is cut into SY_T x SY_T tiles (I, J), I >= J
// (SY_T = 256); one block of SY_NT threads (8 wave64s) reads one tile once
// and uses every element twice:
//   row part     y_I += A_IJ x_J      (for the rows of tile row I)
//   column part  y_J += A_IJ' x_I     (for the columns of tile column J)
// On a diagonal tile the row part takes the elements with c <= r and the
// column part those with c < r, so each element of A is counted exactly as
// often as in the full product; the tile's elements above the diagonal are
// loaded with the rest of the tile (they are inside the matrix) and
// discarded by a select, so their values never reach the result; the
// diagonal tile's upper-right quadrant (rows < SY_T/2, columns >= SY_T/2) lies
// wholly above the diagonal and is not read.
//
// Tile paths.  Tiles whose rows and columns lie inside the matrix (all but
// the last tile row when SY_T does not divide n) read A through a buffer
// resource based at the tile row, so a row's address is a scalar offset and
// the lane's byte offset (the same for every row) is one vector register;
// only the ragged last tile row checks bounds.  The diagonal and edge tiles
// are the first blocks of the launch, so that they overlap with the interior
// tiles instead of forming a tail.
//
// Each wave reads SY_RPW rows of the tile, interleaved with the other waves;
// a tile row is two 1 KiB halves, one wave instruction each (64 lanes x 16
// bytes: lane l holds columns 2l, 2l + 1 of each half), nontemporal as in the
// general product.  The x values of
// a wave's rows are wave-uniform (scalar loads), so no barrier precedes the
// loads of A.  The column part accumulates per lane (its columns
// are fixed) and is summed over the SY_WAVES (8) waves through LDS.  The row part of each
// row is a sum over the 64 lanes; a wave takes its rows in groups of U and
// forms the U sums together by a butterfly that halves the number of values
// per lane at each exchange, then adds within the remaining lane groups.
//
// Every tile writes its two partial vectors (row part, column part; SY_T
// values each) to a workspace; a second kernel sums, for each element, the row
// parts of its tile row and the column parts of its tile column in a fixed
// order (deterministic, no atomics), and writes y.  In CG the tiles also leave
// their shares of p'Ap, and the second kernel applies the iteration's update
// instead of writing q, so an iteration is two launches and the p update.
// The workspace traffic is 2 x 2 x 8 bytes per SY_T elements of A read, i.e.
// 1.6% of the product's bytes at SY_T = 256, yet the workspace writes are what
// the tile size trades against: measured on MI355X at n = 16384, storing them
// cost ~15 us of a 173 us product with 128-wide tiles and ~11 us of the 168 us
// tile launch with 256-wide ones (156 us without the stores), whose finishing
// sum also reads half as much; a block of two adjacent 256-wide tiles stores
// a quarter less but ends the launch later (189 us).
#include "ks_device.h"

namespace ks {

typedef double sy_d2 __attribute__((ext_vector_type(2)));
typedef uint32_t sy_u4 __attribute__((ext_vector_type(4)));

// Word 3 of a gfx9-family buffer resource for raw (untyped) loads.
constexpr int SY_RSRC_WORD3 = 0x00020000;
// Cache policy of the loads of A: nt (streamed once).
constexpr int SY_NT_POLICY = 2;

constexpr int SY_WAVES = SY_NT / WAVE;
constexpr int SY_RPW = SY_T / SY_WAVES;  // rows per wave in a tile (32)
constexpr int SY_H = 2;                  // 1 KiB halves per tile row
constexpr int SY_HW = SY_T / SY_H;       // columns per half (128)
constexpr int SY_UNR_INT = 8;            // rows per group, interior tiles
constexpr int SY_UNR_SPC = 8;            // rows per group, diagonal / edge tiles
constexpr int SY_FACC = 8;               // loads in flight per wave of the finishing kernel
constexpr int SY_FWAVES = 16;            // waves per block of the finishing kernel
static_assert(SY_HW == 2 * WAVE, "one wave instruction covers one half of a tile row");
static_assert(SY_RPW % SY_UNR_INT == 0 && SY_RPW % SY_UNR_SPC == 0, "groups tile the rows");
static_assert(SY_T % SY_FIN == 0, "a finishing block stays inside one tile column");

// Rows of a tile are interleaved over the waves: wave w reads rows w, w + 8,
// w + 16, ... (local row lr = w + SY_WAVES * k), so the block as a whole reads
// consecutive rows at any moment (measured 5% faster than contiguous row
// blocks per wave for the same bytes).
__device__ __forceinline__ int sy_row(int w, int k) { return w + SY_WAVES * k; }

// Shared set-up of a tile block.  The lane's columns inside the tile:
// h * SY_HW + lc and h * SY_HW + lc + 1 for the halves h = 0, 1.
struct SyTile {
    int I, J, t, lane, w, r0, c0, lc;
    double xj[SY_H][2];
};

__device__ __forceinline__ SyTile sy_setup(int n, int I, int J, const double *__restrict__ x) {
    SyTile T;
    T.I = I;
    T.J = J;
    T.t = I * (I + 1) / 2 + J;
    T.lane = threadIdx.x & (WAVE - 1);
    T.w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    T.r0 = I * SY_T;
    T.c0 = J * SY_T;
    T.lc = 2 * T.lane;
#pragma unroll
    for (int h = 0; h < SY_H; ++h) {
        const int c = T.c0 + h * SY_HW + T.lc;
        T.xj[h][0] = c < n ? x[c] : 0.0;
        T.xj[h][1] = c + 1 < n ? x[c + 1] : 0.0;
    }
    return T;
}

// Process one group of U rows (k = k0 .. k0 + U - 1 of the wave) that are
// already loaded: row parts reduced over the lanes into `rows` (LDS), column
// parts accumulated.  xr[u]: x at the group's rows (wave-uniform values).
template <int U, bool DIAG>
__device__ __forceinline__ void sy_group(const SyTile &T, int k0, const sy_d2 (&a)[U][SY_H],
                                         const double (&xr)[U], double *rows,
                                         double (&ca)[SY_H][2]) {
    double racc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int lr = sy_row(T.w, k0 + u);
        double s = 0.0;
#pragma unroll
        for (int h = 0; h < SY_H; ++h) {
            double ar0 = a[u][h].x, ar1 = a[u][h].y, ac0 = ar0, ac1 = ar1;
            if constexpr (DIAG) {
                // row part: c <= r; column part: c < r
                const int c = h * SY_HW + T.lc;
                ar0 = (c <= lr) ? ar0 : 0.0;
                ar1 = (c + 1 <= lr) ? ar1 : 0.0;
                ac0 = (c < lr) ? ac0 : 0.0;
                ac1 = (c + 1 < lr) ? ac1 : 0.0;
            }
            s = fma(ar0, T.xj[h][0], s);
            s = fma(ar1, T.xj[h][1], s);
            ca[h][0] = fma(ac0, xr[u], ca[h][0]);
            ca[h][1] = fma(ac1, xr[u], ca[h][1]);
        }
        racc[u] = s;
    }
    const double v = rows_reduce<U>(racc, T.lane);
    constexpr int LPR = WAVE / U;  // lanes per row after the reduction
    if ((T.lane % LPR) == 0) rows[sy_row(T.w, k0 + T.lane / LPR)] = v;
}

// The tile's output, row parts then column parts (the latter summed over the
// waves), written by the whole block as one contiguous 4 KiB store at its end.
// Storing once per block instead of per row group, with device-scope cache
// policy (sc1), measured 7% faster for the whole kernel: the stores interleave
// less with the stream of loads.
constexpr int SY_STORE_POLICY = 16;  // sc1
//
// With sig != nullptr the block also leaves its share of x'A x (CG: sigma =
// p'Ap), the dot product of its two outputs with x_I and x_J, in sig[tile]:
// the 512 products summed over each wave, then the 8 wave sums in wave order.
__device__ __forceinline__ void sy_store(const SyTile &T, int n, const double (&ca)[SY_H][2],
                                         const double *rows, double (*cs)[SY_T],
                                         const double *__restrict__ x, double *__restrict__ W,
                                         double *__restrict__ sig) {
    __shared__ double sg[SY_WAVES];
    const int q = threadIdx.x & (SY_T - 1);
    // this thread's output is element q of the row part (threads < SY_T) or of
    // the column part; the x value it meets in x'A x
    const int xi = (threadIdx.x < SY_T ? T.r0 : T.c0) + q;
    const double xo = (sig && xi < n) ? x[xi] : 0.0;
#pragma unroll
    for (int h = 0; h < SY_H; ++h) {
        cs[T.w][h * SY_HW + T.lc] = ca[h][0];
        cs[T.w][h * SY_HW + T.lc + 1] = ca[h][1];
    }
    __syncthreads();
    double out;
    if (threadIdx.x < SY_T) {
        out = rows[q];
    } else {
        out = 0.0;
#pragma unroll
        for (int k = 0; k < SY_WAVES; ++k) out += cs[k][q];
    }
    static_assert(SY_NT == 2 * SY_T, "one value per thread");
    typedef uint32_t sy_u2 __attribute__((ext_vector_type(2)));
    const __amdgpu_buffer_rsrc_t ws = __builtin_amdgcn_make_buffer_rsrc(
        W + (size_t)T.t * 2 * SY_T, 0, 2 * SY_T * 8, SY_RSRC_WORD3);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(sy_u2, out), ws, threadIdx.x * 8, 0,
                                          SY_STORE_POLICY);
    if (sig) {
        const double t = wave_sum(xi < n ? out * xo : 0.0);
        if (T.lane == 0) sg[T.w] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < SY_WAVES; ++k) v += sg[k];
            sig[T.t] = v;
        }
    }
}

// Rows of one tile from a buffer resource based at the tile row (tiles whose
// rows and columns all lie inside the matrix): the row offset is a scalar,
// the lane's byte offset one vector register.  On a diagonal tile the second
// half of the rows above the middle is never read (it lies above the
// diagonal; its values stand as zero).
template <bool DIAG>
__device__ __forceinline__ void sy_tile_full(const SyTile &T, int64_t lda, const double *__restrict__ A,
                                             const double *__restrict__ x, double *rows,
                                             double (&ca)[SY_H][2]) {
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(A + (int64_t)T.r0 * lda), 0, (int)((int64_t)SY_T * lda * 8),
        SY_RSRC_WORD3);
    const int coff = (T.c0 + T.lc) * 8;
    const double *xi = x + T.r0;  // x_I: read at wave-uniform indices
#pragma unroll 1
    for (int k0 = 0; k0 < SY_RPW; k0 += SY_UNR_INT) {
        sy_d2 a[SY_UNR_INT][SY_H];
        double xr[SY_UNR_INT];
#pragma unroll
        for (int u = 0; u < SY_UNR_INT; ++u) {
            const int lr = sy_row(T.w, k0 + u);
#pragma unroll
            for (int h = 0; h < SY_H; ++h) {
                if (DIAG && h * SY_HW > lr) {
                    a[u][h] = sy_d2{0.0, 0.0};
                    continue;
                }
                const sy_u4 raw = __builtin_amdgcn_raw_buffer_load_b128(
                    rsrc, coff + h * SY_HW * 8, (int)((int64_t)lr * lda * 8), SY_NT_POLICY);
                a[u][h] = __builtin_bit_cast(sy_d2, raw);
            }
        }
#pragma unroll
        for (int u = 0; u < SY_UNR_INT; ++u) xr[u] = xi[sy_row(T.w, k0 + u)];
        sy_group<SY_UNR_INT, DIAG>(T, k0, a, xr, rows, ca);
    }
}

// The last tile row when SY_T does not divide n: rows and columns at or
// beyond n are not read.
__device__ __forceinline__ void sy_tile_edge(const SyTile &T, int n, int64_t lda,
                                             const double *__restrict__ A,
                                             const double *__restrict__ x, double *rows,
                                             double (&ca)[SY_H][2]) {
    const bool diag = (T.I == T.J);
#pragma unroll 1
    for (int k0 = 0; k0 < SY_RPW; k0 += SY_UNR_SPC) {
        sy_d2 a[SY_UNR_SPC][SY_H];
        double xr[SY_UNR_SPC];
#pragma unroll
        for (int u = 0; u < SY_UNR_SPC; ++u) {
            const int lr = sy_row(T.w, k0 + u);
            const int r = T.r0 + lr;
            const bool rin = r < n;
            const double *row = A + (int64_t)r * lda + T.c0 + T.lc;
#pragma unroll
            for (int h = 0; h < SY_H; ++h) {
                const int c = T.c0 + h * SY_HW + T.lc;
                // on the diagonal tile the upper-right quadrant is never read
                const bool hin = rin && !(diag && h * SY_HW > lr);
                a[u][h] = sy_d2{(hin && c < n) ? row[h * SY_HW] : 0.0,
                                (hin && c + 1 < n) ? row[h * SY_HW + 1] : 0.0};
            }
            xr[u] = rin ? x[r] : 0.0;
        }
        if (diag)
            sy_group<SY_UNR_SPC, true>(T, k0, a, xr, rows, ca);
        else
            sy_group<SY_UNR_SPC, false>(T, k0, a, xr, rows, ca);
    }
}

// One block per tile of the lower triangle.  Blocks are ordered so that the
// few special tiles start first and overlap with the bulk:
//   b < nT                       diagonal tile (b, b)
//   nT <= b < nT + ne            (ragged n only) tile (nT - 1, b - nT) of the last tile row
//   then the interior tiles (I, J), 1 <= I < n / SY_T, J < I, in row order.
// st != nullptr: return at once when the Krylov loop has stopped.
// sig != nullptr: each tile's share of x'A x into sig[tile] (see sy_store).
// b: the block's index in the launch (the request server's batched launches
// pass a solve's local block index).
__device__ __forceinline__ void symv_tile_body(int n, int64_t lda, const double *__restrict__ A,
                                               const double *__restrict__ x, double *__restrict__ W,
                                               const State *st, double *__restrict__ sig, int b) {
    __shared__ double rows[SY_T];
    __shared__ double cs[SY_WAVES][SY_T];
    if (st && (st->flags & F_STOP)) return;
    const int nT = div_up(n, SY_T), nTf = n / SY_T;
    const int ne = (nT > nTf) ? nT - 1 : 0;
    int I, J;
    if (b < nT) {
        I = b;
        J = b;
    } else if (b < nT + ne) {
        I = nT - 1;
        J = b - nT;
    } else {
        tri_ij(b - nT - ne, I, J);
        I += 1;
    }
    const SyTile T = sy_setup(n, I, J, x);
    double ca[SY_H][2] = {{0.0, 0.0}, {0.0, 0.0}};
    if (T.r0 + SY_T > n)
        sy_tile_edge(T, n, lda, A, x, rows, ca);
    else if (I == J)
        sy_tile_full<true>(T, lda, A, x, rows, ca);
    else
        sy_tile_full<false>(T, lda, A, x, rows, ca);
    sy_store(T, n, ca, rows, cs, x, W, sig);
}

__global__ __launch_bounds__(SY_NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void symv_tile_kernel(
    int n, int64_t lda, const double *__restrict__ A, const double *__restrict__ x,
    double *__restrict__ W, const State *st, double *__restrict__ sig) {
    symv_tile_body(n, lda, A, x, W, st, sig, blockIdx.x);
}

// y_j = (row parts of tile row J) + (column parts of tile column J), J = j / SY_T,
// summed in a fixed order: the SY_FWAVES waves take sources w, w + SY_FWAVES,
// ... and their sums are added in wave order.  Every wave calls it; afterwards
// lane l of wave 0 holds y at j0 + l (j0 = fb * SY_FIN, fb the finishing block).
__device__ __forceinline__ double sy_finish_sum(int n, const double *__restrict__ W,
                                                double (*red)[SY_FIN], int lane, int w, int fb) {
    const int j0 = fb * SY_FIN;
    const int J = j0 / SY_T;
    const int jj = j0 - J * SY_T + lane;
    const int nT = div_up(n, SY_T);
    const int nsrc = nT + 1;  // J + 1 row parts, nT - J column parts
    // SY_FACC independent sums keep that many loads in flight per wave; they
    // are added in a fixed order at the end
    double acc[SY_FACC];
#pragma unroll
    for (int q = 0; q < SY_FACC; ++q) acc[q] = 0.0;
    for (int s0 = w; s0 < nsrc; s0 += SY_FWAVES * SY_FACC) {
#pragma unroll
        for (int q = 0; q < SY_FACC; ++q) {
            const int src = s0 + q * SY_FWAVES;
            if (src < nsrc) {
                size_t off;
                if (src <= J) {
                    off = ((size_t)J * (J + 1) / 2 + src) * 2 * SY_T + jj;
                } else {
                    const int Ib = src - 1;  // tiles (Ib, J), Ib = J .. nT - 1
                    off = (((size_t)Ib * (Ib + 1) / 2 + J) * 2 + 1) * SY_T + jj;
                }
                acc[q] += W[off];
            }
        }
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < SY_FACC; ++q) s += acc[q];
    red[w][lane] = s;
    __syncthreads();
    double v = 0.0;
    if (w == 0) {
#pragma unroll
        for (int q = 0; q < SY_FWAVES; ++q) v += red[q][lane];
    }
    return v;
}

// y = A x finished from the tile outputs.  With p != nullptr the block also
// leaves sum_j p_j y_j in partial[block] (CG: sigma = p'q).
__global__ __launch_bounds__(SY_FWAVES * WAVE) void symv_finish_kernel(int n, const double *__restrict__ W,
                                                            double *__restrict__ y,
                                                            const double *__restrict__ p,
                                                            double *__restrict__ partial,
                                                            const State *st) {
    __shared__ double red[SY_FWAVES][SY_FIN];
    if (st && (st->flags & F_STOP)) return;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const double v = sy_finish_sum(n, W, red, lane, w, blockIdx.x);
    if (w == 0) {
        const int j = blockIdx.x * SY_FIN + lane;
        double contrib = 0.0;
        if (j < n) {
            y[j] = v;
            if (p) contrib = p[j] * v;
        }
        if (partial) {
            const double tsum = wave_sum(contrib);
            if (lane == 0) partial[blockIdx.x] = tsum;
        }
    }
}

// CG's finishing kernel with the symmetric product: q_j as above (not stored),
// sigma = p'q as the sum of the tiles' shares (every block adds them in the
// same order, so all blocks hold the same sigma bit for bit), then the
// iteration's update on the block's elements, as the general CG update does:
// block 0 records the iteration (or the breakdown / non-finite sigma) in st,
// x_j += alpha p_j, r_j -= alpha q_j, and the block's r'r and ||x||_inf
// partials (and ||r||_inf when stopping on the backward error).  The vectors and the shares are loaded before the tile outputs
// are summed, so their latency is hidden behind that reduction.
__device__ __forceinline__ void symv_cg_finish_body(int n, const double *__restrict__ W,
                                                    const double *__restrict__ sig, int ntiles,
                                                    const double *__restrict__ p, double *__restrict__ x,
                                                    double *__restrict__ r, State *st,
                                                    double *__restrict__ prho, int nfb, int fb) {
    __shared__ double red[SY_FWAVES][SY_FIN];
    __shared__ double sm[SY_FWAVES];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int j = fb * SY_FIN + lane;
    const int jc = min(j, n - 1);
    double pj = 0.0, xj = 0.0, rj = 0.0;
    if (w == 0) {
        pj = p[jc];
        xj = x[jc];
        rj = r[jc];
    }
    double sg = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += SY_FWAVES * WAVE) sg += sig[i];
    const double rho = st->rho;  // written by the launch before, read with the vectors
    const bool eta = st->eta_tol > 0.0;
    // block 0 of this very launch may set F_STOP (breakdown) while other blocks
    // start: the whole block takes one decision, so no wave leaves before a
    // barrier that the others reach (a launch that sees the new flag would
    // have found sigma unusable and skipped the update all the same)
    if (__syncthreads_or((st->flags & F_STOP) != 0)) return;
    const double qj = sy_finish_sum(n, W, red, lane, w, fb);
    sg = wave_sum(sg);
    if (lane == 0) sm[w] = sg;
    __syncthreads();
    double sigma = 0.0;
#pragma unroll
    for (int k = 0; k < SY_FWAVES; ++k) sigma += sm[k];
    const bool ok = finite_d(sigma) && sigma > 0.0;
    if (fb == 0 && threadIdx.x == 0) {
        st->iters += 1;
        st->sigma = sigma;
        st->rho_prev = rho;
        if (!finite_d(sigma))
            st->flags |= F_NONFIN | F_STOP;
        else if (sigma <= 0.0)
            st->flags |= F_BREAK | F_STOP;
        else
            st->alpha = rho / sigma;
    }
    if (!ok || w != 0) return;
    const double a = rho / sigma;
    double s2 = 0.0, xm = 0.0, rm = 0.0;
    if (j < n) {
        const double xi = fma(a, pj, xj);
        x[j] = xi;
        const double ri = fma(-a, qj, rj);
        r[j] = ri;
        s2 = ri * ri;
        xm = finite_d(xi) ? fabs(xi) : INFINITY;
        rm = finite_d(ri) ? fabs(ri) : INFINITY;
    }
    s2 = wave_sum(s2);
    xm = wave_max(xm);
    if (lane == 0) {
        prho[fb] = s2;
        prho[nfb + fb] = xm;
    }
    if (eta) {
        // ||r||_inf partials for stopping on the backward error
        rm = wave_max(rm);
        if (lane == 0) prho[2 * nfb + fb] = rm;
    }
}

__global__ __launch_bounds__(SY_FWAVES * WAVE) void symv_cg_finish_kernel(
    int n, const double *__restrict__ W, const double *__restrict__ sig, int ntiles,
    const double *__restrict__ p, double *__restrict__ x, double *__restrict__ r, State *st,
    double *__restrict__ prho, int nfb) {
    symv_cg_finish_body(n, W, sig, ntiles, p, x, r, st, prho, nfb, blockIdx.x);
}

int symv_finish_blocks(int n) { return div_up(n, SY_FIN); }

// The request server's batched launches: the same bodies with each solve's
// local block index.
__global__ __launch_bounds__(SY_NT) __attribute__((amdgpu_waves_per_eu(4, 4))) void b_symv_tile_kernel(
    BatchSetT<BatchItemT<double, double>> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    symv_tile_body(it.n, it.lda, it.A, it.p, it.sy, it.st, it.sy + sy_ws_doubles(it.n), l);
}

__global__ __launch_bounds__(SY_FWAVES * WAVE) void b_symv_cg_finish_kernel(
    BatchSetT<BatchItemT<double, double>> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    symv_cg_finish_body(it.n, it.sy, it.sy + sy_ws_doubles(it.n), sy_tiles(it.n), it.p, it.x, it.resid,
                        it.st, symv_cg_rho_part(it.n, it.sy), nb, l);
}

hipError_t batch_symv(int which, const BatchSetT<BatchItemT<double, double>> &bs, int blocks,
                      hipStream_t s) {
    if (bs.count <= 0 || blocks <= 0) return hipSuccess;
    if (which == 0)
        b_symv_tile_kernel<<<blocks, SY_NT, 0, s>>>(bs);
    else
        b_symv_cg_finish_kernel<<<blocks, SY_FWAVES * WAVE, 0, s>>>(bs);
    return hipGetLastError();
}

hipError_t launch_symv(int n, int64_t lda, const double *A, const double *x, double *y,
                       double *W, const State *st, const double *p, double *partial,
                       hipStream_t s) {
    symv_tile_kernel<<<sy_tiles(n), SY_NT, 0, s>>>(n, lda, A, x, W, st, nullptr);
    symv_finish_kernel<<<symv_finish_blocks(n), SY_FWAVES * WAVE, 0, s>>>(n, W, y, p, partial, st);
    return hipGetLastError();
}

hipError_t launch_symv_cg(int n, int64_t lda, const double *A, const double *p, double *x,
                          double *r, double *region, State *st, hipStream_t s) {
    double *W = region;
    double *sig = region + sy_ws_doubles(n);
    const int nfb = symv_finish_blocks(n);
    symv_tile_kernel<<<sy_tiles(n), SY_NT, 0, s>>>(n, lda, A, p, W, st, sig);
    symv_cg_finish_kernel<<<nfb, SY_FWAVES * WAVE, 0, s>>>(n, W, sig, sy_tiles(n), p, x, r, st,
                                                          symv_cg_rho_part(n, region), nfb);
    return hipGetLastError();
}

}  // namespace ks
