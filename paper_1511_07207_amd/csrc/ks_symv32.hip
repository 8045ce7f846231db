// Symmetric product y = A x from the lower triangle of a binary32 A, with
// binary32 vectors and binary32 accumulation: the product of the binary32
// inner solves of iterative refinement (the Krylov section's CG counts one
// matrix-vector product per iteration as its Theta(n^2) part), at half the
// bytes of the general binary32 product, so a refined SPD solve reads a
// quarter of the bytes of a general binary64 one per inner iteration.
//
// The same tiling as the binary64 symmetric product: SY_T x SY_T tiles (I, J),
// I >= J, one block of SY_NT threads (8 wave64s) per tile, every element used
// twice (row part y_I += A_IJ x_J, column part y_J += A_IJ' x_I; on a diagonal
// tile the row part takes c <= r and the column part c < r), rows interleaved
// over the waves, the rows' sums formed eight at a time by the halving
// butterfly, the column parts summed over the waves through LDS, and each
// tile's two partial vectors written once at the block's end for a finishing
// kernel that adds them in a fixed order.  A tile row of binary32 is one
// 1 KiB wave load (16 bytes, four columns, per lane); the diagonal tiles read
// whole rows (their discarded upper quadrant is 64 of 2080 tiles' quarter at
// n = 16384).  CG's shares of p'Ap are formed in binary64.
#include "ks_device.h"

namespace ks {

typedef float s3_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t s3_u4 __attribute__((ext_vector_type(4)));

constexpr int S3_RSRC_WORD3 = 0x00020000;  // gfx9-family raw buffer resource, word 3
constexpr int S3_NT_POLICY = 2;             // loads of A: nt (streamed once)
constexpr int S3_STORE_POLICY = 16;         // workspace stores: sc1
constexpr int S3_WAVES = SY_NT / WAVE;
constexpr int S3_RPW = SY_T / S3_WAVES;     // rows per wave in a tile (32)
constexpr int S3_EPL = 4;                   // columns per lane
constexpr int S3_U = 8;                     // rows per group
constexpr int S3_FACC = 8;                  // loads in flight per wave of the finishing kernels
constexpr int S3_FWAVES = 16;               // waves per finishing block
static_assert(WAVE * S3_EPL == SY_T, "one wave load covers a tile row");
static_assert(S3_RPW % S3_U == 0, "groups tile the rows");
static_assert(SY_T % SY_FIN == 0, "a finishing block stays inside one tile column");

__device__ __forceinline__ int s3_row(int w, int k) { return w + S3_WAVES * k; }

// One group of S3_U rows already loaded: a[u] holds the lane's four columns of
// row s3_row(w, k0 + u), xr[u] x at that row.  Row sums into `rows` (LDS),
// column parts accumulated in ca.
template <bool DIAG>
__device__ __forceinline__ void s3_group(int lane, int w, int k0, const s3_f4 (&a)[S3_U],
                                         const float (&xr)[S3_U], const float (&xj)[S3_EPL],
                                         float *rows, float (&ca)[S3_EPL]) {
    float racc[S3_U];
#pragma unroll
    for (int u = 0; u < S3_U; ++u) {
        const int lr = s3_row(w, k0 + u);
        const float av[S3_EPL] = {a[u].x, a[u].y, a[u].z, a[u].w};
        float s = 0.0f;
#pragma unroll
        for (int e = 0; e < S3_EPL; ++e) {
            float ar = av[e], ac = av[e];
            if constexpr (DIAG) {
                const int c = S3_EPL * lane + e;
                ar = (c <= lr) ? ar : 0.0f;
                ac = (c < lr) ? ac : 0.0f;
            }
            s = fmaf(ar, xj[e], s);
            ca[e] = fmaf(ac, xr[u], ca[e]);
        }
        racc[u] = s;
    }
    const float v = rows_reduce<S3_U>(racc, lane);
    constexpr int LPR = WAVE / S3_U;
    if ((lane % LPR) == 0) rows[s3_row(w, k0 + lane / LPR)] = v;
}

// One block per tile, ordered as the binary64 product's blocks: the diagonal
// tiles, then (ragged n) the last tile row's other tiles, then the interior
// tiles in row order.  st != nullptr: return at once after the Krylov loop
// stopped.  sig != nullptr: the tile's share of x'A x (binary64) in sig[tile].
// b: the block's index in the launch (or a solve's local block index in the
// request server's batched launches).
__device__ __forceinline__ void symv32_tile_body(int n, int64_t lda, const float *__restrict__ A,
                                                 const float *__restrict__ x, float *__restrict__ W,
                                                 const State *st, double *__restrict__ sig, int b) {
    __shared__ float rows[SY_T];
    __shared__ float cs[S3_WAVES][SY_T];
    __shared__ double sg[S3_WAVES];
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
    const int t = I * (I + 1) / 2 + J;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int r0 = I * SY_T, c0 = J * SY_T;
    float xj[S3_EPL], ca[S3_EPL];
#pragma unroll
    for (int e = 0; e < S3_EPL; ++e) {
        const int c = c0 + S3_EPL * lane + e;
        xj[e] = c < n ? x[c] : 0.0f;
        ca[e] = 0.0f;
    }
    const bool diag = (I == J);
    if (r0 + SY_T <= n) {
        // rows and columns inside the matrix: buffer loads, row offset scalar
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(A + (int64_t)r0 * lda), 0, (int)((int64_t)SY_T * lda * 4), S3_RSRC_WORD3);
        const int coff = (c0 + S3_EPL * lane) * 4;
        const float *xi = x + r0;
#pragma unroll 1
        for (int k0 = 0; k0 < S3_RPW; k0 += S3_U) {
            s3_f4 a[S3_U];
            float xr[S3_U];
#pragma unroll
            for (int u = 0; u < S3_U; ++u) {
                const int lr = s3_row(w, k0 + u);
                const s3_u4 raw = __builtin_amdgcn_raw_buffer_load_b128(rsrc, coff, (int)((int64_t)lr * lda * 4),
                                                                        S3_NT_POLICY);
                a[u] = __builtin_bit_cast(s3_f4, raw);
            }
#pragma unroll
            for (int u = 0; u < S3_U; ++u) xr[u] = xi[s3_row(w, k0 + u)];
            if (diag)
                s3_group<true>(lane, w, k0, a, xr, xj, rows, ca);
            else
                s3_group<false>(lane, w, k0, a, xr, xj, rows, ca);
        }
    } else {
        // the last tile row when SY_T does not divide n: nothing at or past n is read
#pragma unroll 1
        for (int k0 = 0; k0 < S3_RPW; k0 += S3_U) {
            s3_f4 a[S3_U];
            float xr[S3_U];
#pragma unroll
            for (int u = 0; u < S3_U; ++u) {
                const int r = r0 + s3_row(w, k0 + u);
                const bool rin = r < n;
                const float *row = A + (int64_t)r * lda + c0 + S3_EPL * lane;
                const int c = c0 + S3_EPL * lane;
                a[u] = s3_f4{(rin && c < n) ? row[0] : 0.0f, (rin && c + 1 < n) ? row[1] : 0.0f,
                             (rin && c + 2 < n) ? row[2] : 0.0f, (rin && c + 3 < n) ? row[3] : 0.0f};
                xr[u] = rin ? x[r] : 0.0f;
            }
            if (diag)
                s3_group<true>(lane, w, k0, a, xr, xj, rows, ca);
            else
                s3_group<false>(lane, w, k0, a, xr, xj, rows, ca);
        }
    }
    // the tile's output: row parts (threads < SY_T) then column parts summed
    // over the waves, one contiguous 2 KiB store
    const int q = threadIdx.x & (SY_T - 1);
    const int xo_i = (threadIdx.x < SY_T ? r0 : c0) + q;
    const float xo = (sig && xo_i < n) ? x[xo_i] : 0.0f;
#pragma unroll
    for (int e = 0; e < S3_EPL; ++e) cs[w][S3_EPL * lane + e] = ca[e];
    __syncthreads();
    float out;
    if (threadIdx.x < SY_T) {
        out = rows[q];
    } else {
        out = 0.0f;
#pragma unroll
        for (int k = 0; k < S3_WAVES; ++k) out += cs[k][q];
    }
    static_assert(SY_NT == 2 * SY_T, "one value per thread");
    const __amdgpu_buffer_rsrc_t ws =
        __builtin_amdgcn_make_buffer_rsrc(W + (size_t)t * 2 * SY_T, 0, 2 * SY_T * 4, S3_RSRC_WORD3);
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, out), ws, threadIdx.x * 4, 0,
                                          S3_STORE_POLICY);
    if (sig) {
        const double tv = wave_sum(xo_i < n ? (double)out * (double)xo : 0.0);
        if (lane == 0) sg[w] = tv;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < S3_WAVES; ++k) v += sg[k];
            sig[t] = v;
        }
    }
}

__global__ __launch_bounds__(SY_NT) void symv32_tile_kernel(int n, int64_t lda, const float *__restrict__ A,
                                                            const float *__restrict__ x,
                                                            float *__restrict__ W, const State *st,
                                                            double *__restrict__ sig) {
    symv32_tile_body(n, lda, A, x, W, st, sig, blockIdx.x);
}

// y_j = (row parts of tile row J) + (column parts of tile column J) in a
// fixed order: wave w takes sources w, w + S3_FWAVES, ..., and the waves'
// sums are added in wave order.  Every wave calls it; afterwards lane l of
// wave 0 holds y at fb * SY_FIN + l (fb the finishing block).
__device__ __forceinline__ float s3_finish_sum(int n, const float *__restrict__ W,
                                               float (*red)[SY_FIN], int lane, int w, int fb) {
    const int j0 = fb * SY_FIN;
    const int J = j0 / SY_T;
    const int jj = j0 - J * SY_T + lane;
    const int nT = div_up(n, SY_T);
    const int nsrc = nT + 1;  // J + 1 row parts, nT - J column parts
    float acc[S3_FACC];
#pragma unroll
    for (int q = 0; q < S3_FACC; ++q) acc[q] = 0.0f;
    for (int s0 = w; s0 < nsrc; s0 += S3_FWAVES * S3_FACC) {
#pragma unroll
        for (int q = 0; q < S3_FACC; ++q) {
            const int src = s0 + q * S3_FWAVES;
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
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < S3_FACC; ++q) s += acc[q];
    red[w][lane] = s;
    __syncthreads();
    float v = 0.0f;
    if (w == 0) {
#pragma unroll
        for (int q = 0; q < S3_FWAVES; ++q) v += red[q][lane];
    }
    return v;
}

__global__ __launch_bounds__(S3_FWAVES * WAVE) void symv32_finish_kernel(int n, const float *__restrict__ W,
                                                                  float *__restrict__ y) {
    __shared__ float red[S3_FWAVES][SY_FIN];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const float v = s3_finish_sum(n, W, red, lane, w, blockIdx.x);
    const int j = blockIdx.x * SY_FIN + lane;
    if (w == 0 && j < n) y[j] = v;
}

// CG's finishing kernel (binary32 vectors): q_j summed as above (not stored),
// sigma = p'q as the binary64 sum of the tiles' shares (the same order in
// every block), then the update on the block's elements as the general CG
// update does in binary32: block 0 records the iteration (or the breakdown /
// non-finite sigma) in st; x_j += alpha p_j, r_j -= alpha q_j with alpha
// rounded to binary32; the block's r'r and ||x||_inf partials (binary64).
__device__ __forceinline__ void symv32_cg_finish_body(int n, const float *__restrict__ W,
                                                      const double *__restrict__ sig, int ntiles,
                                                      const float *__restrict__ p, float *__restrict__ x,
                                                      float *__restrict__ r, State *st,
                                                      double *__restrict__ prho, int nfb, int fb) {
    __shared__ float red[S3_FWAVES][SY_FIN];
    __shared__ double sm[S3_FWAVES];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    const int j = fb * SY_FIN + lane;
    const int jc = min(j, n - 1);
    float pj = 0.0f, xj = 0.0f, rj = 0.0f;
    if (w == 0) {
        pj = p[jc];
        xj = x[jc];
        rj = r[jc];
    }
    double sgv = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += S3_FWAVES * WAVE) sgv += sig[i];
    const double rho = st->rho;  // written by the launch before, read with the vectors
    // block 0 of this launch may set F_STOP (breakdown) while other blocks
    // start: one decision per block, so no wave leaves before a barrier
    if (__syncthreads_or((st->flags & F_STOP) != 0)) return;
    const float qj = s3_finish_sum(n, W, red, lane, w, fb);
    sgv = wave_sum(sgv);
    if (lane == 0) sm[w] = sgv;
    __syncthreads();
    double sigma = 0.0;
#pragma unroll
    for (int k = 0; k < S3_FWAVES; ++k) sigma += sm[k];
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
    const float a = (float)(rho / sigma);
    double s2 = 0.0, xm = 0.0;
    if (j < n) {
        const float xi = fmaf(a, pj, xj);
        x[j] = xi;
        const float ri = fmaf(-a, qj, rj);
        r[j] = ri;
        s2 = (double)ri * (double)ri;
        xm = finite_d((double)xi) ? fabs((double)xi) : INFINITY;
    }
    s2 = wave_sum(s2);
    xm = wave_max(xm);
    if (lane == 0) {
        prho[fb] = s2;
        prho[nfb + fb] = xm;
    }
}

__global__ __launch_bounds__(S3_FWAVES * WAVE) void symv32_cg_finish_kernel(
    int n, const float *__restrict__ W, const double *__restrict__ sig, int ntiles,
    const float *__restrict__ p, float *__restrict__ x, float *__restrict__ r, State *st,
    double *__restrict__ prho, int nfb) {
    symv32_cg_finish_body(n, W, sig, ntiles, p, x, r, st, prho, nfb, blockIdx.x);
}

// The request server's batched launches (binary32 inner CG solves).
__global__ __launch_bounds__(SY_NT) void b_symv32_tile_kernel(BatchSetT<BatchItemT<float, float>> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    symv32_tile_body(it.n, it.lda, it.A, it.p, reinterpret_cast<float *>(it.sy), it.st,
                     it.sy + sy_ws_doubles(it.n), l);
}

__global__ __launch_bounds__(S3_FWAVES * WAVE) void b_symv32_cg_finish_kernel(
    BatchSetT<BatchItemT<float, float>> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    symv32_cg_finish_body(it.n, reinterpret_cast<const float *>(it.sy), it.sy + sy_ws_doubles(it.n),
                          sy_tiles(it.n), it.p, it.x, it.resid, it.st, symv_cg_rho_part(it.n, it.sy), nb,
                          l);
}

hipError_t batch_symv32(int which, const BatchSetT<BatchItemT<float, float>> &bs, int blocks,
                        hipStream_t s) {
    if (bs.count <= 0 || blocks <= 0) return hipSuccess;
    if (which == 0)
        b_symv32_tile_kernel<<<blocks, SY_NT, 0, s>>>(bs);
    else
        b_symv32_cg_finish_kernel<<<blocks, S3_FWAVES * WAVE, 0, s>>>(bs);
    return hipGetLastError();
}

hipError_t launch_symv32(int n, int64_t lda, const float *A, const float *x, float *y, float *W,
                         hipStream_t s) {
    symv32_tile_kernel<<<sy_tiles(n), SY_NT, 0, s>>>(n, lda, A, x, W, nullptr, nullptr);
    symv32_finish_kernel<<<symv_finish_blocks(n), S3_FWAVES * WAVE, 0, s>>>(n, W, y);
    return hipGetLastError();
}

hipError_t launch_symv32_cg(int n, int64_t lda, const float *A, const float *p, float *x, float *r,
                            double *region, State *st, hipStream_t s) {
    float *W = reinterpret_cast<float *>(region);
    double *sig = region + sy_ws_doubles(n);
    const int nfb = symv_finish_blocks(n);
    symv32_tile_kernel<<<sy_tiles(n), SY_NT, 0, s>>>(n, lda, A, p, W, st, sig);
    symv32_cg_finish_kernel<<<nfb, S3_FWAVES * WAVE, 0, s>>>(n, W, sig, sy_tiles(n), p, x, r, st,
                                                            symv_cg_rho_part(n, region), nfb);
    return hipGetLastError();
}

}  // namespace ks
