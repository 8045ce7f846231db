// Device helpers shared by the kernels: wave64 DPP reductions, block
// reductions, deterministic cross-block reductions and bfloat16 conversion.
// gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ks_internal.h"

namespace ks {

// ------------------------------------------------------------ grid barrier
// A barrier across the blocks of a cooperative launch without cache
// maintenance.  An agent-scope release or acquire fence on gfx950 writes back
// or invalidates the XCD's L2 (buffer_wbl2 / buffer_inv) and costs about
// 0.13 us per block per barrier; instead, whatever a block writes for another
// block before the barrier is stored with agent-scope relaxed atomics
// (coherent at device scope) and read back the same way after it.  Block b
// waits for its own stores to complete (vmcnt(0)), meets its threads at a
// block barrier and publishes `done` in bar[b * BAR_STRIDE]; thread t <
// gridDim.x then polls bar[t] until it reaches `done`.  So no block passes
// before every block's coherent writes made before the barrier are visible
// to it.  `done` must grow from one barrier to the next (the words start at
// zero).  Every wait is bounded: false when some poll gave up after
// `spin_limit` tries (the same answer in every thread of the block).
constexpr int WAIT_VMEM = 0x0F70;  // s_waitcnt vmcnt(0) (gfx9 encoding: expcnt, lgkmcnt not waited)

__device__ __forceinline__ bool grid_barrier(uint32_t *bar, uint32_t done, uint32_t spin_limit) {
    __builtin_amdgcn_s_waitcnt(WAIT_VMEM);
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&bar[blockIdx.x * FZ_BAR_STRIDE], done, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    int late = 0;
    if (threadIdx.x < gridDim.x) {
        uint32_t polls = 0;
        while (__hip_atomic_load(&bar[threadIdx.x * FZ_BAR_STRIDE], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) < done) {
            if (++polls > spin_limit) {
                late = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    late = __syncthreads_or(late);
    return late == 0;
}

// coherent (agent-scope relaxed) loads and stores of what crosses a grid barrier
template <typename T>
__device__ __forceinline__ T coh_load(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void coh_store(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- DPP moves
// dpp_ctrl encodings (GFX9 DPP): quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E,
// row_ror:4 = 0x124, row_ror:8 = 0x128.  Every source lane is valid for these
// patterns, so bound_ctrl does not matter.
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
    uint64_t u = __builtin_bit_cast(uint64_t, x);
    int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes of a wave.  The result is exact-order deterministic
// and is read from lane 0 (other lanes may differ in the last bit).
template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
    x += dpp<0xB1>(x);
    x += dpp<0x4E>(x);
    x += dpp<0x124>(x);
    x += dpp<0x128>(x);
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
    x = fmax(x, dpp<0xB1>(x));
    x = fmax(x, dpp<0x4E>(x));
    x = fmax(x, dpp<0x124>(x));
    x = fmax(x, dpp<0x128>(x));
    x = fmax(x, __shfl_xor(x, 16));
    x = fmax(x, __shfl_xor(x, 32));
    return x;
}

// One step of the row butterfly: the lanes whose `mask` bit is 0 keep the
// first half of their K values, the others the second half, each adding the
// partner's copy of the half it keeps.
template <int K, int U, typename V>
__device__ __forceinline__ void rows_fold(V (&v)[U], int lane, int mask) {
    const bool hi = (lane & mask) != 0;
#pragma unroll
    for (int i = 0; i < K / 2; ++i) {
        const V keep = hi ? v[i + K / 2] : v[i];
        const V send = hi ? v[i] : v[i + K / 2];
        v[i] = keep + __shfl_xor(send, mask);
    }
}

// U row sums over the 64 lanes (U = 4, 8 or 16).  Afterwards every lane of
// the lane group g = lane / (64 / U) holds the sum of row g: the halving
// exchanges over lane bits 5, 4, ... leave row g in the lanes whose high bits
// spell g, and the remaining low bits are summed by plain exchanges.
template <int U, typename V>
__device__ __forceinline__ V rows_reduce(V (&v)[U], int lane) {
    static_assert(U == 4 || U == 8 || U == 16, "row group of 4, 8 or 16");
    rows_fold<U, U>(v, lane, 32);
    if constexpr (U >= 4) rows_fold<U / 2, U>(v, lane, 16);
    if constexpr (U >= 8) rows_fold<U / 4, U>(v, lane, 8);
    if constexpr (U >= 16) rows_fold<U / 8, U>(v, lane, 4);
    V s = v[0];
#pragma unroll
    for (int m = 32 / U; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    return s;
}

// Position in the lower triangle: t = i (i + 1) / 2 + j, j <= i  ->  (i, j)
__device__ __forceinline__ void tri_ij(int t, int &I, int &J) {
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (i > 0 && i * (i + 1) / 2 > t) --i;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// Block sum; the result is valid in thread 0 only.  smem: NT/64 entries.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T *smem) {
    constexpr int NW = NT / WAVE;
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    if (lane == 0) smem[w] = v;
    __syncthreads();
    T s = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NW; ++i) s += smem[i];
    }
    return s;
}

template <int NT, typename T>
__device__ __forceinline__ T block_max(T v, T *smem) {
    constexpr int NW = NT / WAVE;
    v = wave_max(v);
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    if (lane == 0) smem[w] = v;
    __syncthreads();
    T s = 0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NW; ++i) s = fmax(s, smem[i]);
    }
    return s;
}

// ------------------------------------------------- cross-block reductions
// A kernel writes one partial per block; the *next* kernel reduces them.  The
// kernel boundary makes the partials visible device-wide, so no atomics or
// device-scope fences are needed (on gfx950 such a fence writes back and
// invalidates the XCD's L2, which costs more than the GEMV itself when every
// block does it).  Every consumer block sums the partials in the same fixed
// order, so all blocks obtain bitwise the same scalar and the result is
// reproducible run to run.

// Sum of partial[i * stride], i < count, returned to every thread of the block.
template <int NT>
__device__ __forceinline__ double reduce_partials_all(const double *partial, int count, int stride) {
    __shared__ double sm_r[NT / WAVE];
    __shared__ double sm_out;
    // the loads go out eight at a time ahead of the adds, which keep the
    // order of the plain strided loop (the same sum bit for bit); a plain loop
    // waits for each load before its add
    double s = 0.0;
    int i = threadIdx.x;
    for (; i + 7 * NT < count; i += 8 * NT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(i + u * NT) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; i < count; i += NT) s += partial[(size_t)i * stride];
    s = block_sum<NT>(s, sm_r);
    if (threadIdx.x == 0) sm_out = s;
    __syncthreads();
    return sm_out;
}

template <int NT>
__device__ __forceinline__ double reduce_partials_max_all(const double *partial, int count,
                                                          int stride) {
    __shared__ double sm_r[NT / WAVE];
    __shared__ double sm_out;
    double s = 0.0;
    int i = threadIdx.x;
    for (; i + 7 * NT < count; i += 8 * NT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(i + u * NT) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s = fmax(s, v[u]);
    }
    for (; i < count; i += NT) s = fmax(s, partial[(size_t)i * stride]);
    s = block_max<NT>(s, sm_r);
    if (threadIdx.x == 0) sm_out = s;
    __syncthreads();
    return sm_out;
}

// ------------------------------------------------------------- conversions
__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xFFFF0000u); }
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// binary32 -> bfloat16, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x0040u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bool finite_d(double x) { return __builtin_isfinite(x); }

// Absolute threshold on ||r||_2: tol ||b||_2, or with backward-error stopping
// tol (||A||_inf ||x||_inf + ||b||_inf) (which bounds eta_inf by tol).
__device__ __forceinline__ double stop_threshold(const State *st, double xinf) {
    return st->eta_tol > 0.0 ? st->eta_tol * (st->anorm_inf * xinf + st->binf) : st->thresh;
}

// GMRES's threshold on its estimate |g(k+1)| = ||r||_2.  With backward-error
// stopping the 2-norm stands in for ||r||_inf through the ratio
// ||r||_2 / ||r||_inf of the cycle's starting (true) residual, so the cycle
// stops near eta_inf = tol rather than ||r||_2 / (...) = tol, which for a
// residual spread over n components is about sqrt(n / (2 ln n)) times
// smaller; the stop is confirmed on eta_inf of the true residual at the end
// of the cycle, and a failed check starts another cycle.
__device__ __forceinline__ double gm_threshold(const State *st) {
    if (!(st->eta_tol > 0.0)) return st->thresh;
    const double ratio = st->resinf > 0.0 ? st->res / st->resinf : 1.0;
    return st->eta_tol * (st->anorm_inf * st->xinf + st->binf) * ratio;
}

// The request server's batched launches: the item of block `bid` in a set
// (offs[i] <= bid < offs[i+1]), its local block index and block count.
template <typename Item>
__device__ __forceinline__ const Item &batch_item(const BatchSetT<Item> &bs, int bid, int &local,
                                                  int &nblk) {
    int lo = 0, hi = bs.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bs.offs[mid] <= bid)
            lo = mid;
        else
            hi = mid - 1;
    }
    local = bid - bs.offs[lo];
    nblk = bs.offs[lo + 1] - bs.offs[lo];
    return bs.items[bs.idx[lo]];
}

}  // namespace ks
