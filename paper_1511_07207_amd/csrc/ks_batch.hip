// Batched launches for the request server: one launch advances the same phase
// of many in-flight solves.  The launch's blocks are the concatenation of each
// solve's own grid; block b finds its solve by binary search in a prefix-sum
// table of block counts and runs the same device body as the single-solve
// kernel with its local block index.  Solves of different sizes therefore
// share every launch, and small solves no longer pay one launch latency each.
// The kernels are templated on the storage of A and of the vectors, so the
// binary64 solves and the binary32 / bfloat16 inner solves of mixed-precision
// requests batch the same way.
#include <type_traits>

#include "ks_gemv_body.h"
#include "ks_vec_body.h"

namespace ks {

// item of block `bid` in a set: offs[i] <= bid < offs[i+1]
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

template <typename TA, typename T>
using BSet = BatchSetT<BatchItemT<TA, T>>;

// GMRES step number of an item (device-resident, advanced by b_gm_advance)
template <typename TA, typename T>
__device__ __forceinline__ int item_k(const BatchItemT<TA, T> &it) { return it.st->kcur; }

// ------------------------------------------------------------ setup
template <typename TA, typename T>
__global__ __launch_bounds__(ONE_NT) void b_vec_stats(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    vec_stats_body<T>(it.n, it.b, it.tol, it.st, it.eta);
}

__global__ __launch_bounds__(GEMV_NT) void b_norm_inf(BSet<double, double> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    norm_inf_body(it.n, it.lda, it.A, it.P.g, l);
}

__global__ __launch_bounds__(ONE_NT) void b_norm_inf_finish(BSet<double, double> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    norm_inf_finish_body(gemv_blocks<double>(it.n), it.st, it.P.g);
}

// r = b - A x into it.resid.  gate: 0 always; 1 when stopped; 3 when the
// GMRES cycle has ended (stopped, or all m steps done)
template <typename TA, typename T>
__device__ __forceinline__ bool resid_gate(const BatchItemT<TA, T> &it, int gate) {
    if (gate == 0) return true;
    const bool stopped = (it.st->flags & F_STOP) != 0;
    if (gate == 1) return stopped;
    return stopped || it.st->kcur >= it.m;
}

template <typename TA, typename T>
__global__ __launch_bounds__(GEMV_NT) void b_residual(BSet<TA, T> bs, int gate) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    if (!resid_gate(it, gate)) return;
    residual_body<TA>(it.n, it.lda, it.A, it.b, it.x, it.resid, it.st, it.P.g, 0, l);
}

template <typename TA, typename T>
__global__ __launch_bounds__(ONE_NT) void b_residual_finish(BSet<TA, T> bs, int gate) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    if (!resid_gate(it, gate)) return;
    residual_finish_body(gemv_blocks<TA>(it.n), it.st, it.P.g, 0);
}

// --------------------------------------------------------------- CG
template <typename TA, typename T>
__global__ __launch_bounds__(VEC_NT) void b_cg_begin(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    cg_begin_body<T>(it.n, it.resid, it.p, it.st, l);
}

template <typename TA, typename T>
__global__ __launch_bounds__(GEMV_NT) void b_cg_matvec(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    cg_matvec_body<TA>(it.n, it.lda, it.A, it.p, it.q, it.st, it.P.g, l);
}

template <typename TA, typename T>
__global__ __launch_bounds__(VEC_NT) void b_cg_update(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    cg_update_body<T>(it.n, it.x, it.resid, it.p, it.q, it.st, it.P.g, gemv_blocks<TA>(it.n), it.P.v,
                      l, nb);
}

template <typename TA, typename T>
__global__ __launch_bounds__(VEC_NT) void b_cg_pupdate(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    cg_pupdate_body<T>(it.n, it.resid, it.p, it.st, it.P.v, vec_blocks(it.n), it.max_iter, l);
}

// ------------------------------------------------------------- GMRES
template <typename TA, typename T>
__global__ __launch_bounds__(VEC_NT) void b_gm_begin(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    gm_begin_body<T>(it.n, it.resid, it.V, it.st, it.ga, l);
    if (l == 0 && threadIdx.x == 0) it.st->kcur = 0;
}

// the step kernels skip an item whose cycle has run all m steps
template <typename TA, typename T>
__global__ __launch_bounds__(GEMV_NT) void b_gm_matvec(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    const int k = item_k(it);
    if (k >= it.m) return;
    gm_matvec_body<TA>(it.n, it.lda, it.A, it.V + (size_t)k * it.ldv, it.resid, it.st, it.P.g, l);
}

template <typename TA, typename T, int MODE>
__global__ __launch_bounds__(CGS_NT) void b_gm_cgs(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    const int k = item_k(it);
    if (k >= it.m) return;
    gm_cgs_body<T, MODE>(it.n, it.ldv, it.V, it.resid, k, it.st, it.ga, it.P, gemv_blocks<TA>(it.n), l,
                         nb);
}

template <typename TA, typename T>
__global__ __launch_bounds__(VEC_NT) void b_gm_givens(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    const int k = item_k(it);
    if (k >= it.m) return;
    gm_givens_body<T>(it.n, it.resid, it.V + (size_t)(k + 1) * it.ldv, k, it.st, it.ga, it.P.nrm,
                      cgs_blocks(it.n), it.max_iter, l);
}

// one thread per item: the step counter moves on after every step launch
// (a stopped cycle keeps counting; its kernels return at once)
template <typename TA, typename T>
__global__ void b_gm_advance(BSet<TA, T> bs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= bs.count) return;
    State *st = bs.items[bs.idx[i]].st;
    if (st->kcur < bs.items[bs.idx[i]].m) st->kcur += 1;
}

// end of cycle (stopped, or m steps done): back substitution and x += V y
template <typename TA, typename T>
__global__ __launch_bounds__(CGS_NT) void b_gm_finish(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    if (!resid_gate(it, 3)) return;
    gm_finish_body<T>(it.n, it.ldv, it.V, it.x, it.st, it.ga, l);
}

// copy every item's State into a contiguous staging array (one host copy)
template <typename TA, typename T>
__global__ void b_gather(BSet<TA, T> bs, State *staging) {
    const int i = blockIdx.x;
    if (i >= bs.count) return;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(bs.items[bs.idx[i]].st);
    uint32_t *dst = reinterpret_cast<uint32_t *>(staging + i);
    for (int w = threadIdx.x; w < (int)(sizeof(State) / 4); w += blockDim.x) dst[w] = src[w];
}

// copy the States at ptrs[0 .. count) into a contiguous staging array
__global__ void b_gather_ptrs(const State *const *ptrs, int count, State *staging) {
    const int i = blockIdx.x;
    if (i >= count) return;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(ptrs[i]);
    uint32_t *dst = reinterpret_cast<uint32_t *>(staging + i);
    for (int w = threadIdx.x; w < (int)(sizeof(State) / 4); w += blockDim.x) dst[w] = src[w];
}

hipError_t gather_states(const State *const *d_ptrs, int count, State *staging, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    b_gather_ptrs<<<count, 64, 0, s>>>(d_ptrs, count, staging);
    return hipGetLastError();
}

// ------------------------------------------------- refinement steps
__global__ __launch_bounds__(VEC_NT) void b_ir_scale(IrSet bs) {
    int l, nb;
    const IrItem &it = batch_item(bs, blockIdx.x, l, nb);
    ir_scale_body(it.n, it.r64, it.rhs, it.st, l);
}

__global__ __launch_bounds__(VEC_NT) void b_ir_zero_d(IrSet bs) {
    int l, nb;
    const IrItem &it = batch_item(bs, blockIdx.x, l, nb);
    fill_body<float>(it.n, it.d, 0.0f, l);
}

__global__ __launch_bounds__(VEC_NT) void b_ir_update(IrSet bs) {
    int l, nb;
    const IrItem &it = batch_item(bs, blockIdx.x, l, nb);
    ir_update_body(it.n, it.x, it.d, &it.st->res, l);
}

// ------------------------------------------------------------- launchers
template <typename TA, typename T>
hipError_t batch_launch(BatchKernel kind, const BSet<TA, T> &bs, int blocks, int gate, hipStream_t s,
                        State *staging) {
    if (bs.count <= 0 || blocks <= 0) return hipSuccess;
    switch (kind) {
        case BK_VEC_STATS: b_vec_stats<TA, T><<<blocks, ONE_NT, 0, s>>>(bs); break;
        case BK_NORM_INF:
        case BK_NORM_INF_FINISH:
            if constexpr (std::is_same<TA, double>::value && std::is_same<T, double>::value) {
                if (kind == BK_NORM_INF)
                    b_norm_inf<<<blocks, GEMV_NT, 0, s>>>(bs);
                else
                    b_norm_inf_finish<<<blocks, ONE_NT, 0, s>>>(bs);
                break;
            } else {
                return hipErrorInvalidValue;
            }
        case BK_RESIDUAL: b_residual<TA, T><<<blocks, GEMV_NT, 0, s>>>(bs, gate); break;
        case BK_RESIDUAL_FINISH: b_residual_finish<TA, T><<<blocks, ONE_NT, 0, s>>>(bs, gate); break;
        case BK_CG_BEGIN: b_cg_begin<TA, T><<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_CG_MATVEC: b_cg_matvec<TA, T><<<blocks, GEMV_NT, 0, s>>>(bs); break;
        case BK_CG_UPDATE: b_cg_update<TA, T><<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_CG_PUPDATE: b_cg_pupdate<TA, T><<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_GM_BEGIN: b_gm_begin<TA, T><<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_GM_MATVEC: b_gm_matvec<TA, T><<<blocks, GEMV_NT, 0, s>>>(bs); break;
        case BK_GM_CGS0: b_gm_cgs<TA, T, 0><<<blocks, CGS_NT, 0, s>>>(bs); break;
        case BK_GM_CGS1: b_gm_cgs<TA, T, 1><<<blocks, CGS_NT, 0, s>>>(bs); break;
        case BK_GM_CGS2: b_gm_cgs<TA, T, 2><<<blocks, CGS_NT, 0, s>>>(bs); break;
        case BK_GM_GIVENS: b_gm_givens<TA, T><<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_GM_ADVANCE: b_gm_advance<TA, T><<<(bs.count + 255) / 256, 256, 0, s>>>(bs); break;
        case BK_GM_FINISH: b_gm_finish<TA, T><<<blocks, CGS_NT, 0, s>>>(bs); break;
        case BK_GATHER: b_gather<TA, T><<<bs.count, 64, 0, s>>>(bs, staging); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t batch_launch<double, double>(BatchKernel, const BSet<double, double> &, int, int,
                                                 hipStream_t, State *);
template hipError_t batch_launch<float, float>(BatchKernel, const BSet<float, float> &, int, int,
                                               hipStream_t, State *);
template hipError_t batch_launch<bf16_t, float>(BatchKernel, const BSet<bf16_t, float> &, int, int,
                                                hipStream_t, State *);

hipError_t ir_batch_launch(IrKernel kind, const IrSet &bs, int blocks, hipStream_t s) {
    if (bs.count <= 0 || blocks <= 0) return hipSuccess;
    switch (kind) {
        case IK_SCALE: b_ir_scale<<<blocks, VEC_NT, 0, s>>>(bs); break;
        case IK_ZERO_D: b_ir_zero_d<<<blocks, VEC_NT, 0, s>>>(bs); break;
        case IK_UPDATE: b_ir_update<<<blocks, VEC_NT, 0, s>>>(bs); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ks
