// Batched launches for the request server: one launch advances the same phase
// of many in-flight solves.  The launch's blocks are the concatenation of each
// solve's own grid; block b finds its solve by binary search in a prefix-sum
// table of block counts and runs the same device body as the single-solve
// kernel with its local block index.  Solves of different sizes therefore
// share every launch, and small solves no longer pay one launch latency each.
#include "ks_gemv_body.h"
#include "ks_vec_body.h"

namespace ks {

// solve index of block `bid` in a set: offs[i] <= bid < offs[i+1]
__device__ __forceinline__ const BatchItem &batch_item(const BatchSet &bs, int bid, int &local,
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

// GMRES step number of an item (device-resident, advanced by b_gm_advance)
__device__ __forceinline__ int item_k(const BatchItem &it) { return it.st->kcur; }

// ------------------------------------------------------------ setup
__global__ __launch_bounds__(ONE_NT) void b_vec_stats(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    vec_stats_body<double>(it.n, it.b, it.tol, it.st, it.eta);
}

__global__ __launch_bounds__(GEMV_NT) void b_norm_inf(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    norm_inf_body(it.n, it.lda, it.A, it.P.g, l);
}

__global__ __launch_bounds__(ONE_NT) void b_norm_inf_finish(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    norm_inf_finish_body(gemv_blocks<double>(it.n), it.st, it.P.g);
}

// r = b - A x into it.resid.  gate: 0 always; 1 when stopped; 3 when the
// GMRES cycle has ended (stopped, or all m steps done)
__device__ __forceinline__ bool resid_gate(const BatchItem &it, int gate) {
    if (gate == 0) return true;
    const bool stopped = (it.st->flags & F_STOP) != 0;
    if (gate == 1) return stopped;
    return stopped || it.st->kcur >= it.m;
}

__global__ __launch_bounds__(GEMV_NT) void b_residual(BatchSet bs, int gate) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    if (!resid_gate(it, gate)) return;
    residual_body<double>(it.n, it.lda, it.A, it.b, it.x, it.resid, it.st, it.P.g, 0, l);
}

__global__ __launch_bounds__(ONE_NT) void b_residual_finish(BatchSet bs, int gate) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    if (!resid_gate(it, gate)) return;
    residual_finish_body(gemv_blocks<double>(it.n), it.st, it.P.g, 0);
}

// --------------------------------------------------------------- CG
__global__ __launch_bounds__(VEC_NT) void b_cg_begin(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    cg_begin_body<double>(it.n, it.resid, it.p, it.st, l);
}

__global__ __launch_bounds__(GEMV_NT) void b_cg_matvec(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    cg_matvec_body<double>(it.n, it.lda, it.A, it.p, it.q, it.st, it.P.g, l);
}

__global__ __launch_bounds__(VEC_NT) void b_cg_update(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    cg_update_body<double>(it.n, it.x, it.resid, it.p, it.q, it.st, it.P.g,
                           gemv_blocks<double>(it.n), it.P.v, l, nb);
}

__global__ __launch_bounds__(VEC_NT) void b_cg_pupdate(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    cg_pupdate_body<double>(it.n, it.resid, it.p, it.st, it.P.v, vec_blocks(it.n), it.max_iter, l);
}

// ------------------------------------------------------------- GMRES
__global__ __launch_bounds__(VEC_NT) void b_gm_begin(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    gm_begin_body<double>(it.n, it.resid, it.V, it.st, it.ga, l);
    if (l == 0 && threadIdx.x == 0) it.st->kcur = 0;
}

// the step kernels skip an item whose cycle has run all m steps
__global__ __launch_bounds__(GEMV_NT) void b_gm_matvec(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    const int k = item_k(it);
    if (k >= it.m) return;
    gm_matvec_body<double>(it.n, it.lda, it.A, it.V + (size_t)k * it.ldv, it.resid, it.st, it.P.g, l);
}

template <int MODE>
__global__ __launch_bounds__(CGS_NT) void b_gm_cgs(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    const int k = item_k(it);
    if (k >= it.m) return;
    gm_cgs_body<double, MODE>(it.n, it.ldv, it.V, it.resid, k, it.st, it.ga, it.P,
                              gemv_blocks<double>(it.n), l, nb);
}

__global__ __launch_bounds__(VEC_NT) void b_gm_givens(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    const int k = item_k(it);
    if (k >= it.m) return;
    gm_givens_body<double>(it.n, it.resid, it.V + (size_t)(k + 1) * it.ldv, k, it.st, it.ga, it.P.nrm,
                           cgs_blocks(it.n), it.max_iter, l);
}

// one thread per item: the step counter moves on after every step launch
// (a stopped cycle keeps counting; its kernels return at once)
__global__ void b_gm_advance(BatchSet bs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= bs.count) return;
    State *st = bs.items[bs.idx[i]].st;
    if (st->kcur < bs.items[bs.idx[i]].m) st->kcur += 1;
}

// end of cycle (stopped, or m steps done): back substitution and x += V y
__global__ __launch_bounds__(CGS_NT) void b_gm_finish(BatchSet bs) {
    int l, nb;
    const BatchItem &it = batch_item(bs, blockIdx.x, l, nb);
    if (!resid_gate(it, 3)) return;
    gm_finish_body<double>(it.n, it.ldv, it.V, it.x, it.st, it.ga, l);
}

// copy every item's State into a contiguous staging array (one host copy)
__global__ void b_gather(BatchSet bs, State *staging) {
    const int i = blockIdx.x;
    if (i >= bs.count) return;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(bs.items[bs.idx[i]].st);
    uint32_t *dst = reinterpret_cast<uint32_t *>(staging + i);
    for (int w = threadIdx.x; w < (int)(sizeof(State) / 4); w += blockDim.x) dst[w] = src[w];
}

// ------------------------------------------------------------- launchers
static inline hipError_t done() { return hipGetLastError(); }

hipError_t batch_launch(BatchKernel kind, const BatchSet &bs, int blocks, int gate, hipStream_t s,
                        State *staging) {
    if (bs.count <= 0 || blocks <= 0) return hipSuccess;
    switch (kind) {
        case BK_VEC_STATS: b_vec_stats<<<blocks, ONE_NT, 0, s>>>(bs); break;
        case BK_NORM_INF: b_norm_inf<<<blocks, GEMV_NT, 0, s>>>(bs); break;
        case BK_NORM_INF_FINISH: b_norm_inf_finish<<<blocks, ONE_NT, 0, s>>>(bs); break;
        case BK_RESIDUAL: b_residual<<<blocks, GEMV_NT, 0, s>>>(bs, gate); break;
        case BK_RESIDUAL_FINISH: b_residual_finish<<<blocks, ONE_NT, 0, s>>>(bs, gate); break;
        case BK_CG_BEGIN: b_cg_begin<<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_CG_MATVEC: b_cg_matvec<<<blocks, GEMV_NT, 0, s>>>(bs); break;
        case BK_CG_UPDATE: b_cg_update<<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_CG_PUPDATE: b_cg_pupdate<<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_GM_BEGIN: b_gm_begin<<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_GM_MATVEC: b_gm_matvec<<<blocks, GEMV_NT, 0, s>>>(bs); break;
        case BK_GM_CGS0: b_gm_cgs<0><<<blocks, CGS_NT, 0, s>>>(bs); break;
        case BK_GM_CGS1: b_gm_cgs<1><<<blocks, CGS_NT, 0, s>>>(bs); break;
        case BK_GM_CGS2: b_gm_cgs<2><<<blocks, CGS_NT, 0, s>>>(bs); break;
        case BK_GM_GIVENS: b_gm_givens<<<blocks, VEC_NT, 0, s>>>(bs); break;
        case BK_GM_ADVANCE: b_gm_advance<<<(bs.count + 255) / 256, 256, 0, s>>>(bs); break;
        case BK_GM_FINISH: b_gm_finish<<<blocks, CGS_NT, 0, s>>>(bs); break;
        case BK_GATHER: b_gather<<<bs.count, 64, 0, s>>>(bs, staging); break;
        default: return hipErrorInvalidValue;
    }
    return done();
}

}  // namespace ks
