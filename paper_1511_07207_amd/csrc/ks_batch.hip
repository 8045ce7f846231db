// Batched launches for the request server: one launch advances the same phase
// of many in-flight solves.  The launch's blocks are the concatenation of each
// solve's own grid; block b finds its solve by binary search in a prefix-sum
// table of block counts and runs the same device body as the single-solve
// kernel with its local block index.  Solves of different sizes therefore
// share every launch, and small solves no longer pay one launch latency each.
// The set-up, restart and cycle-end kernels are templated on the storage of A
// and of the vectors (binary64 solves, binary32 / bfloat16 inner solves of
// mixed-precision requests).  The Krylov steps run as stages: one launch
// holds one position of the step for CG and GMRES solves of every storage
// type (the products one launch per storage), each entry of its table naming
// the item and the body it runs, so a step costs at most seven launches
// whatever the mix of methods and precisions in flight.
#include <type_traits>

#include "ks_gemv_body.h"
#include "ks_vec_body.h"

namespace ks {

template <typename TA, typename T>
using BSet = BatchSetT<BatchItemT<TA, T>>;

// ------------------------------------------------------------ setup
template <typename TA, typename T>
__global__ __launch_bounds__(ONE_NT) void b_vec_stats(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    if (!setup_gate(it)) return;
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

// An inner solve started by a refinement check on the device in this tick
// runs only if that check said go on.
template <typename TA, typename T>
__device__ __forceinline__ bool setup_gate(const BatchItemT<TA, T> &it) {
    return !it.outer || it.outer->ir_next == IR_GO;
}

// r = b - A x into it.resid.  gate: 0 always; 1 when stopped; 3 when the
// GMRES cycle has ended (stopped, or all m steps done).  Gates 1 and 3 are
// closed for a solve whose set-up ended it (no step ran).
template <typename TA, typename T>
__device__ __forceinline__ bool resid_gate(const BatchItemT<TA, T> &it, int gate) {
    if (!setup_gate(it)) return false;
    if (gate == 0) return true;
    if (it.st->flags & F_SETUP_END) return false;
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

// The set-up's own decision, taken at the (re)start as the host drivers take
// it after the set-up: b = 0, a non-finite or already converged residual, or
// no iterations left end the solve before its first step (F_SETUP_END, with
// F_STOP so that the step kernels return at once).  Every block reads the
// same fields, none of which this launch changes, so all take the same
// branch.  A (re)start the host decided after checking the same conditions
// always proceeds.
template <typename TA, typename T>
__device__ __forceinline__ bool begin_gate(const BatchItemT<TA, T> &it, int l) {
    if (!setup_gate(it)) return false;
    const State *st = it.st;
    if (st->bnorm == 0.0 || (st->flags & (F_TRUE_NONFIN | F_TRUE_OK)) || st->iters >= it.max_iter) {
        if (l == 0 && threadIdx.x == 0) it.st->flags |= F_STOP | F_SETUP_END;
        return false;
    }
    return true;
}

// --------------------------------------------------------------- CG
template <typename TA, typename T>
__global__ __launch_bounds__(VEC_NT) void b_cg_begin(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    if (!begin_gate(it, l)) return;
    cg_begin_body<T>(it.n, it.resid, it.p, it.st, l);
}

// ------------------------------------------------------------- GMRES
template <typename TA, typename T>
__global__ __launch_bounds__(VEC_NT) void b_gm_begin(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    if (!begin_gate(it, l)) return;
    gm_begin_body<T>(it.n, it.resid, it.V, it.st, it.ga, l);
    if (l == 0 && threadIdx.x == 0) it.st->kcur = it.st->kcur_odd = 0;
}

// end of cycle (stopped, or m steps done): back substitution and x += V y
template <typename TA, typename T>
__global__ __launch_bounds__(CGS_NT) void b_gm_finish(BSet<TA, T> bs) {
    int l, nb;
    const auto &it = batch_item(bs, blockIdx.x, l, nb);
    if (!resid_gate(it, 3)) return;
    gm_finish_body<T>(it.n, it.ldv, it.V, it.x, it.st, it.ga, l);
}

// ------------------------------------------------------------- stages
// Step `step` of a tick reads the GMRES step number from the counter of its
// parity; the Givens stage's block 0 moves the other counter on (min(k + 1,
// m), also when the step returned at once after a stop), so no block of a
// stage reads a counter that the same stage writes.
template <typename TA, typename T>
__device__ __forceinline__ int stage_k(const BatchItemT<TA, T> &it, int step) {
    return (step & 1) ? it.st->kcur_odd : it.st->kcur;
}

// The kinds a stage holds (stage_of): each stage is its own kernel, so that
// the product stage carries only the product bodies' registers.
__host__ __device__ constexpr int stage_of(int sk) {
    return sk == SK_CG_MATVEC || sk == SK_GM_MATVEC                          ? 1
           : sk == SK_CG_UPDATE || sk == SK_GM_CGS0                          ? 2
           : sk == SK_CG_PUPDATE || sk == SK_SY_PUPDATE || sk == SK_GM_CGS1  ? 3
           : sk == SK_GM_CGS2                         ? 4
                                                      : 5;
}

template <int STAGE, typename TA, typename T>
__device__ __forceinline__ void stage_body(const BatchItemT<TA, T> &it, int sk, int l, int nb, int step) {
    if constexpr (STAGE == 1) {
        if (sk == SK_CG_MATVEC) {
            cg_matvec_body<TA>(it.n, it.lda, it.A, it.p, it.q, it.st, it.P.g, l);
        } else {
            const int k = stage_k(it, step);
            if (k >= it.m) return;
            gm_matvec_body<TA>(it.n, it.lda, it.A, it.V + (size_t)k * it.ldv, it.resid, it.st, it.P.g, l);
        }
    } else if constexpr (STAGE == 2 || STAGE == 3) {
        if (sk == SK_CG_UPDATE) {
            cg_update_body<T>(it.n, it.x, it.resid, it.p, it.q, it.st, it.P.g, gemv_blocks<TA>(it.n),
                              it.P.v, l, nb);
        } else if (sk == SK_CG_PUPDATE) {
            cg_pupdate_body<T>(it.n, it.resid, it.p, it.st, it.P.v, vec_blocks(it.n), it.max_iter, l);
        } else if (sk == SK_SY_PUPDATE) {
            // after the symmetric product's finishing sum: its r'r partials
            cg_pupdate_body<T>(it.n, it.resid, it.p, it.st, symv_cg_rho_part(it.n, it.sy),
                               div_up(it.n, SY_FIN), it.max_iter, l);
        } else {
            const int k = stage_k(it, step);
            if (k >= it.m) return;
            gm_cgs_body<T, STAGE - 2>(it.n, it.ldv, it.V, it.resid, k, it.st, it.ga, it.P,
                                      gemv_blocks<TA>(it.n), l, nb);
        }
    } else if constexpr (STAGE == 4) {
        const int k = stage_k(it, step);
        if (k >= it.m) return;
        gm_cgs_body<T, 2>(it.n, it.ldv, it.V, it.resid, k, it.st, it.ga, it.P, gemv_blocks<TA>(it.n), l, nb);
    } else {
        const int k = stage_k(it, step);
        if (l == 0 && threadIdx.x == 0) {
            const int kn = k < it.m ? k + 1 : k;
            if (step & 1)
                it.st->kcur = kn;
            else
                it.st->kcur_odd = kn;
        }
        if (k >= it.m) return;
        gm_givens_body<T>(it.n, it.resid, it.V + (size_t)(k + 1) * it.ldv, k, it.st, it.ga, it.P.nrm,
                          cgs_blocks(it.n), it.max_iter, l);
    }
}

// DT >= 0: every entry has that storage (the product stage runs one launch
// per storage, each with only its own product bodies' registers: 64 rather
// than 108 VGPRs for the binary64 products); DT < 0: the entry's storage
// decides.
template <int STAGE, int DT>
__global__ __launch_bounds__(256) void b_stage_kernel(StageSet ss, int step) {
    int lo = 0, hi = ss.count - 1;
    const int bid = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ss.offs[mid] <= bid)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int l = bid - ss.offs[lo];
    const int nb = ss.offs[lo + 1] - ss.offs[lo];
    const int slot = ss.idx[lo];
    const int kind = ss.kind[lo];
    const int sk = kind & 255;
    const int dt = DT >= 0 ? DT : kind >> 8;
    if (dt == 0) {
        if constexpr (DT < 0 || DT == 0) stage_body<STAGE>(ss.i64[slot], sk, l, nb, step);
    } else if (dt == 1) {
        if constexpr (DT < 0 || DT == 1) stage_body<STAGE>(ss.i32[slot], sk, l, nb, step);
    } else {
        if constexpr (DT < 0 || DT == 2) stage_body<STAGE>(ss.i16[slot], sk, l, nb, step);
    }
}

hipError_t stage_launch(const StageSet &ss, int stage, int blocks, int step, hipStream_t s) {
    if (ss.count <= 0 || blocks <= 0) return hipSuccess;
    static_assert(GEMV_NT == 256 && VEC_NT == 256 && CGS_NT == 256, "one block shape for every stage");
    switch (stage) {
        case 10: b_stage_kernel<1, 0><<<blocks, 256, 0, s>>>(ss, step); break;
        case 11: b_stage_kernel<1, 1><<<blocks, 256, 0, s>>>(ss, step); break;
        case 12: b_stage_kernel<1, 2><<<blocks, 256, 0, s>>>(ss, step); break;
        case 2: b_stage_kernel<2, -1><<<blocks, 256, 0, s>>>(ss, step); break;
        case 3: b_stage_kernel<3, -1><<<blocks, 256, 0, s>>>(ss, step); break;
        case 4: b_stage_kernel<4, -1><<<blocks, 256, 0, s>>>(ss, step); break;
        case 5: b_stage_kernel<5, -1><<<blocks, 256, 0, s>>>(ss, step); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
    if (it.gated && it.st->ir_next != IR_GO) return;
    ir_scale_body(it.n, it.r64, it.rhs, it.st, l);
}

__global__ __launch_bounds__(VEC_NT) void b_ir_zero_d(IrSet bs) {
    int l, nb;
    const IrItem &it = batch_item(bs, blockIdx.x, l, nb);
    if (it.gated && it.st->ir_next != IR_GO) return;
    fill_body<float>(it.n, it.d, 0.0f, l);
}

// The refinement check of one request on its new outer residual, in the
// order and arithmetic of the host's check (the binary64 comparisons of
// eta_inf with the target, the step limit and half the previous eta_inf), so
// that both reach the same decision.  Anything but IR_GO leaves the inner
// State stopped, so that no kernel of the inner solve runs in this tick.
__global__ void b_ir_decide(IrSet bs) {
    if (threadIdx.x != 0 || (int)blockIdx.x >= bs.count) return;
    const IrItem &it = bs.items[bs.idx[blockIdx.x]];
    const State &h = *it.st;
    int next;
    if (it.first && h.bnorm == 0.0) {
        next = IR_ZERO;
    } else {
        const double den = h.anorm_inf * h.xinf + h.binf;
        const double eta = den > 0.0 ? h.resinf / den : h.resinf;
        if (!finite_d(eta) || (h.flags & F_TRUE_NONFIN))
            next = IR_NONFIN;
        else if (eta <= it.tol)
            next = IR_DONE;
        else if (it.outer_steps >= it.max_outer)
            next = IR_STAG;
        else if (eta > 0.5 * it.eta_prev && it.bad + 1 >= 2 && it.prec != KS_FP64)
            next = IR_PROMOTE;
        else
            next = IR_GO;
    }
    it.st->ir_next = next;
    if (next != IR_GO) it.inner->flags = F_STOP;
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
        case BK_GM_BEGIN: b_gm_begin<TA, T><<<blocks, VEC_NT, 0, s>>>(bs); break;
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
        case IK_DECIDE: b_ir_decide<<<bs.count, 64, 0, s>>>(bs); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ks
