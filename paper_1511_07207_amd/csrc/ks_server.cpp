// Request server: continuous batching of many CG / GMRES(m) solves, binary64
// or mixed precision (inner solve on a binary32 / bfloat16 copy of A with
// binary64 iterative refinement around it).
//
// Requests are queued in arrival order and admitted while the memory budget
// (resident A plus the solve's workspace) and the slot count allow; the queue
// is served first come, first served (no request overtakes an earlier one).
// Each call of ks_server_step is one tick:
//   1. admit from the queue;
//   2. one batched launch per phase and storage type advances every in-flight
//      solve: set-up of the new ones (||A||_inf, ||b||, r0), refinement steps
//      (x += ||r|| d, binary64 residual; r / ||r|| as the next inner
//      right-hand side), (re)starts, then `chunk` iterations of every CG solve
//      and `chunk` Arnoldi steps of every GMRES solve -- binary64 and inner
//      alike -- the gated true residuals and the GMRES cycle ends;
//   3. one gather kernel and one copy bring the State each request's next
//      decision needs to the host, which decides per request exactly as the
//      single-solve drivers do (continue, restart, new cycle, refinement step,
//      precision promotion, done), retires finished requests (latency =
//      completion - submission) and frees their memory.
// Requests that arrive while others run join at the next tick, so their work
// overlaps on the device with the solves already in flight.  A solve's result
// does not depend on what else is batched with it: every block of a batched
// launch runs the same device body on the same data, in the same order, as
// the single-solve kernel, and the host takes the same decisions in the same
// order as the single-solve drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "ks.h"
#include "ks_internal.h"
#include "ks_layout.h"
#include "ks_sched.h"

using namespace ks;

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Phases of a request.  Binary64 solves (and the binary64 finish of a
// mixed-precision request after promotion) go INIT -> BEGIN -> RUN ...;
// mixed-precision requests go INIT -> (check) -> IN_INIT -> IN_BEGIN ->
// IN_RUN ... -> UPDATE -> (check) -> IN_INIT ...
enum Phase { P_QUEUED, P_INIT, P_BEGIN, P_RUN, P_IN_INIT, P_IN_BEGIN, P_IN_RUN, P_UPDATE, P_DONE };

struct Req {
    uint64_t ticket = 0;
    ks_params p{};
    Layout L;
    const double *A = nullptr;
    const double *b = nullptr;
    double *x = nullptr;
    double t_submit = 0.0;
    size_t ws_off = 0, ws_bytes = 0, footprint = 0;
    Phase phase = P_QUEUED;
    int seg = -1;  // workspace segment
    double *sy = nullptr;  // symmetric CG product region (KS_FLAG_SYMMETRIC)
    bool copy_a = false;
    int restarts = 0, cycles = 0;
    BatchItem item{};  // binary64: the solve, or the refinement's outer step
    // mixed precision
    bool ir = false;         // refinement request (until promoted to binary64)
    bool fp64_tail = false;  // promoted: the binary64 solve stopping on the backward error
    int prec = KS_FP64;      // precision of the next inner solve
    int outer = 0, bad = 0, total_iters = 0;
    double eta_prev = INFINITY;
    bool fb_ready = false;
    void *A_low = nullptr;
    float *A_fb = nullptr;
    BatchItemT<float, float> in32{};
    BatchItemT<bf16_t, float> in16{};
    IrItem iri{};
    State last_outer{};  // the outer State of the last refinement check
    ks_info info{};
};

constexpr int SERVER_CG_MAX_RESTARTS = 16;
constexpr int NO_OUTCOME = -100;

}  // namespace

// The workspaces live in device segments allocated as admission needs them
// (SchedPool): a request goes first fit into an existing segment, else into a
// new one of at least SCHED_SEG_MIN bytes, as long as all segments together
// stay within the memory budget (the workspaces of the admitted requests
// never exceed it, so admission is decided by the budget, not by a fixed
// arena).
struct ks_server {
    hipStream_t stream = nullptr;
    size_t budget = 0, in_use = 0;
    int max_inflight = 0;
    int chunk = 16;
    SchedPool pool;
    uint64_t next_ticket = 1;
    std::deque<Req *> queue;
    std::vector<Req *> inflight;
    std::vector<Req *> finished;
    char *dtab = nullptr, *htab = nullptr;
    size_t tab_cap = 0;
    State *dstage = nullptr, *hstage = nullptr;
    size_t stage_cap = 0;
};

namespace {

int grow_buffers(ks_server *sv, size_t tab_bytes, size_t nstage) {
    if (tab_bytes > sv->tab_cap) {
        const size_t cap = std::max(tab_bytes, 2 * sv->tab_cap);
        if (sv->dtab) (void)hipFree(sv->dtab);
        if (sv->htab) (void)hipHostFree(sv->htab);
        sv->dtab = sv->htab = nullptr;
        sv->tab_cap = 0;
        if (hipMalloc((void **)&sv->dtab, cap) != hipSuccess) return KS_ENOMEM;
        if (hipHostMalloc((void **)&sv->htab, cap, hipHostMallocDefault) != hipSuccess) return KS_ENOMEM;
        sv->tab_cap = cap;
    }
    if (nstage > sv->stage_cap) {
        const size_t cap = std::max(nstage, 2 * sv->stage_cap);
        if (sv->dstage) (void)hipFree(sv->dstage);
        if (sv->hstage) (void)hipHostFree(sv->hstage);
        sv->dstage = sv->hstage = nullptr;
        sv->stage_cap = 0;
        if (hipMalloc((void **)&sv->dstage, cap * sizeof(State)) != hipSuccess) return KS_ENOMEM;
        if (hipHostMalloc((void **)&sv->hstage, cap * sizeof(State), hipHostMallocDefault) != hipSuccess)
            return KS_ENOMEM;
        sv->stage_cap = cap;
    }
    return KS_OK;
}

// A workspace for r in the pool (device segments from hipMalloc).  Returns
// false (nothing allocated) when none can be placed within the budget.
bool ws_alloc(ks_server *sv, Req *r) {
    auto dev_alloc = [](size_t bytes) -> char * {
        char *p = nullptr;
        return hipMalloc((void **)&p, bytes) == hipSuccess ? p : nullptr;
    };
    auto dev_free = [](char *p) { (void)hipFree(p); };
    return sv->pool.place_or_reset(r->ws_bytes, sv->inflight.empty(), dev_alloc, dev_free, &r->seg,
                                   &r->ws_off);
}

inline char *ws_base(const ks_server *sv, const Req *r) { return sv->pool.base(r->seg) + r->ws_off; }

// Builds the per-tick table in pinned host memory: item arrays, then for
// every (subset, block shape) an index array and a prefix-sum array of block
// counts.  Device addresses mirror the host offsets (one copy per tick).
class TableBuilder {
   public:
    TableBuilder(char *host, char *dev) : host_(host), dev_(dev) {}
    template <typename T>
    T *array(int count, const T **dev_ptr) {
        const size_t off = off_;
        off_ += align_up(sizeof(T) * (size_t)std::max(count, 1));
        *dev_ptr = reinterpret_cast<const T *>(dev_ + off);
        return reinterpret_cast<T *>(host_ + off);
    }
    static size_t array_bytes(size_t elem, int count) { return align_up(elem * (size_t)std::max(count, 1)); }
    static size_t set_bytes(int count) { return 2 * align_up(sizeof(int) * (size_t)(count + 1)); }
    template <typename Item, typename F>
    BatchSetT<Item> add(const Item *dev_items, const std::vector<int> &idx, F blocks_of, int *total) {
        BatchSetT<Item> bs{};
        const int c = (int)idx.size();
        int *hi = reinterpret_cast<int *>(host_ + off_);
        bs.idx = reinterpret_cast<const int *>(dev_ + off_);
        off_ += align_up(sizeof(int) * (size_t)(c + 1));
        int *ho = reinterpret_cast<int *>(host_ + off_);
        bs.offs = reinterpret_cast<const int *>(dev_ + off_);
        off_ += align_up(sizeof(int) * (size_t)(c + 1));
        int acc = 0;
        for (int i = 0; i < c; ++i) {
            hi[i] = idx[i];
            ho[i] = acc;
            acc += blocks_of(idx[i]);
        }
        ho[c] = acc;
        bs.items = dev_items;
        bs.count = c;
        *total = acc;
        return bs;
    }
    // A stage set over (slot, kind) entries, blocks_of(slot, kind) blocks each.
    template <typename F>
    StageSet stage(const BatchItem *d64, const BatchItemT<float, float> *d32,
                   const BatchItemT<bf16_t, float> *d16, const std::vector<std::pair<int, int>> &e,
                   F blocks_of, int *total) {
        StageSet ss{};
        const int c = (int)e.size();
        int *hi = reinterpret_cast<int *>(host_ + off_);
        ss.idx = reinterpret_cast<const int *>(dev_ + off_);
        off_ += align_up(sizeof(int) * (size_t)(c + 1));
        int *hk = reinterpret_cast<int *>(host_ + off_);
        ss.kind = reinterpret_cast<const int *>(dev_ + off_);
        off_ += align_up(sizeof(int) * (size_t)(c + 1));
        int *ho = reinterpret_cast<int *>(host_ + off_);
        ss.offs = reinterpret_cast<const int *>(dev_ + off_);
        off_ += align_up(sizeof(int) * (size_t)(c + 1));
        int acc = 0;
        for (int i = 0; i < c; ++i) {
            hi[i] = e[i].first;
            hk[i] = e[i].second;
            ho[i] = acc;
            acc += blocks_of(e[i].first, e[i].second);
        }
        ho[c] = acc;
        ss.i64 = d64;
        ss.i32 = d32;
        ss.i16 = d16;
        ss.count = c;
        *total = acc;
        return ss;
    }
    static size_t stage_bytes(int count) { return 3 * align_up(sizeof(int) * (size_t)(count + 1)); }
    size_t bytes() const { return off_; }

   private:
    char *host_, *dev_;
    size_t off_ = 0;
};

// Inner solves of one storage type: the subsets and their block counts.
template <typename TA>
struct InnerSets {
    using Set = BatchSetT<BatchItemT<TA, float>>;
    // set-up, (re)starts and the GMRES cycle ends; the steps run as stages
    Set init_g, init_1, cgb, gmb, gm_g, gm_c, gm_1;
    int n_init_g = 0, n_init_1 = 0, n_cgb = 0, n_gmb = 0, n_gm_g = 0, n_gm_c = 0, n_gm_1 = 0;
};

void finish_metrics(Req *r, const State &h) {
    if (h.bnorm > 0.0 && std::isfinite(h.bnorm)) {
        const double den = h.anorm_inf * h.xinf + h.binf;
        r->info.rel_res = h.res / h.bnorm;
        r->info.backward_err = den > 0.0 ? h.resinf / den : h.resinf;
    } else {
        r->info.rel_res = 0.0;
        r->info.backward_err = 0.0;
    }
}

// h: the binary64 State the outcome is read from (residual of the returned x)
void retire(ks_server *sv, Req *r, const State &h, int status, int iters) {
    r->info.status = status;
    r->info.iters = iters;
    if (r->p.precision != KS_FP64)
        r->info.restarts = 0;  // as the single-solve refinement driver reports
    else
        r->info.restarts = r->p.method == KS_CG ? r->restarts : std::max(0, r->cycles - 1);
    finish_metrics(r, h);
    r->info.elapsed_ms = now_ms() - r->t_submit;
    r->info.outer_iters = r->outer;
    r->info.precision_used = r->prec;
    r->phase = P_DONE;
    sv->pool.release(r->seg, r->ws_off, r->ws_bytes);
    sv->in_use -= r->footprint;
    sv->finished.push_back(r);
}

// Pointers of a request's inner solve (the vectors of the binary32 region of
// its workspace; A_low, or the binary32 copy after a promotion from
// bfloat16), and of its refinement steps.
void setup_inner(Req *r, const Carved &c) {
    const Layout &L = r->L;
    auto vec32 = [&](int i) { return c.v32 + (size_t)i * L.ldv; };
    auto fill = [&](auto &it) {
        it.lda = L.lda_low;
        it.n = r->p.n;
        it.ldv = L.ldv;
        it.m = L.m;
        it.max_iter = r->p.max_iter;
        it.tol = r->p.inner_tol;
        it.eta = 0;
        it.b = vec32(0);
        it.x = vec32(1);
        it.resid = vec32(2);
        if (r->p.method == KS_CG) {
            it.p = vec32(3);
            it.q = vec32(4);
            it.V = nullptr;
        } else {
            it.V = vec32(3);
            it.p = it.q = nullptr;
        }
        it.st = c.st + 1;
        it.P = c.P;
        it.ga = c.ga;
    };
    fill(r->in32);
    fill(r->in16);
    r->in32.sy = r->sy;      // binary32 inner CG on the lower triangle
    r->in16.sy = nullptr;    // bfloat16 inner solves keep the general product
    r->in16.A = (const bf16_t *)r->A_low;
    r->in32.A = (r->p.precision == KS_IR_BF16) ? r->A_fb : (const float *)r->A_low;
    r->iri.n = r->p.n;
    r->iri.r64 = c.v64 + (size_t)(L.nv64 - 1) * L.ldv;
    r->iri.rhs = vec32(0);
    r->iri.d = vec32(1);
    r->iri.x = r->x;
    r->iri.st = c.st;
}

// Switch a refinement request to its binary64 finish: the plain solve from
// the current x, stopping on the backward error (as the single-solve driver).
void to_fp64_tail(Req *r, const Carved &c) {
    r->ir = false;
    r->fp64_tail = true;
    BatchItem &it = r->item;
    it.tol = r->p.tol;
    it.eta = 1;
    it.max_iter = std::max(1, r->p.max_iter);
    const int ldv = r->L.ldv;
    if (r->p.method == KS_CG) {
        it.resid = c.v64;
        it.p = c.v64 + ldv;
        it.q = c.v64 + 2 * (size_t)ldv;
        it.V = nullptr;
    } else {
        it.resid = c.v64;
        it.V = c.v64 + ldv;
        it.p = it.q = nullptr;
    }
    it.sy = r->sy;
    r->restarts = 0;
    r->cycles = 0;
    r->phase = P_INIT;
}

// The refinement check at the head of each outer step (the loop head of the
// single-solve refinement driver), on the outer State h.  Returns a status to
// retire with, or NO_OUTCOME to go on (the next phase is set).
int ir_check(ks_server *sv, Req *r, const State &h) {
    r->last_outer = h;
    const double den = h.anorm_inf * h.xinf + h.binf;
    const double eta = den > 0.0 ? h.resinf / den : h.resinf;
    if (!std::isfinite(eta) || (h.flags & F_TRUE_NONFIN)) return KS_NONFINITE;
    if (eta <= r->p.tol) return KS_OK;
    if (r->outer >= r->p.max_outer) return KS_STAGNATED;
    if (eta > 0.5 * r->eta_prev) {
        if (++r->bad >= 2 && r->prec != KS_FP64) {
            r->prec = (r->prec == KS_IR_BF16) ? KS_IR_FP32 : KS_FP64;
            r->bad = 0;
        }
    } else {
        r->bad = 0;
    }
    r->eta_prev = eta;
    const Carved c = carve(r->L, ws_base(sv, r));
    if (r->prec == KS_FP64) {
        to_fp64_tail(r, c);
        return NO_OUTCOME;
    }
    if (r->prec == KS_IR_FP32 && r->p.precision == KS_IR_BF16 && !r->fb_ready) {
        if (launch_convert(r->p.n, r->item.lda, r->item.A, KS_DT_F32, r->L.lda_low, r->A_fb,
                           sv->stream) != hipSuccess)
            return KS_EHIP;
        r->fb_ready = true;
    }
    r->phase = P_IN_INIT;
    return NO_OUTCOME;
}

// After an inner solve: count it, then either promote (breakdown) and check
// again on the same outer State, or take the refinement step.
int ir_after_inner(ks_server *sv, Req *r, int inner_status, int inner_iters) {
    r->total_iters += inner_iters;
    r->outer++;
    if (inner_status == KS_BREAKDOWN || inner_status == KS_NONFINITE) {
        r->prec = (r->prec == KS_IR_BF16) ? KS_IR_FP32 : KS_FP64;
        r->bad = 0;
        r->eta_prev = INFINITY;
        return ir_check(sv, r, r->last_outer);
    }
    r->phase = P_UPDATE;
    return NO_OUTCOME;
}

template <typename TA, typename F1, typename F2>
void build_inner(TableBuilder &tb, InnerSets<TA> &S, const BatchItemT<TA, float> *dev,
                 const std::vector<int> &init, const std::vector<int> &cgb, const std::vector<int> &gmb,
                 const std::vector<int> &gmr, F1 gsh, F2 vsh,
                 const std::vector<int> &cgs_blocks_of) {
    auto one = [](int) { return 1; };
    auto csh = [&](int i) { return cgs_blocks_of[i]; };
    S.init_g = tb.add(dev, init, gsh, &S.n_init_g);
    S.init_1 = tb.add(dev, init, one, &S.n_init_1);
    S.cgb = tb.add(dev, cgb, vsh, &S.n_cgb);
    S.gmb = tb.add(dev, gmb, vsh, &S.n_gmb);
    S.gm_g = tb.add(dev, gmr, gsh, &S.n_gm_g);
    S.gm_c = tb.add(dev, gmr, csh, &S.n_gm_c);
    S.gm_1 = tb.add(dev, gmr, one, &S.n_gm_1);
}

}  // namespace

extern "C" {

int ks_server_create(ks_server **out, size_t mem_budget_bytes, int32_t max_inflight,
                     int32_t chunk, void *stream) {
    if (!out || mem_budget_bytes == 0 || max_inflight < 1 || chunk < 0) return KS_EINVAL;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return KS_EHIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return KS_EDEVICE;
    ks_server *sv = new (std::nothrow) ks_server();
    if (!sv) return KS_ENOMEM;
    sv->stream = (hipStream_t)stream;
    sv->budget = mem_budget_bytes;
    sv->pool.set_budget(mem_budget_bytes);
    sv->max_inflight = max_inflight;
    // an even number of steps per tick: the GMRES step counter alternates
    // between two State fields by step parity and ends each tick in kcur
    sv->chunk = chunk > 0 ? chunk + (chunk & 1) : 16;
    *out = sv;
    return KS_OK;
}

int ks_server_submit(ks_server *sv, const ks_params *p, const double *d_A, const double *d_b,
                     double *d_x, uint64_t *ticket) {
    if (!sv || !p || !d_A || !d_b || !d_x || !ticket) return KS_EINVAL;
    if (!valid_params(p) || p->nrhs != 1 || (p->method != KS_CG && p->method != KS_GMRES) ||
        p->precision > KS_IR_BF16)
        return KS_EINVAL;
    if ((uintptr_t)d_b % 16 || (uintptr_t)d_x % 16) return KS_EINVAL;
    Req *r = new (std::nothrow) Req();
    if (!r) return KS_ENOMEM;
    r->p = *p;
    r->L = make_layout(p);
    // an A whose rows are not 16-byte aligned is copied into the workspace
    r->copy_a = !a_borrowable(d_A, p->lda);
    r->ws_bytes = r->copy_a ? r->L.total : r->L.total_borrowed;
    r->footprint = r->ws_bytes + (size_t)8 * (size_t)p->n * (size_t)p->lda;
    if (r->footprint > sv->budget) {
        delete r;
        return KS_ETOOLARGE;
    }
    r->A = d_A;
    r->b = d_b;
    r->x = d_x;
    r->ticket = sv->next_ticket++;
    r->t_submit = now_ms();
    r->ir = p->precision != KS_FP64;
    r->prec = p->precision;
    sv->queue.push_back(r);
    *ticket = r->ticket;
    return KS_OK;
}

int ks_server_step(ks_server *sv, int32_t *n_inflight, int32_t *n_queued) {
    if (!sv) return KS_EINVAL;
    hipStream_t s = sv->stream;
    // 1. admission, first come first served
    while (!sv->queue.empty()) {
        Req *r = sv->queue.front();
        if (!sched_admits(sv->in_use, r->footprint, sv->budget, (int)sv->inflight.size(), sv->max_inflight))
            break;
        if (!ws_alloc(sv, r)) break;
        sv->in_use += r->footprint;
        char *ws = ws_base(sv, r);
        const Carved c = carve(r->L, ws);
        r->sy = r->L.sy_bytes ? (double *)(ws + r->L.sy_off) : nullptr;
        BatchItem &it = r->item;
        it.A = r->A;
        it.lda = r->p.lda;
        if (r->copy_a) {
            double *Ac = (double *)(ws + r->L.acopy_off);
            if (launch_copy_pad(r->p.n, r->p.lda, r->A, r->L.lda_pad, Ac, s) != hipSuccess)
                return KS_EHIP;
            it.A = Ac;
            it.lda = r->L.lda_pad;
        }
        it.n = r->p.n;
        it.ldv = r->L.ldv;
        it.m = r->L.m;
        it.b = r->b;
        it.x = r->x;
        it.st = c.st;
        it.P = c.P;
        it.ga = c.ga;
        it.sy = r->ir ? nullptr : r->sy;  // a refinement's outer step makes no CG product
        if (!r->ir) {
            it.max_iter = r->p.max_iter;
            it.tol = r->p.tol;
            it.eta = (r->p.flags & KS_FLAG_STOP_BACKWARD) ? 1 : 0;
            if (r->p.method == KS_CG) {
                it.resid = c.v64;
                it.p = c.v64 + r->L.ldv;
                it.q = c.v64 + 2 * (size_t)r->L.ldv;
                it.V = nullptr;
            } else {
                it.resid = c.v64;
                it.V = c.v64 + r->L.ldv;
                it.p = it.q = nullptr;
            }
        } else {
            // the outer step of the refinement: ||b||, r = b - A x in binary64
            it.max_iter = std::max(1, r->p.max_iter);
            it.tol = 1.0;
            it.eta = 0;
            it.resid = c.v64 + (size_t)(r->L.nv64 - 1) * r->L.ldv;
            it.p = it.q = it.V = nullptr;
            r->A_low = ws + r->L.alow_off;
            r->A_fb = r->L.afb_bytes ? (float *)(ws + r->L.afb_off) : nullptr;
            if (launch_convert(r->p.n, it.lda, it.A,
                               r->p.precision == KS_IR_FP32 ? KS_DT_F32 : KS_DT_BF16, r->L.lda_low,
                               r->A_low, s) != hipSuccess)
                return KS_EHIP;
            setup_inner(r, c);
        }
        r->phase = P_INIT;
        sv->inflight.push_back(r);
        sv->queue.pop_front();
    }
    const int nf = (int)sv->inflight.size();
    if (nf == 0) {
        if (n_inflight) *n_inflight = 0;
        if (n_queued) *n_queued = (int32_t)sv->queue.size();
        return KS_OK;
    }
    // 2. subsets of this tick.  Binary64 items: plain solves and refinement
    // outer steps; inner items by storage type (k = 0 binary32, 1 bfloat16).
    // A solve's set-up, its start and its steps run in the same tick (the
    // start kernels take the set-up's own decision, F_SETUP_END); so do a
    // refinement request's outer residual, its refinement check (on the
    // device, IK_DECIDE) and, when the check says go on, the set-up, start
    // and steps of its next inner solve.
    std::vector<int> init, upd, dec, cg_begin, gm_begin, cg_run, gm_run, in_init_all;
    std::vector<int> in_init[2], in_cgb[2], in_gmb[2], in_cg[2], in_gm[2];
    std::vector<char> gated(nf, 0);
    auto tix = [](const Req *r) { return r->prec == KS_IR_BF16 ? 1 : 0; };
    for (int i = 0; i < nf; ++i) {
        const Req *r = sv->inflight[i];
        const bool cg = r->p.method == KS_CG;
        const bool inner_next = r->ir && (r->phase == P_INIT || r->phase == P_UPDATE);
        if (r->phase == P_INIT) init.push_back(i);
        if (r->phase == P_UPDATE) upd.push_back(i);
        if (inner_next) {
            dec.push_back(i);
            gated[i] = 1;
        }
        switch (r->phase) {
            case P_INIT:
                if (r->ir) break;  // the inner solve below
                // fall through: binary64 set-up, start and steps
            case P_BEGIN:
                (cg ? cg_begin : gm_begin).push_back(i);
                (cg ? cg_run : gm_run).push_back(i);
                break;
            case P_RUN: (cg ? cg_run : gm_run).push_back(i); break;
            default: break;
        }
        if (inner_next || r->phase == P_IN_INIT) {
            in_init[tix(r)].push_back(i);
            in_init_all.push_back(i);
        }
        if (inner_next || r->phase == P_IN_INIT || r->phase == P_IN_BEGIN) {
            (cg ? in_cgb : in_gmb)[tix(r)].push_back(i);
            (cg ? in_cg : in_gm)[tix(r)].push_back(i);
        }
        if (r->phase == P_IN_RUN) (cg ? in_cg : in_gm)[tix(r)].push_back(i);
    }
    size_t need = TableBuilder::array_bytes(sizeof(BatchItem), nf) +
                  TableBuilder::array_bytes(sizeof(BatchItemT<float, float>), nf) +
                  TableBuilder::array_bytes(sizeof(BatchItemT<bf16_t, float>), nf) +
                  TableBuilder::array_bytes(sizeof(IrItem), nf) +
                  TableBuilder::array_bytes(sizeof(State *), 2 * nf);
    need += TableBuilder::set_bytes((int)dec.size());
    need += 2 * TableBuilder::set_bytes((int)init.size()) + 3 * TableBuilder::set_bytes((int)upd.size());
    need += TableBuilder::set_bytes((int)cg_begin.size()) + TableBuilder::set_bytes((int)gm_begin.size());
    need += 2 * TableBuilder::set_bytes((int)cg_run.size()) + 3 * TableBuilder::set_bytes((int)gm_run.size());
    need += TableBuilder::set_bytes((int)in_init_all.size());
    for (int k = 0; k < 2; ++k) {
        need += 2 * TableBuilder::set_bytes((int)in_init[k].size());
        need += TableBuilder::set_bytes((int)in_cgb[k].size()) + TableBuilder::set_bytes((int)in_gmb[k].size());
        need += 3 * TableBuilder::set_bytes((int)in_gm[k].size());
    }
    // the step stages: at most one entry per running item in each; the
    // symmetric products' four sets
    need += 7 * TableBuilder::stage_bytes(nf) + 4 * TableBuilder::set_bytes(nf);
    need += 4096;
    int rc = grow_buffers(sv, need, 2 * (size_t)nf);
    if (rc) return rc;
    TableBuilder tb(sv->htab, sv->dtab);
    const BatchItem *d64;
    const BatchItemT<float, float> *d32;
    const BatchItemT<bf16_t, float> *d16;
    const IrItem *dir;
    const State *const *dptrs;
    BatchItem *h64 = tb.array<BatchItem>(nf, &d64);
    BatchItemT<float, float> *h32 = tb.array<BatchItemT<float, float>>(nf, &d32);
    BatchItemT<bf16_t, float> *h16 = tb.array<BatchItemT<bf16_t, float>>(nf, &d16);
    IrItem *hir = tb.array<IrItem>(nf, &dir);
    const State **hptrs = tb.array<const State *>(2 * nf, &dptrs);
    std::vector<int> cgsb(nf);
    for (int i = 0; i < nf; ++i) {
        const Req *r = sv->inflight[i];
        h64[i] = r->item;
        h64[i].outer = nullptr;
        h32[i] = r->in32;
        h16[i] = r->in16;
        h32[i].outer = h16[i].outer = gated[i] ? r->item.st : nullptr;
        hir[i] = r->iri;
        if (r->ir) {
            hir[i].inner = r->in32.st;
            hir[i].tol = r->p.tol;
            hir[i].eta_prev = r->eta_prev;
            hir[i].outer_steps = r->outer;
            hir[i].max_outer = r->p.max_outer;
            hir[i].bad = r->bad;
            hir[i].prec = r->prec;
            hir[i].first = r->phase == P_INIT;
            hir[i].gated = gated[i];
        }
        cgsb[i] = cgs_blocks(r->p.n);
        // the States the host's next decisions read: the outer (or only)
        // one and the inner one
        hptrs[2 * i] = r->item.st;
        hptrs[2 * i + 1] = r->ir ? r->in32.st : r->item.st;
    }
    auto n_of = [&](int i) { return sv->inflight[i]->p.n; };
    auto g64 = [&](int i) { return gemv_blocks<double>(n_of(i)); };
    auto g32 = [&](int i) { return gemv_blocks<float>(n_of(i)); };
    auto g16 = [&](int i) { return gemv_blocks<bf16_t>(n_of(i)); };
    auto vsh = [&](int i) { return vec_blocks(n_of(i)); };
    auto csh = [&](int i) { return cgsb[i]; };
    auto one = [](int) { return 1; };
    int nb_init_g, nb_init_1, nb_upd_v, nb_upd_g, nb_upd_1, nb_cgb, nb_gmb, nb_cg_g, nb_cg_1, nb_gm_g,
        nb_gm_c, nb_gm_1, nb_in_v;
    const BatchSet s_init_g = tb.add(d64, init, g64, &nb_init_g);
    const BatchSet s_init_1 = tb.add(d64, init, one, &nb_init_1);
    const IrSet s_upd_v = tb.add(dir, upd, vsh, &nb_upd_v);
    const BatchSet s_upd_g = tb.add(d64, upd, g64, &nb_upd_g);
    const BatchSet s_upd_1 = tb.add(d64, upd, one, &nb_upd_1);
    const BatchSet s_cgb = tb.add(d64, cg_begin, vsh, &nb_cgb);
    const BatchSet s_gmb = tb.add(d64, gm_begin, vsh, &nb_gmb);
    const BatchSet s_cg_g = tb.add(d64, cg_run, g64, &nb_cg_g);
    const BatchSet s_cg_1 = tb.add(d64, cg_run, one, &nb_cg_1);
    const BatchSet s_gm_g = tb.add(d64, gm_run, g64, &nb_gm_g);
    const BatchSet s_gm_c = tb.add(d64, gm_run, csh, &nb_gm_c);
    const BatchSet s_gm_1 = tb.add(d64, gm_run, one, &nb_gm_1);
    const IrSet s_in_v = tb.add(dir, in_init_all, vsh, &nb_in_v);
    int nb_dec;
    const IrSet s_dec = tb.add(dir, dec, one, &nb_dec);
    InnerSets<float> S32;
    InnerSets<bf16_t> S16;
    build_inner(tb, S32, d32, in_init[0], in_cgb[0], in_gmb[0], in_gm[0], g32, vsh, cgsb);
    build_inner(tb, S16, d16, in_init[1], in_cgb[1], in_gmb[1], in_gm[1], g16, vsh, cgsb);
    // the step stages (one launch per stage position for the CG and GMRES
    // items of every storage type; the products one launch per storage)
    std::vector<std::pair<int, int>> e1[3], e2, e3, e4, e5;
    // CG on the lower triangle (binary64 solves, binary32 inner solves):
    // product and update in the batched symmetric launches, p update in stage 3
    std::vector<int> sy64, sy32;
    auto add_cg = [&](const std::vector<int> &v, int dt) {
        for (int i : v) {
            const Req *r = sv->inflight[i];
            const bool sym = (dt == 0 && r->item.sy) || (dt == 1 && r->in32.sy);
            if (sym) {
                (dt == 0 ? sy64 : sy32).push_back(i);
                e3.push_back({i, SK_SY_PUPDATE | dt << 8});
                continue;
            }
            e1[dt].push_back({i, SK_CG_MATVEC | dt << 8});
            e2.push_back({i, SK_CG_UPDATE | dt << 8});
            e3.push_back({i, SK_CG_PUPDATE | dt << 8});
        }
    };
    auto add_gm = [&](const std::vector<int> &v, int dt) {
        for (int i : v) {
            e1[dt].push_back({i, SK_GM_MATVEC | dt << 8});
            e2.push_back({i, SK_GM_CGS0 | dt << 8});
            e3.push_back({i, SK_GM_CGS1 | dt << 8});
            e4.push_back({i, SK_GM_CGS2 | dt << 8});
            e5.push_back({i, SK_GM_GIVENS | dt << 8});
        }
    };
    add_cg(cg_run, 0);
    add_cg(in_cg[0], 1);
    add_cg(in_cg[1], 2);
    add_gm(gm_run, 0);
    add_gm(in_gm[0], 1);
    add_gm(in_gm[1], 2);
    auto stage_blocks = [&](int i, int kind) {
        const int sk = kind & 255, dt = kind >> 8;
        if (sk == SK_CG_MATVEC || sk == SK_GM_MATVEC)
            return dt == 0 ? g64(i) : dt == 1 ? g32(i) : g16(i);
        if (sk == SK_GM_CGS0 || sk == SK_GM_CGS1 || sk == SK_GM_CGS2) return cgsb[i];
        return vec_blocks(n_of(i));
    };
    StageSet ss1[3];
    int nb1[3], nb2, nb3, nb4, nb5;
    for (int k = 0; k < 3; ++k) ss1[k] = tb.stage(d64, d32, d16, e1[k], stage_blocks, &nb1[k]);
    const StageSet ss2 = tb.stage(d64, d32, d16, e2, stage_blocks, &nb2);
    const StageSet ss3 = tb.stage(d64, d32, d16, e3, stage_blocks, &nb3);
    const StageSet ss4 = tb.stage(d64, d32, d16, e4, stage_blocks, &nb4);
    const StageSet ss5 = tb.stage(d64, d32, d16, e5, stage_blocks, &nb5);
    auto tiles_of = [&](int i) { return sy_tiles(n_of(i)); };
    auto fin_of = [&](int i) { return symv_finish_blocks(n_of(i)); };
    int nb_sy64t, nb_sy64f, nb_sy32t, nb_sy32f;
    const BatchSet s_sy64t = tb.add(d64, sy64, tiles_of, &nb_sy64t);
    const BatchSet s_sy64f = tb.add(d64, sy64, fin_of, &nb_sy64f);
    const BatchSetT<BatchItemT<float, float>> s_sy32t = tb.add(d32, sy32, tiles_of, &nb_sy32t);
    const BatchSetT<BatchItemT<float, float>> s_sy32f = tb.add(d32, sy32, fin_of, &nb_sy32f);
    if (tb.bytes() > sv->tab_cap) return KS_ENOMEM;
    if (hipMemcpyAsync(sv->dtab, sv->htab, tb.bytes(), hipMemcpyHostToDevice, s) != hipSuccess)
        return KS_EHIP;
#define BL(kind, set, nb, gate)                                                             \
    do {                                                                                    \
        if (batch_launch(kind, set, nb, gate, s, sv->dstage) != hipSuccess) return KS_EHIP; \
    } while (0)
#define IL(kind, set, nb)                                                    \
    do {                                                                     \
        if (ir_batch_launch(kind, set, nb, s) != hipSuccess) return KS_EHIP; \
    } while (0)
    // set-up of the newly admitted solves (and of a binary64 finish after promotion)
    BL(BK_NORM_INF, s_init_g, nb_init_g, 0);
    BL(BK_NORM_INF_FINISH, s_init_1, nb_init_1, 0);
    BL(BK_VEC_STATS, s_init_1, nb_init_1, 0);
    BL(BK_RESIDUAL, s_init_g, nb_init_g, 0);
    BL(BK_RESIDUAL_FINISH, s_init_1, nb_init_1, 0);
    // refinement steps: x += ||r|| d, then the binary64 residual
    IL(IK_UPDATE, s_upd_v, nb_upd_v);
    BL(BK_RESIDUAL, s_upd_g, nb_upd_g, 0);
    BL(BK_RESIDUAL_FINISH, s_upd_1, nb_upd_1, 0);
    // the refinement check on the new outer residual (device)
    IL(IK_DECIDE, s_dec, nb_dec);
    // inner set-up: rhs = r / ||r||, d = 0, ||rhs||, r_in = rhs - A_low d
    IL(IK_SCALE, s_in_v, nb_in_v);
    IL(IK_ZERO_D, s_in_v, nb_in_v);
    BL(BK_VEC_STATS, S32.init_1, S32.n_init_1, 0);
    BL(BK_RESIDUAL, S32.init_g, S32.n_init_g, 0);
    BL(BK_RESIDUAL_FINISH, S32.init_1, S32.n_init_1, 0);
    BL(BK_VEC_STATS, S16.init_1, S16.n_init_1, 0);
    BL(BK_RESIDUAL, S16.init_g, S16.n_init_g, 0);
    BL(BK_RESIDUAL_FINISH, S16.init_1, S16.n_init_1, 0);
    // (re)starts, new GMRES cycles and the starts after a set-up
    BL(BK_CG_BEGIN, s_cgb, nb_cgb, 0);
    BL(BK_GM_BEGIN, s_gmb, nb_gmb, 0);
    BL(BK_CG_BEGIN, S32.cgb, S32.n_cgb, 0);
    BL(BK_GM_BEGIN, S32.gmb, S32.n_gmb, 0);
    BL(BK_CG_BEGIN, S16.cgb, S16.n_cgb, 0);
    BL(BK_GM_BEGIN, S16.gmb, S16.n_gmb, 0);
    // iterations of every running solve: per step, the products (one launch
    // per storage), then the four stages of the updates and Gram-Schmidt /
    // Givens work of every CG and GMRES solve
#define SL(set, stage, nb, step)                                                      \
    do {                                                                              \
        if (stage_launch(set, stage, nb, step, s) != hipSuccess) return KS_EHIP;      \
    } while (0)
#define SY(fn, which, set, nb)                                                     \
    do {                                                                           \
        if (fn(which, set, nb, s) != hipSuccess) return KS_EHIP;                    \
    } while (0)
    for (int c = 0; c < sv->chunk; ++c) {
        for (int k = 0; k < 3; ++k) SL(ss1[k], 10 + k, nb1[k], c);
        SY(batch_symv, 0, s_sy64t, nb_sy64t);
        SY(batch_symv32, 0, s_sy32t, nb_sy32t);
        SL(ss2, 2, nb2, c);
        SY(batch_symv, 1, s_sy64f, nb_sy64f);
        SY(batch_symv32, 1, s_sy32f, nb_sy32f);
        SL(ss3, 3, nb3, c);
        SL(ss4, 4, nb4, c);
        SL(ss5, 5, nb5, c);
    }
#undef SL
#undef SY
    // true residual of stopped binary64 CG solves (an inner CG stops on its
    // recursive residual alone); end of finished GMRES cycles
    BL(BK_RESIDUAL, s_cg_g, nb_cg_g, 1);
    BL(BK_RESIDUAL_FINISH, s_cg_1, nb_cg_1, 1);
    BL(BK_GM_FINISH, s_gm_c, nb_gm_c, 3);
    BL(BK_RESIDUAL, s_gm_g, nb_gm_g, 3);
    BL(BK_RESIDUAL_FINISH, s_gm_1, nb_gm_1, 3);
    BL(BK_GM_FINISH, S32.gm_c, S32.n_gm_c, 3);
    BL(BK_RESIDUAL, S32.gm_g, S32.n_gm_g, 3);
    BL(BK_RESIDUAL_FINISH, S32.gm_1, S32.n_gm_1, 3);
    BL(BK_GM_FINISH, S16.gm_c, S16.n_gm_c, 3);
    BL(BK_RESIDUAL, S16.gm_g, S16.n_gm_g, 3);
    BL(BK_RESIDUAL_FINISH, S16.gm_1, S16.n_gm_1, 3);
#undef BL
#undef IL
    if (gather_states(dptrs, 2 * nf, sv->dstage, s) != hipSuccess) return KS_EHIP;
    if (hipMemcpyAsync(sv->hstage, sv->dstage, 2 * (size_t)nf * sizeof(State), hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return KS_EHIP;
    // 3. decisions, as in the single-solve drivers: ho is a request's outer
    // (or only) State, hi its inner solve's
    std::vector<Req *> keep;
    keep.reserve(nf);
    bool zero_fill = false;
    for (int i = 0; i < nf; ++i) {
        Req *r = sv->inflight[i];
        const State &ho = sv->hstage[2 * i], &hi = sv->hstage[2 * i + 1];
        const bool cg = r->p.method == KS_CG;
        const Phase ph = r->phase;
        int done = NO_OUTCOME;
        State out = ho;  // the binary64 State the outcome is read from
        int iters = ho.iters;
        // the inner solve after its set-up and the steps of this tick: the
        // loop head of the single-solve drivers when the set-up ended it,
        // else the end of its pass (or of a GMRES cycle)
        auto inner_after = [&]() -> int {
            const int f = hi.flags;
            int st_in = NO_OUTCOME;
            if (f & F_SETUP_END) {
                if (hi.bnorm == 0.0)
                    st_in = KS_OK;
                else if (f & F_TRUE_NONFIN)
                    st_in = KS_NONFINITE;
                else if (f & F_TRUE_OK)
                    st_in = KS_OK;
                else
                    st_in = KS_MAXITER;
            } else {
                const bool ended = cg ? (f & F_STOP) != 0 : ((f & F_STOP) != 0 || hi.kcur >= r->L.m);
                if (!ended) {
                    r->phase = P_IN_RUN;
                } else if (cg) {
                    if (f & F_BREAK)
                        st_in = KS_BREAKDOWN;
                    else if (f & F_NONFIN)
                        st_in = KS_NONFINITE;
                    else
                        st_in = (f & F_CONV) ? KS_OK : KS_MAXITER;
                } else {
                    if (f & F_BREAK)
                        st_in = KS_BREAKDOWN;
                    else if ((f & F_NONFIN) || (f & F_TRUE_NONFIN))
                        st_in = KS_NONFINITE;
                    else if (f & F_TRUE_OK)
                        st_in = KS_OK;
                    else if (hi.iters >= r->p.max_iter)
                        st_in = KS_MAXITER;
                    else
                        r->phase = P_IN_BEGIN;  // next cycle of the inner GMRES
                }
            }
            return st_in != NO_OUTCOME ? ir_after_inner(sv, r, st_in, hi.iters) : NO_OUTCOME;
        };
        if (r->ir && (ph == P_INIT || ph == P_UPDATE)) {
            // the refinement check on the new outer residual ran on the
            // device; the host repeats it (same arithmetic) to keep its
            // counters, and the two must agree
            if (ph == P_INIT && ho.bnorm == 0.0) {
                if (ho.ir_next != IR_ZERO) return KS_EHIP;
                if (launch_fill<double>(r->p.n, r->x, 0.0, s) != hipSuccess) return KS_EHIP;
                zero_fill = true;
                r->last_outer = ho;
                r->last_outer.res = r->last_outer.resinf = 0.0;
                done = KS_OK;
            } else {
                const int prec0 = r->prec;
                done = ir_check(sv, r, ho);
                if (done == KS_EHIP) return KS_EHIP;
                const bool go = done == NO_OUTCOME && r->prec == prec0 && r->phase == P_IN_INIT;
                if (go != (ho.ir_next == IR_GO)) return KS_EHIP;
                // on go, the inner set-up, start and steps ran in this tick
                if (go) done = inner_after();
            }
            if (done == KS_EHIP) return KS_EHIP;
            out = r->last_outer;
            iters = r->total_iters;
        } else if (ph == P_IN_INIT || ph == P_IN_BEGIN || ph == P_IN_RUN) {
            done = inner_after();
            if (done == KS_EHIP) return KS_EHIP;
            out = r->last_outer;
            iters = r->total_iters;
        } else if (ph == P_INIT && (ho.flags & F_SETUP_END)) {
            // binary64 set-up that ended the solve (the drivers' loop head)
            const int f = ho.flags;
            if (ho.bnorm == 0.0) {
                if (launch_fill<double>(r->p.n, r->x, 0.0, s) != hipSuccess) return KS_EHIP;
                zero_fill = true;
                out.res = out.resinf = 0.0;
                done = KS_OK;
            } else if (f & F_TRUE_NONFIN) {
                done = KS_NONFINITE;
            } else if (f & F_TRUE_OK) {
                done = KS_OK;
            } else {
                done = KS_MAXITER;
            }
        } else {
            // a binary64 solve's steps (after its set-up, a restart or a new cycle)
            const int f = ho.flags;
            const bool ended = cg ? (f & F_STOP) != 0 : ((f & F_STOP) != 0 || ho.kcur >= r->L.m);
            if (!ended) {
                r->phase = P_RUN;
            } else {
                if (!cg) r->cycles++;
                if (f & F_BREAK)
                    done = KS_BREAKDOWN;
                else if ((f & F_NONFIN) || (f & F_TRUE_NONFIN))
                    done = KS_NONFINITE;
                else if (f & F_TRUE_OK)
                    done = KS_OK;
                else if (ho.iters >= r->item.max_iter)
                    done = KS_MAXITER;
                else if (cg && r->restarts >= SERVER_CG_MAX_RESTARTS)
                    done = KS_STAGNATED;
                else {
                    if (cg) r->restarts++;
                    r->phase = P_BEGIN;
                }
            }
        }
        if (done != NO_OUTCOME && r->fp64_tail) {
            // binary64 finish of a refinement request: one more outer step;
            // success is decided on the backward error of the result
            r->outer++;
            iters = r->total_iters + ho.iters;
            finish_metrics(r, ho);
            if (r->info.backward_err <= r->p.tol) done = KS_OK;
        }
        if (done != NO_OUTCOME) {
            retire(sv, r, out, done, iters);
        } else {
            keep.push_back(r);
        }
    }
    if (zero_fill && hipStreamSynchronize(s) != hipSuccess) return KS_EHIP;
    sv->inflight.swap(keep);
    if (n_inflight) *n_inflight = (int32_t)sv->inflight.size();
    if (n_queued) *n_queued = (int32_t)sv->queue.size();
    return KS_OK;
}

int ks_server_poll(ks_server *sv, uint64_t *tickets, ks_info *infos, int32_t cap, int32_t *n_done) {
    if (!sv || !n_done || cap < 0 || (cap > 0 && (!tickets || !infos))) return KS_EINVAL;
    const int k = std::min<int>(cap, (int)sv->finished.size());
    for (int i = 0; i < k; ++i) {
        tickets[i] = sv->finished[i]->ticket;
        infos[i] = sv->finished[i]->info;
        delete sv->finished[i];
    }
    sv->finished.erase(sv->finished.begin(), sv->finished.begin() + k);
    *n_done = k;
    return KS_OK;
}

int ks_server_stats(const ks_server *sv, size_t *bytes_in_use, int32_t *n_inflight,
                    int32_t *n_queued) {
    if (!sv) return KS_EINVAL;
    if (bytes_in_use) *bytes_in_use = sv->in_use;
    if (n_inflight) *n_inflight = (int32_t)sv->inflight.size();
    if (n_queued) *n_queued = (int32_t)sv->queue.size();
    return KS_OK;
}

void ks_server_free(ks_server *sv) {
    if (!sv) return;
    (void)hipStreamSynchronize(sv->stream);
    for (Req *r : sv->queue) delete r;
    for (Req *r : sv->inflight) delete r;
    for (Req *r : sv->finished) delete r;
    for (const SchedSegment &sg : sv->pool.segments()) (void)hipFree(sg.base);
    if (sv->dtab) (void)hipFree(sv->dtab);
    if (sv->htab) (void)hipHostFree(sv->htab);
    if (sv->dstage) (void)hipFree(sv->dstage);
    if (sv->hstage) (void)hipHostFree(sv->hstage);
    delete sv;
}

}  // extern "C"
