// Request server: continuous batching of many binary64 CG / GMRES(m) solves.
//
// Requests are queued in arrival order and admitted while the memory budget
// (resident A plus the solve's workspace) and the slot count allow; the queue
// is served first come, first served (no request overtakes an earlier one).
// Each call of ks_server_step is one tick:
//   1. admit from the queue;
//   2. one batched launch per phase advances every in-flight solve: set-up of
//      the new ones (||A||_inf, ||b||, r0), (re)starts, then `chunk`
//      iterations of every CG solve and `chunk` Arnoldi steps of every GMRES
//      solve, the gated true residuals and the GMRES cycle ends;
//   3. one gather kernel and one copy bring every solve's State to the host,
//      which decides per request (continue, restart, new cycle, done) exactly
//      as the single-solve drivers do, retires finished requests (latency =
//      completion - submission) and frees their memory.
// Requests that arrive while others run join at the next tick, so their work
// overlaps on the device with the solves already in flight.  A solve's result
// does not depend on what else is batched with it: every block of a batched
// launch runs the same device body on the same data, in the same order, as
// the single-solve kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "ks.h"
#include "ks_internal.h"
#include "ks_layout.h"

using namespace ks;

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over a device arena, in 256-byte units, with
// coalescing of neighbouring free ranges.
class Arena {
   public:
    void init(size_t size) {
        free_.clear();
        free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rem = it->second - bytes, noff = it->first + bytes;
                free_.erase(it);
                if (rem) free_[noff] = rem;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

   private:
    std::map<size_t, size_t> free_;
};

enum Phase { P_QUEUED, P_INIT, P_BEGIN, P_RUN, P_DONE };

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
    bool copy_a = false;
    int restarts = 0, cycles = 0;
    BatchItem item{};
    ks_info info{};
};

constexpr int SERVER_CG_MAX_RESTARTS = 16;

}  // namespace

struct ks_server {
    hipStream_t stream = nullptr;
    size_t budget = 0, in_use = 0;
    int max_inflight = 0;
    int chunk = 16;
    char *arena_dev = nullptr;
    size_t arena_bytes = 0;
    Arena arena;
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

// Builds the per-tick table in pinned host memory: the items, then for every
// (subset, block shape) an index array and a prefix-sum array of block counts.
class TableBuilder {
   public:
    TableBuilder(char *host, char *dev) : host_(host), dev_(dev) {}
    size_t reserve_items(int count) {
        items_off_ = off_;
        off_ += align_up(sizeof(BatchItem) * (size_t)std::max(count, 1));
        return items_off_;
    }
    BatchItem *items() { return reinterpret_cast<BatchItem *>(host_ + items_off_); }
    // sizes only (first pass)
    static size_t set_bytes(int count) { return 2 * align_up(sizeof(int) * (size_t)(count + 1)); }
    template <typename F>
    BatchSet add(const std::vector<int> &idx, F blocks_of, int *total) {
        BatchSet bs{};
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
        bs.items = reinterpret_cast<const BatchItem *>(dev_ + items_off_);
        bs.count = c;
        *total = acc;
        return bs;
    }
    size_t bytes() const { return off_; }

   private:
    char *host_, *dev_;
    size_t off_ = 0, items_off_ = 0;
};

void retire(ks_server *sv, Req *r, const State &h, int status) {
    r->info.status = status;
    r->info.iters = h.iters;
    r->info.restarts = r->p.method == KS_CG ? r->restarts : std::max(0, r->cycles - 1);
    if (h.bnorm > 0.0 && std::isfinite(h.bnorm)) {
        const double den = h.anorm_inf * h.xinf + h.binf;
        r->info.rel_res = h.res / h.bnorm;
        r->info.backward_err = den > 0.0 ? h.resinf / den : h.resinf;
    } else {
        r->info.rel_res = 0.0;
        r->info.backward_err = 0.0;
    }
    r->info.elapsed_ms = now_ms() - r->t_submit;
    r->info.precision_used = KS_FP64;
    r->phase = P_DONE;
    sv->arena.release(r->ws_off, r->ws_bytes);
    sv->in_use -= r->footprint;
    sv->finished.push_back(r);
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
    sv->max_inflight = max_inflight;
    sv->chunk = chunk > 0 ? chunk : 16;
    // workspaces only (A stays where the caller keeps it): a fraction of the budget
    sv->arena_bytes = align_up(std::min<size_t>(mem_budget_bytes, (size_t)4 << 30));
    if (hipMalloc((void **)&sv->arena_dev, sv->arena_bytes) != hipSuccess) {
        delete sv;
        return KS_ENOMEM;
    }
    sv->arena.init(sv->arena_bytes);
    *out = sv;
    return KS_OK;
}

int ks_server_submit(ks_server *sv, const ks_params *p, const double *d_A, const double *d_b,
                     double *d_x, uint64_t *ticket) {
    if (!sv || !p || !d_A || !d_b || !d_x || !ticket) return KS_EINVAL;
    if (!valid_params(p) || p->precision != KS_FP64 || p->nrhs != 1 || p->method == KS_BICGSTAB)
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
    if (r->footprint > sv->budget || align_up(r->ws_bytes) > sv->arena_bytes) {
        delete r;
        return KS_ETOOLARGE;
    }
    r->A = d_A;
    r->b = d_b;
    r->x = d_x;
    r->ticket = sv->next_ticket++;
    r->t_submit = now_ms();
    sv->queue.push_back(r);
    *ticket = r->ticket;
    return KS_OK;
}

int ks_server_step(ks_server *sv, int32_t *n_inflight, int32_t *n_queued) {
    if (!sv) return KS_EINVAL;
    // 1. admission, first come first served
    while (!sv->queue.empty() && (int)sv->inflight.size() < sv->max_inflight) {
        Req *r = sv->queue.front();
        if (sv->in_use + r->footprint > sv->budget) break;
        size_t off = 0;
        if (!sv->arena.alloc(r->ws_bytes, &off)) break;
        r->ws_off = off;
        sv->in_use += r->footprint;
        const Carved c = carve(r->L, sv->arena_dev + off);
        BatchItem &it = r->item;
        it.A = r->A;
        it.lda = r->p.lda;
        if (r->copy_a) {
            double *Ac = (double *)(sv->arena_dev + off + r->L.acopy_off);
            if (launch_copy_pad(r->p.n, r->p.lda, r->A, r->L.lda_pad, Ac, sv->stream) != hipSuccess)
                return KS_EHIP;
            it.A = Ac;
            it.lda = r->L.lda_pad;
        }
        it.n = r->p.n;
        it.ldv = r->L.ldv;
        it.m = r->L.m;
        it.max_iter = r->p.max_iter;
        it.tol = r->p.tol;
        it.eta = (r->p.flags & KS_FLAG_STOP_BACKWARD) ? 1 : 0;
        it.b = r->b;
        it.x = r->x;
        it.st = c.st;
        it.P = c.P;
        it.ga = c.ga;
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
    // 2. subsets of this tick
    std::vector<int> init, cg_begin, gm_begin, cg_run, gm_run, all(nf);
    for (int i = 0; i < nf; ++i) {
        const Req *r = sv->inflight[i];
        all[i] = i;
        const bool cg = r->p.method == KS_CG;
        if (r->phase == P_INIT) init.push_back(i);
        if (r->phase == P_BEGIN) (cg ? cg_begin : gm_begin).push_back(i);
        if (r->phase == P_BEGIN || r->phase == P_RUN) (cg ? cg_run : gm_run).push_back(i);
    }
    size_t need = align_up(sizeof(BatchItem) * (size_t)nf);
    need += 4 * TableBuilder::set_bytes((int)init.size());
    need += TableBuilder::set_bytes((int)cg_begin.size()) + TableBuilder::set_bytes((int)gm_begin.size());
    need += 4 * TableBuilder::set_bytes((int)cg_run.size()) + 5 * TableBuilder::set_bytes((int)gm_run.size());
    need += TableBuilder::set_bytes(nf) + 4096;
    int rc = grow_buffers(sv, need, (size_t)nf);
    if (rc) return rc;
    TableBuilder tb(sv->htab, sv->dtab);
    tb.reserve_items(nf);
    for (int i = 0; i < nf; ++i) tb.items()[i] = sv->inflight[i]->item;
    auto n_of = [&](int i) { return sv->inflight[i]->p.n; };
    auto gemv_sh = [&](int i) { return gemv_blocks<double>(n_of(i)); };
    auto vec_sh = [&](int i) { return vec_blocks(n_of(i)); };
    auto cgs_sh = [&](int i) { return cgs_blocks(n_of(i)); };
    auto one_sh = [&](int) { return 1; };
    int nb_init_g, nb_init_1, nb_cgb, nb_gmb, nb_cg_g, nb_cg_v, nb_cg_1, nb_gm_g, nb_gm_c, nb_gm_v,
        nb_gm_1, nb_all;
    const BatchSet s_init_g = tb.add(init, gemv_sh, &nb_init_g);
    const BatchSet s_init_1 = tb.add(init, one_sh, &nb_init_1);
    const BatchSet s_cgb = tb.add(cg_begin, vec_sh, &nb_cgb);
    const BatchSet s_gmb = tb.add(gm_begin, vec_sh, &nb_gmb);
    const BatchSet s_cg_g = tb.add(cg_run, gemv_sh, &nb_cg_g);
    const BatchSet s_cg_v = tb.add(cg_run, vec_sh, &nb_cg_v);
    const BatchSet s_cg_1 = tb.add(cg_run, one_sh, &nb_cg_1);
    const BatchSet s_gm_g = tb.add(gm_run, gemv_sh, &nb_gm_g);
    const BatchSet s_gm_c = tb.add(gm_run, cgs_sh, &nb_gm_c);
    const BatchSet s_gm_v = tb.add(gm_run, vec_sh, &nb_gm_v);
    const BatchSet s_gm_1 = tb.add(gm_run, one_sh, &nb_gm_1);
    const BatchSet s_all = tb.add(all, one_sh, &nb_all);
    hipStream_t s = sv->stream;
    if (hipMemcpyAsync(sv->dtab, sv->htab, tb.bytes(), hipMemcpyHostToDevice, s) != hipSuccess)
        return KS_EHIP;
#define BL(kind, set, nb, gate)                                                       \
    do {                                                                              \
        if (batch_launch(kind, set, nb, gate, s, sv->dstage) != hipSuccess) return KS_EHIP; \
    } while (0)
    // set-up of the newly admitted solves
    BL(BK_NORM_INF, s_init_g, nb_init_g, 0);
    BL(BK_NORM_INF_FINISH, s_init_1, nb_init_1, 0);
    BL(BK_VEC_STATS, s_init_1, nb_init_1, 0);
    BL(BK_RESIDUAL, s_init_g, nb_init_g, 0);
    BL(BK_RESIDUAL_FINISH, s_init_1, nb_init_1, 0);
    // (re)starts and new GMRES cycles
    BL(BK_CG_BEGIN, s_cgb, nb_cgb, 0);
    BL(BK_GM_BEGIN, s_gmb, nb_gmb, 0);
    // iterations of every running solve
    for (int c = 0; c < sv->chunk; ++c) {
        BL(BK_CG_MATVEC, s_cg_g, nb_cg_g, 0);
        BL(BK_CG_UPDATE, s_cg_v, nb_cg_v, 0);
        BL(BK_CG_PUPDATE, s_cg_v, nb_cg_v, 0);
        BL(BK_GM_MATVEC, s_gm_g, nb_gm_g, 0);
        BL(BK_GM_CGS0, s_gm_c, nb_gm_c, 0);
        BL(BK_GM_CGS1, s_gm_c, nb_gm_c, 0);
        BL(BK_GM_CGS2, s_gm_c, nb_gm_c, 0);
        BL(BK_GM_GIVENS, s_gm_v, nb_gm_v, 0);
        BL(BK_GM_ADVANCE, s_gm_1, nb_gm_1, 0);
    }
    // true residual of stopped CG solves; end of finished GMRES cycles
    BL(BK_RESIDUAL, s_cg_g, nb_cg_g, 1);
    BL(BK_RESIDUAL_FINISH, s_cg_1, nb_cg_1, 1);
    BL(BK_GM_FINISH, s_gm_c, nb_gm_c, 3);
    BL(BK_RESIDUAL, s_gm_g, nb_gm_g, 3);
    BL(BK_RESIDUAL_FINISH, s_gm_1, nb_gm_1, 3);
    BL(BK_GATHER, s_all, nb_all, 0);
#undef BL
    if (hipMemcpyAsync(sv->hstage, sv->dstage, (size_t)nf * sizeof(State), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return KS_EHIP;
    // 3. decisions, as in the single-solve drivers
    std::vector<Req *> keep;
    keep.reserve(nf);
    bool zero_fill = false;
    for (int i = 0; i < nf; ++i) {
        Req *r = sv->inflight[i];
        const State &h = sv->hstage[i];
        const int f = h.flags;
        const bool cg = r->p.method == KS_CG;
        int done = -100;
        if (r->phase == P_INIT) {
            if (h.bnorm == 0.0) {
                if (launch_fill<double>(r->p.n, r->x, 0.0, sv->stream) != hipSuccess) return KS_EHIP;
                zero_fill = true;
                done = KS_OK;
            } else if (f & F_TRUE_NONFIN) {
                done = KS_NONFINITE;
            } else if (f & F_TRUE_OK) {
                done = KS_OK;
            } else if (h.iters >= r->p.max_iter) {
                done = KS_MAXITER;
            } else {
                r->phase = P_BEGIN;
            }
        } else {
            const bool ended = cg ? (f & F_STOP) != 0 : ((f & F_STOP) != 0 || h.kcur >= r->L.m);
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
                else if (h.iters >= r->p.max_iter)
                    done = KS_MAXITER;
                else if (cg && r->restarts >= SERVER_CG_MAX_RESTARTS)
                    done = KS_STAGNATED;
                else {
                    if (cg) r->restarts++;
                    r->phase = P_BEGIN;
                }
            }
        }
        if (done != -100) {
            State hs = h;
            if (r->phase == P_INIT && h.bnorm == 0.0) hs.res = hs.resinf = 0.0;
            retire(sv, r, hs, done);
        } else {
            keep.push_back(r);
        }
    }
    if (zero_fill && hipStreamSynchronize(sv->stream) != hipSuccess) return KS_EHIP;
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
    if (sv->arena_dev) (void)hipFree(sv->arena_dev);
    if (sv->dtab) (void)hipFree(sv->dtab);
    if (sv->htab) (void)hipHostFree(sv->htab);
    if (sv->dstage) (void)hipFree(sv->dstage);
    if (sv->hstage) (void)hipHostFree(sv->hstage);
    delete sv;
}

}  // extern "C"
