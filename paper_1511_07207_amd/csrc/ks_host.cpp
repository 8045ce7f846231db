// Host side of the dense Krylov library: workspace layout, the CG / GMRES(m)
// / iterative-refinement drivers and the C ABI of ks.h.
//
// The drivers follow the host flow of the paper's parallel-implementation
// section (device memory, launch grid, kernels, copy back), with every
// per-iteration scalar kept on the device: the host enqueues a chunk of
// iterations, then reads the 256-byte State once to decide whether to go on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "ks.h"
#include "ks_internal.h"
#include "ks_layout.h"

using namespace ks;

#define HIPCHK(expr)                          \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) return KS_EHIP; \
    } while (0)

struct ks_solver {
    ks_params p{};
    Layout L;
    int n = 0;
    int64_t lda = 0;
    const double *A = nullptr;
    void *A_low = nullptr;
    float *A_fb = nullptr;
    bool fb_ready = false;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    bool own_ws = false;
    State *st = nullptr;     // outer / plain solve
    State *st_in = nullptr;  // IR inner solve
    State *host = nullptr;   // pinned mirror of both
    Partials P{};
    GmArrays ga{};
    double *v64 = nullptr;
    float *v32 = nullptr;
    double *sy = nullptr;     // tile partials of the symmetric product (KS_FLAG_SYMMETRIC)
    bool fz = false;          // fused small-n binary64 CG (one launch per iteration)
    uint32_t *fzbar = nullptr;  // grid-barrier flags of its persistent launch
    // GMRES-IR: the binary32 LU in A_low, its pivots, permutation, and the
    // first zero pivot's column + 1 (0: nonsingular)
    int *lu_piv = nullptr, *lu_perm = nullptr, *lu_info = nullptr;
    // the persistent substitutions' exchange words (null: one launch per
    // 64-row step, KS_FLAG_NO_PERSIST)
    uint64_t *ts_xw = nullptr;
    int lu_sing = 0;
    int chol_notpd = 0;  // CG-IR: 1 + the first column with a non-positive pivot
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> tev;  // timing event pairs of A*v launches
    int tev_used = 0;
    double gemv_ms = 0.0;
    int gemv_calls = 0;
    std::vector<int> tpos;  // position in the polling chunk of each timed launch
    int tchunk_pos = 0;     // launches in the current polling chunk so far
    long long tcall = 0;    // launches so far in this solve (timing sample)
    double anorm_inf = 0.0;
    // multi-right-hand-side
    double *mr64 = nullptr;   // X, R, P, Q, Qpart (binary64)
    float *mr32 = nullptr;    // D, R, P, Q, rhs, Qpart (binary32, IR inner solve)
    ColState *cols = nullptr, *cols_in = nullptr;
    ColState *host_cols = nullptr;
    double *mr_part = nullptr;
    std::vector<ks_info> col_info;

    double *vec64(int i) const { return v64 + (size_t)i * L.ldv; }
    double *mrb64(int i) const { return mr64 + (size_t)i * L.mr_block_elems; }
    float *mrb32(int i) const { return mr32 + (size_t)i * L.mr_block_elems; }
    float *vec32(int i) const { return v32 + (size_t)i * L.ldv; }
    bool timing() const { return (p.flags & KS_FLAG_TIMING) != 0; }
};

namespace {

int check_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KS_EHIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return KS_EHIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return KS_EDEVICE;
    return KS_OK;
}

int sync_state(ks_solver *s) {
    HIPCHK(hipMemcpyAsync(s->host, s->st, 2 * sizeof(State), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    // a persistent kernel's bounded wait gave up (the fused CG, the
    // preconditioner's substitutions): its results are not to be used
    if (s->host[0].sync_fail || s->host[1].sync_fail) return KS_EHIP;
    return KS_OK;
}

// Timing of A*v launches: an event pair around every launch, or around one
// in p.timing_every (counted over the solve); each pair keeps its launch's
// position in the polling chunk, and after the sync only the pairs of the
// chunk's first `real` launches count (the rest returned at once).
int timing_pair(ks_solver *s, hipEvent_t *a, hipEvent_t *b) {
    *a = *b = nullptr;
    if (!s->timing()) return KS_OK;
    const int pos = s->tchunk_pos++;
    const long long call = s->tcall++;
    if (s->p.timing_every > 1 && call % s->p.timing_every != 0) return KS_OK;
    while ((int)s->tev.size() < 2 * (s->tev_used + 1)) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        s->tev.push_back(e);
    }
    if ((int)s->tpos.size() < s->tev_used + 1) s->tpos.resize(s->tev_used + 1);
    s->tpos[s->tev_used] = pos;
    *a = s->tev[2 * s->tev_used];
    *b = s->tev[2 * s->tev_used + 1];
    s->tev_used++;
    return KS_OK;
}

int timed_collect(ks_solver *s, int real) {
    if (!s->timing()) return KS_OK;
    for (int i = 0; i < s->tev_used; ++i) {
        if (s->tpos[i] >= real) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, s->tev[2 * i], s->tev[2 * i + 1]));
        s->gemv_ms += ms;
        s->gemv_calls++;
    }
    s->tev_used = 0;
    s->tchunk_pos = 0;
    return KS_OK;
}

int poll_chunk(const ks_solver *s) {
    if (s->p.poll_every > 0) return s->p.poll_every;
    if (s->n >= 8192) return 8;
    if (s->n >= 2048) return 16;
    return 32;
}

// CG and GMRES: an iteration launched after the stop costs only launches that
// return at once, while a poll costs a host round trip, so the chunk between
// polls is 32 iterations at every n (measured at n = 16384: CG 164.0 ms with
// 8, 162.5 ms with 32, no better beyond; GMRES(30) unchanged)
// polls of one bounded grid-barrier wait of a persistent launch (each a
// memory round trip and a short sleep: about a second in all)
constexpr uint32_t FZ_SPIN_LIMIT = 1u << 20;

int poll_chunk_krylov(const ks_solver *s) {
    return s->p.poll_every > 0 ? s->p.poll_every : 32;
}

struct Outcome {
    int status = KS_OK;
    int iters = 0;
    int restarts = 0;
};

// ------------------------------------------------------------------ CG
// Plain conjugate gradient (binary64 or, as the inner solve, binary32 on a
// low-precision A).  `outer` = true: confirm on the true residual and restart
// from the current x when it fails (binary64 solve); false: one pass, stop on
// the recursive residual (inner solve).
template <typename TA, typename T>
int run_cg(ks_solver *s, State *st, int state_index, const TA *A, int64_t lda, const T *b, T *x,
           T *r, T *p, T *q, double tol, int max_iter, bool outer, Outcome *out, int eta = 0) {
    const int n = s->n;
    hipStream_t sm = s->stream;
    HIPCHK(launch_vec_stats<T>(n, b, tol, st, sm, eta));
    HIPCHK((launch_residual<TA, T>(n, lda, A, b, x, r, st, s->P, 0, sm)));
    int rc = sync_state(s);
    if (rc) return rc;
    const State *h = &s->host[state_index];
    if (h->bnorm == 0.0) {
        HIPCHK(launch_fill<T>(n, x, T(0), sm));
        out->status = KS_OK;
        out->iters = 0;
        return KS_OK;
    }
    int restarts = 0;
    bool first = true;
    for (;;) {
        const int f = h->flags;
        if (f & F_TRUE_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
        if (f & F_TRUE_OK) {
            out->status = KS_OK;
            break;
        }
        if (h->iters >= max_iter) {
            out->status = KS_MAXITER;
            break;
        }
        if (!first) {
            if (restarts >= CG_MAX_RESTARTS) {
                out->status = KS_STAGNATED;
                break;
            }
            ++restarts;
        }
        first = false;
        HIPCHK(launch_cg_begin<T>(n, r, p, st, sm));
        bool done = false;
        // binary64 at small n: one fused launch per iteration (same arithmetic)
        bool fused = false;
        if constexpr (std::is_same<TA, double>::value && std::is_same<T, double>::value)
            fused = s->fz && eta == 0;
        if (fused) {
            if constexpr (std::is_same<TA, double>::value && std::is_same<T, double>::value) {
                const int ng = gemv_blocks<double>(n);
                double *const vec[6] = {r, s->vec64(3), p, s->vec64(4), q, s->vec64(5)};
                double *const pg[2] = {s->P.g, s->P.g + ng};
                HIPCHK(launch_fz_start(n, lda, A, p, q, st, pg[0], sm));
                // n <= fz_persist_max_n(): the iterations up to the stop (or
                // max_iter) in one cooperative launch, grid barriers between them
                const bool persist = n <= fz_persist_max_n() && s->fzbar &&
                                     !(s->p.flags & KS_FLAG_NO_PERSIST);
                int k = 0;
                while (!done) {
                    const int it0 = h->iters;
                    if (persist) {
                        const int steps = std::max(1, max_iter - it0);
                        HIPCHK(launch_fz_persist(n, lda, A, x, vec, st, pg, k & 1, steps, max_iter,
                                                 s->fzbar, FZ_SPIN_LIMIT, sm));
                        k += steps;
                    } else {
                        const int chunk = std::max(1, std::min(poll_chunk_krylov(s), max_iter - it0));
                        for (int c = 0; c < chunk; ++c, ++k) {
                            hipEvent_t e0, e1;
                            if ((rc = timing_pair(s, &e0, &e1))) return rc;
                            if (e0) HIPCHK(hipEventRecord(e0, sm));
                            HIPCHK(launch_fz_step(n, lda, A, x, vec, st, pg, k & 1, max_iter, sm));
                            if (e1) HIPCHK(hipEventRecord(e1, sm));
                        }
                    }
                    HIPCHK(launch_fz_publish(st, k & 1, sm));
                    if (outer) HIPCHK((launch_residual<TA, T>(n, lda, A, b, x, r, st, s->P, 1, sm)));
                    if ((rc = sync_state(s))) return rc;
                    if (h->sync_fail) return KS_EHIP;
                    if ((rc = timed_collect(s, h->iters - it0))) return rc;
                    done = (h->flags & F_STOP) != 0;
                }
            }
        }
        while (!done) {
            const int it0 = h->iters;
            const int chunk = std::max(1, std::min(poll_chunk_krylov(s), max_iter - it0));
            for (int c = 0; c < chunk; ++c) {
                hipEvent_t e0, e1;
                if ((rc = timing_pair(s, &e0, &e1))) return rc;
                if (e0) HIPCHK(hipEventRecord(e0, sm));
                bool symmetric = false;
                if (s->sy) {
                    // product and update in two launches (the timed pair
                    // covers both; the update adds 5 vector passes to A's bytes)
                    if constexpr (std::is_same<TA, double>::value && std::is_same<T, double>::value) {
                        HIPCHK(launch_symv_cg(n, lda, A, p, x, r, s->sy, st, sm));
                        symmetric = true;
                    } else if constexpr (std::is_same<TA, float>::value && std::is_same<T, float>::value) {
                        HIPCHK(launch_symv32_cg(n, lda, A, p, x, r, s->sy, st, sm));
                        symmetric = true;
                    }
                    if (symmetric) {
                        if (e1) HIPCHK(hipEventRecord(e1, sm));
                        HIPCHK(launch_cg_pupdate_from<T>(n, r, p, st, symv_cg_rho_part(n, s->sy),
                                                         symv_finish_blocks(n), max_iter, sm));
                    }
                }
                if (!symmetric) {
                    HIPCHK((launch_cg_matvec<TA, T>(n, lda, A, p, q, st, s->P, sm)));
                    if (e1) HIPCHK(hipEventRecord(e1, sm));
                    HIPCHK(launch_cg_update<T>(n, x, r, p, q, st, s->P, gemv_blocks<TA>(n), sm));
                    HIPCHK(launch_cg_pupdate<T>(n, r, p, st, s->P, max_iter, sm));
                }
            }
            if (outer) HIPCHK((launch_residual<TA, T>(n, lda, A, b, x, r, st, s->P, 1, sm)));
            if ((rc = sync_state(s))) return rc;
            if ((rc = timed_collect(s, h->iters - it0))) return rc;
            done = (h->flags & F_STOP) != 0;
        }
        const int f2 = h->flags;
        if (f2 & F_BREAK) {
            out->status = KS_BREAKDOWN;
            break;
        }
        if (f2 & F_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
        if (!outer) {
            out->status = (f2 & F_CONV) ? KS_OK : KS_MAXITER;
            break;
        }
        // F_CONV or F_MAXIT: the gated residual kernel has refreshed F_TRUE_OK
    }
    out->iters = h->iters;
    out->restarts = restarts;
    return KS_OK;
}

// ---------------------------------------------------------------- GMRES
template <typename TA, typename T>
int run_gmres(ks_solver *s, State *st, int state_index, const TA *A, int64_t lda, const T *b,
              T *x, T *w, T *V, double tol, int max_iter, Outcome *out, int eta = 0) {
    const int n = s->n, m = s->ga.m, ldv = s->L.ldv;
    hipStream_t sm = s->stream;
    HIPCHK(launch_vec_stats<T>(n, b, tol, st, sm, eta));
    HIPCHK((launch_residual<TA, T>(n, lda, A, b, x, w, st, s->P, 0, sm)));
    int rc = sync_state(s);
    if (rc) return rc;
    const State *h = &s->host[state_index];
    if (h->bnorm == 0.0) {
        HIPCHK(launch_fill<T>(n, x, T(0), sm));
        out->status = KS_OK;
        out->iters = 0;
        return KS_OK;
    }
    int cycles = 0;
    for (;;) {
        const int f = h->flags;
        if (f & F_TRUE_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
        if (f & F_TRUE_OK) {
            out->status = KS_OK;
            break;
        }
        if (h->iters >= max_iter) {
            out->status = KS_MAXITER;
            break;
        }
        HIPCHK(launch_gm_begin<T>(n, w, V, st, s->ga, sm));
        const int chunk = poll_chunk_krylov(s);
        int k = 0;
        bool stopped = false;
        while (k < m && !stopped) {
            const int it0 = h->iters;
            const int kend = std::min(m, k + chunk);
            for (; k < kend; ++k) {
                hipEvent_t e0, e1;
                if ((rc = timing_pair(s, &e0, &e1))) return rc;
                HIPCHK((launch_gm_step<TA, T>(n, lda, A, ldv, V, w, k, st, s->ga, s->P, max_iter,
                                              sm, e0, e1)));
            }
            if (kend < m) {
                if ((rc = sync_state(s))) return rc;
                if ((rc = timed_collect(s, h->iters - it0))) return rc;
                stopped = (h->flags & F_STOP) != 0;
            } else {
                // last chunk of the cycle: finish, residual, then one sync
                HIPCHK(launch_gm_finish<T>(n, ldv, V, x, st, s->ga, sm));
                HIPCHK((launch_residual<TA, T>(n, lda, A, b, x, w, st, s->P, 0, sm)));
                if ((rc = sync_state(s))) return rc;
                if ((rc = timed_collect(s, h->iters - it0))) return rc;
                stopped = true;
                k = m;
            }
        }
        if (k < m) {
            // cycle ended early: finish it
            HIPCHK(launch_gm_finish<T>(n, ldv, V, x, st, s->ga, sm));
            HIPCHK((launch_residual<TA, T>(n, lda, A, b, x, w, st, s->P, 0, sm)));
            if ((rc = sync_state(s))) return rc;
        }
        ++cycles;
        const int f2 = h->flags;
        if (f2 & F_BREAK) {
            out->status = KS_BREAKDOWN;
            break;
        }
        if (f2 & F_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
    }
    out->iters = h->iters;
    out->restarts = std::max(0, cycles - 1);
    return KS_OK;
}

// ------------------------------------------------------------- BiCGSTAB
// Same host flow as run_cg: one pass of the recurrence from the current x,
// then (binary64) confirmation on the true residual and a restart with a new
// shadow residual when it fails.  vec = {r, r0, p, v, s, t}.  Each iteration
// makes up to two products; max_iter bounds the products.
template <typename TA, typename T>
int run_bicgstab(ks_solver *s, State *st, int state_index, const TA *A, int64_t lda, const T *b,
                 T *x, T *const vec[6], double tol, int max_iter, bool outer, Outcome *out,
                 int eta = 0) {
    const int n = s->n;
    hipStream_t sm = s->stream;
    T *r = vec[0];
    HIPCHK(launch_vec_stats<T>(n, b, tol, st, sm, eta));
    HIPCHK((launch_residual<TA, T>(n, lda, A, b, x, r, st, s->P, 0, sm)));
    int rc = sync_state(s);
    if (rc) return rc;
    const State *h = &s->host[state_index];
    if (h->bnorm == 0.0) {
        HIPCHK(launch_fill<T>(n, x, T(0), sm));
        out->status = KS_OK;
        out->iters = 0;
        return KS_OK;
    }
    int restarts = 0;
    bool first = true;
    for (;;) {
        const int f = h->flags;
        if (f & F_TRUE_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
        if (f & F_TRUE_OK) {
            out->status = KS_OK;
            break;
        }
        if (h->iters >= max_iter) {
            out->status = KS_MAXITER;
            break;
        }
        if (!first) {
            if (restarts >= CG_MAX_RESTARTS) {
                out->status = KS_STAGNATED;
                break;
            }
            ++restarts;
        }
        first = false;
        HIPCHK(launch_bs_begin<T>(n, r, vec[1], vec[2], st, sm));
        bool done = false;
        while (!done) {
            const int it0 = h->iters;
            const int chunk = std::max(1, std::min(poll_chunk(s), div_up(max_iter - it0, 2)));
            for (int c = 0; c < chunk; ++c) {
                hipEvent_t ev[4];
                if ((rc = timing_pair(s, &ev[0], &ev[1]))) return rc;
                if ((rc = timing_pair(s, &ev[2], &ev[3]))) return rc;
                HIPCHK((launch_bs_iteration<TA, T>(n, lda, A, x, vec, st, s->P, max_iter, sm, ev[0],
                                                   ev[1], ev[2], ev[3])));
            }
            if (outer) HIPCHK((launch_residual<TA, T>(n, lda, A, b, x, r, st, s->P, 1, sm)));
            if ((rc = sync_state(s))) return rc;
            if ((rc = timed_collect(s, h->iters - it0))) return rc;
            done = (h->flags & F_STOP) != 0;
        }
        const int f2 = h->flags;
        if (f2 & F_BREAK) {
            out->status = KS_BREAKDOWN;
            break;
        }
        if (f2 & F_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
        if (!outer) {
            out->status = (f2 & F_CONV) ? KS_OK : KS_MAXITER;
            break;
        }
        // F_CONV or F_MAXIT (after a full or a half step): the gated residual
        // kernel has refreshed F_TRUE_OK
    }
    out->iters = h->iters;
    out->restarts = restarts;
    return KS_OK;
}

// ------------------------------------------------- Jacobi / Gauss-Seidel
// Shared start: ||b||, diag(A) (zero -> breakdown) and the true residual of
// x0.  Returns 1 when the solve is already decided (out filled), 0 to go on.
int stationary_start(ks_solver *s, const double *b, double *x, double *r, double *d, double tol,
                     int eta, Outcome *out, int *rc) {
    const int n = s->n;
    hipStream_t sm = s->stream;
    State *st = s->st;
    *rc = KS_OK;
    if ((*rc = launch_vec_stats<double>(n, b, tol, st, sm, eta) ? KS_EHIP : KS_OK)) return 1;
    if ((*rc = launch_st_diag(n, s->lda, s->A, d, st, sm) ? KS_EHIP : KS_OK)) return 1;
    if ((*rc = launch_residual<double, double>(n, s->lda, s->A, b, x, r, st, s->P, 0, sm)
                   ? KS_EHIP
                   : KS_OK))
        return 1;
    if ((*rc = sync_state(s))) return 1;
    const State *h = &s->host[0];
    out->iters = 0;
    out->restarts = 0;
    if (h->bnorm == 0.0) {
        if ((*rc = launch_fill<double>(n, x, 0.0, sm) ? KS_EHIP : KS_OK)) return 1;
        out->status = KS_OK;
        return 1;
    }
    if (h->flags & F_TRUE_NONFIN) {
        out->status = KS_NONFINITE;
        return 1;
    }
    if (h->flags & F_BREAK) {
        out->status = KS_BREAKDOWN;
        return 1;
    }
    return 0;
}

// status of a stopped stationary loop from its flags
int stationary_status(int f) {
    if (f & F_NONFIN) return KS_NONFINITE;
    if (f & F_BREAK) return KS_BREAKDOWN;
    if (f & F_CONV) return KS_OK;
    return KS_MAXITER;
}

// Jacobi: [r = b - A x (partials)] -> [decide on x] -> [x += r / d], the
// residual of each iterate being the true one.
int run_jacobi(ks_solver *s, const double *b, double *x, double tol, int max_iter, Outcome *out,
               int eta) {
    const int n = s->n;
    hipStream_t sm = s->stream;
    State *st = s->st;
    double *r = s->vec64(0), *d = s->vec64(1);
    int rc;
    if (stationary_start(s, b, x, r, d, tol, eta, out, &rc)) return rc;
    const State *h = &s->host[0];
    const int nb = gemv_blocks<double>(n);
    HIPCHK(launch_st_begin(st, sm));
    bool done = false;
    while (!done) {
        const int it0 = h->iters;
        const int chunk = std::max(1, std::min(poll_chunk(s), max_iter - it0 + 1));
        for (int c = 0; c < chunk; ++c) {
            HIPCHK(launch_st_decide(nb, st, s->P.g, max_iter, sm));
            HIPCHK(launch_jacobi_update(n, x, r, d, st, sm));
            hipEvent_t e0, e1;
            if ((rc = timing_pair(s, &e0, &e1))) return rc;
            if (e0) HIPCHK(hipEventRecord(e0, sm));
            HIPCHK((launch_residual_rows<double, double>(n, s->lda, s->A, b, x, r, st, s->P.g, 2,
                                                         sm)));
            if (e1) HIPCHK(hipEventRecord(e1, sm));
        }
        if ((rc = sync_state(s))) return rc;
        if ((rc = timed_collect(s, h->iters - it0))) return rc;
        done = (h->flags & F_STOP) != 0;
    }
    out->status = stationary_status(h->flags);
    out->iters = h->iters;
    return KS_OK;
}

// Gauss-Seidel: [u = U x, c = b - u, residual of x as u_prev - u] ->
// [decide on x] -> [forward substitution (D + L) x = c].  The residual from
// the difference of products is the true one up to rounding; a stop is
// confirmed on the true residual and the sweeps resume if it disagrees.
int run_gauss_seidel(ks_solver *s, const double *b, double *x, double tol, int max_iter,
                     Outcome *out, int eta) {
    const int n = s->n;
    hipStream_t sm = s->stream;
    State *st = s->st;
    double *r = s->vec64(0), *d = s->vec64(1), *c = s->vec64(4);
    double *u[2] = {s->vec64(2), s->vec64(3)};
    int rc;
    if (stationary_start(s, b, x, r, d, tol, eta, out, &rc)) return rc;
    const State *h = &s->host[0];
    // a sweep is ceil(n / 64) dependent launches: poll often, so that few
    // sweeps run (as no-ops) past the stop
    const int poll = s->p.poll_every > 0 ? s->p.poll_every : (n >= 4096 ? 1 : n >= 1024 ? 4 : 16);
    int restarts = 0, k = 0;
    bool first = true;
    for (;;) {
        const int f = h->flags;
        if (f & F_TRUE_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
        if (f & F_TRUE_OK) {
            out->status = KS_OK;
            break;
        }
        if (h->iters >= max_iter) {
            out->status = KS_MAXITER;
            break;
        }
        if (!first) {
            if (restarts >= CG_MAX_RESTARTS) {
                out->status = KS_STAGNATED;
                break;
            }
            ++restarts;
        }
        HIPCHK(launch_st_begin(st, sm));
        bool with_res = false;  // the cycle's first test uses the true residual's partials
        bool done = false;
        while (!done) {
            const int it0 = h->iters;
            for (int i = 0; i < poll; ++i, ++k) {
                hipEvent_t e0, e1;
                if ((rc = timing_pair(s, &e0, &e1))) return rc;
                if (e0) HIPCHK(hipEventRecord(e0, sm));
                HIPCHK(launch_gs_upper(n, s->lda, s->A, b, x, u[(k + 1) & 1], u[k & 1], c, st,
                                       s->P.g, with_res ? 1 : 0, sm));
                if (e1) HIPCHK(hipEventRecord(e1, sm));
                HIPCHK(launch_st_decide(with_res ? gs_upper_blocks(n) : gemv_blocks<double>(n), st,
                                        s->P.g, max_iter, sm));
                HIPCHK(launch_gs_sweep(n, s->lda, s->A, x, c, st, sm));
                with_res = true;
            }
            if ((rc = sync_state(s))) return rc;
            // the upper product before the stopping decision ran as well
            const bool stopped = (h->flags & F_STOP) != 0;
            if ((rc = timed_collect(s, h->iters - it0 + (stopped ? 1 : 0)))) return rc;
            done = stopped;
        }
        first = false;
        const int f2 = h->flags;
        if (f2 & (F_NONFIN | F_BREAK)) {
            out->status = stationary_status(f2);
            break;
        }
        // converged or at the limit by the recurrence: confirm on b - A x
        HIPCHK((launch_residual<double, double>(n, s->lda, s->A, b, x, r, st, s->P, 0, sm)));
        if ((rc = sync_state(s))) return rc;
    }
    out->iters = h->iters;
    out->restarts = restarts;
    return KS_OK;
}

// ------------------------------------------------------------ GMRES-IR
// The binary32 block LU of A (in A_low) and the permutation of its pivots:
// (P v)_i = v[perm[i]], composed on the host from the row interchanges.
int lu_setup(ks_solver *s) {
    const int n = s->n;
    hipStream_t sm = s->stream;
    const size_t ln = (size_t)round_up(n, 64);
    s->lu_piv = (int *)(s->ws + s->L.lu_off);
    s->lu_perm = s->lu_piv + ln;
    s->lu_info = s->lu_perm + ln;  // the factorization's work area
    HIPCHK(launch_lu_factor(n, s->L.lda_low, (float *)s->A_low, s->lu_piv, s->lu_info, sm));
    std::vector<int> piv(n), perm(n);
    int info[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(piv.data(), s->lu_piv, sizeof(int) * n, hipMemcpyDeviceToHost, sm));
    HIPCHK(hipMemcpyAsync(info, s->lu_info, sizeof(info), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipStreamSynchronize(sm));
    if (info[1]) return KS_EHIP;  // a panel's grid barrier timed out
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int k = 0; k < n; ++k) {
        if (piv[k] < 0 || piv[k] >= n) return KS_EHIP;  // cannot happen; never trust a bad index
        std::swap(perm[k], perm[piv[k]]);
    }
    HIPCHK(hipMemcpyAsync(s->lu_perm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, sm));
    HIPCHK(hipStreamSynchronize(sm));
    s->lu_sing = info[0];
    return KS_OK;
}

// Inner solve of GMRES-IR: restarted GMRES(m) in binary64 on
// M^-1 A d = M^-1 rhs from d = 0 (M = P^-1 L U in binary32), relative
// tolerance tol on the preconditioned residual, at most max_iter products.
// Every Arnoldi step is the product, M^-1 (the substitutions), then the
// Gram-Schmidt passes and the Givens rotation of the plain GMRES.
int run_gmres_lu(ks_solver *s, const double *rhs, double *d, double tol, int max_iter,
                 Outcome *out) {
    const int n = s->n, m = s->ga.m, ldv = s->L.ldv;
    hipStream_t sm = s->stream;
    State *st = s->st_in;
    const float *LU = (const float *)s->A_low;
    const int64_t ldl = s->L.lda_low;
    double *w = s->vec64(0), *V = s->vec64(1);
    double *t = s->vec64(s->L.nv64 - 2);
    HIPCHK(launch_fill<double>(n, d, 0.0, sm));
    // thresh = tol ||M^-1 rhs||; the residual of d = 0 is M^-1 rhs itself
    HIPCHK(launch_lu_apply(n, ldl, LU, s->lu_perm, rhs, w, t, s->P.g, s->ts_xw, &st->sync_fail, sm));
    HIPCHK(launch_vec_stats<double>(n, w, tol, st, sm, 0));
    HIPCHK(launch_lu_res_finish(n, st, s->P.g, sm));
    int rc = sync_state(s);
    if (rc) return rc;
    const State *h = &s->host[1];
    int cycles = 0;
    for (;;) {
        const int f = h->flags;
        if (f & F_TRUE_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
        if (f & F_TRUE_OK) {
            out->status = KS_OK;
            break;
        }
        if (h->iters >= max_iter) {
            out->status = KS_MAXITER;
            break;
        }
        HIPCHK(launch_gm_begin<double>(n, w, V, st, s->ga, sm));
        // one step per host check: a stopped step would still run the
        // substitutions (they do not test the stop flag)
        for (int k = 0; k < m; ++k) {
            HIPCHK((launch_gm_matvec<double, double>(n, s->lda, s->A, V + (size_t)k * ldv, w, st,
                                                     s->P, sm)));
            HIPCHK(launch_lu_apply(n, ldl, LU, s->lu_perm, w, w, t, s->P.g, s->ts_xw, &st->sync_fail, sm));
            HIPCHK(launch_gm_ortho<double>(n, ldv, V, w, k, st, s->ga, s->P, gemv_blocks<double>(n),
                                           max_iter, sm));
            if ((rc = sync_state(s))) return rc;
            if (h->flags & F_STOP) break;
        }
        HIPCHK(launch_gm_finish<double>(n, ldv, V, d, st, s->ga, sm));
        // the preconditioned residual M^-1 (rhs - A d)
        HIPCHK((launch_residual_rows<double, double>(n, s->lda, s->A, rhs, d, w, st, s->P.g, 0, sm)));
        HIPCHK(launch_lu_apply(n, ldl, LU, s->lu_perm, w, w, t, s->P.g, s->ts_xw, &st->sync_fail, sm));
        HIPCHK(launch_lu_res_finish(n, st, s->P.g, sm));
        if ((rc = sync_state(s))) return rc;
        ++cycles;
        const int f2 = h->flags;
        if (f2 & F_BREAK) {
            out->status = KS_BREAKDOWN;
            break;
        }
        if (f2 & F_NONFIN) {
            out->status = KS_NONFINITE;
            break;
        }
    }
    out->iters = h->iters;
    out->restarts = std::max(0, cycles - 1);
    return KS_OK;
}

// ------------------------------------------------------------- CG-IR
// The binary32 block Cholesky factor of A (in A_low: L below, L^T above).
int chol_setup(ks_solver *s) {
    hipStream_t sm = s->stream;
    int *info = (int *)(s->ws + s->L.lu_off);
    HIPCHK(hipMemsetAsync(info, 0, sizeof(int), sm));
    HIPCHK(launch_chol_factor(s->n, s->L.lda_low, (float *)s->A_low, info, sm));
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, info, sizeof(int), hipMemcpyDeviceToHost, sm));
    HIPCHK(hipStreamSynchronize(sm));
    s->chol_notpd = h;
    return KS_OK;
}

// Inner solve of CG-IR: CG in binary64 on A d = rhs from d = 0,
// preconditioned by M = L L^T (binary32 factor), stopping at
// ||rhs - A d||_2 <= tol ||rhs||_2 on the recursive residual or after
// max_iter products.  The state is polled after every iteration: the
// substitutions of an iteration launched after the stop would still run.
int run_pcg_chol(ks_solver *s, const double *rhs, double *d, double tol, int max_iter, Outcome *out) {
    const int n = s->n, nv = s->L.nv64;
    hipStream_t sm = s->stream;
    State *st = s->st_in;
    const float *L = (const float *)s->A_low;
    const int64_t ldl = s->L.lda_low;
    double *r = s->vec64(0), *p = s->vec64(1), *q = s->vec64(2), *z = s->vec64(nv - 2);
    double *rz_part = s->P.w;
    HIPCHK(launch_fill<double>(n, d, 0.0, sm));
    HIPCHK(launch_vec_stats<double>(n, rhs, tol, st, sm, 0));
    HIPCHK(launch_chol_apply(n, ldl, L, rhs, z, s->ts_xw, &st->sync_fail, sm));
    HIPCHK(launch_pcg_dot(n, rhs, z, st, rz_part, sm));
    HIPCHK(launch_cg_begin<double>(n, rhs, r, st, sm));  // r = rhs, flags cleared
    HIPCHK(launch_pcg_begin(n, z, p, st, rz_part, sm));
    int rc = sync_state(s);
    if (rc) return rc;
    const State *h = &s->host[1];
    if (h->bnorm == 0.0) {
        out->status = KS_OK;
        out->iters = 0;
        return KS_OK;
    }
    if (h->flags & F_TRUE_NONFIN) {
        out->status = KS_NONFINITE;
        out->iters = 0;
        return KS_OK;
    }
    while (!(h->flags & F_STOP)) {
        if (h->iters >= max_iter) break;
        HIPCHK((launch_cg_matvec<double, double>(n, s->lda, s->A, p, q, st, s->P, sm)));
        HIPCHK(launch_cg_update<double>(n, d, r, p, q, st, s->P, gemv_blocks<double>(n), sm));
        HIPCHK(launch_chol_apply(n, ldl, L, r, z, s->ts_xw, &st->sync_fail, sm));
        HIPCHK(launch_pcg_dot(n, r, z, st, rz_part, sm));
        HIPCHK(launch_pcg_pupdate(n, z, p, st, s->P.v, rz_part, max_iter, sm));
        if ((rc = sync_state(s))) return rc;
    }
    const int f = h->flags;
    if (f & F_NONFIN)
        out->status = KS_NONFINITE;
    else if (f & F_BREAK)
        out->status = KS_BREAKDOWN;
    else if (f & F_CONV)
        out->status = KS_OK;
    else
        out->status = KS_MAXITER;
    out->iters = h->iters;
    return KS_OK;
}

// Metrics of the returned x from the State the solve left behind: every exit
// path of the drivers ends with a true-residual kernel and a sync, so the
// host mirror holds ||b||, ||r|| and the infinity norms of r, x and b.
void metrics_from_state(const ks_solver *s, ks_info *info) {
    const State &h = s->host[0];
    if (!(h.bnorm > 0.0)) {
        info->rel_res = 0.0;
        info->backward_err = 0.0;
        return;
    }
    const double den = h.anorm_inf * h.xinf + h.binf;
    info->rel_res = h.res / h.bnorm;
    info->backward_err = den > 0.0 ? h.resinf / den : h.resinf;
}

int solve_fp64(ks_solver *s, const double *b, double *x, double tol, int max_iter, Outcome *o,
               int eta) {
    if (s->p.method == KS_JACOBI) return run_jacobi(s, b, x, tol, max_iter, o, eta);
    if (s->p.method == KS_GAUSS_SEIDEL) return run_gauss_seidel(s, b, x, tol, max_iter, o, eta);
    if (s->p.method == KS_CG)
        return run_cg<double, double>(s, s->st, 0, s->A, s->lda, b, x, s->vec64(0), s->vec64(1),
                                      s->vec64(2), tol, max_iter, true, o, eta);
    if (s->p.method == KS_BICGSTAB) {
        double *const vec[6] = {s->vec64(0), s->vec64(1), s->vec64(2),
                                s->vec64(3), s->vec64(4), s->vec64(5)};
        return run_bicgstab<double, double>(s, s->st, 0, s->A, s->lda, b, x, vec, tol, max_iter,
                                            true, o, eta);
    }
    return run_gmres<double, double>(s, s->st, 0, s->A, s->lda, b, x, s->vec64(0), s->vec64(1),
                                     tol, max_iter, o, eta);
}

// ----------------------------------------------- multi-right-hand-side CG
int sync_mr(ks_solver *s) {
    HIPCHK(hipMemcpyAsync(s->host, s->st, 2 * sizeof(State), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(s->host_cols, s->cols, 2 * (size_t)KS_MAX_NRHS * sizeof(ColState),
                          hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return KS_OK;
}

// Lockstep CG on s columns.  outer = true: binary64 solve confirmed on the
// true residual, failing columns restarted (as the one-column solve); false:
// one pass stopped on the recursive residuals (refinement inner solve).
// status[j], iters[j], restarts[j] receive each column's outcome.
template <typename T>
int run_mrhs(ks_solver *s, State *st, ColState *cols, int ci, const T *A, int64_t lda, const T *B,
             int ldb, T *X, T *R, T *P, T *Q, T *Qpart, double tol, int max_iter, bool outer,
             std::vector<int> &status, std::vector<int> &restarts) {
    const int n = s->n, ns = s->p.nrhs, ldv = s->L.ldv;
    hipStream_t sm = s->stream;
    double *pa = s->mr_part, *pb = s->mr_part + (size_t)mr_blocks(n) * KS_MAX_NRHS;
    HIPCHK(launch_mr_stats<T>(n, ns, B, ldb, tol, cols, st, sm));
    HIPCHK(launch_mr_residual<T>(n, lda, A, ns, B, ldb, X, Qpart, R, ldv, s->mr_part, cols, st, 0, sm));
    int rc = sync_mr(s);
    if (rc) return rc;
    const ColState *hc = s->host_cols + (size_t)ci * KS_MAX_NRHS;
    const State *h = &s->host[ci];
    status.assign(ns, -100);
    restarts.assign(ns, 0);
    std::vector<char> started(ns, 0);
    for (int j = 0; j < ns; ++j)
        if (hc[j].bnorm == 0.0) {
            HIPCHK(launch_fill<T>(n, X + (size_t)j * ldv, T(0), sm));
            status[j] = KS_OK;
        }
    for (;;) {
        uint64_t mask = 0;
        for (int j = 0; j < ns; ++j) {
            if (status[j] != -100) continue;
            const int f = hc[j].flags;
            if (f & F_TRUE_NONFIN)
                status[j] = KS_NONFINITE;
            else if (f & F_TRUE_OK)
                status[j] = KS_OK;
            else if (started[j] && (f & F_BREAK))
                status[j] = KS_BREAKDOWN;
            else if (started[j] && (f & F_NONFIN))
                status[j] = KS_NONFINITE;
            else if (hc[j].iters >= max_iter)
                status[j] = KS_MAXITER;
            else if (started[j] && restarts[j] >= CG_MAX_RESTARTS)
                status[j] = KS_STAGNATED;
            else {
                if (started[j]) ++restarts[j];
                started[j] = 1;
                mask |= 1ull << j;
            }
        }
        if (!mask) break;
        HIPCHK(launch_mr_begin<T>(n, ns, R, P, ldv, cols, st, mask, sm));
        bool done = false;
        while (!done) {
            const int it0 = h->iters;
            const int chunk = std::max(1, std::min(poll_chunk(s), max_iter));
            for (int c = 0; c < chunk; ++c) {
                hipEvent_t e0, e1;
                if ((rc = timing_pair(s, &e0, &e1))) return rc;
                HIPCHK(launch_mr_iteration<T>(n, lda, A, ns, X, R, P, Q, Qpart, ldv, pa, pb, cols, st,
                                              max_iter, sm, e0, e1));
            }
            if (outer)
                HIPCHK(launch_mr_residual<T>(n, lda, A, ns, B, ldb, X, Qpart, R, ldv, s->mr_part, cols,
                                             st, 1, sm));
            if ((rc = sync_mr(s))) return rc;
            if ((rc = timed_collect(s, h->iters - it0))) return rc;
            done = (h->flags & F_STOP) != 0;
        }
        if (!outer) {
            for (int j = 0; j < ns; ++j) {
                if (status[j] != -100) continue;
                const int f = hc[j].flags;
                status[j] = (f & F_CONV)     ? KS_OK
                            : (f & F_BREAK)  ? KS_BREAKDOWN
                            : (f & F_NONFIN) ? KS_NONFINITE
                                             : KS_MAXITER;
            }
            break;
        }
    }
    return KS_OK;
}

int solve_mrhs_fp64(ks_solver *s, const double *B, double *Xuser, ks_info *info, Outcome *o) {
    const int n = s->n, ns = s->p.nrhs, ldv = s->L.ldv;
    hipStream_t sm = s->stream;
    double *X = s->mrb64(0), *R = s->mrb64(1), *P = s->mrb64(2), *Q = s->mrb64(3),
           *Qp = s->mrb64(4);
    HIPCHK(launch_mr_copy<double>(n, ns, Xuser, n, X, ldv, sm));
    std::vector<int> status, restarts;
    int rc = run_mrhs<double>(s, s->st, s->cols, 0, s->A, s->lda, B, n, X, R, P, Q, Qp, s->p.tol,
                              s->p.max_iter, true, status, restarts);
    if (rc) return rc;
    HIPCHK(launch_mr_copy<double>(n, ns, X, ldv, Xuser, n, sm));
    s->col_info.assign(ns, ks_info{});
    o->status = KS_OK;
    o->iters = s->host[0].iters;
    info->rel_res = 0.0;
    info->backward_err = 0.0;
    for (int j = 0; j < ns; ++j) {
        const ColState &c = s->host_cols[j];
        ks_info &ci = s->col_info[j];
        ci.status = status[j];
        ci.iters = c.iters;
        ci.restarts = restarts[j];
        const double den = s->host[0].anorm_inf * c.xinf + c.binf;
        ci.rel_res = c.bnorm > 0.0 ? c.res / c.bnorm : 0.0;
        ci.backward_err = c.bnorm > 0.0 ? (den > 0.0 ? c.resinf / den : c.resinf) : 0.0;
        ci.precision_used = KS_FP64;
        o->status = std::max(o->status, status[j]);
        o->restarts = std::max(o->restarts, restarts[j]);
        info->rel_res = std::max(info->rel_res, ci.rel_res);
        info->backward_err = std::max(info->backward_err, ci.backward_err);
    }
    return KS_OK;
}

// Refinement around lockstep CG: binary64 residuals R = B - A X, per-column
// backward error; inner lockstep CG on the binary32 copy of A for the active
// columns (MFMA binary32 contraction); X_j += ||r_j|| d_j.
int solve_mrhs_ir(ks_solver *s, const double *B, double *Xuser, ks_info *info, Outcome *o) {
    const int n = s->n, ns = s->p.nrhs, ldv = s->L.ldv;
    hipStream_t sm = s->stream;
    double *X = s->mrb64(0), *R = s->mrb64(1), *Qp = s->mrb64(4);
    float *D = s->mrb32(0), *R32 = s->mrb32(1), *P32 = s->mrb32(2), *Q32 = s->mrb32(3),
          *rhs = s->mrb32(4), *Qp32 = s->mrb32(5);
    const float *A32 = (const float *)s->A_low;
    const int64_t ll = s->L.lda_low;
    HIPCHK(launch_mr_copy<double>(n, ns, Xuser, n, X, ldv, sm));
    HIPCHK(launch_mr_stats<double>(n, ns, B, n, 1.0, s->cols, s->st, sm));
    HIPCHK(launch_mr_residual<double>(n, s->lda, s->A, ns, B, n, X, Qp, R, ldv, s->mr_part, s->cols,
                                      s->st, 0, sm));
    int rc = sync_mr(s);
    if (rc) return rc;
    const ColState *hc = s->host_cols;
    const double anorm = s->host[0].anorm_inf;
    std::vector<int> status(ns, -100), bad(ns, 0), inner_iters(ns, 0);
    std::vector<double> eta_prev(ns, INFINITY);
    int outer = 0;
    auto eta_of = [&](int j) {
        const double den = anorm * hc[j].xinf + hc[j].binf;
        return den > 0.0 ? hc[j].resinf / den : hc[j].resinf;
    };
    for (int j = 0; j < ns; ++j)
        if (hc[j].bnorm == 0.0) {
            HIPCHK(launch_fill<double>(n, X + (size_t)j * ldv, 0.0, sm));
            status[j] = KS_OK;
        }
    for (;;) {
        uint64_t mask = 0;
        for (int j = 0; j < ns; ++j) {
            if (status[j] != -100) continue;
            const double eta = eta_of(j);
            if (!std::isfinite(eta) || (hc[j].flags & F_TRUE_NONFIN))
                status[j] = KS_NONFINITE;
            else if (eta <= s->p.tol)
                status[j] = KS_OK;
            else if (outer >= s->p.max_outer)
                status[j] = KS_STAGNATED;
            else {
                if (eta > 0.5 * eta_prev[j]) {
                    if (++bad[j] >= 2) {
                        status[j] = KS_STAGNATED;
                        continue;
                    }
                } else {
                    bad[j] = 0;
                }
                eta_prev[j] = eta;
                mask |= 1ull << j;
            }
        }
        if (!mask) break;
        HIPCHK(launch_mr_ir_scale(n, ns, R, ldv, rhs, s->cols, mask, sm));
        HIPCHK(launch_fill<float>((int)std::min<size_t>((size_t)ns * ldv, 0x7fffffff), D, 0.0f, sm));
        std::vector<int> ist, irs;
        rc = run_mrhs<float>(s, s->st_in, s->cols_in, 1, A32, ll, rhs, ldv, D, R32, P32, Q32, Qp32,
                             s->p.inner_tol, s->p.max_iter, false, ist, irs);
        if (rc) return rc;
        for (int j = 0; j < ns; ++j)
            if ((mask >> j) & 1ull) {
                inner_iters[j] += s->host_cols[KS_MAX_NRHS + j].iters;
                if (ist[j] == KS_BREAKDOWN || ist[j] == KS_NONFINITE) status[j] = KS_BREAKDOWN;
            }
        HIPCHK(launch_mr_ir_update(n, ns, X, D, ldv, s->cols, mask, sm));
        HIPCHK(launch_mr_residual<double>(n, s->lda, s->A, ns, B, n, X, Qp, R, ldv, s->mr_part, s->cols,
                                          s->st, 0, sm));
        if ((rc = sync_mr(s))) return rc;
        ++outer;
    }
    HIPCHK(launch_mr_copy<double>(n, ns, X, ldv, Xuser, n, sm));
    s->col_info.assign(ns, ks_info{});
    o->status = KS_OK;
    o->iters = 0;
    info->rel_res = 0.0;
    info->backward_err = 0.0;
    info->outer_iters = outer;
    info->precision_used = KS_IR_FP32;
    for (int j = 0; j < ns; ++j) {
        ks_info &ci = s->col_info[j];
        ci.status = status[j];
        ci.iters = inner_iters[j];
        ci.outer_iters = outer;
        ci.rel_res = hc[j].bnorm > 0.0 ? hc[j].res / hc[j].bnorm : 0.0;
        ci.backward_err = hc[j].bnorm > 0.0 ? eta_of(j) : 0.0;
        ci.precision_used = KS_IR_FP32;
        o->status = std::max(o->status, status[j]);
        o->iters = std::max(o->iters, inner_iters[j]);
        info->rel_res = std::max(info->rel_res, ci.rel_res);
        info->backward_err = std::max(info->backward_err, ci.backward_err);
    }
    return KS_OK;
}

// ------------------------------------------------- iterative refinement
// Outer binary64 loop: r = b - A x; stop at eta_inf <= tol; inner solve of
// A_low d = r/||r|| (binary32 vectors); x += ||r|| d.  Precision is promoted
// bfloat16 -> binary32 -> binary64 when the backward error fails to halve
// twice, or the inner solve breaks down.
int solve_ir(ks_solver *s, const double *b, double *x, ks_info *info, Outcome *o) {
    const int n = s->n, m = s->ga.m;
    hipStream_t sm = s->stream;
    double *r64 = s->vec64(s->L.nv64 - 1);
    float *rhs = s->vec32(0), *d = s->vec32(1);
    int prec = s->p.precision;
    int total_iters = 0, outer = 0, bad = 0, rc;
    double eta_prev = INFINITY;
    HIPCHK(launch_vec_stats<double>(n, b, 1.0, s->st, sm));
    HIPCHK((launch_residual<double, double>(n, s->lda, s->A, b, x, r64, s->st, s->P, 0, sm)));
    if ((rc = sync_state(s))) return rc;
    const State *h = &s->host[0];
    if (h->bnorm == 0.0) {
        HIPCHK(launch_fill<double>(n, x, 0.0, sm));
        o->status = KS_OK;
        info->rel_res = 0.0;
        info->backward_err = 0.0;
        info->precision_used = prec;
        return KS_OK;
    }
    const double binf = h->binf, bnorm = h->bnorm;
    s->anorm_inf = h->anorm_inf;
    if ((prec == KS_IR_LU32 && s->lu_sing) || (prec == KS_IR_CHOL32 && s->chol_notpd)) {
        // the binary32 factorization met a zero (LU) or non-positive (Cholesky) pivot
        info->rel_res = h->res / bnorm;
        const double den0 = s->anorm_inf * h->xinf + binf;
        info->backward_err = den0 > 0.0 ? h->resinf / den0 : h->resinf;
        info->precision_used = prec;
        o->status = KS_BREAKDOWN;
        return KS_OK;
    }
    for (;;) {
        const double den = s->anorm_inf * h->xinf + binf;
        const double eta = den > 0.0 ? h->resinf / den : h->resinf;
        info->rel_res = h->res / bnorm;
        info->backward_err = eta;
        if (!std::isfinite(eta) || (h->flags & F_TRUE_NONFIN)) {
            o->status = KS_NONFINITE;
            break;
        }
        if (eta <= s->p.tol) {
            o->status = KS_OK;
            break;
        }
        if (outer >= s->p.max_outer) {
            o->status = KS_STAGNATED;
            break;
        }
        if (eta > 0.5 * eta_prev) {
            if (++bad >= 2 && prec != KS_FP64) {
                prec = (prec == KS_IR_BF16) ? KS_IR_FP32 : KS_FP64;
                bad = 0;
            }
        } else {
            bad = 0;
        }
        eta_prev = eta;
        if (prec == KS_FP64) {
            // finish in binary64 from the current x, stopping on the backward error
            Outcome o64;
            if ((rc = solve_fp64(s, b, x, s->p.tol, std::max(1, s->p.max_iter), &o64, 1))) return rc;
            total_iters += o64.iters;
            ++outer;
            HIPCHK((launch_residual<double, double>(n, s->lda, s->A, b, x, r64, s->st, s->P, 0,
                                                    sm)));
            if ((rc = sync_state(s))) return rc;
            const double den2 = s->anorm_inf * h->xinf + binf;
            info->rel_res = h->res / bnorm;
            info->backward_err = den2 > 0.0 ? h->resinf / den2 : h->resinf;
            o->status = (info->backward_err <= s->p.tol) ? KS_OK : o64.status;
            if (o->status == KS_OK && o64.status != KS_OK && info->backward_err > s->p.tol)
                o->status = o64.status;
            break;
        }
        if (prec == KS_IR_LU32) {
            // GMRES-IR: correction from the preconditioned GMRES in binary64
            Outcome oi;
            double *dl = s->vec64(s->L.nv64 - 3);
            if ((rc = run_gmres_lu(s, r64, dl, s->p.inner_tol, s->p.max_iter, &oi))) return rc;
            total_iters += oi.iters;
            ++outer;
            if (oi.status == KS_BREAKDOWN || oi.status == KS_NONFINITE) {
                prec = KS_FP64;
                bad = 0;
                eta_prev = INFINITY;
                continue;
            }
            HIPCHK(launch_lu_xupdate(n, x, dl, sm));
            HIPCHK((launch_residual<double, double>(n, s->lda, s->A, b, x, r64, s->st, s->P, 0, sm)));
            if ((rc = sync_state(s))) return rc;
            continue;
        }
        if (prec == KS_IR_CHOL32) {
            // CG-IR: correction from the preconditioned CG in binary64
            Outcome oi;
            double *dl = s->vec64(s->L.nv64 - 3);
            if ((rc = run_pcg_chol(s, r64, dl, s->p.inner_tol, s->p.max_iter, &oi))) return rc;
            total_iters += oi.iters;
            ++outer;
            if (oi.status == KS_BREAKDOWN || oi.status == KS_NONFINITE) {
                prec = KS_FP64;
                bad = 0;
                eta_prev = INFINITY;
                continue;
            }
            HIPCHK(launch_lu_xupdate(n, x, dl, sm));
            HIPCHK((launch_residual<double, double>(n, s->lda, s->A, b, x, r64, s->st, s->P, 0, sm)));
            if ((rc = sync_state(s))) return rc;
            continue;
        }
        if (prec == KS_IR_FP32 && s->p.precision == KS_IR_BF16 && !s->fb_ready) {
            HIPCHK(launch_convert(n, s->lda, s->A, KS_DT_F32, s->L.lda_low, s->A_fb, sm));
            s->fb_ready = true;
        }
        // inner solve on the low-precision copy
        HIPCHK(launch_ir_scale_cast(n, r64, rhs, s->st, sm));
        HIPCHK(launch_fill<float>(n, d, 0.0f, sm));
        Outcome oi;
        const int64_t ll = s->L.lda_low;
        if (s->p.method == KS_CG) {
            float *ri = s->vec32(2), *pi = s->vec32(3), *qi = s->vec32(4);
            if (prec == KS_IR_BF16)
                rc = run_cg<bf16_t, float>(s, s->st_in, 1, (const bf16_t *)s->A_low, ll, rhs, d, ri, pi,
                                           qi, s->p.inner_tol, s->p.max_iter, false, &oi);
            else
                rc = run_cg<float, float>(s, s->st_in, 1,
                                          (s->p.precision == KS_IR_BF16) ? s->A_fb : (const float *)s->A_low,
                                          ll, rhs, d, ri, pi, qi, s->p.inner_tol, s->p.max_iter, false,
                                          &oi);
        } else if (s->p.method == KS_BICGSTAB) {
            float *const vi[6] = {s->vec32(2), s->vec32(3), s->vec32(4),
                                  s->vec32(5), s->vec32(6), s->vec32(7)};
            if (prec == KS_IR_BF16)
                rc = run_bicgstab<bf16_t, float>(s, s->st_in, 1, (const bf16_t *)s->A_low, ll, rhs, d,
                                                 vi, s->p.inner_tol, s->p.max_iter, false, &oi);
            else
                rc = run_bicgstab<float, float>(s, s->st_in, 1,
                                                (s->p.precision == KS_IR_BF16) ? s->A_fb
                                                                               : (const float *)s->A_low,
                                                ll, rhs, d, vi, s->p.inner_tol, s->p.max_iter, false,
                                                &oi);
        } else {
            float *wi = s->vec32(2), *Vi = s->vec32(3);
            if (prec == KS_IR_BF16)
                rc = run_gmres<bf16_t, float>(s, s->st_in, 1, (const bf16_t *)s->A_low, ll, rhs, d, wi, Vi,
                                              s->p.inner_tol, s->p.max_iter, &oi);
            else
                rc = run_gmres<float, float>(s, s->st_in, 1,
                                             (s->p.precision == KS_IR_BF16) ? s->A_fb
                                                                            : (const float *)s->A_low,
                                             ll, rhs, d, wi, Vi, s->p.inner_tol, s->p.max_iter, &oi);
        }
        (void)m;
        if (rc) return rc;
        total_iters += oi.iters;
        ++outer;
        if (oi.status == KS_BREAKDOWN || oi.status == KS_NONFINITE) {
            // the low-precision copy is not usable (e.g. indefinite): promote
            prec = (prec == KS_IR_BF16) ? KS_IR_FP32 : KS_FP64;
            bad = 0;
            eta_prev = INFINITY;
            continue;
        }
        HIPCHK(launch_ir_update(n, x, d, &s->st->res, sm));
        HIPCHK((launch_residual<double, double>(n, s->lda, s->A, b, x, r64, s->st, s->P, 0, sm)));
        if ((rc = sync_state(s))) return rc;
    }
    o->iters = total_iters;
    info->outer_iters = outer;
    info->precision_used = prec;
    return KS_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int ks_params_init(ks_params *p, int32_t n, int32_t method) {
    if (!p || n < 1 ||
        (method != KS_CG && method != KS_GMRES && method != KS_BICGSTAB && method != KS_JACOBI &&
         method != KS_GAUSS_SEIDEL))
        return KS_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->n = n;
    p->method = method;
    p->lda = n;
    p->precision = KS_FP64;
    p->max_iter = 10 * n;
    p->tol = 1e-10;
    p->restart = 30;
    p->max_outer = 30;
    p->inner_tol = 1e-4;
    p->poll_every = 0;
    p->flags = 0;
    p->nrhs = 1;
    p->timing_every = 0;
    return KS_OK;
}

int ks_workspace_bytes(const ks_params *p, size_t *bytes) {
    if (!valid_params(p) || !bytes) return KS_EINVAL;
    *bytes = make_layout(p).total;
    return KS_OK;
}

int ks_workspace_bytes_borrowed(const ks_params *p, size_t *bytes) {
    if (!valid_params(p) || !bytes) return KS_EINVAL;
    *bytes = make_layout(p).total_borrowed;
    return KS_OK;
}

int ks_create(ks_solver **out, const ks_params *p, const double *dA, void *d_ws, size_t ws_bytes,
              void *stream) {
    if (!out || !valid_params(p) || !dA) return KS_EINVAL;
    if (d_ws && ((uintptr_t)d_ws % ALIGN) != 0) return KS_EINVAL;
    if (!d_ws && ws_bytes != 0) return KS_EINVAL;
    int rc = check_device();
    if (rc) return rc;
    Layout L = make_layout(p);
    const bool borrow = a_borrowable(dA, p->lda);
    const size_t need = borrow ? L.total_borrowed : L.total;
    ks_solver *s = new (std::nothrow) ks_solver();
    if (!s) return KS_ENOMEM;
    s->p = *p;
    s->L = L;
    s->n = p->n;
    s->stream = (hipStream_t)stream;
    if (d_ws) {
        if (ws_bytes < need) {
            delete s;
            return KS_ENOMEM;
        }
        s->ws = (char *)d_ws;
    } else {
        if (hipMalloc((void **)&s->ws, need) != hipSuccess) {
            delete s;
            return KS_ENOMEM;
        }
        s->own_ws = true;
    }
    if (hipHostMalloc((void **)&s->host, 2 * sizeof(State), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess) {
        ks_free(s);
        return KS_EHIP;
    }
    {
        const Carved c = carve(L, s->ws);
        s->st = c.st;
        s->st_in = c.st + 1;
        s->ga = c.ga;
        s->P = c.P;
        s->v64 = c.v64;
        s->v32 = c.v32;
        if (L.sy_bytes) s->sy = (double *)(s->ws + L.sy_off);
        // the layout holds the second copies of r, p, q for the fused CG
        s->fz = p->method == KS_CG && p->nrhs == 1 && p->n <= FZ_MAX_N && !s->sy && L.nv64 >= 6;
        if (s->fz && L.bar_off) s->fzbar = (uint32_t *)(s->ws + L.bar_off);
    }
    if (p->nrhs > 1) {
        s->mr64 = (double *)(s->ws + L.mr_off);
        s->mr32 = (float *)(s->ws + L.mr_off + (4 + (size_t)mr_splits(p->n, 8)) * L.mr_block_elems * sizeof(double));
        s->cols = (ColState *)(s->ws + L.mr_cols_off);
        s->cols_in = s->cols + KS_MAX_NRHS;
        s->mr_part = (double *)(s->ws + L.mr_part_off);
        if (hipHostMalloc((void **)&s->host_cols, 2 * (size_t)KS_MAX_NRHS * sizeof(ColState),
                          hipHostMallocDefault) != hipSuccess) {
            ks_free(s);
            return KS_EHIP;
        }
    }
    hipStream_t sm = s->stream;
    // zero the states and the small arrays
    if (hipMemsetAsync(s->ws, 0, L.part_off, sm) != hipSuccess) {
        ks_free(s);
        return KS_EHIP;
    }
    if (borrow) {
        s->A = dA;
        s->lda = p->lda;
    } else {
        double *Ac = (double *)(s->ws + L.acopy_off);
        if (launch_copy_pad(p->n, p->lda, dA, L.lda_pad, Ac, sm) != hipSuccess) {
            ks_free(s);
            return KS_EHIP;
        }
        s->A = Ac;
        s->lda = L.lda_pad;
    }
    if (launch_norm_inf(p->n, s->lda, s->A, s->st, s->P, sm) != hipSuccess) {
        ks_free(s);
        return KS_EHIP;
    }
    if (p->precision != KS_FP64) {
        s->A_low = s->ws + L.alow_off;
        if (p->precision == KS_IR_BF16) s->A_fb = (float *)(s->ws + L.afb_off);
        const int dt = (p->precision == KS_IR_BF16) ? KS_DT_BF16 : KS_DT_F32;
        if (launch_convert(p->n, s->lda, s->A, dt, L.lda_low, s->A_low, sm) != hipSuccess) {
            ks_free(s);
            return KS_EHIP;
        }
    }
    if ((p->precision == KS_IR_CHOL32 || p->precision == KS_IR_LU32) && !(p->flags & KS_FLAG_NO_PERSIST))
        s->ts_xw = (uint64_t *)(s->ws + L.lu_off + 2 * (size_t)round_up(p->n, 64) * sizeof(int) + LU_WORK_BYTES);
    if (p->precision == KS_IR_CHOL32 && (rc = chol_setup(s))) {
        ks_free(s);
        return rc;
    }
    if (p->precision == KS_IR_LU32 && (rc = lu_setup(s))) {
        ks_free(s);
        return rc;
    }
    *out = s;
    return KS_OK;
}

int ks_solve(ks_solver *s, const double *d_b, double *d_x, ks_info *info) {
    if (!s || !d_b || !d_x) return KS_EINVAL;
    if ((uintptr_t)d_b % 16 || (uintptr_t)d_x % 16) return KS_EINVAL;
    ks_info local;
    if (!info) info = &local;
    std::memset(info, 0, sizeof(*info));
    info->precision_used = s->p.precision;
    s->gemv_ms = 0.0;
    s->gemv_calls = 0;
    s->tcall = 0;
    s->tchunk_pos = 0;
    s->tev_used = 0;
    HIPCHK(hipEventRecord(s->ev0, s->stream));
    Outcome o;
    int rc;
    if (s->p.nrhs > 1) {
        if (s->p.precision == KS_FP64)
            rc = solve_mrhs_fp64(s, d_b, d_x, info, &o);
        else
            rc = solve_mrhs_ir(s, d_b, d_x, info, &o);
        if (rc) return rc;
        HIPCHK(hipEventRecord(s->ev1, s->stream));
    } else if (s->p.precision == KS_FP64) {
        rc = solve_fp64(s, d_b, d_x, s->p.tol, s->p.max_iter, &o,
                        (s->p.flags & KS_FLAG_STOP_BACKWARD) ? 1 : 0);
        if (rc) return rc;
        HIPCHK(hipEventRecord(s->ev1, s->stream));
        metrics_from_state(s, info);
    } else {
        rc = solve_ir(s, d_b, d_x, info, &o);
        if (rc) return rc;
        HIPCHK(hipEventRecord(s->ev1, s->stream));
    }
    HIPCHK(hipEventSynchronize(s->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    info->elapsed_ms = ms;
    info->status = o.status;
    info->iters = o.iters;
    info->restarts = o.restarts;
    info->gemv_ms = s->gemv_ms;
    info->gemv_calls = s->gemv_calls;
    return o.status;
}

int ks_arnoldi(ks_solver *s, const double *d_v0, int32_t k, double *d_V, double *d_H,
               int32_t *k_done) {
    if (!s || !d_v0 || !d_V || !d_H || !k_done) return KS_EINVAL;
    if ((uintptr_t)d_v0 % 16) return KS_EINVAL;
    if (s->p.method != KS_GMRES || s->p.precision != KS_FP64 || k < 1 || k > s->ga.m)
        return KS_EINVAL;
    const int n = s->n, ldv = s->L.ldv;
    hipStream_t sm = s->stream;
    double *w = s->vec64(0), *V = s->vec64(1);
    HIPCHK(launch_vec_stats<double>(n, d_v0, 0.0, s->st, sm));
    HIPCHK(hipMemcpyAsync(&s->st->res, &s->st->bnorm, sizeof(double), hipMemcpyDeviceToDevice, sm));
    HIPCHK(hipMemsetAsync(s->ga.H, 0, sizeof(double) * (size_t)(s->ga.m + 1) * s->ga.m, sm));
    HIPCHK(launch_gm_begin<double>(n, d_v0, V, s->st, s->ga, sm));
    const int big = 0x7fffffff;
    for (int c = 0; c < k; ++c)
        HIPCHK((launch_gm_step<double, double>(n, s->lda, s->A, ldv, V, w, c, s->st, s->ga, s->P,
                                               big, sm, nullptr, nullptr)));
    int rc = sync_state(s);
    if (rc) return rc;
    const int kd = s->host[0].k_done;
    *k_done = kd;
    HIPCHK(hipMemcpy2DAsync(d_V, (size_t)n * sizeof(double), V, (size_t)ldv * sizeof(double),
                            (size_t)n * sizeof(double), (size_t)kd + 1, hipMemcpyDeviceToDevice, sm));
    if (kd > 0)
        HIPCHK(hipMemcpy2DAsync(d_H, (size_t)k * sizeof(double), s->ga.H,
                                (size_t)s->ga.m * sizeof(double), (size_t)k * sizeof(double),
                                (size_t)kd + 1, hipMemcpyDeviceToDevice, sm));
    HIPCHK(hipStreamSynchronize(sm));
    return KS_OK;
}

int ks_column_info(const ks_solver *s, int32_t j, ks_info *info) {
    if (!s || !info || j < 0 || j >= (int32_t)s->col_info.size()) return KS_EINVAL;
    *info = s->col_info[j];
    return KS_OK;
}

void ks_free(ks_solver *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (hipEvent_t e : s->tev) (void)hipEventDestroy(e);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    if (s->host) (void)hipHostFree(s->host);
    if (s->host_cols) (void)hipHostFree(s->host_cols);
    if (s->own_ws && s->ws) (void)hipFree(s->ws);
    delete s;
}

const char *ks_strerror(int status) {
    switch (status) {
        case KS_OK: return "converged";
        case KS_MAXITER: return "iteration limit reached";
        case KS_BREAKDOWN: return "breakdown (CG: p'Ap <= 0; GMRES: singular Hessenberg)";
        case KS_STAGNATED: return "stagnated";
        case KS_NONFINITE: return "non-finite value";
        case KS_EINVAL: return "invalid argument";
        case KS_ENOMEM: return "workspace too small or allocation failed";
        case KS_EHIP: return "HIP runtime error";
        case KS_EDEVICE: return "device is not gfx950";
        default: return "unknown status";
    }
}

int ks_gemv(int32_t n, int64_t lda, int32_t a_dtype, const void *dA, const void *d_v, void *d_y,
            void *stream) {
    if (n < 1 || lda < n || !dA || !d_v || !d_y) return KS_EINVAL;
    size_t es = (a_dtype == KS_DT_F64) ? 8 : (a_dtype == KS_DT_F32) ? 4 : (a_dtype == KS_DT_BF16) ? 2 : 0;
    if (!es) return KS_EINVAL;
    if ((uintptr_t)dA % 16 || (lda * es) % 16 || (uintptr_t)d_v % 16 || (uintptr_t)d_y % 16)
        return KS_EINVAL;
    HIPCHK(launch_gemv(n, lda, a_dtype, dA, d_v, d_y, (hipStream_t)stream));
    return KS_OK;
}

int ks_gemm_mr_workspace_bytes(int32_t n, int32_t s, int32_t a_dtype, size_t *bytes) {
    const int es = (a_dtype == KS_DT_F64) ? 8 : (a_dtype == KS_DT_F32) ? 4 : 0;
    if (n < 1 || s < 1 || s > KS_MAX_NRHS || !es || !bytes) return KS_EINVAL;
    *bytes = mr_product_ws_bytes(n, s, es);
    return KS_OK;
}

int ks_gemm_mr(int32_t n, int64_t lda, int32_t a_dtype, const void *dA, int32_t s, const void *d_P,
               int64_t ldv, void *d_Q, void *d_ws, size_t ws_bytes, void *stream) {
    const int es = (a_dtype == KS_DT_F64) ? 8 : (a_dtype == KS_DT_F32) ? 4 : 0;
    if (n < 1 || lda < n || ldv < n || s < 1 || s > KS_MAX_NRHS || !es || !dA || !d_P || !d_Q ||
        !d_ws)
        return KS_EINVAL;
    if ((uintptr_t)dA % 16 || (lda * es) % 16 || (uintptr_t)d_ws % 16) return KS_EINVAL;
    if (ws_bytes < mr_product_ws_bytes(n, s, es)) return KS_ENOMEM;
    hipStream_t st = (hipStream_t)stream;
    if (es == 8)
        HIPCHK(launch_mr_product<double>(n, lda, (const double *)dA, s, (const double *)d_P, ldv,
                                         (double *)d_Q, d_ws, st));
    else
        HIPCHK(launch_mr_product<float>(n, lda, (const float *)dA, s, (const float *)d_P, ldv,
                                        (float *)d_Q, d_ws, st));
    return KS_OK;
}

int ks_symv_workspace_bytes(int32_t n, size_t *bytes) {
    if (n < 1 || !bytes) return KS_EINVAL;
    *bytes = sy_ws_doubles(n) * sizeof(double);
    return KS_OK;
}

int ks_symv(int32_t n, int64_t lda, const double *dA, const double *d_x, double *d_y, void *d_ws,
            size_t ws_bytes, void *stream) {
    if (n < 1 || lda < n || !dA || !d_x || !d_y || !d_ws) return KS_EINVAL;
    if ((uintptr_t)dA % 16 || (lda * 8) % 16 || (uintptr_t)d_x % 16 || (uintptr_t)d_y % 16 ||
        (uintptr_t)d_ws % 16)
        return KS_EINVAL;
    if (ws_bytes < sy_ws_doubles(n) * sizeof(double)) return KS_ENOMEM;
    HIPCHK(launch_symv(n, lda, dA, d_x, d_y, (double *)d_ws, nullptr, nullptr, nullptr,
                       (hipStream_t)stream));
    return KS_OK;
}

int ks_symv_f32(int32_t n, int64_t lda, const float *dA, const float *d_x, float *d_y, void *d_ws,
                size_t ws_bytes, void *stream) {
    if (n < 1 || lda < n || !dA || !d_x || !d_y || !d_ws) return KS_EINVAL;
    if ((uintptr_t)dA % 16 || (lda * 4) % 16 || (uintptr_t)d_x % 16 || (uintptr_t)d_y % 16 ||
        (uintptr_t)d_ws % 16)
        return KS_EINVAL;
    if (ws_bytes < sy_ws_doubles(n) * sizeof(float)) return KS_ENOMEM;
    HIPCHK(launch_symv32(n, lda, dA, d_x, d_y, (float *)d_ws, (hipStream_t)stream));
    return KS_OK;
}

int ks_lu32_factor(int32_t n, int64_t lda, const double *d_A, int64_t lda_lu, float *d_LU,
                   int32_t *d_piv, int32_t *info, void *stream) {
    if (n < 1 || n > LU_MAX_N || lda < n || lda_lu < n || !d_A || !d_LU || !d_piv || !info)
        return KS_EINVAL;
    int rc = check_device();
    if (rc) return rc;
    hipStream_t sm = (hipStream_t)stream;
    void *work = nullptr;
    HIPCHK(hipMalloc(&work, LU_WORK_BYTES));
    int h[2] = {0, 0};
    hipError_t e = launch_convert(n, lda, d_A, KS_DT_F32, lda_lu, d_LU, sm);
    if (e == hipSuccess) e = launch_lu_factor(n, lda_lu, d_LU, d_piv, work, sm);
    if (e == hipSuccess) e = hipMemcpyAsync(h, work, sizeof(h), hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    const hipError_t ef = hipFree(work);
    if (e != hipSuccess || ef != hipSuccess || h[1]) return KS_EHIP;
    *info = h[0];
    return KS_OK;
}

int ks_chol32_factor(int32_t n, int64_t lda, const double *d_A, int64_t ldl, float *d_L,
                     int32_t *info, void *stream) {
    if (n < 1 || lda < n || ldl < n || ldl % 4 || !d_A || !d_L || !info || (uintptr_t)d_L % 16)
        return KS_EINVAL;
    int rc = check_device();
    if (rc) return rc;
    hipStream_t sm = (hipStream_t)stream;
    int *dinfo = nullptr;
    HIPCHK(hipMalloc((void **)&dinfo, sizeof(int)));
    int h = 0;
    hipError_t e = hipMemsetAsync(dinfo, 0, sizeof(int), sm);
    if (e == hipSuccess) e = launch_convert(n, lda, d_A, KS_DT_F32, ldl, d_L, sm);
    if (e == hipSuccess) e = launch_chol_factor(n, ldl, d_L, dinfo, sm);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, dinfo, sizeof(int), hipMemcpyDeviceToHost, sm);
    if (e == hipSuccess) e = hipStreamSynchronize(sm);
    const hipError_t ef = hipFree(dinfo);
    if (e != hipSuccess || ef != hipSuccess) return KS_EHIP;
    *info = h;
    return KS_OK;
}

int ks_convert(int32_t n, int64_t lda_src, const double *d_src, int32_t dst_dtype, int64_t lda_dst,
               void *d_dst, void *stream) {
    if (n < 1 || lda_src < n || lda_dst < n || !d_src || !d_dst) return KS_EINVAL;
    if (dst_dtype != KS_DT_F32 && dst_dtype != KS_DT_BF16 && dst_dtype != KS_DT_F64) return KS_EINVAL;
    HIPCHK(launch_convert(n, lda_src, d_src, dst_dtype, lda_dst, d_dst, (hipStream_t)stream));
    return KS_OK;
}

int ks_read_ceiling(const void *d_src, size_t bytes, double *d_sink, void *stream) {
    if (!d_src || !d_sink || bytes == 0 || bytes % 16) return KS_EINVAL;
    if ((uintptr_t)d_src % 16) return KS_EINVAL;
    HIPCHK(launch_read_ceiling(d_src, bytes, d_sink, (hipStream_t)stream));
    return KS_OK;
}

}  // extern "C"
