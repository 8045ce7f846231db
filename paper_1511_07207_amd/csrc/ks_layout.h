// Workspace layout of one solve (shared by the single-solve API and the
// request server): validation of the parameters and the byte offsets of every
// region inside the caller's (or the server's) device workspace.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "ks.h"
#include "ks_internal.h"

namespace ks {
constexpr int CG_MAX_RESTARTS = 16;  // true-residual restarts before "stagnated"
constexpr size_t ALIGN = 256;

inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
    int ldv = 0;
    int m = 0;
    size_t st_off = 0;      // two State structs: [0] outer / plain, [1] inner
    size_t gm_off = 0;      // GMRES small arrays (binary64)
    size_t part_off = 0;    // block partials (regions of Partials)
    size_t part_count = 0;
    size_t pg = 0, pv = 0, ph = 0, pn = 0, pw = 0;  // region sizes in doubles
    size_t v64_off = 0;     // binary64 vectors
    int nv64 = 0;
    size_t v32_off = 0;     // binary32 vectors (IR inner solve)
    int nv32 = 0;
    size_t acopy_off = 0;   // padded binary64 copy of A (when not borrowed)
    size_t acopy_bytes = 0;
    int64_t lda_pad = 0;
    size_t alow_off = 0;    // binary32 / bfloat16 copy of A (IR)
    size_t alow_bytes = 0;
    size_t afb_off = 0;     // binary32 copy used after a bfloat16 -> binary32 fallback
    size_t afb_bytes = 0;
    int64_t lda_low = 0;
    // multi-right-hand-side blocks (nrhs > 1): X, R, P, Q and S partial Q's,
    // each sp16 columns of ldv elements, plus per-column states
    int sp16 = 0;
    size_t mr_off = 0, mr_block_elems = 0, mr_cols_off = 0, mr_part_off = 0, mr_part_count = 0;
    // tile partials of the symmetric product (KS_FLAG_SYMMETRIC)
    size_t sy_off = 0, sy_bytes = 0;
    // GMRES-IR: pivots, permutation and info of the binary32 LU
    size_t lu_off = 0;
    // fused small-n CG: grid-barrier flags of its persistent launch
    size_t bar_off = 0;
    size_t total = 0;
    size_t total_borrowed = 0;
};

inline size_t gm_doubles(int m) { return (size_t)(m + 1) * m * 2 + 2 * (size_t)m + (m + 1) + m + (m + 1); }

inline bool valid_params(const ks_params *p) {
    if (!p) return false;
    if (p->n < 1 || p->lda < p->n || p->timing_every < 0) return false;
    if (p->method != KS_CG && p->method != KS_GMRES && p->method != KS_BICGSTAB &&
        p->method != KS_JACOBI && p->method != KS_GAUSS_SEIDEL)
        return false;
    // the stationary methods: binary64, one right-hand side, general storage
    if ((p->method == KS_JACOBI || p->method == KS_GAUSS_SEIDEL) &&
        (p->precision != KS_FP64 || p->nrhs != 1 || (p->flags & KS_FLAG_SYMMETRIC)))
        return false;
    if (p->precision < KS_FP64 || p->precision > KS_IR_CHOL32) return false;
    // CG-IR with the binary32 Cholesky factor: CG, one right-hand side
    if (p->precision == KS_IR_CHOL32 &&
        (p->method != KS_CG || p->nrhs != 1 || (p->flags & KS_FLAG_SYMMETRIC)))
        return false;
    // GMRES-IR with the binary32 LU: GMRES, one right-hand side, n <= LU_MAX_N
    if (p->precision == KS_IR_LU32 &&
        (p->method != KS_GMRES || p->nrhs != 1 || p->n > LU_MAX_N || (p->flags & KS_FLAG_SYMMETRIC)))
        return false;
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return false;
    if (p->max_iter < 0) return false;
    if (p->method == KS_GMRES && (p->restart < 1 || p->restart > KS_MAX_RESTART)) return false;
    if (p->precision != KS_FP64) {
        if (!(p->inner_tol > 0.0) || p->max_outer < 1) return false;
    }
    if (p->nrhs < 1 || p->nrhs > KS_MAX_NRHS) return false;
    if (p->nrhs > 1 && (p->method != KS_CG || p->precision == KS_IR_BF16)) return false;
    if ((p->flags & KS_FLAG_SYMMETRIC) && (p->method != KS_CG || p->nrhs != 1)) return false;
    return true;
}

inline Layout make_layout(const ks_params *p) {
    Layout L;
    const int n = p->n;
    L.ldv = (int)round_up(n, 64);
    L.m = (p->method == KS_GMRES) ? p->restart : 1;
    size_t off = 0;
    L.st_off = off;
    off = align_up(off + 2 * sizeof(State));
    L.gm_off = off;
    off = align_up(off + gm_doubles(L.m) * sizeof(double));
    L.pg = (size_t)round_up((int64_t)gemv_blocks_max(n) * 3, 32);
    L.pv = (size_t)round_up(3 * vec_blocks(n), 32);
    L.ph = (size_t)round_up((size_t)cgs_blocks(n) * (L.m + 1), 32);
    L.pn = (size_t)round_up(cgs_blocks(n), 32);
    // BiCGSTAB's x/r update partials; CG-IR's r'z partials
    L.pw = (p->method == KS_BICGSTAB || p->precision == KS_IR_CHOL32)
               ? (size_t)round_up(4 * vec_blocks(n), 32)
               : 0;
    L.part_count = L.pg + L.pv + 2 * L.ph + L.pn + L.pw;
    L.part_off = off;
    off = align_up(off + L.part_count * sizeof(double));
    // binary64 vectors: CG r, p, q; GMRES w, V(0..m); BiCGSTAB r, r0, p, v, s, t;
    // Jacobi r, diag(A); Gauss-Seidel r, diag(A), U x twice, b - U x;
    // IR adds the outer residual
    const int nkry = (p->method == KS_CG)            ? 3
                     : (p->method == KS_BICGSTAB)    ? 6
                     : (p->method == KS_JACOBI)      ? 2
                     : (p->method == KS_GAUSS_SEIDEL) ? 5
                                                     : 1 + (L.m + 1);
    // binary64 CG at n <= FZ_MAX_N runs the fused kernel: r, p, q twice
    const bool fused = p->method == KS_CG && p->nrhs == 1 && n <= FZ_MAX_N;
    L.nv64 = fused ? 6 : nkry;
    if (p->precision != KS_FP64) L.nv64 += 1;
    // GMRES-IR: the inner GMRES runs in binary64 (its w, V), plus the
    // correction d and the preconditioner's scratch t
    if (p->precision == KS_IR_LU32) L.nv64 += 2;
    // CG-IR with the Cholesky factor: the inner PCG runs in binary64 on the
    // CG vectors (r, p, q) plus the correction d and z = M^-1 r
    if (p->precision == KS_IR_CHOL32) L.nv64 += 2;
    L.v64_off = off;
    off = align_up(off + (size_t)L.nv64 * L.ldv * sizeof(double));
    // binary32 vectors of the inner solve: rhs, d, then the method's vectors
    L.nv32 = 0;
    if (p->precision == KS_IR_FP32 || p->precision == KS_IR_BF16) L.nv32 = 2 + nkry;
    L.v32_off = off;
    off = align_up(off + (size_t)L.nv32 * L.ldv * sizeof(float));
    if (p->nrhs > 1) {
        L.sp16 = (int)round_up(p->nrhs, 16);
        L.mr_block_elems = (size_t)L.sp16 * L.ldv;
        const size_t es = sizeof(double);
        L.mr_off = off;
        // X, R, P, Q + mr_splits(n, 8) partial products (binary64); the IR
        // inner solve adds its binary32 D, R, P, Q, rhs and partials below
        off = align_up(off + (4 + (size_t)mr_splits(n, 8)) * L.mr_block_elems * es);
        if (p->precision == KS_IR_FP32)
            off = align_up(off + (5 + (size_t)mr_splits(n, 4)) * L.mr_block_elems * sizeof(float));
        L.mr_cols_off = off;
        off = align_up(off + 2 * (size_t)KS_MAX_NRHS * sizeof(ColState));
        L.mr_part_count = 3 * (size_t)mr_blocks(n) * KS_MAX_NRHS;
        L.mr_part_off = off;
        off = align_up(off + L.mr_part_count * sizeof(double));
    }
    if (p->flags & KS_FLAG_SYMMETRIC) {
        L.sy_bytes = (sy_ws_doubles(n) + (p->method == KS_CG ? sy_cg_doubles(n) : 0)) * sizeof(double);
        L.sy_off = off;
        off = align_up(off + L.sy_bytes);
    }
    if (fused) {
        L.bar_off = off;
        off = align_up(off + (size_t)FZ_BAR_MAX_WORDS * sizeof(uint32_t));
    }
    if (p->precision == KS_IR_LU32 || p->precision == KS_IR_CHOL32) {
        // pivots, the permutation, the LU factorization's work area (whose
        // first word is its info word; the Cholesky factorization uses one
        // info word at the start of the region), then the words the
        // persistent substitutions exchange
        L.lu_off = off;
        off = align_up(off + 2 * (size_t)round_up(n, 64) * sizeof(int) + LU_WORK_BYTES +
                       ts_persist_words(n) * sizeof(uint64_t));
    }
    L.lda_low = round_up(n, 64);
    if (p->precision == KS_IR_FP32 || p->precision == KS_IR_LU32 || p->precision == KS_IR_CHOL32) {
        L.alow_bytes = (size_t)n * L.lda_low * sizeof(float);
    } else if (p->precision == KS_IR_BF16) {
        L.alow_bytes = (size_t)n * L.lda_low * sizeof(uint16_t);
        L.afb_bytes = (size_t)n * L.lda_low * sizeof(float);
    }
    L.alow_off = off;
    off = align_up(off + L.alow_bytes);
    L.afb_off = off;
    off = align_up(off + L.afb_bytes);
    L.total_borrowed = off;
    L.lda_pad = round_up(n, 64);
    L.acopy_bytes = (size_t)n * L.lda_pad * sizeof(double);
    L.acopy_off = off;
    off = align_up(off + L.acopy_bytes);
    L.total = off;
    return L;
}

inline bool a_borrowable(const double *A, int64_t lda) {
    return ((uintptr_t)A % 16 == 0) && ((lda * 8) % 16 == 0);
}


// Pointers of the regions inside a workspace starting at ws.
struct Carved {
    State *st = nullptr;
    GmArrays ga{};
    Partials P{};
    double *v64 = nullptr;
    float *v32 = nullptr;
};

inline Carved carve(const Layout &L, char *ws) {
    Carved c;
    c.st = (State *)(ws + L.st_off);
    double *g = (double *)(ws + L.gm_off);
    const int m = L.m;
    c.ga.m = m;
    c.ga.H = g;
    g += (size_t)(m + 1) * m;
    c.ga.R = g;
    g += (size_t)(m + 1) * m;
    c.ga.cs = g;
    g += m;
    c.ga.sn = g;
    g += m;
    c.ga.g = g;
    g += m + 1;
    c.ga.y = g;
    g += m;
    c.ga.h1 = g;
    double *pp = (double *)(ws + L.part_off);
    c.P.g = pp;
    pp += L.pg;
    c.P.v = pp;
    pp += L.pv;
    c.P.h1 = pp;
    pp += L.ph;
    c.P.h2 = pp;
    pp += L.ph;
    c.P.nrm = pp;
    pp += L.pn;
    c.P.w = L.pw ? pp : nullptr;
    c.v64 = (double *)(ws + L.v64_off);
    c.v32 = (float *)(ws + L.v32_off);
    return c;
}

}  // namespace ks
