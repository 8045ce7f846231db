// Device bodies of the vector kernels (inner products, saxpy updates,
// Gram-Schmidt, Givens least squares), called with an explicit block index by
// the single-solve kernels and by the server's batched kernels.
#pragma once
#include "ks_device.h"

namespace ks {

constexpr double HAPPY_FACTOR = 1e-14;  // h(k+1,k) <= this * ||A v_k||

// ------------------------------------------------- ||b||_2 and ||b||_inf

template <typename T>
__device__ __forceinline__ void vec_stats_body(int n, const T *__restrict__ b, double tol, State *st,
                                               int eta) {
    __shared__ double sm[ONE_NT / WAVE];
    double s2 = 0.0, mx = 0.0;
    for (int i = threadIdx.x; i < n; i += ONE_NT) {
        const double v = (double)b[i];
        s2 += v * v;
        mx = fmax(mx, finite_d(v) ? fabs(v) : INFINITY);
    }
    const double ss = block_sum<ONE_NT>(s2, sm);
    __syncthreads();
    const double bm = block_max<ONE_NT>(mx, sm);
    if (threadIdx.x == 0) {
        const double bn = sqrt(ss);
        st->bnorm = bn;
        st->binf = bm;
        st->thresh = tol * bn;
        st->eta_tol = eta ? tol : 0.0;
        st->xinf_it = 0.0;
        st->iters = 0;
        st->k_done = 0;
        st->flags = finite_d(bn) ? 0 : (F_TRUE_NONFIN | F_STOP);
    }
}

// ------------------------------------------------------------------- CG
// x += alpha p, r -= alpha q with alpha = rho / sigma, sigma = p'q reduced
// from the matrix-vector product's partials; r'r partials for the next kernel.
// prho: [r'r partials (nblk)][||x||_inf partials (nblk)][||r||_inf partials
// (nblk, only when stopping on the backward error)], nblk = vec_blocks(n)
template <typename T>
__device__ __forceinline__ void cg_update_body(int n, T *__restrict__ x, T *__restrict__ r,
                                               const T *__restrict__ p, const T *__restrict__ q,
                                               State *st, const double *__restrict__ psigma,
                                               int nsigma, double *__restrict__ prho, int bid,
                                               int nblk) {
    __shared__ double sm[VEC_NT / WAVE];
    // the vectors are loaded before the partials are reduced and the stop
    // flag is tested after that barrier, so that the loads overlap with the
    // reduction's round trip (a launch after the stop loads and discards them)
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
    T xv[VEC_EPT], rv[VEC_EPT], pv[VEC_EPT], qv[VEC_EPT];
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = min(base + e * VEC_NT, n - 1);
        xv[e] = x[i];
        rv[e] = r[i];
        pv[e] = p[i];
        qv[e] = q[i];
    }
    const double rho = st->rho;  // written by the launch before, read with the vectors
    const double eta_tol = st->eta_tol;
    const double sigma = reduce_partials_all<VEC_NT>(psigma, nsigma, 1);
    if (st->flags & F_STOP) return;
    const bool ok = finite_d(sigma) && sigma > 0.0;
    if (bid == 0 && threadIdx.x == 0) {
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
    if (!ok) return;
    const T a = (T)(rho / sigma);
    double s2 = 0.0, xm = 0.0, rm = 0.0;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) {
            const T xi = fma(a, pv[e], xv[e]);
            x[i] = xi;
            const T ri = fma(-a, qv[e], rv[e]);
            r[i] = ri;
            s2 += (double)ri * (double)ri;
            xm = fmax(xm, finite_d((double)xi) ? fabs((double)xi) : INFINITY);
            rm = fmax(rm, finite_d((double)ri) ? fabs((double)ri) : INFINITY);
        }
    }
    const double t = block_sum<VEC_NT>(s2, sm);
    __syncthreads();
    const double tx = block_max<VEC_NT>(xm, sm);
    if (threadIdx.x == 0) {
        prho[bid] = t;
        prho[nblk + bid] = tx;
    }
    if (eta_tol > 0.0) {
        __syncthreads();
        const double tr = block_max<VEC_NT>(rm, sm);
        if (threadIdx.x == 0) prho[2 * nblk + bid] = tr;
    }
}

// rho' = r'r; stop on the recursive residual or the iteration limit;
// otherwise beta = rho' / rho and p = r + beta p.  Stopping on the backward
// error compares ||r||_inf of the recursive residual with
// tol (||A||_inf ||x||_inf + ||b||_inf) (the infinity norms of the iterate's
// partials), i.e. eta_inf of the recursive residual itself.
template <typename T>
__device__ __forceinline__ void cg_pupdate_body(int n, const T *__restrict__ r, T *__restrict__ p,
                                                State *st, const double *__restrict__ prho, int nrho,
                                                int max_iter, int bid) {
    // r and p are loaded before the partials are reduced, the stop flag
    // tested after that barrier (as in the update kernel)
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
    T rv[VEC_EPT], pv[VEC_EPT];
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = min(base + e * VEC_NT, n - 1);
        rv[e] = r[i];
        pv[e] = p[i];
    }
    // the scalars this launch does not change, read with the vectors
    // rather than after the reduction's barriers
    const double eta_tol = st->eta_tol, thresh = st->thresh, rho_prev = st->rho_prev;
    const double anorm_inf = st->anorm_inf, binf = st->binf;
    const int iters = st->iters;
    const double rho_new = reduce_partials_all<VEC_NT>(prho, nrho, 1);
    if (st->flags & F_STOP) return;
    const double xinf = eta_tol > 0.0 ? reduce_partials_max_all<VEC_NT>(prho + nrho, nrho, 1) : 0.0;
    const double rinf =
        eta_tol > 0.0 ? reduce_partials_max_all<VEC_NT>(prho + 2 * nrho, nrho, 1) : 0.0;
    const bool conv = eta_tol > 0.0 ? rinf <= eta_tol * (anorm_inf * xinf + binf)
                                    : sqrt(rho_new) <= thresh;
    int stop = 0;
    if (!finite_d(rho_new))
        stop = F_NONFIN | F_STOP;
    else if (conv)
        stop = F_CONV | F_STOP;
    else if (iters >= max_iter)
        stop = F_MAXIT | F_STOP;
    const double beta = rho_new / rho_prev;
    if (bid == 0 && threadIdx.x == 0) {
        st->xinf_it = xinf;
        if (stop) {
            st->flags |= stop;
        } else {
            st->beta = beta;
            st->rho = rho_new;
        }
    }
    if (stop) return;
    const T bt = (T)beta;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) p[i] = fma(bt, pv[e], rv[e]);
    }
}

template <typename T>
__device__ __forceinline__ void cg_begin_body(int n, const T *__restrict__ r, T *__restrict__ p,
                                              State *st, int bid) {
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) p[i] = r[i];
    }
    if (bid == 0 && threadIdx.x == 0) st->flags &= ~INNER_FLAGS;
}

// ------------------------------------------------ refinement and helpers
// r32 = (float)(r / ||r||) with ||r|| = st->res (the inner right-hand side)
__device__ __forceinline__ void ir_scale_body(int n, const double *__restrict__ r,
                                              float *__restrict__ r32, const State *st, int bid) {
    const double s = st->res;
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) r32[i] = (float)(r[i] / s);
    }
}

// x += (*scale) (double) d   (the refinement step, scale = ||r|| of the outer residual)
__device__ __forceinline__ void ir_update_body(int n, double *__restrict__ x,
                                               const float *__restrict__ d, const double *scale,
                                               int bid) {
    const double s = *scale;
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) x[i] = fma(s, (double)d[i], x[i]);
    }
}

template <typename T>
__device__ __forceinline__ void fill_body(int n, T *__restrict__ x, T value, int bid) {
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) x[i] = value;
    }
}

// ------------------------------------------------------------- BiCGSTAB
// Start of a pass from the current x: shadow residual r0 = r and p = r (the
// first search direction of the recurrence with p = v = 0); rho = r0'r is the
// residual kernel's r'r.
template <typename T>
__device__ __forceinline__ void bs_begin_body(int n, const T *__restrict__ r, T *__restrict__ r0,
                                              T *__restrict__ p, State *st, int bid) {
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) {
            const T ri = r[i];
            r0[i] = ri;
            p[i] = ri;
        }
    }
    if (bid == 0 && threadIdx.x == 0) {
        st->flags &= ~INNER_FLAGS;
        st->xinf_it = st->xinf;
    }
}

// alpha = rho / (r0'v) from the product's partials; s = r - alpha v; s's
// partials for the next kernel.  Block 0 counts the product.
template <typename T>
__device__ __forceinline__ void bs_supdate_body(int n, const T *__restrict__ r, const T *__restrict__ v,
                                                T *__restrict__ s, State *st,
                                                const double *__restrict__ pr0v, int nr0v,
                                                double *__restrict__ pss, int bid) {
    __shared__ double sm[VEC_NT / WAVE];
    if (st->flags & F_STOP) return;
    const double r0v = reduce_partials_all<VEC_NT>(pr0v, nr0v, 1);
    const double rho = st->rho;
    const bool ok = finite_d(r0v) && r0v != 0.0;
    if (bid == 0 && threadIdx.x == 0) {
        st->iters += 1;
        if (!finite_d(r0v))
            st->flags |= F_NONFIN | F_STOP;
        else if (r0v == 0.0)
            st->flags |= F_BREAK | F_STOP;
        else
            st->alpha = rho / r0v;
    }
    if (!ok) return;
    const T a = (T)(rho / r0v);
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
    double s2 = 0.0;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) {
            const T si = fma(-a, v[i], r[i]);
            s[i] = si;
            s2 += (double)si * (double)si;
        }
    }
    const double t = block_sum<VEC_NT>(s2, sm);
    if (threadIdx.x == 0) pss[bid] = t;
}

// Half step (F_HALF from the product kernel): x += alpha p and nothing else.
// Otherwise omega = t's / t't, x += alpha p + omega s, r = s - omega t, and
// partials of r'r, r0'r and ||x||_inf into pw = [nblk][nblk][nblk].  Block 0
// counts the second product and keeps rho in rho_prev for the next kernel.
template <typename T>
__device__ __forceinline__ void bs_xrupdate_body(int n, T *__restrict__ x, T *__restrict__ r,
                                                 const T *__restrict__ r0, const T *__restrict__ p,
                                                 const T *__restrict__ s, const T *__restrict__ t,
                                                 State *st, const double *__restrict__ pt, int npt,
                                                 double *__restrict__ pw, int bid, int nblk) {
    __shared__ double sm[VEC_NT / WAVE];
    const int f = st->flags;
    if (f & F_STOP) return;
    const T a = (T)st->alpha;
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
    if (f & F_HALF) {
#pragma unroll
        for (int e = 0; e < VEC_EPT; ++e) {
            const int i = base + e * VEC_NT;
            if (i < n) x[i] = fma(a, p[i], x[i]);
        }
        return;
    }
    const double ts = reduce_partials_all<VEC_NT>(pt, npt, 2);
    const double tt = reduce_partials_all<VEC_NT>(pt + 1, npt, 2);
    const bool ok = finite_d(tt) && tt != 0.0;
    const double om = ts / tt;
    if (bid == 0 && threadIdx.x == 0) {
        st->iters += 1;
        st->rho_prev = st->rho;
        if (!finite_d(tt))
            st->flags |= F_NONFIN | F_STOP;
        else if (tt == 0.0)
            st->flags |= F_BREAK | F_STOP;
        else
            st->omega = om;
    }
    if (!ok) return;
    const T w = (T)om;
    double rr = 0.0, r0r = 0.0, xm = 0.0, rm = 0.0;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) {
            const T si = s[i];
            const T xi = fma(w, si, fma(a, p[i], x[i]));
            x[i] = xi;
            const T ri = fma(-w, t[i], si);
            r[i] = ri;
            rr += (double)ri * (double)ri;
            r0r += (double)r0[i] * (double)ri;
            xm = fmax(xm, finite_d((double)xi) ? fabs((double)xi) : INFINITY);
            rm = fmax(rm, finite_d((double)ri) ? fabs((double)ri) : INFINITY);
        }
    }
    const double t0 = block_sum<VEC_NT>(rr, sm);
    __syncthreads();
    const double t1 = block_sum<VEC_NT>(r0r, sm);
    __syncthreads();
    const double t2 = block_max<VEC_NT>(xm, sm);
    if (threadIdx.x == 0) {
        pw[bid] = t0;
        pw[nblk + bid] = t1;
        pw[2 * nblk + bid] = t2;
    }
    if (st->eta_tol > 0.0) {
        __syncthreads();
        const double t3 = block_max<VEC_NT>(rm, sm);
        if (threadIdx.x == 0) pw[3 * nblk + bid] = t3;
    }
}

// Stop tests on the recursive residual (tolerance, product budget), then the
// breakdowns omega = 0 and r0'r = 0; otherwise beta = (rho'/rho)(alpha/omega)
// and p = r + beta (p - omega v).  After a half step block 0 only sets F_STOP
// (every block returns in that case, so the flag write cannot race).
template <typename T>
__device__ __forceinline__ void bs_pupdate_body(int n, const T *__restrict__ r, const T *__restrict__ v,
                                                T *__restrict__ p, State *st,
                                                const double *__restrict__ pw, int nw, int max_iter,
                                                int bid) {
    const int f = st->flags;
    if (f & F_STOP) return;
    if (f & F_HALF) {
        if (bid == 0 && threadIdx.x == 0) st->flags = f | F_STOP;
        return;
    }
    const double rr = reduce_partials_all<VEC_NT>(pw, nw, 1);
    const double rho_new = reduce_partials_all<VEC_NT>(pw + nw, nw, 1);
    const double eta_tol = st->eta_tol;
    const double xinf = eta_tol > 0.0 ? reduce_partials_max_all<VEC_NT>(pw + 2 * nw, nw, 1) : 0.0;
    const double rinf = eta_tol > 0.0 ? reduce_partials_max_all<VEC_NT>(pw + 3 * nw, nw, 1) : 0.0;
    const double rho = st->rho_prev, alpha = st->alpha, om = st->omega;
    // backward-error stopping: ||r||_inf of the recursive residual against
    // tol (||A||_inf ||x||_inf + ||b||_inf)
    const bool conv = eta_tol > 0.0 ? rinf <= eta_tol * (st->anorm_inf * xinf + st->binf)
                                    : sqrt(rr) <= st->thresh;
    int stop = 0;
    if (!finite_d(rr))
        stop = F_NONFIN | F_STOP;
    else if (conv)
        stop = F_CONV | F_STOP;
    else if (st->iters >= max_iter)
        stop = F_MAXIT | F_STOP;
    else if (om == 0.0)
        stop = F_BREAK | F_STOP;
    else if (!finite_d(rho_new))
        stop = F_NONFIN | F_STOP;
    else if (rho_new == 0.0)
        stop = F_BREAK | F_STOP;
    const double beta = (rho_new / rho) * (alpha / om);
    if (bid == 0 && threadIdx.x == 0) {
        st->xinf_it = xinf;
        if (stop) {
            st->flags |= stop;
        } else {
            st->beta = beta;
            st->rho = rho_new;
        }
    }
    if (stop) return;
    const T bt = (T)beta, w = (T)om;
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) p[i] = fma(bt, fma(-w, v[i], p[i]), r[i]);
    }
}

// ---------------------------------------------------------------- GMRES
// v_0 = r / beta, g = beta e_1 (beta = ||r|| from the residual kernel).
template <typename T>
__device__ __forceinline__ void gm_begin_body(int n, const T *__restrict__ r, T *__restrict__ v0,
                                              State *st, GmArrays ga, int bid) {
    const double beta = st->res;
    const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
    for (int e = 0; e < VEC_EPT; ++e) {
        const int i = base + e * VEC_NT;
        if (i < n) v0[i] = (T)((double)r[i] / beta);
    }
    if (bid == 0) {
        for (int j = threadIdx.x; j <= ga.m; j += VEC_NT) ga.g[j] = (j == 0) ? beta : 0.0;
        if (threadIdx.x == 0) {
            st->k_done = 0;
            st->flags &= ~INNER_FLAGS;
        }
    }
}

// Classical Gram-Schmidt against the k+1 basis vectors V_0..V_k, one row per
// thread (the projection of the paper's GMRES pseudo-code, applied twice).
// MODE 0: partials of h1 = V'w (block 0 also finishes ||A v_k|| and counts the
//         step).
// MODE 1: h1 from the partials; w -= V h1; partials of h2 = V'w.
// MODE 2: h2 from the partials; w -= V h2; H(:,k) = h1 + h2; partials of ||w||^2.
template <typename T, int MODE>
__device__ __forceinline__ void gm_cgs_body(int n, int ldv, const T *__restrict__ V, T *__restrict__ w,
                                            int k, State *st, GmArrays ga, Partials P, int ngemv,
                                            int bid, int nb) {
    constexpr int NW = CGS_NT / WAVE;
    __shared__ double red[NW][KS_MAX_RESTART + 1];
    __shared__ double hs[KS_MAX_RESTART + 1];
    __shared__ double sm[NW];
    if (st->flags & F_STOP) return;
    const int kk = k + 1;
    const int stride = ga.m + 1;
    const int i = bid * CGS_NT + threadIdx.x;
    const bool valid = i < n;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    if constexpr (MODE == 0) {
        if (bid == 0) {
            const double s2 = reduce_partials_all<CGS_NT>(P.g, ngemv, 1);
            if (threadIdx.x == 0) {
                st->avk = sqrt(s2);
                st->iters += 1;
            }
        }
    }
    double wi = valid ? (double)w[i] : 0.0;
    if constexpr (MODE >= 1) {
        const double *src = (MODE == 1) ? P.h1 : P.h2;
        // one wave per coefficient: lanes take blocks lane, lane+64, ... in order
        for (int j = wv; j < kk; j += NW) {
            double s = 0.0;
            for (int b = lane; b < nb; b += WAVE) s += src[(size_t)b * stride + j];
            s = wave_sum(s);
            if (lane == 0) hs[j] = s;
        }
        __syncthreads();
        if (bid == 0) {
            for (int j = threadIdx.x; j < kk; j += CGS_NT) {
                if (MODE == 1)
                    ga.h1[j] = hs[j];
                else
                    ga.H[(size_t)j * ga.m + k] = ga.h1[j] + hs[j];
            }
        }
        if (valid) {
            double s = 0.0;
            for (int j = 0; j < kk; ++j) s = fma((double)V[(size_t)j * ldv + i], hs[j], s);
            const T wn = (T)(wi - s);
            w[i] = wn;
            wi = (double)wn;
        }
    }
    if constexpr (MODE <= 1) {
        double *dst = (MODE == 0) ? P.h1 : P.h2;
        // eight coefficients at a time: their wave sums together by the
        // halving butterfly (lane group lane / 8 ends with coefficient j0 + g)
        for (int j0 = 0; j0 < kk; j0 += 8) {
            double prod[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                prod[u] = (valid && j0 + u < kk) ? (double)V[(size_t)(j0 + u) * ldv + i] * wi : 0.0;
            const double t = rows_reduce<8>(prod, lane);
            if (lane % 8 == 0 && j0 + lane / 8 < kk) red[wv][j0 + lane / 8] = t;
        }
        __syncthreads();
        for (int j = threadIdx.x; j < kk; j += CGS_NT) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NW; ++q) s += red[q][j];
            dst[(size_t)bid * stride + j] = s;
        }
    } else {
        const double t = block_sum<CGS_NT>(wi * wi, sm);
        if (threadIdx.x == 0) P.nrm[bid] = t;
    }
}

// h(k+1,k) = ||w|| from the partials; v_{k+1} = w / h(k+1,k) unless the step
// is a happy breakdown; block 0 applies the Givens rotations to column k of H,
// forms the new rotation, updates g and decides whether the cycle stops.
template <typename T>
__device__ __forceinline__ void gm_givens_body(int n, const T *__restrict__ w, T *__restrict__ vnext,
                                               int k, State *st, GmArrays ga,
                                               const double *__restrict__ pnrm, int nnrm,
                                               int max_iter, int bid) {
    if (st->flags & F_STOP) return;
    const double hk1 = sqrt(reduce_partials_all<VEC_NT>(pnrm, nnrm, 1));
    const double avk = st->avk;
    if (finite_d(hk1) && finite_d(avk) && hk1 > HAPPY_FACTOR * avk) {
        const int base = bid * VEC_NT * VEC_EPT + threadIdx.x;
#pragma unroll
        for (int e = 0; e < VEC_EPT; ++e) {
            const int i = base + e * VEC_NT;
            if (i < n) vnext[i] = (T)((double)w[i] / hk1);
        }
    }
    if (bid != 0) return;
    // block 0: column k of H and the earlier rotations go to LDS with all
    // threads, then one thread rotates the column there (a single thread
    // reading them from memory waits for every load in turn)
    __shared__ double col[KS_MAX_RESTART + 1], rcs[KS_MAX_RESTART], rsn[KS_MAX_RESTART];
    const int m = ga.m;
    double *H = ga.H, *R = ga.R;
    for (int j = threadIdx.x; j <= k; j += VEC_NT) col[j] = H[(size_t)j * m + k];
    for (int q = threadIdx.x; q < k; q += VEC_NT) {
        rcs[q] = ga.cs[q];
        rsn[q] = ga.sn[q];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    H[(size_t)(k + 1) * m + k] = hk1;
    col[k + 1] = hk1;
    for (int q = 0; q < k; ++q) {
        const double a = col[q], bb = col[q + 1];
        col[q] = rcs[q] * a + rsn[q] * bb;
        col[q + 1] = -rsn[q] * a + rcs[q] * bb;
    }
    const double akk = col[k], bk = col[k + 1];
    const double rho = hypot(akk, bk);
    for (int j = 0; j <= k + 1; ++j) R[(size_t)j * m + k] = col[j];
    st->hk1 = hk1;
    if (!finite_d(rho) || !finite_d(avk)) {
        st->flags |= F_NONFIN | F_STOP;
    } else if (rho == 0.0) {
        st->flags |= F_BREAK | F_STOP;
    } else {
        const double c = akk / rho, sn = bk / rho;
        ga.cs[k] = c;
        ga.sn[k] = sn;
        R[(size_t)k * m + k] = rho;
        R[(size_t)(k + 1) * m + k] = 0.0;
        const double gk = ga.g[k];
        ga.g[k + 1] = -sn * gk;
        ga.g[k] = c * gk;
        st->k_done = k + 1;
        if (hk1 <= HAPPY_FACTOR * avk)
            st->flags |= F_HAPPY | F_STOP;
        else if (fabs(ga.g[k + 1]) <= gm_threshold(st))
            st->flags |= F_CONV | F_STOP;
        else if (st->iters >= max_iter)
            st->flags |= F_MAXIT | F_STOP;
    }
}

// End of a cycle: R y = g by back substitution (each block redundantly, it is
// at most m x m), then x += V y for the block's rows.
template <typename T>
__device__ __forceinline__ void gm_finish_body(int n, int ldv, const T *__restrict__ V,
                                               T *__restrict__ x, const State *st, GmArrays ga,
                                               int bid) {
    __shared__ double y[KS_MAX_RESTART];
    const int kd = st->k_done;
    if (kd <= 0) return;
    if (threadIdx.x == 0) {
        const int m = ga.m;
        for (int r = kd - 1; r >= 0; --r) {
            double s = ga.g[r];
            for (int j = r + 1; j < kd; ++j) s -= ga.R[(size_t)r * m + j] * y[j];
            y[r] = s / ga.R[(size_t)r * m + r];
        }
        if (bid == 0)
            for (int j = 0; j < kd; ++j) ga.y[j] = y[j];
    }
    __syncthreads();
    const int i = bid * CGS_NT + threadIdx.x;
    if (i < n) {
        double s = 0.0;
        for (int j = 0; j < kd; ++j) s = fma((double)V[(size_t)j * ldv + i], y[j], s);
        x[i] = (T)((double)x[i] + s);
    }
}

}  // namespace ks
