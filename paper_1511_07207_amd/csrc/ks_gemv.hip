// Single-solve launches of the matrix-vector kernels (bodies in ks_gemv_body.h).
#include "ks_gemv_body.h"

namespace ks {

template <typename TA>
__global__ __launch_bounds__(GEMV_NT) void gemv_plain_kernel(int n, int64_t lda, const TA *__restrict__ A,
                                                             const typename ATraits<TA>::TV *__restrict__ v,
                                                             typename ATraits<TA>::TV *__restrict__ y) {
    gemv_plain_body<TA>(n, lda, A, v, y, blockIdx.x);
}

template <typename TA>
__global__ __launch_bounds__(GEMV_NT) void cg_matvec_kernel(int n, int64_t lda, const TA *__restrict__ A,
                                                            const typename ATraits<TA>::TV *__restrict__ p,
                                                            typename ATraits<TA>::TV *__restrict__ q,
                                                            const State *st, double *partial) {
    cg_matvec_body<TA>(n, lda, A, p, q, st, partial, blockIdx.x);
}

template <typename TA>
__global__ __launch_bounds__(GEMV_NT) void gm_matvec_kernel(int n, int64_t lda, const TA *__restrict__ A,
                                                            const typename ATraits<TA>::TV *__restrict__ vk,
                                                            typename ATraits<TA>::TV *__restrict__ w,
                                                            const State *st, double *partial) {
    gm_matvec_body<TA>(n, lda, A, vk, w, st, partial, blockIdx.x);
}

template <typename TA>
__global__ __launch_bounds__(GEMV_NT) void residual_kernel(int n, int64_t lda, const TA *__restrict__ A,
                                                           const typename ATraits<TA>::TV *__restrict__ b,
                                                           const typename ATraits<TA>::TV *__restrict__ x,
                                                           typename ATraits<TA>::TV *__restrict__ r,
                                                           const State *st, double *partial, int gate) {
    residual_body<TA>(n, lda, A, b, x, r, st, partial, gate, blockIdx.x);
}

__global__ __launch_bounds__(ONE_NT) void residual_finish_kernel(int nblocks, State *st,
                                                                 const double *partial, int gate) {
    residual_finish_body(nblocks, st, partial, gate);
}

template <typename TA>
__global__ __launch_bounds__(GEMV_NT) void bs_vmatvec_kernel(int n, int64_t lda, const TA *__restrict__ A,
                                                             const typename ATraits<TA>::TV *__restrict__ p,
                                                             const typename ATraits<TA>::TV *__restrict__ r0,
                                                             typename ATraits<TA>::TV *__restrict__ v,
                                                             const State *st, double *partial) {
    bs_vmatvec_body<TA>(n, lda, A, p, r0, v, st, partial, blockIdx.x);
}

template <typename TA>
__global__ __launch_bounds__(GEMV_NT) void bs_tmatvec_kernel(int n, int64_t lda, const TA *__restrict__ A,
                                                             const typename ATraits<TA>::TV *__restrict__ s,
                                                             typename ATraits<TA>::TV *__restrict__ t,
                                                             State *st, const double *__restrict__ pss,
                                                             int nss, int max_iter, double *partial) {
    bs_tmatvec_body<TA>(n, lda, A, s, t, st, pss, nss, max_iter, partial, blockIdx.x);
}

__global__ __launch_bounds__(GEMV_NT) void norm_inf_kernel(int n, int64_t lda, const double *__restrict__ A,
                                                           double *partial) {
    norm_inf_body(n, lda, A, partial, blockIdx.x);
}

__global__ __launch_bounds__(ONE_NT) void norm_inf_finish_kernel(int nblocks, State *st,
                                                                 const double *partial) {
    norm_inf_finish_body(nblocks, st, partial);
}

// ------------------------------------------------------------- launchers
hipError_t launch_gemv(int n, int64_t lda, int a_dtype, const void *A, const void *v, void *y,
                       hipStream_t s) {
    dim3 block(GEMV_NT);
    switch (a_dtype) {
        case KS_DT_F64:
            gemv_plain_kernel<double><<<gemv_blocks<double>(n), block, 0, s>>>(n, lda, (const double *)A,
                                                             (const double *)v, (double *)y);
            break;
        case KS_DT_F32:
            gemv_plain_kernel<float><<<gemv_blocks<float>(n), block, 0, s>>>(n, lda, (const float *)A,
                                                            (const float *)v, (float *)y);
            break;
        case KS_DT_BF16:
            gemv_plain_kernel<bf16_t><<<gemv_blocks<bf16_t>(n), block, 0, s>>>(n, lda, (const bf16_t *)A,
                                                             (const float *)v, (float *)y);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TA, typename T>
hipError_t launch_residual(int n, int64_t lda, const TA *A, const T *b, const T *x, T *r,
                           State *st, Partials P, int gate, hipStream_t s) {
    const int nb = gemv_blocks<TA>(n);
    residual_kernel<TA><<<nb, GEMV_NT, 0, s>>>(n, lda, A, b, x, r, st, P.g, gate);
    residual_finish_kernel<<<1, ONE_NT, 0, s>>>(nb, st, P.g, gate);
    return hipGetLastError();
}

template <typename TA, typename T>
hipError_t launch_residual_rows(int n, int64_t lda, const TA *A, const T *b, const T *x, T *r,
                                const State *st, double *partial, int gate, hipStream_t s) {
    residual_kernel<TA><<<gemv_blocks<TA>(n), GEMV_NT, 0, s>>>(n, lda, A, b, x, r, st, partial, gate);
    return hipGetLastError();
}

template <typename TA, typename T>
hipError_t launch_cg_matvec(int n, int64_t lda, const TA *A, const T *p, T *q, State *st,
                            Partials P, hipStream_t s) {
    cg_matvec_kernel<TA><<<gemv_blocks<TA>(n), GEMV_NT, 0, s>>>(n, lda, A, p, q, st, P.g);
    return hipGetLastError();
}

template <typename TA, typename T>
hipError_t launch_gm_matvec(int n, int64_t lda, const TA *A, const T *vk, T *w, State *st,
                            Partials P, hipStream_t s) {
    gm_matvec_kernel<TA><<<gemv_blocks<TA>(n), GEMV_NT, 0, s>>>(n, lda, A, vk, w, st, P.g);
    return hipGetLastError();
}

template <typename TA, typename T>
hipError_t launch_bs_vmatvec(int n, int64_t lda, const TA *A, const T *p, const T *r0, T *v,
                             State *st, Partials P, hipStream_t s) {
    bs_vmatvec_kernel<TA><<<gemv_blocks<TA>(n), GEMV_NT, 0, s>>>(n, lda, A, p, r0, v, st, P.g);
    return hipGetLastError();
}

template <typename TA, typename T>
hipError_t launch_bs_tmatvec(int n, int64_t lda, const TA *A, const T *sv, T *t, State *st,
                             Partials P, int max_iter, hipStream_t s) {
    bs_tmatvec_kernel<TA><<<gemv_blocks<TA>(n), GEMV_NT, 0, s>>>(n, lda, A, sv, t, st, P.v,
                                                                 vec_blocks(n), max_iter, P.g);
    return hipGetLastError();
}

hipError_t launch_norm_inf(int n, int64_t lda, const double *A, State *st, Partials P,
                           hipStream_t s) {
    const int nb = gemv_blocks<double>(n);
    norm_inf_kernel<<<nb, GEMV_NT, 0, s>>>(n, lda, A, P.g);
    norm_inf_finish_kernel<<<1, ONE_NT, 0, s>>>(nb, st, P.g);
    return hipGetLastError();
}

#define KS_INST_GEMV(TA, T)                                                                      \
    template hipError_t launch_residual<TA, T>(int, int64_t, const TA *, const T *, const T *,  \
                                               T *, State *, Partials, int, hipStream_t);        \
    template hipError_t launch_residual_rows<TA, T>(int, int64_t, const TA *, const T *,         \
                                                    const T *, T *, const State *, double *, int, \
                                                    hipStream_t);                                \
    template hipError_t launch_cg_matvec<TA, T>(int, int64_t, const TA *, const T *, T *,        \
                                                State *, Partials, hipStream_t);                 \
    template hipError_t launch_gm_matvec<TA, T>(int, int64_t, const TA *, const T *, T *,        \
                                                State *, Partials, hipStream_t);                 \
    template hipError_t launch_bs_vmatvec<TA, T>(int, int64_t, const TA *, const T *, const T *, \
                                                 T *, State *, Partials, hipStream_t);           \
    template hipError_t launch_bs_tmatvec<TA, T>(int, int64_t, const TA *, const T *, T *,       \
                                                 State *, Partials, int, hipStream_t);

KS_INST_GEMV(double, double)
KS_INST_GEMV(float, float)
KS_INST_GEMV(bf16_t, float)

}  // namespace ks
