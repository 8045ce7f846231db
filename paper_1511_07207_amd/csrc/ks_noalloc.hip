// The symmetric product without a caller workspace: ks_symv_noalloc.
//
// ks_symv's tile kernel leaves two partial vectors per tile in a workspace
// the caller allocates (ks_symv_workspace_bytes).  For callers that cannot
// allocate device memory, this entry point puts those partials in `scratch`,
// a file-scope device array of fixed size (enough for n <= KS_SYMV_NOALLOC_MAX_N)
// that every GPU the library runs on holds from the code object's load until
// the process ends.  The kernels are ks_symv's own, so the result is the same
// bit for bit.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address of each GPU's copy is taken once per device with
// hipGetSymbolAddress (on the first call made while that device is current)
// and only that address is handed to kernels.
//
// Nothing in the array has to start at zero: every tile block writes all 2 x
// SY_T values of its partials before the finishing kernel, later on the same
// stream, reads them.  Calls that overlap in time on one GPU (other streams,
// other host threads) share the array and race; serialize them.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>

#include "ks.h"
#include "ks_internal.h"

using namespace ks;

namespace {

constexpr int NOALLOC_TILE_ROWS = KS_SYMV_NOALLOC_MAX_N / SY_T;
constexpr size_t NOALLOC_DOUBLES =
    (size_t)NOALLOC_TILE_ROWS * (NOALLOC_TILE_ROWS + 1) / 2 * 2 * SY_T;
static_assert(KS_SYMV_NOALLOC_MAX_N % SY_T == 0, "the maximum order is a whole number of tiles");

constexpr int NOALLOC_MAX_DEVICES = 64;

}  // namespace

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {

std::mutex g_scratch_mu;
double *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of the current device's copy of `scratch`, looked up on
// the first call for that device.
int scratch_for_current_device(double **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KS_EHIP;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return KS_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return KS_EHIP;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return KS_EDEVICE;
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return KS_EHIP;
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return KS_OK;
}

}  // namespace

extern "C" int ks_symv_noalloc(int32_t n, int64_t lda, const double *d_A, const double *d_x,
                               double *d_y, void *stream) {
    if (n < 1 || lda < n || !d_A || !d_x || !d_y) return KS_EINVAL;
    if (n > KS_SYMV_NOALLOC_MAX_N || sy_ws_doubles(n) > NOALLOC_DOUBLES) return KS_ETOOLARGE;
    if ((uintptr_t)d_A % 16 || (lda * 8) % 16 || (uintptr_t)d_x % 16 || (uintptr_t)d_y % 16)
        return KS_EINVAL;
    double *W = nullptr;
    const int rc = scratch_for_current_device(&W);
    if (rc) return rc;
    if (launch_symv(n, lda, d_A, d_x, d_y, W, nullptr, nullptr, nullptr, (hipStream_t)stream) !=
        hipSuccess)
        return KS_EHIP;
    return KS_OK;
}
