// Allocation-free variant of ttsvd_tsqr_r: the reduction tree's triangular
// factors live in a fixed device array of this translation unit instead of a
// caller or stream-ordered workspace, so the call makes no device allocation.
#include <mutex>

#include "common.h"
#include "driver.h"
#include "kernels.h"

namespace ttsvd {
namespace {

constexpr size_t kScratchBytes = size_t(TTSVD_NOALLOC_SCRATCH_BYTES);
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

// The library's only file-scope device buffer.  Host code never passes its
// name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returned for the current device (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_ptr(void **out) {
    int dev = 0;
    TTSVD_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(TTSVD_EUNSUPPORTED, "tsqr_r_noalloc: device %d", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(TTSVD_EHIP, "tsqr_r_noalloc: hipGetSymbolAddress: %s",
                             hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return TTSVD_OK;
}

}  // namespace
}  // namespace ttsvd

using namespace ttsvd;

extern "C" {

int ttsvd_tsqr_r_noalloc(const void *W, int dtype, int64_t rows, int64_t cols, int64_t ld,
                         double *R, int64_t ldr, hipStream_t stream) {
    clear_error();
    if (!W || !R) return set_error(TTSVD_EINVAL, "tsqr_r_noalloc: NULL pointer");
    if (rows < 1 || cols < 1 || ld < rows || ldr < cols)
        return set_error(TTSVD_EINVAL,
                         "tsqr_r_noalloc: bad sizes rows=%lld cols=%lld ld=%lld ldr=%lld",
                         (long long)rows, (long long)cols, (long long)ld, (long long)ldr);
    if (!valid_dtype(dtype)) return set_error(TTSVD_EUNSUPPORTED, "tsqr_r_noalloc: dtype %d", dtype);
    if (cols > 1024) return set_error(TTSVD_EUNSUPPORTED, "tsqr_r_noalloc: cols > 1024");
    const size_t need = tsqr_workspace_bytes(dtype, rows, cols);
    if (need > kScratchBytes)
        return set_error(TTSVD_EINVAL,
                         "tsqr_r_noalloc: %lld x %lld needs %zu bytes of scratch, more than the "
                         "fixed %zu (use ttsvd_tsqr_r with a workspace)",
                         (long long)rows, (long long)cols, need, kScratchBytes);
    void *ws = nullptr;
    const int rc = scratch_ptr(&ws);
    if (rc != TTSVD_OK) return rc;
    return tsqr_launch(W, dtype, rows, cols, ld, R, ldr, ws, kScratchBytes, stream);
}

}  // extern "C"
