// Host-side helpers shared by the single-tensor and the batched drivers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <vector>

#include "ttsvd.h"

namespace ttsvd {

bool valid_dtype(int dt);

__host__ __device__ constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Shapes of every step for the rank upper bounds (the no-tolerance ranks):
// step i (1 <= i < d, 0-based mode index) has m = dims[i] rb[i+1] columns.
struct StepShape {
    int64_t m, rows, K, rb;  // columns, rows, min(rows, m), rank bound
};

// Fills steps[1..d-1] and the rank bounds rb[0..d]; validates dims.
int plan_steps(const int64_t *dims, int d, int64_t r_max, std::vector<StepShape> &steps,
               std::vector<int64_t> &rb, int64_t &nbar_out);

// Library-owned device buffers (workspaces and result cores): a per-device
// cache of hipMalloc blocks reused across calls.  cache_acquire returns a
// block of at least `bytes` bytes that no other call holds (NULL if the
// allocation fails); cache_release hands it back, and the caller releases
// only once no pending device work uses the block (after synchronising the
// stream that used it, or from a host callback enqueued on that stream).
// Blocks stay mapped between calls, so repeated calls neither map nor clear
// memory; idle blocks beyond kCacheIdleBytes per device are freed.
void *cache_acquire(size_t bytes);
void cache_release(void *p);
// cache_release enqueued on stream s: runs once the work before it is done.
hipError_t cache_release_async(void *p, hipStream_t s);

// Result cores: cache blocks released by ttsvd_tt_free after a device
// synchronisation (so, as with hipFree, no pending work can still read them).
void *result_alloc(size_t bytes);
void result_free(void *p);

// Pinned host staging buffer of at least `bytes` bytes owned by the calling
// thread (grown on demand, kept for the thread's lifetime); device<->host
// copies of results and metadata go through it, so they are plain DMA
// transfers ordered on their stream.  NULL if the allocation fails.
void *pinned_stage(size_t bytes);

// Cooperative launch that starts only after every earlier cooperative launch
// of the library on this device has finished (whatever its stream): two
// grid-synchronising kernels that each hold part of the GPU while waiting for
// the rest could otherwise wait on each other.
hipError_t coop_launch(const void *fn, dim3 grid, dim3 block, void **args, size_t lds,
                       hipStream_t s);

// Device buffer shared by the results of one batched call: the last
// ttsvd_tt_free of those results releases it.
struct SharedDev {
    void *ptr = nullptr;
    std::atomic<int> refs{0};
};

// Owner of the library-allocated outputs of one ttsvd_tt.
struct TTPriv {
    double *cores_dev = nullptr;   // own allocation (single-tensor path)
    SharedDev *shared = nullptr;   // shared allocation (batched path)
    std::vector<double *> sigma_host;
};

}  // namespace ttsvd
