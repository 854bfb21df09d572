// Optional per-launch timing of the library's kernels with HIP events on the
// launch stream.  Disabled by default; when disabled the hooks cost one
// relaxed atomic load.
#pragma once

#include <hip/hip_runtime.h>

namespace ttsvd {

// Records a start event on s for a kernel named `name` that moves `bytes`
// algorithmic bytes and performs `flops` floating point operations.
void prof_begin(hipStream_t s, const char *name, double bytes, double flops);
// Records the matching stop event on s.
void prof_end(hipStream_t s);
// Whether recording is on.
bool prof_on();
// Adds a record measured by other means (e.g. device clocks), in ms.
void prof_add(const char *name, double ms, double bytes, double flops);

}  // namespace ttsvd
