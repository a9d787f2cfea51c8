// Small synchronous transfers between device and host for the solver's
// decisions (ranks, pivot counts, convergence flags, norms).  See readback.hip.
#pragma once
#include <cstddef>

#include "common.h"

namespace t2s2 {

// Copy bytes from device memory d to host memory h after all earlier work on
// stream s; returns once h holds the data.  Up to kReadbackMax bytes go
// through a pinned host mailbox written by a kernel (no runtime
// synchronisation); larger reads, or a host thread whose mailbox could not be
// allocated, use hipMemcpyAsync + hipStreamSynchronize.  Errors of earlier
// work on s are reported as Error, as a stream synchronisation would.
void host_read(hipStream_t s, void* h, const void* d, size_t bytes);

// Copy bytes from host memory h to device memory d after all earlier work
// on stream s; returns once the copy is complete (h may be reused).
void host_write(hipStream_t s, void* d, const void* h, size_t bytes);

constexpr size_t kReadbackMax = 64 * 1024;

}  // namespace t2s2
