// mda_internal.h -- library-internal hooks used by the serving engine.
#pragma once

#include <stdint.h>

#include <functional>

#include "mda.h"

namespace mda {

// Device allocations made by the calling thread are stream-ordered
// (hipMallocAsync / hipFreeAsync on the owning run's stream).
void set_stream_ordered_alloc(bool on);

// 1 when every kernel of the run's launch has finished, 0 while it runs, -1 on error.
int run_finished(mda_run *r);

// Records an error for mda_last_error and returns code.
int set_error(int code, const char *msg);

// Device bytes held by the QUBO handle.
int64_t qubo_device_bytes(const mda_qubo *q);

// Called once, from da_run_free, after the run's device memory (and its
// reference to the QUBO) has been released.
void set_release_hook(mda_run *r, std::function<void()> hook);

}  // namespace mda
