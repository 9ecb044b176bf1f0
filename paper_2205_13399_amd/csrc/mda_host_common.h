// mda_host_common.h -- host-side pieces shared by the library's translation
// units: error reporting, the device allocator behind mda_set_allocator, and
// the fixed-point tables of the acceptance test (the quantised -ln(u) and the
// geometric temperature schedule).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mda.h"

namespace mda {

// Records a formatted message for mda_last_error and returns code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::mda::fail(MDA_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// One device allocation, with what it takes to release it.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    mda_free_fn release = nullptr;
    void *ctx = nullptr;
    bool async = false;
};

// Device buffers of one handle, from the installed allocator (or hipMalloc),
// stream-ordered when the calling thread asked for it (the serving engine).
struct DevPool {
    std::vector<DevBuf> bufs;
    int64_t total = 0;

    void *alloc_bytes(size_t bytes, hipStream_t stream);
    template <class T>
    T *alloc(size_t count, hipStream_t stream)
    {
        return static_cast<T *>(alloc_bytes(count * sizeof(T), stream));
    }
    void release_all();
};

// Quantised -ln(u): LNT[k] = round(-ln((k + 1/2) / 4096) * 2^16).
void threshold_table(int32_t *lnt);

// Largest scaled temperature T = floor(256 delta) a run accepts.
constexpr double kMaxTemp = (double)((int64_t)1 << 43);

// Geometric cooling evaluated at the top of every step; T_t = floor(256 delta_t),
// until the temperature stops changing.  Returns the number of entries.
int64_t temperature_table(double delta0, double deltaf, double xi, int64_t steps, std::vector<int64_t> &T);

}  // namespace mda
