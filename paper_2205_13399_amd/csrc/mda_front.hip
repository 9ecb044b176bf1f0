// mda_front.hip -- device pre-filter of the candidates for the merged
// non-dominated archive (Sec. 3.3): among the entries gathered from every
// replica's archive, those dominated by an entry of strictly smaller E1 are
// dropped before the host merge.
#include <algorithm>

#include "mda_device.h"

namespace mda {

// Pre-filter of gathered entries before the host merge: entries are binned by
// E1 over [lo, hi]; an entry whose E2 is not below the smallest E2 of every
// lower bin is dominated by an entry with strictly smaller E1 and is dropped.
// The survivors are compacted in arbitrary order (the host sorts them).
constexpr int kFrontBins = 16384;

__device__ __forceinline__ int front_bin(int64_t e1, int64_t lo, int64_t hi)
{
    const int64_t span = hi - lo + 1;
    return (int)(((e1 - lo) * (int64_t)kFrontBins) / span);
}

__global__ void k_front_range(const FrontEntry *ent, int64_t count, long long *lohi)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x) {
        atomicMin(&lohi[0], (long long)ent[k].e1);
        atomicMax(&lohi[1], (long long)ent[k].e1);
    }
}

__global__ void k_front_binmin(const FrontEntry *ent, int64_t count, const long long *lohi, long long *binmin)
{
    const int64_t lo = lohi[0], hi = lohi[1];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        atomicMin(&binmin[front_bin(ent[k].e1, lo, hi)], (long long)ent[k].e2);
}

// best[b] = min over bins below b of binmin (one block of 1024 threads).
__global__ void __launch_bounds__(1024) k_front_prefix(const long long *binmin, long long *best)
{
    __shared__ long long part[1024];
    constexpr int per = kFrontBins / 1024;
    const int t = (int)threadIdx.x;
    long long mn = LLONG_MAX;
    for (int q = 0; q < per; ++q) mn = min(mn, binmin[t * per + q]);
    part[t] = mn;
    __syncthreads();
    // exclusive prefix minimum over the 1024 chunk minima (serial in thread 0: tiny)
    if (t == 0) {
        long long run = LLONG_MAX;
        for (int c = 0; c < 1024; ++c) {
            const long long v = part[c];
            part[c] = run;
            run = min(run, v);
        }
    }
    __syncthreads();
    long long run = part[t];
    for (int q = 0; q < per; ++q) {
        best[t * per + q] = run;
        run = min(run, binmin[t * per + q]);
    }
}

__global__ void k_front_keep(const FrontEntry *ent, int64_t count, const long long *lohi, const long long *best,
                             FrontEntry *out, unsigned long long *nout)
{
    const int64_t lo = lohi[0], hi = lohi[1];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x) {
        const FrontEntry e = ent[k];
        if (e.e2 < best[front_bin(e.e1, lo, hi)]) {
            const unsigned long long at = atomicAdd(nout, 1ull);
            out[at] = e;
        }
    }
}

__global__ void k_front_init(long long *lohi, long long *binmin, unsigned long long *nout)
{
    for (int k = (int)(blockIdx.x * blockDim.x + threadIdx.x); k < kFrontBins; k += (int)(gridDim.x * blockDim.x))
        binmin[k] = LLONG_MAX;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        lohi[0] = LLONG_MAX;
        lohi[1] = LLONG_MIN;
        *nout = 0;
    }
}

size_t front_filter_scratch()
{
    return (2 + 2 * (size_t)kFrontBins + 1) * sizeof(long long);
}

hipError_t launch_front_filter(const FrontEntry *ent, int64_t count, void *scratch, FrontEntry *out,
                               unsigned long long *nout, hipStream_t stream)
{
    long long *lohi = (long long *)scratch;
    long long *binmin = lohi + 2;
    long long *best = binmin + kFrontBins;
    const int grid = (int)std::min<int64_t>(4096, (count + 255) / 256 + 1);
    hipLaunchKernelGGL(k_front_init, dim3(64), dim3(256), 0, stream, lohi, binmin, nout);
    hipLaunchKernelGGL(k_front_range, dim3(grid), dim3(256), 0, stream, ent, count, lohi);
    hipLaunchKernelGGL(k_front_binmin, dim3(grid), dim3(256), 0, stream, ent, count, lohi, binmin);
    hipLaunchKernelGGL(k_front_prefix, dim3(1), dim3(1024), 0, stream, binmin, best);
    hipLaunchKernelGGL(k_front_keep, dim3(grid), dim3(256), 0, stream, ent, count, lohi, best, out, nout);
    return hipGetLastError();
}

}  // namespace mda
