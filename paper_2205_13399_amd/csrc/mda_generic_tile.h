// mda_generic_tile.h -- launchers of the K-objective kernels for one K
// (MDA_GK), every slot count S with K * S <= 64 (register resident); included by the translation
// unit of that K so that the K compile in parallel.
#pragma once

#include "mda_generic.h"

namespace mda {

#define MDA_GCAT2(a, b) a##b
#define MDA_GCAT(a, b) MDA_GCAT2(a, b)

hipError_t MDA_GCAT(launch_generic_k, MDA_GK)(int S, const GRunDesc *run, const int32_t *lnt, unsigned int *next,
                                             int grid, int block, size_t dyn_lds, hipStream_t stream, int R)
{
    const int nd_grid = (R * 64 + 255) / 256;
    switch (S) {
#define GX(SS)                                                                                               \
    case SS: {                                                                                               \
        if (MDA_GK * SS > 64) return hipErrorInvalidValue;                                                   \
        auto kern = k_generic<MDA_GK, (MDA_GK * SS <= 64 ? SS : 8)>;                                         \
        const hipError_t ea = hipFuncSetAttribute((const void *)kern,                                        \
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds); \
        if (ea != hipSuccess) return ea;                                                                     \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), dyn_lds, stream, run, lnt, next);                  \
        break;                                                                                               \
    }
        GX(8) GX(16) GX(32) GX(64)
#undef GX
    default:
        return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_gnondominated<MDA_GK>), dim3(nd_grid), dim3(256), 0, stream, run);
    return hipGetLastError();
}

hipError_t MDA_GCAT(generic_occupancy_k, MDA_GK)(int S, int block, size_t dyn_lds, int *blocks_per_cu)
{
    switch (S) {
#define GX(SS)                                                                                                 \
    case SS: {                                                                                                 \
        auto kern = k_generic<MDA_GK, (MDA_GK * SS <= 64 ? SS : 8)>;                                           \
        const hipError_t ea = hipFuncSetAttribute((const void *)kern,                                          \
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds);   \
        if (ea != hipSuccess) return ea;                                                                       \
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, block, dyn_lds);              \
    }
        GX(8) GX(16) GX(32) GX(64)
#undef GX
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t MDA_GCAT(launch_gfront_k, MDA_GK)(const GRunDesc *run, int r0, int nr, const int64_t *offs, int64_t total,
                                            GFrontEntry *cand, GFrontEntry *ref, GFrontEntry *keep,
                                            unsigned long long *nkeep, hipStream_t stream)
{
    hipLaunchKernelGGL((k_ggather<MDA_GK>), dim3((nr + 3) / 4), dim3(256), 0, stream, run, r0, nr, offs, cand, ref);
    hipLaunchKernelGGL((k_gfilter<MDA_GK>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, cand, total,
                       ref, nr * (MDA_GK + 1), keep, nkeep);
    return hipGetLastError();
}

hipError_t MDA_GCAT(launch_gexact_k, MDA_GK)(const GFrontEntry *keep, int64_t n, GFrontEntry *front,
                                            unsigned long long *nfront, hipStream_t stream)
{
    if (n > 0)
        hipLaunchKernelGGL((k_gexact<MDA_GK>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, keep, n, front,
                           nfront);
    return hipGetLastError();
}

}  // namespace mda
