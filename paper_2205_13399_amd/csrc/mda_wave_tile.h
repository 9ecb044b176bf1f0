// mda_wave_tile.h -- launchers of one register tile of the one-wave kernels;
// included by the translation unit of that tile (MDA_TILE).
#pragma once

#include "mda_wave.h"

namespace mda {

#define MDA_CAT2(a, b) a##b
#define MDA_CAT(a, b) MDA_CAT2(a, b)

// Dynamic LDS of the persistent kernel: 4096 words per wave, 64 KB for the
// largest block (four waves).
inline size_t persistent_lds(int block)
{
    return (size_t)(block / 64) * 4096 * sizeof(int32_t);
}

#ifdef MDA_F64
// int64 differences: one build, the natural register budget (its state is
// twice that of the int32 build, so a second wave per SIMD would only spill).
hipError_t MDA_CAT(launch_persistent64_ns, MDA_TILE)(const RunDesc *runs, const WorkItem *work, int nwork,
                                                    const int32_t *lnt, unsigned int *next, int grid, int block,
                                                    hipStream_t stream)
{
    hipLaunchKernelGGL((k_persistent<MDA_TILE, 1, 1>), dim3(grid), dim3(block), persistent_lds(block), stream, runs,
                       work, nwork, lnt, next);
    return hipGetLastError();
}

hipError_t MDA_CAT(persistent64_occupancy_ns, MDA_TILE)(int block, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent<MDA_TILE, 1, 1>, block,
                                                        persistent_lds(block));
}
#else
// From 40 slots up a second build holds two waves per SIMD (see k_persistent).
constexpr int kTileOcc2 = MDA_TILE >= 40 ? 2 : 1;

hipError_t MDA_CAT(launch_persistent_ns, MDA_TILE)(int occ, const RunDesc *runs, const WorkItem *work, int nwork,
                                                  const int32_t *lnt, unsigned int *next, int grid, int block,
                                                  hipStream_t stream)
{
    const size_t lds = persistent_lds(block);
    if (occ >= 2 && kTileOcc2 == 2) {
        hipLaunchKernelGGL((k_persistent<MDA_TILE, kTileOcc2, 0>), dim3(grid), dim3(block), lds, stream, runs, work,
                           nwork, lnt, next);
    } else {
        hipLaunchKernelGGL((k_persistent<MDA_TILE, 1, 0>), dim3(grid), dim3(block), lds, stream, runs, work, nwork,
                           lnt, next);
    }
    return hipGetLastError();
}

hipError_t MDA_CAT(persistent_occupancy_ns, MDA_TILE)(int occ, int block, int *blocks_per_cu)
{
    const size_t lds = persistent_lds(block);
    if (occ >= 2 && kTileOcc2 == 2) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent<MDA_TILE, kTileOcc2, 0>, block,
                                                            lds);
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persistent<MDA_TILE, 1, 0>, block, lds);
}

hipError_t MDA_CAT(launch_plain_ns, MDA_TILE)(const RunDesc *run, int R, uint32_t steps, const int32_t *lnt, int block,
                                             hipStream_t stream)
{
    const int wpb = block / 64;
    const int grid = (R + wpb - 1) / wpb;
    hipLaunchKernelGGL(k_plain_init<MDA_TILE>, dim3(grid), dim3(block), 0, stream, run);
    for (uint32_t t = 1; t <= steps; ++t)
        hipLaunchKernelGGL(k_plain_step<MDA_TILE>, dim3(grid), dim3(block), 0, stream, run, t, lnt);
    hipLaunchKernelGGL(k_plain_final<MDA_TILE>, dim3(grid), dim3(block), 0, stream, run);
    return hipGetLastError();
}
#endif

}  // namespace mda
