// mda_group_tile.h -- launchers of one register tile of the workgroup form;
// included by the translation unit of that tile (MDA_TILE).
#pragma once

#include "mda_group.h"

namespace mda {

#define MDA_GCAT2(a, b) a##b
#define MDA_GCAT(a, b) MDA_GCAT2(a, b)

// From 24 slots up a second build holds two workgroups per CU (see k_group).
constexpr int kGroupTileOcc2 = MDA_TILE >= 24 ? 2 : 1;

hipError_t MDA_GCAT(launch_group_ns, MDA_TILE)(int occ, int wr, int wc, const RunDesc *runs, const WorkItem *work,
                                               int nwork, const int32_t *lnt, int grid, hipStream_t stream)
{
    const dim3 block(64 * wr * wc);
    if (occ >= 2 && kGroupTileOcc2 == 2)
        hipLaunchKernelGGL((k_group<MDA_TILE, kGroupTileOcc2>), dim3(grid), block, 0, stream, runs, work, nwork, lnt,
                           wr, wc);
    else
        hipLaunchKernelGGL((k_group<MDA_TILE, 1>), dim3(grid), block, 0, stream, runs, work, nwork, lnt, wr, wc);
    return hipGetLastError();
}

hipError_t MDA_GCAT(group_occupancy_ns, MDA_TILE)(int occ, int wr, int wc, int *blocks_per_cu)
{
    const int threads = 64 * wr * wc;
    if (occ >= 2 && kGroupTileOcc2 == 2)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_group<MDA_TILE, kGroupTileOcc2>, threads, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_group<MDA_TILE, 1>, threads, 0);
}

}  // namespace mda
