// mda_wave_tile.h -- launchers of one register tile of the one-wave kernels;
// included by the translation unit of that tile (MDA_TILE).
#pragma once

#include "mda_wave.h"

namespace mda {

#define MDA_CAT2(a, b) a##b
#define MDA_CAT(a, b) MDA_CAT2(a, b)

// Dynamic LDS of the persistent kernel: kWaveLds words per wave (the 4096-word
// table and the flip's staging words), 68 KB for the largest block (four
// waves).
inline size_t persistent_lds(int block)
{
    return (size_t)(block / 64) * kWaveLds * sizeof(int32_t);
}

// Kernel of step variant sv (the six values of MDA_STEP_VARIANTS), or
// nullptr for a value out of range.
template <int OCC, int F64>
static const void *persistent_kernel(int sv)
{
    switch (sv) {
#define X(PV, AM) \
    case PV * 2 + AM: return reinterpret_cast<const void *>(&k_persistent<MDA_TILE, OCC, F64, PV * 2 + AM>);
        MDA_STEP_VARIANTS(X)
#undef X
    default: return nullptr;
    }
}

static hipError_t launch_kernel(const void *k, const RunDesc *runs, const WorkItem *work, int nwork,
                                const int32_t *lnt, unsigned int *next, int grid, int block, hipStream_t stream)
{
    if (!k) return hipErrorInvalidValue;
    void *args[] = {(void *)&runs, (void *)&work, (void *)&nwork, (void *)&lnt, (void *)&next};
    return hipLaunchKernel(k, dim3(grid), dim3(block), args, persistent_lds(block), stream);
}

#ifdef MDA_F64
// int64 differences: one build, the natural register budget (its state is
// twice that of the int32 build, so a second wave per SIMD would only spill).
hipError_t MDA_CAT(launch_persistent64_ns, MDA_TILE)(int sv, const RunDesc *runs, const WorkItem *work, int nwork,
                                                    const int32_t *lnt, unsigned int *next, int grid, int block,
                                                    hipStream_t stream)
{
    return launch_kernel(persistent_kernel<1, 1>(sv), runs, work, nwork, lnt, next, grid, block, stream);
}

hipError_t MDA_CAT(persistent64_occupancy_ns, MDA_TILE)(int sv, int block, int *blocks_per_cu)
{
    const void *k = persistent_kernel<1, 1>(sv);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, block, persistent_lds(block));
}
#else
// From 32 slots up a second build holds two waves per SIMD (see k_persistent).
constexpr int kTileOcc2 = MDA_TILE >= 32 ? 2 : 1;

static const void *persistent_kernel_occ(int occ, int sv)
{
    return (occ >= 2 && kTileOcc2 == 2) ? persistent_kernel<kTileOcc2, 0>(sv) : persistent_kernel<1, 0>(sv);
}

hipError_t MDA_CAT(launch_persistent_ns, MDA_TILE)(int occ, int sv, const RunDesc *runs, const WorkItem *work,
                                                  int nwork, const int32_t *lnt, unsigned int *next, int grid,
                                                  int block, hipStream_t stream)
{
    return launch_kernel(persistent_kernel_occ(occ, sv), runs, work, nwork, lnt, next, grid, block, stream);
}

hipError_t MDA_CAT(persistent_occupancy_ns, MDA_TILE)(int occ, int sv, int block, int *blocks_per_cu)
{
    const void *k = persistent_kernel_occ(occ, sv);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, block, persistent_lds(block));
}

// Plain step kernel of step variant sv, or nullptr for a value out of range.
static const void *plain_step_kernel(int sv)
{
    switch (sv) {
#define X(PV, AM) \
    case PV * 2 + AM: return reinterpret_cast<const void *>(&k_plain_step<MDA_TILE, PV * 2 + AM>);
        MDA_STEP_VARIANTS(X)
#undef X
    default: return nullptr;
    }
}

hipError_t MDA_CAT(launch_plain_ns, MDA_TILE)(int sv, const RunDesc *run, int R, uint32_t steps, const int32_t *lnt,
                                             int block, hipStream_t stream)
{
    const void *k = plain_step_kernel(sv);
    if (!k) return hipErrorInvalidValue;
    const int wpb = block / 64;
    const int grid = (R + wpb - 1) / wpb;
    hipLaunchKernelGGL(k_plain_init<MDA_TILE>, dim3(grid), dim3(block), 0, stream, run);
    for (uint32_t t = 1; t <= steps; ++t) {
        uint32_t tt = t;
        void *args[] = {(void *)&run, (void *)&tt, (void *)&lnt};
        const hipError_t e = hipLaunchKernel(k, dim3(grid), dim3(block), args, 0, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_plain_final<MDA_TILE>, dim3(grid), dim3(block), 0, stream, run);
    return hipGetLastError();
}
#endif

}  // namespace mda
