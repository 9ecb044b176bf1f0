// mda_group.hip -- launchers of the workgroup form (one replica over WR x WC
// waves; the kernel is in mda_group.h).  Each register tile is instantiated in
// its own translation unit (mda_group_ns*.hip) so that the tiles compile in
// parallel.
#include <hip/hip_runtime.h>

#include "mda_desc.h"

namespace mda {

constexpr int kMaxGroupWavesHost = 8;

#define MDA_GNS_LIST(X) X(8) X(16) X(24) X(32) X(40) X(48) X(56) X(64)

#define MDA_GROUP_DECL(N)                                                                                \
    hipError_t launch_group_ns##N(int occ, int wr, int wc, const RunDesc *runs, const WorkItem *work,   \
                                  int nwork, const int32_t *lnt, int grid, hipStream_t stream);          \
    hipError_t group_occupancy_ns##N(int occ, int wr, int wc, int *blocks_per_cu);
MDA_GNS_LIST(MDA_GROUP_DECL)
#undef MDA_GROUP_DECL

int group_waves_limit(int ns)
{
    return ns <= 16 ? kMaxGroupWavesHost : 4;
}

hipError_t launch_group(int ns, int occ, int wr, int wc, const RunDesc *runs, const WorkItem *work, int nwork,
                        const int32_t *lnt, int grid, hipStream_t stream)
{
    if (wr < 1 || wc < 1 || wr * wc > group_waves_limit(ns)) return hipErrorInvalidValue;
    switch (ns) {
#define X(N) \
    case N:  \
        return launch_group_ns##N(occ, wr, wc, runs, work, nwork, lnt, grid, stream);
        MDA_GNS_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t group_occupancy(int ns, int occ, int wr, int wc, int *blocks_per_cu)
{
    switch (ns) {
#define X(N) \
    case N:  \
        return group_occupancy_ns##N(occ, wr, wc, blocks_per_cu);
        MDA_GNS_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace mda
