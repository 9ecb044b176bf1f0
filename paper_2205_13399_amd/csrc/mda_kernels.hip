// mda_kernels.hip -- kernels of the multi-objective Digital Annealer that are
// built once (non-dominated flags, gather of flagged archive entries, the dense
// QUBO builder) and the dispatch of the one-wave annealing kernels (mda_wave.h)
// to their per-tile translation units (mda_wave_ns*.hip).
#include "mda_wave.h"

namespace mda {

// Non-dominated flags of every archive member within its replica's archive
// (Algorithm 3, final line), one wave per replica.
__global__ void __launch_bounds__(256) k_nondominated(const RunDesc *runs, const WorkItem *work, int nwork)
{
    const int lane = __lane_id();
    const int item = uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (item >= nwork) return;
    const WorkItem w = {ro(work)[item].run, ro(work)[item].replica};
    Desc &D = ro(runs)[uni(w.run)];
    const int r = uni(w.replica);
    const int s = D.s;
    int asz = uni((int)rw(D.st)[(size_t)r * kStWords + kStArch]);
    asz = asz < 0 ? 0 : (asz > s ? s : asz);
    // the archive is only read here, so the scan goes through the constant
    // path: the entries compared against are uniform and load as scalars, 8 at
    // a time so that their latencies overlap
    const MDA_CONST int64_t *AE = ro(D.archE) + (size_t)r * s * 2;
    MDA_GLOBAL uint8_t *nd = rw(D.nd) + (size_t)r * s;
    int count = 0;
    for (int b = 0; b < asz; b += 64) {
        const int e = b + lane;
        const int ec = e < asz ? e : asz - 1;
        const int64_t a1 = AE[2 * ec], a2 = AE[2 * ec + 1];
        bool dom = false;
        int f = 0;
        for (; f + 8 <= asz; f += 8) {
            int64_t q1[8], q2[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                q1[k] = AE[2 * (f + k)];
                q2[k] = AE[2 * (f + k) + 1];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) dom |= dominates(q1[k], q2[k], a1, a2);
        }
        for (; f < asz; ++f) dom |= dominates(AE[2 * f], AE[2 * f + 1], a1, a2);
        if (e < asz) {
            nd[e] = dom ? 0 : 1;
            count += dom ? 0 : 1;
        }
    }
    count = wave_sum(count);
    if (lane == 0) rw(D.st)[(size_t)r * kStWords + kStNd] = count;
}

// Gathers the flagged (non-dominated) entries of replicas [r0, r0 + nr) of one
// run into out, replica k's entries at out[offs[k] ...] in slot order.  One
// wave per replica; offs holds the exclusive prefix sum of the counts that
// k_nondominated wrote.
__global__ void __launch_bounds__(256) k_front_gather(const int64_t *archE, const uint8_t *ndf, const int64_t *st,
                                                      int s, int r0, int nr, const int64_t *offs, FrontEntry *out)
{
    const int lane = __lane_id();
    const int k = uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (k >= nr) return;
    const int r = r0 + k;
    int asz = uni((int)rw(st)[(size_t)r * kStWords + kStArch]);
    asz = asz < 0 ? 0 : (asz > s ? s : asz);
    const MDA_GLOBAL int64_t *AE = rw(archE) + (size_t)r * s * 2;
    const MDA_GLOBAL uint8_t *nd = rw(ndf) + (size_t)r * s;
    MDA_GLOBAL FrontEntry *o = rw(out) + rw(offs)[k];
    int base = 0;
    for (int b = 0; b < asz; b += 64) {
        const int e = b + lane;
        const bool keep = e < asz && nd[e] != 0;
        const uint64_t mask = __ballot(keep);
        if (keep) {
            const int rank = base + __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            o[rank].e1 = AE[2 * e];
            o[rank].e2 = AE[2 * e + 1];
            o[rank].replica = r;
            o[rank].slot = e;
        }
        base += __popcll(mask);
    }
}

// Dense P_k of the bQAP QUBO built on the device.  Row a = (i, u) is stored
// as n blocks of ld entries, P[a][(j, v)] at j * ld + v, zero for v >= n
// (ld = n: the plain m x m layout):
// P[a][b] = F[i][j] D[u][v] + F[j][i] D[v][u] + 2 alpha [(i == j) != (u == v)]
// off the diagonal, F[i][i] D[u][u] - 2 alpha on it.
__global__ void k_build_dense(int n, int ld, const int32_t *__restrict__ F, const int32_t *__restrict__ Dm,
                              int32_t two_alpha, int32_t *__restrict__ P)
{
    const int m = n * n;
    const size_t row = (size_t)n * ld;
    const size_t total = (size_t)m * row;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
        const int a = (int)(k / row);
        const int j = (int)((k % row) / ld), v = (int)(k % ld);
        if (v >= n) {
            P[k] = 0;
            continue;
        }
        const int b = j * n + v;
        const int i = a / n, u = a % n;
        uint32_t val;
        if (a == b) {
            val = (uint32_t)(F[i * n + i] * Dm[u * n + u]) - (uint32_t)two_alpha;
        } else {
            val = (uint32_t)(F[i * n + j] * Dm[u * n + v]) + (uint32_t)(F[j * n + i] * Dm[v * n + u]);
            if ((i == j) != (u == v)) val += (uint32_t)two_alpha;
        }
        P[k] = (int32_t)val;
    }
}

// ---------------------------------------------------------------- host launchers

#define MDA_NS_LIST(X) X(8) X(16) X(24) X(28) X(32) X(40) X(48) X(52) X(56) X(64)


// Register slots of the one-wave kernels for n facilities: the next multiple
// of 8, except 28 for 25 to 28 and 52 for 49 to 52 facilities (four slots
// fewer of registers and of per-step work than 32 and 56).
int ns_for(int n)
{
    const int ns = ((n + 7) / 8) * 8;
    if ((ns == 32 || ns == 56) && n <= ns - 4) return ns - 4;
    return ns < 8 ? 8 : ns;
}

// Per-tile launchers, each defined in the translation unit that instantiates
// that tile (mda_wave_ns*.hip), so that the tiles compile in parallel.
#define MDA_WAVE_DECL(N)                                                                                   \
    hipError_t launch_persistent_ns##N(int occ, int sv, const RunDesc *runs, const WorkItem *work,         \
                                       int nwork, const int32_t *lnt, unsigned int *next, int grid,        \
                                       int block, hipStream_t stream);                                     \
    hipError_t persistent_occupancy_ns##N(int occ, int sv, int block, int *blocks_per_cu);                \
    hipError_t launch_plain_ns##N(int sv, const RunDesc *run, int R, uint32_t steps, const int32_t *lnt,    \
                                  int block, hipStream_t stream);                                          \
    hipError_t launch_persistent64_ns##N(int sv, const RunDesc *runs, const WorkItem *work, int nwork,     \
                                         const int32_t *lnt, unsigned int *next, int grid, int block,      \
                                         hipStream_t stream);                                              \
    hipError_t persistent64_occupancy_ns##N(int sv, int block, int *blocks_per_cu);
MDA_NS_LIST(MDA_WAVE_DECL)
#undef MDA_WAVE_DECL

__global__ void k_zero_counter(unsigned int *p)
{
    if (threadIdx.x == 0) *p = 0u;
}

hipError_t launch_zero_counter(unsigned int *p, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, p);
    return hipGetLastError();
}

// The persistent launch of one tile and step variant sv, preceded by the
// zeroing of its work-item counter (a kernel, so that the pair can be captured
// into a graph).
hipError_t launch_persistent(int ns, int occ, int f64, int sv, const RunDesc *runs, const WorkItem *work, int nwork,
                             const int32_t *lnt, unsigned int *next, int grid, int block, hipStream_t stream)
{
    if (sv < 0 || sv >= kStepVariants) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, next);
    switch (ns) {
#define X(N)                                                                                       \
    case N:                                                                                        \
        return f64 ? launch_persistent64_ns##N(sv, runs, work, nwork, lnt, next, grid, block, stream) \
                   : launch_persistent_ns##N(occ, sv, runs, work, nwork, lnt, next, grid, block, stream);
        MDA_NS_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t persistent_occupancy(int ns, int occ, int f64, int sv, int block, int *blocks_per_cu)
{
    switch (ns) {
#define X(N)                                                                     \
    case N:                                                                      \
        return f64 ? persistent64_occupancy_ns##N(sv, block, blocks_per_cu)      \
                   : persistent_occupancy_ns##N(occ, sv, block, blocks_per_cu);
        MDA_NS_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_plain(int ns, int sv, const RunDesc *run, int R, uint32_t steps, const int32_t *lnt, int block,
                        hipStream_t stream)
{
    switch (ns) {
#define X(N) \
    case N:  \
        return launch_plain_ns##N(sv, run, R, steps, lnt, block, stream);
        MDA_NS_LIST(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}



// Best archive entry of each of R replicas: least E_1, lowest slot on ties
// (one wave per replica).
__global__ void __launch_bounds__(256) k_best(const RunDesc *run, int64_t *e1_out, int32_t *slot_out)
{
    const int lane = __lane_id();
    const int r = uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    Desc &D = *ro(run);
    if (r >= D.R) return;
    const int s = D.s;
    int asz = uni((int)rw(D.st)[(size_t)r * kStWords + kStArch]);
    asz = asz < 0 ? 0 : (asz > s ? s : asz);
    const MDA_GLOBAL int64_t *AE = rw(D.archE) + (size_t)r * s * 2;
    int64_t be = INT64_MAX;
    int bs = INT_MAX;
    for (int e = lane; e < asz; e += 64) {
        const int64_t v = AE[2 * (size_t)e];
        if (v < be) {
            be = v;
            bs = e;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t ov = __shfl_xor(be, off);
        const int os = __shfl_xor(bs, off);
        if (ov < be || (ov == be && os < bs)) {
            be = ov;
            bs = os;
        }
    }
    if (lane == 0) {
        e1_out[r] = be;
        slot_out[r] = bs == INT_MAX ? -1 : bs;
    }
}

hipError_t launch_best(const RunDesc *run, int R, int64_t *e1, int32_t *slot, hipStream_t stream)
{
    hipLaunchKernelGGL(k_best, dim3((R + 3) / 4), dim3(256), 0, stream, run, e1, slot);
    return hipGetLastError();
}

hipError_t launch_nondominated(const RunDesc *runs, const WorkItem *work, int nwork, hipStream_t stream)
{
    const int block = 256;
    const int grid = (nwork * 64 + block - 1) / block;
    hipLaunchKernelGGL(k_nondominated, dim3(grid), dim3(block), 0, stream, runs, work, nwork);
    return hipGetLastError();
}

hipError_t launch_front_gather(const int64_t *archE, const uint8_t *nd, const int64_t *st, int s, int r0, int nr,
                               const int64_t *offs, FrontEntry *out, hipStream_t stream)
{
    const int block = 256;
    const int grid = (nr * 64 + block - 1) / block;
    hipLaunchKernelGGL(k_front_gather, dim3(grid), dim3(block), 0, stream, archE, nd, st, s, r0, nr, offs, out);
    return hipGetLastError();
}

hipError_t launch_build_dense(int n, int ld, const int32_t *F, const int32_t *Dm, int32_t two_alpha, int32_t *P,
                              hipStream_t stream)
{
    const size_t total = (size_t)n * n * n * ld;
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_build_dense, dim3((unsigned)blocks), dim3(256), 0, stream, n, ld, F, Dm, two_alpha, P);
    return hipGetLastError();
}


}  // namespace mda
