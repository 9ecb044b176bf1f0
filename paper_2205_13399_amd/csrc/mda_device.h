// mda_device.h -- device helpers shared by the one-wave and the workgroup
// annealing kernels of the MI355X multi-objective Digital Annealer: address
// spaces, the Philox4x32-10 block function, wave-level reductions, the replica
// register state and the acceptance-rule and update-path tags.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "mda_desc.h"

#define MDA_CONST __attribute__((address_space(4)))
#define MDA_GLOBAL __attribute__((address_space(1)))
#define MDA_LDS __attribute__((address_space(3)))

namespace mda {

// Read-only operands are read through the constant address space (scalar
// loads when the address is wave-uniform); buffers the kernels write go
// through the global address space.
using Desc = const MDA_CONST RunDesc;

template <class T>
__device__ __forceinline__ const MDA_CONST T *ro(const T *p)
{
    return (const MDA_CONST T *)p;
}

template <class T>
__device__ __forceinline__ MDA_GLOBAL T *rw(T *p)
{
    return (MDA_GLOBAL T *)p;
}

// ---------------------------------------------------------------- utilities

struct U4 {
    uint32_t x, y, z, w;
};

// Philox4x32-10 block function (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds, each multiplying words 0 and 2 by the round multipliers and mixing
// the high halves with words 1, 3 and the key; the key advances by the two
// Weyl increments between rounds.
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
    // the round keys are derived here, at each call, instead of being hoisted
    // out of the annealing loop into twenty long-lived scalar registers
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t a = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t b = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t y0 = (uint32_t)(b >> 32) ^ c1 ^ k0;
        const uint32_t y2 = (uint32_t)(a >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)b;
        c3 = (uint32_t)a;
        c0 = y0;
        c2 = y2;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t scale32(uint32_t w, uint32_t c)
{
    return (uint32_t)(((uint64_t)w * c) >> 32);   // floor(w * c / 2^32), uniform in [0, c)
}

__device__ __forceinline__ int32_t rl(int32_t v, int lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ uint64_t rl64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int uni(int v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int64_t uni64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lane of the k-th (0-based) set bit of a wave-uniform mask.
__device__ __forceinline__ int kth_lane(uint64_t M, int k, int lane)
{
    const uint64_t below = M & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
    const bool hit = ((M >> lane) & 1ull) && (__popcll(below) == k);
    return uni(__ffsll((long long)__ballot(hit)) - 1);
}

// Index of the next work item from a launch's counter (one atomic per call,
// made by lane 0 and broadcast to the wave).
__device__ __forceinline__ int next_item(unsigned int *next, int lane)
{
    unsigned int v = 0;
    if (lane == 0) v = atomicAdd(next, 1u);
    return uni((int)v);
}

// p dominates q (Section 3.3): p_k <= q_k for every k, not equal in all.  With
// d_k = q_k - p_k (energies stay far inside int64), the bitwise OR of the d_k
// is negative when some d_k is, zero when all are, and positive exactly when p
// dominates q: one sign test, no per-objective compare masks.
__device__ __forceinline__ bool dominates(int64_t p1, int64_t p2, int64_t q1, int64_t q2)
{
    return ((q1 - p1) | (q2 - p2)) > 0;
}

// Returns p unchanged but hides its value from the optimiser, so loads made
// through it stay on the (rare) path that uses them instead of being hoisted
// into registers for the whole annealing loop.
__device__ __forceinline__ Desc *cold(Desc *p)
{
    uint64_t v = (uint64_t)p;
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    asm volatile("" : "+v"(lo), "+v"(hi));
    lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
    hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)hi);
    return (Desc *)(((uint64_t)hi << 32) | lo);
}

// Same for a wave-uniform integer: conditions derived from the result are
// evaluated where they are used instead of being kept live across the loop.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return __builtin_amdgcn_readfirstlane(v);
}

// Per-lane value hidden from the optimiser: cold code that starts from it
// cannot be hoisted out of the annealing loop into long-lived registers.
__device__ __forceinline__ int opaque_lane(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Wave-wide sum of a per-lane integer.
__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return uni(v);
}

// Four int32 (a 16-byte LDS read of uniform data, e.g. staged flow rows).
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));

// Wave-wide sum of a per-lane int (every lane active) by DPP moves: sums of
// 2, 4, 8 and 16 lanes within each row of 16 (row shifts by 1, 2, 4, 8 with
// zero fill), then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31
// into rows 2 and 3; lane 63 ends with the total.  Fields packed into v add
// independently as long as no field's total overflows into the next.
__device__ __forceinline__ int wave_sum_dpp(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Wave-wide minimum of a per-lane int (every lane active), by the same DPP
// moves as wave_sum_dpp; lanes without a source take INT_MAX.
__device__ __forceinline__ int wave_min_dpp(int v)
{
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x111, 0xF, 0xF, false));   // row_shr:1
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x112, 0xF, 0xF, false));   // row_shr:2
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x114, 0xF, 0xF, false));   // row_shr:4
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x118, 0xF, 0xF, false));   // row_shr:8
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x142, 0xA, 0xF, false));   // row_bcast:15
    v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// Fields read on every step, kept in scalar registers.
struct Hot {
    int n;
    int escape;
    int trace_R;
    uint32_t steps, ntab, key0, key1;
    int64_t beta;
    const MDA_CONST uint32_t *thrmax;
    const MDA_CONST int64_t *thrmax64;
    const MDA_CONST int64_t *T;
};

__device__ __forceinline__ Hot load_hot(Desc *Dp)
{
    Hot h;
    h.n = Dp->n;
    h.escape = Dp->escape;
    h.trace_R = Dp->trace_R;
    h.steps = Dp->steps;
    h.ntab = Dp->ntab;
    h.key0 = Dp->key0;
    h.key1 = Dp->key1;
    h.beta = Dp->beta;
    h.thrmax = ro(Dp->thrmax);
    h.thrmax64 = ro(Dp->thrmax64);
    h.T = ro(Dp->T);
    return h;
}

// ---------------------------------------------------------------- replica state

// Energy-difference type of a run: int32 while every local field fits it
// (the build-time bound), int64 beyond.  U is its unsigned counterpart (the
// field updates wrap there), kMax the value of lanes beyond n, kDeadV the
// value of slots beyond n (see kDead).
template <class FT>
struct Wide;
template <>
struct Wide<int32_t> {
    using U = uint32_t;
    static constexpr int32_t kMax = INT_MAX;
    static constexpr int32_t kDeadV = 1 << 30;
};
template <>
struct Wide<int64_t> {
    using U = uint64_t;
    static constexpr int64_t kMax = INT64_MAX;
    static constexpr int64_t kDeadV = (int64_t)1 << 60;
};

__device__ __forceinline__ int32_t rlf(int32_t v, int lane)
{
    return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ int64_t rlf(int64_t v, int lane)
{
    return (int64_t)rl64((uint64_t)v, lane);
}

// Slots in the group of 8 that starts at slot g: 8, or fewer in the last
// group when NS is not a multiple of 8 (for a multiple of 8 the condition
// folds away and the loops compile exactly as with the plain bound).
#define MDA_GROUP_SLOTS(NS, g) (((NS) % 8 == 0) ? 8 : ((NS) - (g) < 8 ? (NS) - (g) : 8))

template <int NS, class FT = int32_t>
struct Replica {
    FT e1[NS], e2[NS];        // dE_k of bit (slot i, this lane)
    uint64_t xm;              // bit i = x_{i, lane}
    int64_t E1, E2, Eoff;
    int64_t moves, scanned, rngb, detailed;
    int32_t asize;
    // per group of 8 slots (the last one holds 4 when NS is 4 mod 8), the
    // lane's least combined difference (max of the two for the strict rule,
    // min for the lenient one); it only changes when the fields do, so it is
    // recomputed after a move or restart only
    FT gmin[(NS + 7) / 8];
};

// Update paths (template argument PV): dense rows of P_k, or the Kronecker
// column with one product per objective (D or F symmetric) or two.
enum : int { kPvDense = 0, kPvKronSym = 1, kPvKronGen = 2 };

// Value held by slots beyond n (facilities that do not exist).  Such a slot
// only ever receives the +-2 alpha_k penalty of flips in its own column, whose
// sum is 2 alpha_k times the change of that column's occupation, so it stays
// within [kDead - 2 alpha n, kDead + 2 alpha n], inside (0, 2^31) because the
// host checks 2 alpha n < 2^30.  The exact acceptance test masks these slots
// out; their value only decides whether the cheap "can anything be accepted"
// test passes.
constexpr int32_t kDead = 1 << 30;

// Wave-wide sum of a per-lane int64.
__device__ __forceinline__ int64_t wave_sum64(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int lo = __shfl_xor((int)(uint32_t)v, off);
        const int hi = __shfl_xor((int)(uint32_t)((uint64_t)v >> 32), off);
        v += (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
    return uni64(v);
}

// Acceptance rule (template argument AM): strict (Eq. pacceptms) or lenient
// (Eq. pacceptml).
enum : int { kAmStrict = 0, kAmLenient = 1 };

// Offset and reach of the cheap "can any bit be accepted" test of a step whose
// largest acceptance threshold is thrmax: a bit can only be accepted when its
// combined difference is at most the reach.  int32 differences: every real dE
// is at most 2^31 - 2 (build-time bound), so capping the offset and the reach
// at 2^31 - 2 keeps all comparisons exact while slots and lanes beyond n, which
// hold INT_MAX, never qualify.  int64 differences: the offset (at most steps *
// beta) and the threshold (below 2^39) stay far below the dead values (2^60
// and up).
template <class FT>
__device__ __forceinline__ FT capped_offset(int64_t Eoff)
{
    return sizeof(FT) == 8 ? (FT)Eoff : (FT)(Eoff < (int64_t)(INT_MAX - 1) ? Eoff : (int64_t)(INT_MAX - 1));
}

template <class FT>
__device__ __forceinline__ FT step_reach(int64_t Eoff, int64_t thrmax)
{
    const int64_t Xl = (int64_t)capped_offset<FT>(Eoff) + thrmax;
    return sizeof(FT) == 8 ? (FT)Xl : (FT)(Xl < (int64_t)(INT_MAX - 1) ? Xl : (int64_t)(INT_MAX - 1));
}

// Steps, from the present one and at most rem, whose cheap test fails while
// the fields stay as they are: with the offset escape such a step only raises
// the offset by beta, so step k of the stretch has offset Eoff + k beta and a
// candidate first appears at the least k with Eoff + k beta + thr >= least
// (thr the constant largest threshold; least <= 2^31 - 2 for int32 differences,
// so the caps of step_reach do not change the answer).
__device__ __forceinline__ uint32_t quiet_steps(int64_t least, int64_t Eoff, int64_t thr, int64_t beta, uint32_t rem)
{
    const int64_t need = least - thr - Eoff;
    if (need <= 0) return 0u;
    uint64_t k;
    if (need <= (int64_t)UINT32_MAX && beta <= (int64_t)UINT32_MAX) {
        const uint32_t nd = (uint32_t)need, b = (uint32_t)beta;
        k = (uint64_t)(nd / b + (nd % b != 0u ? 1u : 0u));
    } else {
        k = (uint64_t)need / (uint64_t)beta + ((uint64_t)need % (uint64_t)beta != 0u ? 1u : 0u);
    }
    return k < (uint64_t)rem ? (uint32_t)k : rem;
}

// Index into the temperature tables for step t (the schedule is constant after
// its last entry).
__device__ __forceinline__ uint32_t table_index(uint32_t t, uint32_t ntab)
{
    return ((t < ntab) ? t : ntab) - 1u;
}

__device__ __forceinline__ int path_variant(Desc *Dp)
{
    return Dp->path == kPathDense ? kPvDense : (Dp->kform == kKronGen ? kPvKronGen : kPvKronSym);
}

// Update path and acceptance rule of a run, as one switch value.
__device__ __forceinline__ int step_variant(Desc *Dp)
{
    return run_step_variant(Dp->path, Dp->kform, Dp->accept);
}

// The differences d_k = dE_k of bit (slot js, lane jl), js uniform: a switch
// on js (a tree of scalar branches) reaches one readlane of the slot's
// register per objective, where a select over every slot would take 2 NS
// vector instructions.
template <int NS, class FT>
__device__ __forceinline__ void pick_diffs(const Replica<NS, FT> &S, int js, int jl, FT &d1, FT &d2)
{
    switch (js) {
#define MDA_PICK(I)                                   \
    case I:                                           \
        if (I < NS) {                                 \
            d1 = rlf(S.e1[I < NS ? I : 0], jl);       \
            d2 = rlf(S.e2[I < NS ? I : 0], jl);       \
        }                                             \
        break;
        MDA_PICK(0) MDA_PICK(1) MDA_PICK(2) MDA_PICK(3) MDA_PICK(4) MDA_PICK(5) MDA_PICK(6) MDA_PICK(7)
        MDA_PICK(8) MDA_PICK(9) MDA_PICK(10) MDA_PICK(11) MDA_PICK(12) MDA_PICK(13) MDA_PICK(14) MDA_PICK(15)
        MDA_PICK(16) MDA_PICK(17) MDA_PICK(18) MDA_PICK(19) MDA_PICK(20) MDA_PICK(21) MDA_PICK(22) MDA_PICK(23)
        MDA_PICK(24) MDA_PICK(25) MDA_PICK(26) MDA_PICK(27) MDA_PICK(28) MDA_PICK(29) MDA_PICK(30) MDA_PICK(31)
        MDA_PICK(32) MDA_PICK(33) MDA_PICK(34) MDA_PICK(35) MDA_PICK(36) MDA_PICK(37) MDA_PICK(38) MDA_PICK(39)
        MDA_PICK(40) MDA_PICK(41) MDA_PICK(42) MDA_PICK(43) MDA_PICK(44) MDA_PICK(45) MDA_PICK(46) MDA_PICK(47)
        MDA_PICK(48) MDA_PICK(49) MDA_PICK(50) MDA_PICK(51) MDA_PICK(52) MDA_PICK(53) MDA_PICK(54) MDA_PICK(55)
        MDA_PICK(56) MDA_PICK(57) MDA_PICK(58) MDA_PICK(59) MDA_PICK(60) MDA_PICK(61) MDA_PICK(62) MDA_PICK(63)
#undef MDA_PICK
    default: break;
    }
}

// Slot js (uniform) of every lane takes one more term of the flip: c_k with
// the lane's sign for that slot ((c ^ m) + b is c or -c in wrapping
// arithmetic).  A switch on js (a tree of scalar branches) reaches the slot's
// registers, where a select in every slot's update would take 2 NS vector
// instructions.
template <int NS, class FT>
__device__ __forceinline__ void add_to_slot(Replica<NS, FT> &S, int js, uint64_t xmx, typename Wide<FT>::U c1,
                                            typename Wide<FT>::U c2)
{
    using UT = typename Wide<FT>::U;
    switch (js) {
#define MDA_FIX(I)                                                                 \
    case I:                                                                        \
        if (I < NS) {                                                              \
            constexpr int i = I < NS ? I : 0;                                      \
            const UT b = (UT)((xmx >> i) & 1ull);                                  \
            const UT m = (UT)0 - b;                                                \
            S.e1[i] = (FT)((UT)S.e1[i] + (c1 ^ m) + b);                            \
            S.e2[i] = (FT)((UT)S.e2[i] + (c2 ^ m) + b);                            \
        }                                                                          \
        break;
        MDA_FIX(0) MDA_FIX(1) MDA_FIX(2) MDA_FIX(3) MDA_FIX(4) MDA_FIX(5) MDA_FIX(6) MDA_FIX(7)
        MDA_FIX(8) MDA_FIX(9) MDA_FIX(10) MDA_FIX(11) MDA_FIX(12) MDA_FIX(13) MDA_FIX(14) MDA_FIX(15)
        MDA_FIX(16) MDA_FIX(17) MDA_FIX(18) MDA_FIX(19) MDA_FIX(20) MDA_FIX(21) MDA_FIX(22) MDA_FIX(23)
        MDA_FIX(24) MDA_FIX(25) MDA_FIX(26) MDA_FIX(27) MDA_FIX(28) MDA_FIX(29) MDA_FIX(30) MDA_FIX(31)
        MDA_FIX(32) MDA_FIX(33) MDA_FIX(34) MDA_FIX(35) MDA_FIX(36) MDA_FIX(37) MDA_FIX(38) MDA_FIX(39)
        MDA_FIX(40) MDA_FIX(41) MDA_FIX(42) MDA_FIX(43) MDA_FIX(44) MDA_FIX(45) MDA_FIX(46) MDA_FIX(47)
        MDA_FIX(48) MDA_FIX(49) MDA_FIX(50) MDA_FIX(51) MDA_FIX(52) MDA_FIX(53) MDA_FIX(54) MDA_FIX(55)
        MDA_FIX(56) MDA_FIX(57) MDA_FIX(58) MDA_FIX(59) MDA_FIX(60) MDA_FIX(61) MDA_FIX(62) MDA_FIX(63)
#undef MDA_FIX
    default: break;
    }
}

}  // namespace mda
