// mda_wave.h -- one-wave-per-replica kernels of the multi-objective Digital Annealer
// (Ayodele et al., GECCO 2022, arXiv:2205.13399) on the bi-objective QAP.
//
// Layout: one replica per wave64.  Lane u holds location u; register slot i
// holds facility i, so bit a = i*n + u lives in slot i of lane u (n <= 64).
// Each lane keeps the two energy differences dE_1[a], dE_2[a] of its bits
// (Eq. cale with the sign (1 - 2 x_a) folded in) and its column of x as a
// 64-bit mask.  All arithmetic is integer: int32 differences (bounded by the
// build-time row check), int64 energies, offset and thresholds.
//
// One annealing step (Algorithm 3, with the offset of Algorithm 1):
//  1. per lane: min over its slots of max(dE_1, dE_2) (strict) or
//     min(dE_1, dE_2) (lenient); one ballot tells whether any bit can be
//     accepted at all (dE <= E_offset + the largest threshold of this step);
//  2. only then: exact acceptance per bit, drawing the Philox block of a group
//     of eight facilities only when some bit of it is neither certainly
//     accepted (S = 0) nor certainly rejected (S > largest threshold);
//  3. uniform choice of one accepted bit in ascending bit order (scalar);
//  4. field update: dense rows of P_k from HBM, or the Kronecker column
//     rebuilt from F_k, D and alpha_k with 24-bit multiply-adds;
//  5. archive update (Algorithm 4 or 5) against the archive in HBM.
// The random stream is counter-based on (seed, step, replica, bit group), so
// the result does not depend on the launch shape or on which draws are skipped.
#pragma once

#include "mda_device.h"

namespace mda {

// Flips bit (js, jl) whose current differences are d1, d2: E_k += dE_k(j);
// for every other bit a, dE_k[a] += (x_a == x_j ? +1 : -1) * P_k[a][j];
// dE_k(j) = -dE_k(j).  The per-slot code is the same for every slot; the
// own-row penalty of slot js and the new value of bit j are added to slot js
// afterwards (add_to_slot).
// Column entries fit int32 (build-time bound); the differences are updated in
// the unsigned counterpart UT of their type FT, where the additions wrap.
// LDS words of one wave of the persistent kernel: the 4096-entry -ln (or
// threshold) table, then kStageWords of staging for the flipped facility's
// flow rows (four rows of 64 lanes).
constexpr int kStageWords = 256;
constexpr int kWaveLds = 4096 + kStageWords;

template <int NS, int PV, class FT>
__device__ __forceinline__ void flip(Desc *Dp, int n_, Replica<NS, FT> &S, int js, int jl, FT d1, FT d2, int lane_,
                                     MDA_LDS int32_t *stage)
{
    using UT = typename Wide<FT>::U;
    const int n = opaque(n_);
    const int lane = opaque_lane(lane_);
    const bool live = lane < n;
    const uint64_t xj = (rl64(S.xm, jl) >> js) & 1ull;
    const uint64_t xmx = S.xm ^ (0ull - xj);   // bit i set where x_{i,lane} != x_j
    S.E1 += d1;
    S.E2 += d2;
    Desc &D = *cold(Dp);
    if (PV == kPvDense) {
        // Row j of P_k holds every column entry, penalty and diagonal included;
        // bit j itself gets -2 d - P_jj on top of P_jj.
        const int j = js * n + jl;
        const UT c1 = (lane == jl) ? (UT)(-2 * d1) - (UT)(FT)ro(D.diag1)[js * kLD + jl] : (UT)0;
        const UT c2 = (lane == jl) ? (UT)(-2 * d2) - (UT)(FT)ro(D.diag2)[js * kLD + jl] : (UT)0;
        // bit j's own entry (added first: the additions commute)
        add_to_slot<NS, FT>(S, js, xmx, c1, c2);
        // rows of n x n entries: lanes beyond n read a clamped (in-bounds)
        // index and take 0
        const MDA_CONST int32_t *r1 = ro(D.P1) + (size_t)j * (size_t)(n * n);
        const MDA_CONST int32_t *r2 = ro(D.P2) + (size_t)j * (size_t)(n * n);
        const int ul = live ? lane : 0;
#pragma unroll
        for (int g = 0; g < NS; g += 8) {
            // at most 16 row loads in flight (keeps the register budget)
            asm volatile("" : "+v"(r1), "+v"(r2));
            uint32_t t1[8], t2[8];
#pragma unroll
            for (int f = 0; f < MDA_GROUP_SLOTS(NS, g); ++f) {
                const int i = g + f;
                t1[f] = (i < n) ? (uint32_t)r1[i * n + ul] : 0u;
                t2[f] = (i < n) ? (uint32_t)r2[i * n + ul] : 0u;
                t1[f] = live ? t1[f] : 0u;
                t2[f] = live ? t2[f] : 0u;
            }
#pragma unroll
            for (int f = 0; f < MDA_GROUP_SLOTS(NS, g); ++f) {
                const int i = g + f;
                const UT b = (UT)((xmx >> i) & 1ull);
                const UT m = (UT)0 - b;
                const UT u1 = (UT)(FT)(int32_t)t1[f];
                const UT u2 = (UT)(FT)(int32_t)t2[f];
                S.e1[i] = (FT)((UT)S.e1[i] + (u1 ^ m) + b);
                S.e2[i] = (FT)((UT)S.e2[i] + (u2 ^ m) + b);
            }
        }
    } else {
        // P_k[(i,u)][(js,jl)] = KA_k[js][i] DA[jl][u] (+ KB_k[js][i] DB[jl][u])
        //                       + 2 alpha_k [(i == js) != (u == jl)]
        // Slot i != js adds the penalty vector q_k = 2 alpha_k [u == jl]; slot js
        // adds r_k = 2 alpha_k [u != jl] instead, except at lane jl where the
        // term is chosen so that dE_k(j) becomes -d_k.
        // operand rows are padded to kLD entries with zeros, so lanes beyond n load 0
        const int32_t dv = ro(D.DA)[jl * kLD + lane];
        const int32_t dw = (PV == kPvKronGen) ? ro(D.DB)[jl * kLD + lane] : 0;
        const int32_t fa1 = ro(D.KA1)[js * kLD + lane];
        const int32_t fa2 = ro(D.KA2)[js * kLD + lane];
        const int32_t fb1 = (PV == kPvKronGen) ? ro(D.KB1)[js * kLD + lane] : 0;
        const int32_t fb2 = (PV == kPvKronGen) ? ro(D.KB2)[js * kLD + lane] : 0;
        // The rows (one entry per lane) go through the wave's staging words
        // in LDS and come back as uniform 16-byte reads, four slots each, in
        // place of one readlane per slot and objective.
        stage[lane] = fa1;
        stage[64 + lane] = fa2;
        if (PV == kPvKronGen) {
            stage[128 + lane] = fb1;
            stage[192 + lane] = fb2;
        }
        const MDA_LDS v4i32 *s4 = (const MDA_LDS v4i32 *)stage;
        const UT ta1 = (UT)(FT)D.two_alpha1, ta2 = (UT)(FT)D.two_alpha2;
        const bool atj = lane == jl;
        const UT q1 = atj ? ta1 : (UT)0, q2 = atj ? ta2 : (UT)0;
        UT own1 = (UT)(FT)__mul24(rl(fa1, js), dv), own2 = (UT)(FT)__mul24(rl(fa2, js), dv);
        if (PV == kPvKronGen) {
            own1 += (UT)(FT)__mul24(rl(fb1, js), dw);
            own2 += (UT)(FT)__mul24(rl(fb2, js), dw);
        }
        const UT r1 = atj ? (UT)(-2 * d1) - own1 : (live ? ta1 : (UT)0);
        const UT r2 = atj ? (UT)(-2 * d2) - own2 : (live ? ta2 : (UT)0);
        // slot js takes r_k in place of q_k (added first: the additions
        // commute, and fewer values are live here than after the loop)
        add_to_slot<NS, FT>(S, js, xmx, r1 - q1, r2 - q2);
#pragma unroll
        for (int g = 0; g < NS; g += 4) {
            const v4i32 a1 = s4[g / 4], a2 = s4[16 + g / 4];
            v4i32 b1 = a1, b2 = a2;
            if (PV == kPvKronGen) {
                b1 = s4[32 + g / 4];
                b2 = s4[48 + g / 4];
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int i = g + f;
                // wrapping arithmetic: each product and the column entry fit int32
                UT t1 = (UT)(FT)__mul24(a1[f], dv) + q1;
                UT t2 = (UT)(FT)__mul24(a2[f], dv) + q2;
                if (PV == kPvKronGen) {
                    t1 += (UT)(FT)__mul24(b1[f], dw);
                    t2 += (UT)(FT)__mul24(b2[f], dw);
                }
                const UT b = (UT)((xmx >> i) & 1ull);
                const UT m = (UT)0 - b;
                S.e1[i] = (FT)((UT)S.e1[i] + (t1 ^ m) + b);
                S.e2[i] = (FT)((UT)S.e2[i] + (t2 ^ m) + b);
            }
        }
    }
    S.xm ^= (lane == jl) ? (1ull << js) : 0ull;
}

// Fields and energies of the solution in S.xm computed from scratch:
// g_k[a] = d_k[a] + sum_{b in x, b != a} P_k[a][b], dE_k[a] = (1 - 2 x_a) g_k[a],
// E_k = q_k + sum_{a in x} (d_k[a] + g_k[a]) / 2 (Eq. qubo).  The column sums
// run over the set bits; the penalty part 2 alpha_k [(i == i') != (u == u')]
// is counted from the row and column occupation of x.
template <int NS, int PV, class FT>
__device__ __forceinline__ void fields_from_scratch(Desc *Dp, Replica<NS, FT> &S, int lane_)
{
    using UT = typename Wide<FT>::U;
    const int lane = opaque_lane(lane_);
    Desc &D = *cold(Dp);
    const int n = opaque(D.n);
    const bool live = lane < n;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        S.e1[i] = 0;
        S.e2[i] = 0;
    }
    // sum over set bits b = (bi, bu) of the cost part of column b
    uint64_t todo = live ? S.xm : 0ull;
    for (;;) {
        const uint64_t bb = __ballot(todo != 0ull);
        if (bb == 0ull) break;
        const int bu = __ffsll((long long)bb) - 1;
        const int bi = uni(__ffsll((long long)rl64(todo, bu)) - 1);
        if (PV == kPvDense) {
            const MDA_CONST int32_t *r1 = ro(D.P1) + (size_t)(bi * n + bu) * (size_t)(n * n);
            const MDA_CONST int32_t *r2 = ro(D.P2) + (size_t)(bi * n + bu) * (size_t)(n * n);
            const int ul = live ? lane : 0;
#pragma unroll
            for (int g = 0; g < NS; g += 8) {
                asm volatile("" : "+v"(r1), "+v"(r2));
#pragma unroll
                for (int f = 0; f < MDA_GROUP_SLOTS(NS, g); ++f) {
                    const int i = g + f;
                    const UT v1 = (i < n) ? (UT)(FT)r1[i * n + ul] : (UT)0;
                    const UT v2 = (i < n) ? (UT)(FT)r2[i * n + ul] : (UT)0;
                    S.e1[i] = (FT)((UT)S.e1[i] + (live ? v1 : (UT)0));
                    S.e2[i] = (FT)((UT)S.e2[i] + (live ? v2 : (UT)0));
                }
            }
        } else {
            const int32_t dv = ro(D.DA)[bu * kLD + lane];
            const int32_t dw = (PV == kPvKronGen) ? ro(D.DB)[bu * kLD + lane] : 0;
            const int32_t fa1 = ro(D.KA1)[bi * kLD + lane];
            const int32_t fa2 = ro(D.KA2)[bi * kLD + lane];
            const int32_t fb1 = (PV == kPvKronGen) ? ro(D.KB1)[bi * kLD + lane] : 0;
            const int32_t fb2 = (PV == kPvKronGen) ? ro(D.KB2)[bi * kLD + lane] : 0;
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                UT t1 = (UT)(FT)__mul24(rl(fa1, i), dv);
                UT t2 = (UT)(FT)__mul24(rl(fa2, i), dv);
                if (PV == kPvKronGen) {
                    t1 += (UT)(FT)__mul24(rl(fb1, i), dw);
                    t2 += (UT)(FT)__mul24(rl(fb2, i), dw);
                }
                S.e1[i] = (FT)((UT)S.e1[i] + t1);
                S.e2[i] = (FT)((UT)S.e2[i] + t2);
            }
        }
        todo ^= (lane == bu) ? (1ull << bi) : 0ull;
    }
    // Self term, penalty counts, diagonal, sign; energies.
    const uint64_t xl = live ? S.xm : 0ull;
    const uint32_t cu = (uint32_t)__popcll(xl);   // bits set in this lane's column
    const UT ta1 = (UT)(FT)D.two_alpha1, ta2 = (UT)(FT)D.two_alpha2;
    const int32_t lslot = live ? 0 : 1;            // lanes beyond n
    int64_t acc1 = 0, acc2 = 0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const bool on = (xl >> i) & 1ull;
        const bool ok = live && i < n;
        const uint32_t ri = (uint32_t)__popcll(__ballot(on));   // bits set in row i
        const UT dg1 = (UT)(FT)ro(D.diag1)[i * kLD + lane];   // padded: 0 beyond n
        const UT dg2 = (UT)(FT)ro(D.diag2)[i * kLD + lane];
        UT g1 = (UT)S.e1[i] + dg1, g2 = (UT)S.e2[i] + dg2;
        if (PV == kPvDense) {
            // the row of b = a added P_aa = d_a
            g1 -= on ? dg1 : (UT)0;
            g2 -= on ? dg2 : (UT)0;
        } else {
            // the Kronecker column of b = a added twice its cost part
            // C_aa = d_a + 2 alpha (both products of the off-diagonal form)
            g1 -= on ? (UT)2 * (dg1 + ta1) : (UT)0;
            g2 -= on ? (UT)2 * (dg2 + ta2) : (UT)0;
            const UT cnt = (UT)(ri + cu - (on ? 2u : 0u));
            g1 += cnt * ta1;
            g2 += cnt * ta2;
        }
        acc1 += on ? (int64_t)(FT)g1 + (int64_t)(FT)dg1 : 0;
        acc2 += on ? (int64_t)(FT)g2 + (int64_t)(FT)dg2 : 0;
        const FT s1 = on ? -(FT)g1 : (FT)g1;
        const FT s2 = on ? -(FT)g2 : (FT)g2;
        S.e1[i] = ok ? s1 : (lslot ? Wide<FT>::kMax : Wide<FT>::kDeadV);
        S.e2[i] = ok ? s2 : (lslot ? Wide<FT>::kMax : Wide<FT>::kDeadV);
    }
    S.E1 = D.q1 + wave_sum64(acc1) / 2;
    S.E2 = D.q2 + wave_sum64(acc2) / 2;
}

// Continue from archive member p (Algorithm 3, escape by restart).
template <int NS, int PV, class FT>
__device__ __forceinline__ void restart_from(Desc *Dp, int n, Replica<NS, FT> &S, int r, int p, int lane)
{
    Desc &D = *cold(Dp);
    const MDA_GLOBAL uint64_t *ax = rw(D.archX) + ((size_t)r * D.s + p) * (size_t)n;
    S.xm = (lane < n) ? ax[lane] : 0ull;
    fields_from_scratch<NS, PV>(Dp, S, lane);
}

// Archive update after a move: Algorithm 4 (explore) or 5 (exploit).
template <int NS, class FT>
__device__ __forceinline__ void archive_update(Desc *Dp, int n, Replica<NS, FT> &S, int r, uint32_t t, int lane_,
                                               uint32_t key0, uint32_t key1)
{
    const int lane = opaque_lane(lane_);
    Desc &D = *cold(Dp);
    const int s = D.s;
    MDA_GLOBAL int64_t *AE = rw(D.archE) + (size_t)r * s * 2;
    MDA_GLOBAL uint64_t *AX = rw(D.archX) + (size_t)r * s * (size_t)n;
    const int asz = S.asize;
    const int64_t E1 = S.E1, E2 = S.E2;
    int slot = -1;
    if (D.archive == 0) {
        // first member that x dominates; kAB blocks of 64 members are read at
        // once (indices clamped into the archive, so every read is in bounds).
        // The archives do not fit the caches, so each round trip waits on
        // memory: 8 blocks per trip beat 4 and 16 on the benchmark launch.
        // The loads of a round trip are issued before any of their values is
        // tested, and lanes past the end take their test through a bitwise
        // AND: a short-circuit test let the compiler move each load under its
        // own branch, one memory wait per block.
        constexpr int kAB = 8;
        for (int b = 0; b < asz; b += 64 * kAB) {
            int64_t a1[kAB], a2[kAB];
#pragma unroll
            for (int q = 0; q < kAB; ++q) {
                const int e = b + 64 * q + lane;
                const int ec = e < asz ? e : asz - 1;
                a1[q] = AE[2 * ec];
                a2[q] = AE[2 * ec + 1];
            }
            uint64_t M[kAB];
#pragma unroll
            for (int q = 0; q < kAB; ++q) {
                const int e = b + 64 * q + lane;
                M[q] = __ballot((e < asz) & dominates(E1, E2, a1[q], a2[q]));
            }
            int q = -1;
#pragma unroll
            for (int qq = kAB - 1; qq >= 0; --qq) q = M[qq] ? qq : q;
            if (q >= 0) {
                uint64_t Mq = M[0];
#pragma unroll
                for (int qq = 1; qq < kAB; ++qq) Mq = (q == qq) ? M[qq] : Mq;
                const int f = __ffsll((long long)Mq) - 1;
                S.scanned += 64 * q + f + 1;
                slot = b + 64 * q + f;
                break;
            }
            S.scanned += (asz - b < 64 * kAB) ? (asz - b) : 64 * kAB;
        }
    } else {
        // Algorithm 5: nothing may dominate x; then a random member of
        // B = {y : x dominates y} is replaced, or x is appended.
        int nb = 0;
        bool rejected = false;
        for (int b = 0; b < asz; b += 64) {
            const int e = b + lane;
            bool z = false, y = false;
            if (e < asz) {
                const int64_t a1 = AE[2 * e], a2 = AE[2 * e + 1];
                z = dominates(a1, a2, E1, E2);
                y = dominates(E1, E2, a1, a2);
            }
            S.scanned += (asz - b < 64) ? (asz - b) : 64;
            if (__ballot(z)) {
                rejected = true;
                break;
            }
            nb += __popcll(__ballot(y));
        }
        if (rejected) return;
        if (nb > 0) {
            const U4 o = philox10(0u, t, (uint32_t)r, kTagArc, key0, key1);
            int k = (int)scale32((uint32_t)uni((int)o.x), (uint32_t)nb);
            for (int b = 0; b < asz; b += 64) {
                const int e = b + lane;
                bool y = false;
                if (e < asz) y = dominates(E1, E2, AE[2 * e], AE[2 * e + 1]);
                const uint64_t M = __ballot(y);
                const int pc = __popcll(M);
                if (k < pc) {
                    slot = b + kth_lane(M, k, lane);
                    break;
                }
                k -= pc;
            }
        }
    }
    if (slot < 0 && asz < s) {
        slot = asz;
        S.asize = asz + 1;
    }
    slot = uni(slot);
    if (slot >= 0) {
        if (lane == 0) {
            AE[2 * slot] = E1;
            AE[2 * slot + 1] = E2;
        }
        if (lane < n) AX[(size_t)slot * n + lane] = S.xm;
    }
}

// Random start (Algorithm 3): bit (i, u) is bit i of the 64-bit word
// (o.x, o.y) of Philox block (0, u); fields and energies from scratch.
template <int NS, int PV, class FT>
__device__ __forceinline__ void init_replica(Desc *Dp, Replica<NS, FT> &S, int r, int lane)
{
    Desc &D = *cold(Dp);
    const int n = opaque(D.n);
    const U4 o = philox10((uint32_t)lane, 0u, (uint32_t)r, kTagInit, D.key0, D.key1);
    const uint64_t nmask = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    S.xm = (lane < n) ? ((((uint64_t)o.y << 32) | o.x) & nmask) : 0ull;
    S.Eoff = 0;
    S.moves = S.scanned = S.rngb = S.detailed = 0;
    S.asize = 0;
    fields_from_scratch<NS, PV>(Dp, S, lane);
}

// Least combined difference of every group of 8 slots (see Replica::gmin).
template <int NS, int AM, class FT>
__device__ __forceinline__ void group_minima(Replica<NS, FT> &S)
{
#pragma unroll
    for (int g = 0; g < NS; g += 8) {
        FT gm = Wide<FT>::kMax;
#pragma unroll
        for (int f = 0; f < MDA_GROUP_SLOTS(NS, g); ++f)
            gm = min(gm, AM == kAmStrict ? max(S.e1[g + f], S.e2[g + f]) : min(S.e1[g + f], S.e2[g + f]));
        S.gmin[g >> 3] = gm;
    }
}

// Least combined difference over the whole replica (every slot and lane):
// the cheap test of a step passes exactly when it is within the step's reach.
template <int NS, class FT>
__device__ __forceinline__ FT wave_least(const Replica<NS, FT> &S)
{
    FT mn = Wide<FT>::kMax;
#pragma unroll
    for (int g = 0; g < (NS + 7) / 8; ++g) mn = min(mn, S.gmin[g]);
    if (sizeof(FT) == 4) return (FT)wave_min_dpp((int)mn);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint64_t u = (uint64_t)(int64_t)mn;
        const int lo = __shfl_xor((int)(uint32_t)u, off), hi = __shfl_xor((int)(uint32_t)(u >> 32), off);
        mn = min(mn, (FT)(int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
    }
    return (FT)uni64((int64_t)mn);
}

// One annealing step t of replica r whose largest acceptance threshold
// (T_t * LNT[0]) >> 24 is thrmax.  Returns the flipped bit or -1.  lnt is the
// -ln table; with THR (int32 differences at the schedule's final, constant
// temperature) it holds the thresholds (T * LNT[k]) >> 24 themselves,
// saturated at 2^32 - 1 (above every statistic, so the decisions are the same).
template <int NS, int PV, int AM, class FT, class LP, bool THR = false>
__device__ __forceinline__ int anneal_step(Desc *Dp, const Hot &H, Replica<NS, FT> &S, int r, uint32_t t, int lane_,
                                           LP lnt, int64_t thrmax, MDA_LDS int32_t *stage)
{
    constexpr bool strict = AM == kAmStrict;
    using UT = typename Wide<FT>::U;
    const int lane = lane_;
    const int n = H.n;
    const uint64_t actmask = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
    const uint32_t ti = table_index(t, H.ntab);
    const FT EoC = capped_offset<FT>(S.Eoff);
    const FT X = step_reach<FT>(S.Eoff, thrmax);

    // 1. can any bit be accepted?  The minimum is kept per group of 8 slots so
    // that step 2 passes over groups in which no lane comes within reach.
    const FT *gmin = S.gmin;
    FT mn = Wide<FT>::kMax;
#pragma unroll
    for (int g = 0; g < (NS + 7) / 8; ++g) mn = min(mn, gmin[g]);
    const uint64_t cand = __ballot(mn <= X) & actmask;

    int j = -1;
    if (cand) {
        S.detailed++;
        const int lane = opaque_lane(lane_);
        // 2. exact acceptance, 8 facilities per random block.  The threshold
        // (T * LNT[k]) >> 24 is formed exactly: with T = Th 2^24 + Tl (T < 2^43,
        // so Th < 2^19; LNT < 2^20) it equals Th LNT + ((Tl LNT) >> 24), and the
        // statistic is compared with it in 64 bits.
        const int64_t T = THR ? 0 : H.T[ti];
        const uint32_t Th = (uint32_t)((uint64_t)T >> 24), Tl = (uint32_t)T & 0xFFFFFFu;
        uint64_t acc = 0;
        const int ng = opaque(n);
#pragma unroll
        for (int g = 0; g < NS; g += 8) {
            // a group whose slots all exceed X on every lane has neither
            // certain nor possible acceptances and draws no random block
            if (g < ng && __ballot(gmin[g >> 3] <= X)) {
                // slots g .. g+7 that are facilities (< n)
                const uint32_t slots = (ng - g >= 8) ? 0xFFu : ((1u << (ng - g)) - 1u);
                uint32_t certain = 0, maybe = 0;
#pragma unroll
                for (int f = 0; f < MDA_GROUP_SLOTS(NS, g); ++f) {
                    const int i = g + f;
                    // the statistic S is 0 exactly when the combined difference is at
                    // most the offset, and above every threshold when it exceeds X
                    const FT v = strict ? max(S.e1[i], S.e2[i]) : min(S.e1[i], S.e2[i]);
                    const bool sure = v <= EoC;
                    const bool near = v <= X;
                    certain |= sure ? (1u << f) : 0u;
                    maybe |= (near && !sure) ? (1u << f) : 0u;
                }
                certain &= slots;
                maybe &= slots;
                if (__ballot(maybe != 0u)) {
                    S.rngb++;
                    const U4 o = philox10(((uint32_t)(g >> 3) << 16) | (uint32_t)lane, t, (uint32_t)r,
                                          kTagAcc, H.key0, H.key1);
                    // the eight -ln lookups are issued together (one LDS wait
                    // per block, not one per slot) and all eight slots are
                    // tested without a branch (no exec-mask switching per
                    // slot); slots that are not undecided keep their decision
                    // through the mask
                    uint32_t Lv[8];
#pragma unroll
                    for (int f = 0; f < 8; ++f) {
                        const uint32_t w = (f < 2) ? o.x : (f < 4) ? o.y : (f < 6) ? o.z : o.w;
                        Lv[f] = (uint32_t)lnt[(w >> (16 * (f & 1))) & 0xFFFu];
                    }
#pragma unroll
                    for (int f = 0; f < MDA_GROUP_SLOTS(NS, g); ++f) {
                        const int i = g + f;
                        // u_k = max(0, dE_k - E_offset) < 2^31 for a real int32 bit, so
                        // the strict sum stays below 2^32
                        const UT u1 = (UT)(max(S.e1[i], EoC) - EoC);
                        const UT u2 = (UT)(max(S.e2[i], EoC) - EoC);
                        const UT Sx = strict ? (u1 + u2) : (u1 < u2 ? u1 : u2);
                        uint32_t ok;
                        if (THR) {
                            ok = (uint64_t)Sx <= (uint64_t)Lv[f] ? 1u : 0u;
                        } else {
                            const uint32_t L = Lv[f] & 0xFFFFFu;
                            const uint64_t low = (uint64_t)Tl * (uint64_t)L;   // 24 x 20 bits
                            const uint64_t t64 = (uint64_t)Th * (uint64_t)L + (low >> 24);
                            ok = (uint64_t)Sx <= t64 ? 1u : 0u;
                        }
                        certain |= ((maybe >> f) & ok) << f;
                    }
                }
                acc |= (uint64_t)certain << g;
            }
        }
        // 3. uniform choice in ascending bit order a = i*n + u.  The wave's
        // count of accepted bits per group of eight slots (three groups per
        // word in 10-bit fields, at most 512 each), then per slot of the
        // chosen group (four per word in 8-bit fields, at most 64 each), then
        // the lane: the (slot, lane) of the k-th accepted bit, slot-major.
        constexpr int NG = (NS + 7) / 8;
        int gtot[NG];
#pragma unroll
        for (int w = 0; w < NG; w += 3) {
            int packed = 0;
#pragma unroll
            for (int q = 0; q < 3 && w + q < NG; ++q)
                packed |= __popc((uint32_t)(acc >> (8 * (w + q))) & 0xFFu) << (10 * q);
            const int sum = wave_sum_dpp(packed);
#pragma unroll
            for (int q = 0; q < 3 && w + q < NG; ++q) gtot[w + q] = (sum >> (10 * q)) & 0x3FF;
        }
        int cnt = 0;
#pragma unroll
        for (int g = 0; g < NG; ++g) cnt += gtot[g];
        if (cnt > 0) {
            const U4 o = philox10(0u, t, (uint32_t)r, kTagSel, H.key0, H.key1);
            int k = (int)scale32((uint32_t)uni((int)o.x), (uint32_t)cnt);
            int gs = 0, before = 0, run = 0;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const bool here = run <= k && k < run + gtot[g];
                gs = here ? g : gs;
                before = here ? run : before;
                run += gtot[g];
            }
            gs = uni(gs);
            k -= before;
            const uint32_t gb = (uint32_t)(acc >> (8 * gs)) & 0xFFu;
            const int lo4 = wave_sum_dpp((int)((gb & 1u) | ((gb >> 1) & 1u) << 8 | ((gb >> 2) & 1u) << 16 |
                                               ((gb >> 3) & 1u) << 24));
            const int hi4 = wave_sum_dpp((int)(((gb >> 4) & 1u) | ((gb >> 5) & 1u) << 8 | ((gb >> 6) & 1u) << 16 |
                                               ((gb >> 7) & 1u) << 24));
            int fs = 0;
            before = 0;
            run = 0;
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                const int c = ((f < 4 ? lo4 : hi4) >> (8 * (f & 3))) & 0xFF;
                const bool here = run <= k && k < run + c;
                fs = here ? f : fs;
                before = here ? run : before;
                run += c;
            }
            k -= before;
            const int js = uni(8 * gs + fs);
            const int jl = kth_lane(__ballot((acc >> js) & 1ull), k, lane);
            FT d1 = 0, d2 = 0;
            pick_diffs<NS, FT>(S, js, jl, d1, d2);
            // 4. move, 5. archive
            flip<NS, PV>(Dp, n, S, js, jl, d1, d2, lane, stage);
            group_minima<NS, AM>(S);
            S.moves++;
            archive_update<NS, FT>(Dp, n, S, r, t, lane, H.key0, H.key1);
            j = js * n + jl;
        }
    }
    // No accepted flip: raise the offset (Algorithm 1) or restart from the archive
    // (Algorithm 3).  Written as straight-line selects and an if-then so that the
    // replica state never merges at an if/else.
    const bool moved = j >= 0;
    S.Eoff = moved ? 0 : ((H.escape == 0) ? S.Eoff + H.beta : S.Eoff);
    if (!moved && H.escape != 0 && S.asize > 0) {
        const U4 o = philox10(0u, t, (uint32_t)r, kTagArc, H.key0, H.key1);
        const int p = (int)scale32((uint32_t)uni((int)o.y), (uint32_t)S.asize);
        restart_from<NS, PV>(Dp, n, S, r, p, lane);
        group_minima<NS, AM>(S);
    }
    if (r < H.trace_R && lane == 0) rw(cold(Dp)->trace)[(size_t)r * H.steps + (t - 1u)] = j;
    return j;
}

// Final state of replica r: x, canonical local fields h_k = sign * dE_k - d_k, scalars.
template <int NS, class FT>
__device__ __forceinline__ void export_replica(Desc *Dp, const Replica<NS, FT> &S, int r, int lane)
{
    Desc &D = *cold(Dp);
    const int n = opaque(D.n);
    const int m = D.m;
    rw(D.x)[(size_t)r * 64 + lane] = (lane < n) ? S.xm : 0ull;
    if (lane < n) {
        MDA_GLOBAL int64_t *h1 = rw(D.h) + (size_t)r * 2 * m;
        MDA_GLOBAL int64_t *h2 = h1 + m;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (i < n) {
                const int a = i * n + lane;
                const bool on = (S.xm >> i) & 1ull;
                const FT g1 = on ? -S.e1[i] : S.e1[i];
                const FT g2 = on ? -S.e2[i] : S.e2[i];
                h1[a] = (int64_t)g1 - ro(D.diag1)[i * kLD + lane];
                h2[a] = (int64_t)g2 - ro(D.diag2)[i * kLD + lane];
            }
        }
    }
    if (lane == 0) {
        MDA_GLOBAL int64_t *st = rw(D.st) + (size_t)r * kStWords;
        st[kStE1] = S.E1;
        st[kStE2] = S.E2;
        st[kStEoff] = S.Eoff;
        st[kStMoves] = S.moves;
        st[kStScanned] = S.scanned;
        st[kStRng] = S.rngb;
        st[kStArch] = S.asize;
        st[kStDetailed] = S.detailed;
    }
}

// ---------------------------------------------------------------- kernels

// Largest threshold of table entry k: the saturated 32-bit table for int32
// differences, the int64 one for int64 differences.
template <class FT>
__device__ __forceinline__ int64_t thr_entry(const Hot &H, uint32_t k)
{
    return sizeof(FT) == 8 ? H.thrmax64[k] : (int64_t)H.thrmax[k];
}

// Trace entries (no flip) of the k steps from t of a replica that records its
// trajectory.
__device__ __forceinline__ void quiet_trace(Desc *Dp, const Hot &H, int r, uint32_t t, uint32_t k, int lane)
{
    if (r < H.trace_R) {
        MDA_GLOBAL int32_t *tr = rw(cold(Dp)->trace) + (size_t)r * H.steps + (t - 1u);
        for (uint32_t i = (uint32_t)lane; i < k; i += 64u) tr[i] = -1;
    }
}

// All steps of one replica with its state in registers.  tab is the wave's
// 4096 words of LDS: the -ln table (copied from lnt_g) while the temperature
// changes; from step ntab on, where it stays at its last value, the int32 build
// replaces each LNT[k] by the threshold (T * LNT[k]) >> 24 of that temperature.
template <int NS, int PV, int AM, class FT>
__device__ __forceinline__ void run_replica(Desc *Dp, int r, int lane, MDA_LDS int32_t *tab,
                                            const MDA_GLOBAL int32_t *lnt_g)
{
    constexpr bool wide = sizeof(FT) == 8;
#pragma unroll 8
    for (int k = lane; k < 4096; k += 64) tab[k] = lnt_g[k];
    Replica<NS, FT> S;
    init_replica<NS, PV>(Dp, S, r, lane);
    group_minima<NS, AM>(S);
    const Hot H = load_hot(Dp);
    // With the offset escape a step whose cheap test fails does nothing but
    // raise the offset by beta.  Such steps are decided against the replica's
    // least combined difference, which only changes with a move, by the scalar
    // unit alone: one by one while the temperature changes, a whole stretch at
    // once (quiet_steps) after that.
    const bool skip = H.escape == 0;
    FT least = wave_least(S);
    // the next step's threshold is loaded one step ahead
    int64_t thr = thr_entry<FT>(H, 0);
    const uint32_t cool = wide ? H.steps : ((H.ntab - 1u < H.steps) ? H.ntab - 1u : H.steps);
    uint32_t t = 1;
    for (; t <= cool; ++t) {
        // entry of step t + 1: min(t + 1, ntab) - 1 = min(t, ntab - 1), ntab >= 1
        const int64_t thr_next = thr_entry<FT>(H, (t < H.ntab - 1u) ? t : H.ntab - 1u);
        if (skip && least > step_reach<FT>(S.Eoff, thr)) {
            S.Eoff += H.beta;
            quiet_trace(Dp, H, r, t, 1u, lane);
        } else if (anneal_step<NS, PV, AM>(Dp, H, S, r, t, lane, (const MDA_LDS int32_t *)tab, thr, tab + 4096) >= 0) {
            least = wave_least(S);
        }
        thr = thr_next;
    }
    if (!wide && t <= H.steps) {
        const uint64_t T = (uint64_t)H.T[H.ntab - 1u];
#pragma unroll 8
        for (int k = lane; k < 4096; k += 64) {
            // T < 2^43 and LNT < 2^20: the product fits 64 bits
            const uint64_t v = (T * (uint64_t)((uint32_t)tab[k] & 0xFFFFFu)) >> 24;
            tab[k] = (int32_t)(uint32_t)(v < 0xFFFFFFFFull ? v : 0xFFFFFFFFull);
        }
        while (t <= H.steps) {
            if (skip) {
                const uint32_t k = quiet_steps((int64_t)least, S.Eoff, thr, H.beta, H.steps - t + 1u);
                if (k > 0u) {
                    S.Eoff += (int64_t)k * H.beta;
                    quiet_trace(Dp, H, r, t, k, lane);
                    t += k;
                    continue;
                }
            }
            if (anneal_step<NS, PV, AM, FT, const MDA_LDS int32_t *, true>(Dp, H, S, r, t, lane,
                                                                         (const MDA_LDS int32_t *)tab, thr,
                                                                         tab + 4096) >= 0)
                least = wave_least(S);
            ++t;
        }
    }
    export_replica<NS>(Dp, S, r, lane);
}

#define MDA_STEP_VARIANTS(X)                                                                          \
    X(kPvDense, kAmStrict) X(kPvDense, kAmLenient) X(kPvKronSym, kAmStrict) X(kPvKronSym, kAmLenient) \
    X(kPvKronGen, kAmStrict) X(kPvKronGen, kAmLenient)

// Persistent form: wave w of the grid runs work item w, then whichever item
// comes next in the list when it finishes (W waves in the grid; the host
// orders the items largest first), each for all of its steps with the replica
// state in registers.  Replicas of one instance can differ a lot in length (an
// archive that grows large makes every move scan it), so a fixed assignment of
// items to waves would leave the launch waiting for its unluckiest wave.
// Every item of a launch has step variant SV (update path and acceptance
// rule; the host groups the work list by it), so the kernel holds one variant
// of the step: a build with all six behind a switch needs twice the scratch of
// the two-wave budget and is 4.5 % slower on the n = 50 benchmark launch.
// From 32 slots up the kernel holds one wave per SIMD (OCC = 1); the OCC = 2
// build keeps part of the cold-path state (initial fields, restarts, archive
// scans) in scratch so that a second wave per SIMD hides the latency of the
// first.  The host takes it when a launch has more replicas than one wave per
// SIMD can hold at once (n = 50 benchmark launch: 2.45 s -> 1.69 s; three
// waves spill the step's own state and are slower).
// F64 = 1: the int64-difference build (one wave per SIMD).
template <int NS, int OCC, int F64, int SV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC))) k_persistent(const RunDesc *runs, const WorkItem *work, int nwork,
                                                    const int32_t *lnt_, unsigned int *next)
{
    using FT = typename std::conditional<F64 != 0, int64_t, int32_t>::type;
    // dynamic LDS: kWaveLds words per wave, the table read at random by the
    // exact acceptance test (see run_replica), then the flip's staging words
    extern __shared__ int32_t wave_tab[];
    MDA_LDS int32_t *tab = (MDA_LDS int32_t *)(wave_tab + (threadIdx.x >> 6) * kWaveLds);
    const MDA_GLOBAL int32_t *lnt = (const MDA_GLOBAL int32_t *)lnt_;
    const int lane = __lane_id();
    const int wpb = (int)(blockDim.x >> 6);
    const int wave = uni((int)(blockIdx.x * wpb + (threadIdx.x >> 6)));
    const int nwaves = (int)gridDim.x * wpb;
    // work items are taken in list order (largest first): a wave's first is
    // its own index, every later one comes from the launch's counter (zero at
    // launch), so that waves whose replicas run long take fewer of them
    for (int item = wave; item < nwork; item = nwaves + next_item(next, lane)) {
        const WorkItem w = {ro(work)[item].run, ro(work)[item].replica};
        Desc *Dp = ro(runs) + uni(w.run);
        const int r = uni(w.replica);
        // (an item of another variant is never planned into this launch)
        if (step_variant(Dp) == SV) run_replica<NS, SV / 2, SV % 2, FT>(Dp, r, lane, tab, lnt);
    }
}

// Plain form: state lives in HBM between launches (one launch per step).
template <int NS>
__device__ __forceinline__ void plain_load(Desc *Dp, Replica<NS> &S, int r, int lane)
{
    Desc &D = *Dp;
    const MDA_GLOBAL int32_t *pe = rw(D.pe) + (size_t)r * 2 * NS * 64;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        S.e1[i] = pe[i * 64 + lane];
        S.e2[i] = pe[(NS + i) * 64 + lane];
    }
    S.xm = rw(D.x)[(size_t)r * 64 + lane];
    const MDA_GLOBAL int64_t *st = rw(D.st) + (size_t)r * kStWords;
    S.E1 = uni64(st[kStE1]);
    S.E2 = uni64(st[kStE2]);
    S.Eoff = uni64(st[kStEoff]);
    S.moves = uni64(st[kStMoves]);
    S.scanned = uni64(st[kStScanned]);
    S.rngb = uni64(st[kStRng]);
    S.asize = uni((int)st[kStArch]);
    S.detailed = uni64(st[kStDetailed]);
}

template <int NS>
__device__ __forceinline__ void plain_store(Desc *Dp, const Replica<NS> &S, int r, int lane)
{
    Desc &D = *cold(Dp);
    MDA_GLOBAL int32_t *pe = rw(D.pe) + (size_t)r * 2 * NS * 64;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        pe[i * 64 + lane] = S.e1[i];
        pe[(NS + i) * 64 + lane] = S.e2[i];
    }
    rw(D.x)[(size_t)r * 64 + lane] = S.xm;
    if (lane == 0) {
        MDA_GLOBAL int64_t *st = rw(D.st) + (size_t)r * kStWords;
        st[kStE1] = S.E1;
        st[kStE2] = S.E2;
        st[kStEoff] = S.Eoff;
        st[kStMoves] = S.moves;
        st[kStScanned] = S.scanned;
        st[kStRng] = S.rngb;
        st[kStArch] = S.asize;
        st[kStDetailed] = S.detailed;
    }
}

template <int NS>
__global__ void __launch_bounds__(256) k_plain_init(const RunDesc *run)
{
    const int lane = __lane_id();
    const int r = uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    Desc *Dp = ro(run);
    if (r >= Dp->R) return;
    Replica<NS> S;
    switch (path_variant(Dp)) {
    case kPvDense: init_replica<NS, kPvDense>(Dp, S, r, lane); break;
    case kPvKronSym: init_replica<NS, kPvKronSym>(Dp, S, r, lane); break;
    default: init_replica<NS, kPvKronGen>(Dp, S, r, lane); break;
    }
    plain_store<NS>(Dp, S, r, lane);
}

template <int NS, int PV, int AM>
__device__ __forceinline__ void plain_step_one(Desc *Dp, int r, uint32_t t, int lane, const MDA_GLOBAL int32_t *lnt)
{
    Replica<NS> S;
    plain_load<NS>(Dp, S, r, lane);
    group_minima<NS, AM>(S);
    const Hot H = load_hot(Dp);
    // staging words of the flip: 256 per wave of the block (at most four)
    __shared__ __align__(16) int32_t plain_stage[4 * kStageWords];
    anneal_step<NS, PV, AM>(Dp, H, S, r, t, lane, lnt, H.thrmax[table_index(t, H.ntab)],
                            (MDA_LDS int32_t *)(plain_stage + (threadIdx.x >> 6) * kStageWords));
    plain_store<NS>(Dp, S, r, lane);
}

// One annealing step of every replica of the run, built per step variant SV
// (the run's own; the host launches the matching build).
template <int NS, int SV>
__global__ void __launch_bounds__(256) k_plain_step(const RunDesc *run, uint32_t t, const int32_t *lnt_)
{
    const int lane = __lane_id();
    const int r = uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    Desc *Dp = ro(run);
    if (r >= Dp->R || step_variant(Dp) != SV) return;
    const MDA_GLOBAL int32_t *lnt = (const MDA_GLOBAL int32_t *)lnt_;
    plain_step_one<NS, SV / 2, SV % 2>(Dp, r, t, lane, lnt);
}

template <int NS>
__global__ void __launch_bounds__(256) k_plain_final(const RunDesc *run)
{
    const int lane = __lane_id();
    const int r = uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    Desc *Dp = ro(run);
    if (r >= Dp->R) return;
    Replica<NS> S;
    plain_load<NS>(Dp, S, r, lane);
    export_replica<NS>(Dp, S, r, lane);
}

}  // namespace mda
