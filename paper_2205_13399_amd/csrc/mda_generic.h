// mda_generic.h -- the multi-objective Digital Annealer with K objectives on a
// generic QUBO (any m x m matrices Q_k, Eq. qubo): the extension beyond two
// objectives that the paper's Conclusion names, with the acceptance rules of
// Eqs. pacceptms / pacceptml summed or minimised over K objectives and K-way
// dominance in the archive updates of Algorithms 4 and 5.
//
// Layout: one replica per wave64.  Lane l holds the S consecutive bits
// a = l*S .. l*S + S - 1 (S a multiple of 8, S <= 64), so a group of eight
// slots of a lane is one Philox block of the random-number contract (bits
// a >> 3), and the flipped bit's row of the symmetric P_k streams coalesced
// from HBM: each lane reads its own S consecutive entries.  Per slot and
// objective the lane keeps the energy difference with the sign (1 - 2 x_a)
// folded in (int32: the build-time bound keeps every local field inside it);
// bits beyond m hold INT_MAX and never qualify.
#pragma once

#include "mda_device.h"

namespace mda {

constexpr int kMaxK = 4;

// Statistics block of a generic run (int64 words).
enum : int32_t {
    kGE = 0,            // E_1 .. E_K at kGE + k
    kGEoff = 4, kGMoves = 5, kGScanned = 6, kGRng = 7, kGArch = 8, kGDetailed = 9, kGNd = 10, kGWords = 16
};

struct GRunDesc {
    int32_t m, K, S, nl;       // bits, objectives, slots per lane, lanes holding bits (ceil(m / S))
    int32_t s;                 // archive capacity
    int32_t accept, archive, escape;
    int32_t R, trace_R;
    uint32_t key0, key1;
    uint32_t steps, ntab;
    int64_t beta;
    int64_t q[kMaxK];          // constants q_k
    int64_t ld;                // row stride of P_k: 64 S entries (zero beyond m)
    const int32_t *P;          // [K][m][ld]: P_k[a][b] at (k m + a) ld + b
    const int64_t *T;          // fixed-point temperature per table entry
    const int64_t *thrmax;     // (T * LNT[0]) >> 24 per table entry
    uint64_t *x;               // [R][64]: lane l's word, bit s = x of bit l S + s
    int64_t *h;                // [R][K][m] final local fields
    int64_t *st;               // [R][kGWords]
    int64_t *archE;            // [R][s][K]
    uint64_t *archX;           // [R][s][nl]
    uint8_t *nd;               // [R][s]
    int32_t *trace;            // [trace_R][steps]
};

using GDesc = const MDA_CONST GRunDesc;

template <int K, int S>
struct GRep {
    int32_t e[K][S];          // dE_k of bit l S + s, sign folded in
    uint64_t xm;              // bit s = x of bit l S + s
    int64_t E[K];
    int64_t Eoff, moves, scanned, rngb, detailed;
    int32_t asize;
    int32_t gmin[S / 8];      // per group of 8 slots: least combined difference
};

__device__ __forceinline__ GDesc *gcold(GDesc *p)
{
    uint64_t v = (uint64_t)p;
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    asm volatile("" : "+v"(lo), "+v"(hi));
    lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
    hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)hi);
    return (GDesc *)(((uint64_t)hi << 32) | lo);
}

// p dominates q over K objectives (Section 3.3): <= in every one, not equal in
// all; as for two objectives, exactly when the OR of the q_k - p_k is positive.
template <int K>
__device__ __forceinline__ bool gdom(const int64_t *p, const int64_t *q)
{
    int64_t o = q[0] - p[0];
#pragma unroll
    for (int k = 1; k < K; ++k) o |= q[k] - p[k];
    return o > 0;
}

template <int K, int S, int AM>
__device__ __forceinline__ void g_minima(GRep<K, S> &G)
{
#pragma unroll
    for (int g = 0; g < S; g += 8) {
        int32_t gm = INT_MAX;
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            int32_t v = G.e[0][g + f];
#pragma unroll
            for (int k = 1; k < K; ++k) v = AM == kAmStrict ? max(v, G.e[k][g + f]) : min(v, G.e[k][g + f]);
            gm = min(gm, v);
        }
        G.gmin[g >> 3] = gm;
    }
}

// Fields and energies of the solution in G.xm from scratch: every set bit b
// adds its row of P_k (the symmetric form, diagonal P_bb) to all bits; then
// h_k[a] = that sum minus P_aa x_a, dE_k[a] = (1 - 2 x_a)(P_aa + h_k[a]) and
// E_k = q_k + sum_{a in x} P_aa + (sum_{a in x} h_k[a]) / 2 (Eq. qubo).
template <int K, int S>
__device__ __forceinline__ void g_scratch(GDesc *Dp, GRep<K, S> &G, int lane_)
{
    const int lane = opaque_lane(lane_);
    GDesc &D = *gcold(Dp);
    const int m = D.m;
    const int64_t ld = D.ld;
    const int a0 = lane * S;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int s = 0; s < S; ++s) G.e[k][s] = 0;
    uint64_t todo = G.xm;
    for (;;) {
        const uint64_t bb = __ballot(todo != 0ull);
        if (bb == 0ull) break;
        const int bl = __ffsll((long long)bb) - 1;
        const int bs = uni(__ffsll((long long)rl64(todo, bl)) - 1);
        const int b = bl * S + bs;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const MDA_CONST int32_t *row = ro(D.P) + ((int64_t)k * m + b) * ld + a0;
#pragma unroll
            for (int s = 0; s < S; ++s) G.e[k][s] = (int32_t)((uint32_t)G.e[k][s] + (uint32_t)row[s]);
        }
        todo ^= (lane == bl) ? (1ull << bs) : 0ull;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        int64_t acc = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int a = a0 + s;
            const bool live = a < m;
            const bool on = (G.xm >> s) & 1ull;
            const int32_t d = live ? ro(D.P)[((int64_t)k * m + a) * ld + a] : 0;
            const int32_t h = (int32_t)((uint32_t)G.e[k][s] - (on ? (uint32_t)d : 0u));
            acc += on ? (int64_t)d * 2 + h : 0;
            const int32_t g = (int32_t)((uint32_t)d + (uint32_t)h);
            G.e[k][s] = live ? (on ? -g : g) : INT_MAX;
        }
        G.E[k] = D.q[k] + wave_sum64(acc) / 2;
    }
}

// Random start: bit a = bit (a & 31) of word (a >> 5) & 3 of the block
// (a >> 7, 0, r, INIT); a lane's S <= 64 bits lie in at most two blocks.
template <int K, int S>
__device__ __forceinline__ void g_init(GDesc *Dp, GRep<K, S> &G, int r, int lane)
{
    GDesc &D = *gcold(Dp);
    const int m = D.m;
    const int a0 = lane * S;
    const uint32_t b0 = (uint32_t)(a0 >> 7);
    const U4 o0 = philox10(b0, 0u, (uint32_t)r, kTagInit, D.key0, D.key1);
    const U4 o1 = philox10(b0 + 1u, 0u, (uint32_t)r, kTagInit, D.key0, D.key1);
    uint64_t xm = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int a = a0 + s;
        const bool first = (uint32_t)(a >> 7) == b0;
        const int wi = (a >> 5) & 3;
        const uint32_t w = wi == 0 ? (first ? o0.x : o1.x) : wi == 1 ? (first ? o0.y : o1.y)
                         : wi == 2 ? (first ? o0.z : o1.z) : (first ? o0.w : o1.w);
        const uint64_t bit = (a < m) ? (uint64_t)((w >> (a & 31)) & 1u) : 0ull;
        xm |= bit << s;
    }
    G.xm = xm;
    G.Eoff = 0;
    G.moves = G.scanned = G.rngb = G.detailed = 0;
    G.asize = 0;
    g_scratch<K, S>(Dp, G, lane);
}

// Archive update after a move: Algorithm 4 (explore) or 5 (exploit), K-way.
// The scans read the wave's copy of the archive energies in LDS (objective
// k of member e at AL[k s + e]); an insertion writes both that copy and the
// archive in HBM.
template <int K, int S>
__device__ __forceinline__ void g_archive(GDesc *Dp, GRep<K, S> &G, int r, uint32_t t, int lane_,
                                          MDA_LDS int64_t *AL)
{
    const int lane = opaque_lane(lane_);
    GDesc &D = *gcold(Dp);
    const int s = D.s, nl = D.nl;
    MDA_GLOBAL int64_t *AE = rw(D.archE) + (size_t)r * s * K;
    MDA_GLOBAL uint64_t *AX = rw(D.archX) + (size_t)r * s * nl;
    const int asz = G.asize;
    int64_t E[K];
#pragma unroll
    for (int k = 0; k < K; ++k) E[k] = G.E[k];
    int slot = -1;
    if (D.archive == 0) {
        // first member that x dominates, 4 blocks of 64 members per round trip
        // (all reads of a trip issued before any test; lanes past the end
        // through a bitwise AND, not a branch per block)
        constexpr int kAB = 4;
        for (int b = 0; b < asz; b += 64 * kAB) {
            int64_t a[kAB][K];
#pragma unroll
            for (int q = 0; q < kAB; ++q) {
                const int e = b + 64 * q + lane;
                const int ec = e < asz ? e : asz - 1;
#pragma unroll
                for (int k = 0; k < K; ++k) a[q][k] = AL[k * s + ec];
            }
            uint64_t M[kAB];
#pragma unroll
            for (int q = 0; q < kAB; ++q) {
                const int e = b + 64 * q + lane;
                M[q] = __ballot((e < asz) & gdom<K>(E, a[q]));
            }
            int q = -1;
#pragma unroll
            for (int qq = kAB - 1; qq >= 0; --qq) q = M[qq] ? qq : q;
            if (q >= 0) {
                uint64_t Mq = M[0];
#pragma unroll
                for (int qq = 1; qq < kAB; ++qq) Mq = (q == qq) ? M[qq] : Mq;
                const int f = __ffsll((long long)Mq) - 1;
                G.scanned += 64 * q + f + 1;
                slot = b + 64 * q + f;
                break;
            }
            G.scanned += (asz - b < 64 * kAB) ? (asz - b) : 64 * kAB;
        }
    } else {
        int nb = 0;
        bool rejected = false;
        for (int b = 0; b < asz; b += 64) {
            const int e = b + lane;
            bool z = false, y = false;
            if (e < asz) {
                int64_t a[K];
#pragma unroll
                for (int k = 0; k < K; ++k) a[k] = AL[k * s + e];
                z = gdom<K>(a, E);
                y = gdom<K>(E, a);
            }
            G.scanned += (asz - b < 64) ? (asz - b) : 64;
            if (__ballot(z)) {
                rejected = true;
                break;
            }
            nb += __popcll(__ballot(y));
        }
        if (rejected) return;
        if (nb > 0) {
            const U4 o = philox10(0u, t, (uint32_t)r, kTagArc, D.key0, D.key1);
            int k = (int)scale32((uint32_t)uni((int)o.x), (uint32_t)nb);
            for (int b = 0; b < asz; b += 64) {
                const int e = b + lane;
                bool y = false;
                if (e < asz) {
                    int64_t a[K];
#pragma unroll
                    for (int kk = 0; kk < K; ++kk) a[kk] = AL[kk * s + e];
                    y = gdom<K>(E, a);
                }
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
        G.asize = asz + 1;
    }
    slot = uni(slot);
    if (slot >= 0) {
        if (lane < K) {
            int64_t v = E[0];
#pragma unroll
            for (int k = 1; k < K; ++k) v = (lane == k) ? E[k] : v;
            AE[(size_t)slot * K + lane] = v;
            AL[lane * s + slot] = v;
        }
        if (lane < nl) AX[(size_t)slot * nl + lane] = G.xm;
    }
}

// One annealing step t (Algorithm 3 with the offset of Algorithm 1, readings
// G1-G3).  Returns the flipped bit or -1.  With THR (steps at the schedule's
// final, constant temperature) lnt holds the thresholds (T * LNT[k]) >> 24
// themselves, each below 2^32 - 1.
template <int K, int S, int AM, bool THR = false>
__device__ __forceinline__ int g_step(GDesc *Dp, GRep<K, S> &G, int r, uint32_t t, int lane_,
                                      const MDA_LDS int32_t *lnt, int64_t thrmax, MDA_LDS int64_t *AL)
{
    constexpr bool strict = AM == kAmStrict;
    GDesc &Dh = *Dp;
    const int lane = lane_;
    const int nl = Dh.nl;
    const uint64_t livelanes = (nl >= 64) ? ~0ull : ((1ull << nl) - 1ull);
    const uint32_t ti = table_index(t, Dh.ntab);
    // every real dE is at most 2^31 - 2 (build-time bound): capping the offset
    // and the largest threshold there keeps the comparisons exact
    const int32_t EoC = (int32_t)(G.Eoff < (int64_t)(INT_MAX - 1) ? G.Eoff : (int64_t)(INT_MAX - 1));
    const int64_t Xl = (int64_t)EoC + thrmax;
    const int32_t X = (int32_t)(Xl < (int64_t)(INT_MAX - 1) ? Xl : (int64_t)(INT_MAX - 1));
    int32_t mn = INT_MAX;
#pragma unroll
    for (int g = 0; g < S / 8; ++g) mn = min(mn, G.gmin[g]);
    const uint64_t cand = __ballot(mn <= X) & livelanes;
    int j = -1;
    if (cand) {
        G.detailed++;
        const int lane = opaque_lane(lane_);
        const int64_t T = THR ? 0 : ro(Dh.T)[ti];
        const uint32_t Th = (uint32_t)((uint64_t)T >> 24), Tl = (uint32_t)T & 0xFFFFFFu;
        uint64_t acc = 0;
#pragma unroll
        for (int g = 0; g < S; g += 8) {
            if (__ballot(G.gmin[g >> 3] <= X)) {
                uint32_t certain = 0, maybe = 0;
#pragma unroll
                for (int f = 0; f < 8; ++f) {
                    int32_t v = G.e[0][g + f];
#pragma unroll
                    for (int k = 1; k < K; ++k) v = strict ? max(v, G.e[k][g + f]) : min(v, G.e[k][g + f]);
                    const bool sure = v <= EoC;
                    const bool near = v <= X;
                    certain |= sure ? (1u << f) : 0u;
                    maybe |= (near && !sure) ? (1u << f) : 0u;
                }
                if (__ballot(maybe != 0u)) {
                    G.rngb++;
                    const U4 o = philox10((uint32_t)(lane * (S / 8) + (g >> 3)), t, (uint32_t)r, kTagAcc,
                                          Dh.key0, Dh.key1);
                    uint32_t Lv[8];
#pragma unroll
                    for (int f = 0; f < 8; ++f) {
                        const uint32_t w = (f < 2) ? o.x : (f < 4) ? o.y : (f < 6) ? o.z : o.w;
                        Lv[f] = (uint32_t)lnt[(w >> (16 * (f & 1) + 4)) & 0xFFFu];
                    }
#pragma unroll
                    for (int f = 0; f < 8; ++f) {
                        // S = sum (strict) or least (lenient) of max(0, dE_k - E_offset)
                        uint64_t Sx = 0;
#pragma unroll
                        for (int k = 0; k < K; ++k) {
                            const uint64_t u = (uint64_t)(uint32_t)(max(G.e[k][g + f], EoC) - EoC);
                            Sx = strict ? Sx + u : (k == 0 ? u : (u < Sx ? u : Sx));
                        }
                        uint64_t thr;
                        if (THR) {
                            thr = (uint64_t)Lv[f];
                        } else {
                            const uint32_t L = Lv[f] & 0xFFFFFu;
                            const uint64_t low = (uint64_t)Tl * (uint64_t)L;
                            thr = (uint64_t)Th * (uint64_t)L + (low >> 24);
                        }
                        certain |= ((maybe >> f) & (Sx <= thr ? 1u : 0u)) << f;
                    }
                }
                acc |= (uint64_t)certain << g;
            }
        }
        // uniform choice in ascending bit order a = l S + s: lane of the k-th
        // accepted bit from the exclusive prefix of the per-lane counts (one
        // ballot per bit of a count), then the slot within the lane
        const int c = __popcll(acc);
        const int cnt = wave_sum_dpp(c);
        if (cnt > 0) {
            const U4 o = philox10(0u, t, (uint32_t)r, kTagSel, Dh.key0, Dh.key1);
            const int k = (int)scale32((uint32_t)uni((int)o.x), (uint32_t)cnt);
            const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            int excl = 0;
#pragma unroll
            for (int b = 0; b < 7; ++b) excl += __popcll(__ballot((c >> b) & 1) & below) << b;
            const int jl = uni(__ffsll((long long)__ballot(excl <= k && k < excl + c)) - 1);
            int kk = k - rl(excl, jl);
            uint64_t msk = rl64(acc, jl);
            for (; kk > 0; --kk) msk &= msk - 1ull;
            const int js = uni(__ffsll((long long)msk) - 1);
            // flip bit j = jl S + js
            j = jl * S + js;
            GDesc &D = *gcold(Dp);
            const int m = D.m;
            const int64_t ld = D.ld;
            const uint64_t xj = (rl64(G.xm, jl) >> js) & 1ull;
            const uint64_t xmx = G.xm ^ (0ull - xj);   // bit s set where x_a != x_j
            const bool atj = lane == jl;
#pragma unroll
            for (int k2 = 0; k2 < K; ++k2) {
                int32_t v = 0;
#pragma unroll
                for (int s = 0; s < S; ++s) v = (s == js) ? G.e[k2][s] : v;
                const int32_t d = rl(v, jl);
                G.E[k2] += d;
                const MDA_CONST int32_t *row = ro(D.P) + ((int64_t)k2 * m + j) * ld + lane * S;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    // dE_k[a] += (x_a == x_j ? +1 : -1) P_k[a][j]; dE_k[j] becomes -dE_k[j]
                    const uint32_t b = (uint32_t)(xmx >> s) & 1u;
                    const uint32_t msk2 = 0u - b;
                    const int32_t upd = (int32_t)((uint32_t)G.e[k2][s] + (((uint32_t)row[s]) ^ msk2) + b);
                    G.e[k2][s] = (atj && s == js) ? -d : upd;
                }
            }
            G.xm ^= atj ? (1ull << js) : 0ull;
            g_minima<K, S, AM>(G);
            G.moves++;
            g_archive<K, S>(Dp, G, r, t, lane, AL);
        }
    }
    const bool moved = j >= 0;
    G.Eoff = moved ? 0 : ((Dh.escape == 0) ? G.Eoff + Dh.beta : G.Eoff);
    if (!moved && Dh.escape != 0 && G.asize > 0) {
        const int lane = opaque_lane(lane_);
        const U4 o = philox10(0u, t, (uint32_t)r, kTagArc, Dh.key0, Dh.key1);
        const int p = (int)scale32((uint32_t)uni((int)o.y), (uint32_t)G.asize);
        GDesc &D = *gcold(Dp);
        const MDA_GLOBAL uint64_t *ax = rw(D.archX) + ((size_t)r * D.s + p) * (size_t)D.nl;
        G.xm = (lane < D.nl) ? ax[lane] : 0ull;
        g_scratch<K, S>(Dp, G, lane);
        g_minima<K, S, AM>(G);
    }
    if (r < Dh.trace_R && lane == 0) rw(gcold(Dp)->trace)[(size_t)r * Dh.steps + (t - 1u)] = j;
    return j;
}

template <int K, int S>
__device__ __forceinline__ void g_export(GDesc *Dp, const GRep<K, S> &G, int r, int lane)
{
    GDesc &D = *gcold(Dp);
    const int m = D.m;
    const int64_t ld = D.ld;
    rw(D.x)[(size_t)r * 64 + lane] = (lane < D.nl) ? G.xm : 0ull;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        MDA_GLOBAL int64_t *h = rw(D.h) + ((size_t)r * K + k) * m;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int a = lane * S + s;
            if (a < m) {
                const bool on = (G.xm >> s) & 1ull;
                const int32_t d = ro(D.P)[((int64_t)k * m + a) * ld + a];
                h[a] = (int64_t)(on ? -G.e[k][s] : G.e[k][s]) - d;
            }
        }
    }
    if (lane == 0) {
        MDA_GLOBAL int64_t *st = rw(D.st) + (size_t)r * kGWords;
#pragma unroll
        for (int k = 0; k < K; ++k) st[kGE + k] = G.E[k];
        st[kGEoff] = G.Eoff;
        st[kGMoves] = G.moves;
        st[kGScanned] = G.scanned;
        st[kGRng] = G.rngb;
        st[kGArch] = G.asize;
        st[kGDetailed] = G.detailed;
    }
}

// Least of the group minima over the live lanes: a step's cheap test passes
// exactly when it is within the step's reach.
template <int K, int S>
__device__ __forceinline__ int32_t g_least(const GRep<K, S> &G, int nl, int lane)
{
    int32_t mn = INT_MAX;
#pragma unroll
    for (int g = 0; g < S / 8; ++g) mn = min(mn, G.gmin[g]);
    mn = lane < nl ? mn : INT_MAX;
    return wave_min_dpp(mn);
}

// Trace entries (no flip) of the q steps from t of a replica that records its
// trajectory.
__device__ __forceinline__ void g_quiet_trace(GDesc *Dp, int trace_R, int r, uint32_t t, uint32_t q, int lane)
{
    if (r < trace_R) {
        GDesc &D = *gcold(Dp);
        MDA_GLOBAL int32_t *tr = rw(D.trace) + (size_t)r * D.steps + (t - 1u);
        for (uint32_t i = (uint32_t)lane; i < q; i += 64u) tr[i] = -1;
    }
}

// thrt: the block's thresholds at the final temperature, or NULL when some
// would not fit 32 bits (then every step forms its thresholds from lnt).
template <int K, int S, int AM>
__device__ __forceinline__ void g_run(GDesc *Dp, int r, int lane, const MDA_LDS int32_t *lnt,
                                      const MDA_LDS int32_t *thrt, MDA_LDS int64_t *AL)
{
    GRep<K, S> G;
    g_init<K, S>(Dp, G, r, lane);
    g_minima<K, S, AM>(G);
    const uint32_t steps = Dp->steps, ntab = Dp->ntab;
    const MDA_CONST int64_t *thrmax = ro(Dp->thrmax);
    // With the offset escape a step whose cheap test fails does nothing but
    // raise the offset: such steps are decided against the replica's least
    // combined difference (live lanes), which only changes with a move, by the
    // scalar unit alone: one by one while the temperature changes, a whole
    // stretch at once (quiet_steps) at the final temperature.
    const bool skip = Dp->escape == 0;
    const int64_t beta = Dp->beta;
    const int trace_R = Dp->trace_R;
    int32_t least = g_least<K, S>(G, Dp->nl, lane);
    int64_t thr = thrmax[0];
    const uint32_t cool = (thrt == nullptr || ntab - 1u > steps) ? steps : ntab - 1u;
    uint32_t t = 1;
    for (; t <= cool; ++t) {
        const int64_t thr_next = thrmax[(t < ntab - 1u) ? t : ntab - 1u];
        if (skip && (int64_t)least > (int64_t)step_reach<int32_t>(G.Eoff, thr)) {
            G.Eoff += beta;
            g_quiet_trace(Dp, trace_R, r, t, 1u, lane);
        } else if (g_step<K, S, AM>(Dp, G, r, t, lane, lnt, thr, AL) >= 0) {
            least = g_least<K, S>(G, Dp->nl, lane);
        }
        thr = thr_next;
    }
    while (t <= steps) {
        if (skip) {
            const uint32_t q = quiet_steps((int64_t)least, G.Eoff, thr, beta, steps - t + 1u);
            if (q > 0u) {
                G.Eoff += (int64_t)q * beta;
                g_quiet_trace(Dp, trace_R, r, t, q, lane);
                t += q;
                continue;
            }
        }
        if (g_step<K, S, AM, true>(Dp, G, r, t, lane, thrt, thr, AL) >= 0) least = g_least<K, S>(G, Dp->nl, lane);
        ++t;
    }
    g_export<K, S>(Dp, G, r, lane);
}

// Persistent form: wave w of the grid runs replica w, then whichever replica
// comes next when it finishes (from the launch's counter, zero at launch).
// Dynamic LDS: s * K int64 archive energies per wave of the block.
template <int K, int S>
__global__ void __launch_bounds__(256) k_generic(const GRunDesc *run, const int32_t *lnt_, unsigned int *next)
{
    __shared__ int32_t lnt_lds[4096];
    __shared__ int32_t thr_lds[4096];
    extern __shared__ int64_t garch_lds[];
    // every wave of the launch runs the same schedule: the thresholds of the
    // final temperature, (T * LNT[k]) >> 24, are formed once per block
    const uint64_t Tf = (uint64_t)ro(run)->T[ro(run)->ntab - 1u];
    const bool use_thr = ((Tf * (uint64_t)(((const MDA_GLOBAL int32_t *)lnt_)[0] & 0xFFFFF)) >> 24) < 0xFFFFFFFFull;
    for (int k = (int)threadIdx.x; k < 4096; k += (int)blockDim.x) {
        const int32_t L = ((const MDA_GLOBAL int32_t *)lnt_)[k];
        lnt_lds[k] = L;
        thr_lds[k] = (int32_t)(uint32_t)((Tf * (uint64_t)(L & 0xFFFFF)) >> 24);
    }
    __syncthreads();
    const MDA_LDS int32_t *lnt = (const MDA_LDS int32_t *)lnt_lds;
    const MDA_LDS int32_t *thrt = use_thr ? (const MDA_LDS int32_t *)thr_lds : nullptr;
    const int lane = __lane_id();
    const int wpb = (int)(blockDim.x >> 6);
    const int wave = uni((int)(blockIdx.x * wpb + (threadIdx.x >> 6)));
    const int nwaves = (int)gridDim.x * wpb;
    GDesc *Dp = ro(run);
    const int R = Dp->R;
    const bool strict = Dp->accept == 0;
    MDA_LDS int64_t *AL = (MDA_LDS int64_t *)(garch_lds + (size_t)(threadIdx.x >> 6) * Dp->s * K);
    for (int r = wave; r < R; r = nwaves + next_item(next, lane)) {
        if (strict) g_run<K, S, kAmStrict>(Dp, r, lane, lnt, thrt, AL);
        else g_run<K, S, kAmLenient>(Dp, r, lane, lnt, thrt, AL);
    }
}

// Non-dominated flags within each replica's archive (K-way), one wave per replica.
template <int K>
__global__ void __launch_bounds__(256) k_gnondominated(const GRunDesc *run)
{
    const int lane = __lane_id();
    const int r = uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    GDesc &D = *ro(run);
    if (r >= D.R) return;
    const int s = D.s;
    int asz = uni((int)rw(D.st)[(size_t)r * kGWords + kGArch]);
    asz = asz < 0 ? 0 : (asz > s ? s : asz);
    const MDA_CONST int64_t *AE = ro(D.archE) + (size_t)r * s * K;
    MDA_GLOBAL uint8_t *nd = rw(D.nd) + (size_t)r * s;
    int count = 0;
    for (int b = 0; b < asz; b += 64) {
        const int e = b + lane;
        const int ec = e < asz ? e : asz - 1;
        int64_t a[K];
#pragma unroll
        for (int k = 0; k < K; ++k) a[k] = AE[(size_t)ec * K + k];
        bool dom = false;
        for (int f = 0; f < asz; ++f) {
            int64_t q[K];
#pragma unroll
            for (int k = 0; k < K; ++k) q[k] = AE[(size_t)f * K + k];
            dom |= gdom<K>(q, a);
        }
        if (e < asz) {
            nd[e] = dom ? 0 : 1;
            count += dom ? 0 : 1;
        }
    }
    count = wave_sum(count);
    if (lane == 0) rw(D.st)[(size_t)r * kGWords + kGNd] = count;
}

// ---- merged non-dominated front of several replicas (K-way, Section 3.3) ----

struct GFrontEntry {
    int64_t e[kMaxK];
    int32_t rep, slot;
};

// One wave per replica r0 + k: its flagged (non-dominated within its archive)
// entries appended at offs[k] in slot order (offs has nr + 1 entries: the host
// prefix of the flag counts), and K + 1 of them as reference points: the entry
// of least energy sum and, for each objective, the entry of least energy in it
// (lowest slot on ties), or entries of INT64_MAX energies if there is none.
template <int K>
__global__ void __launch_bounds__(256) k_ggather(const GRunDesc *run, int r0, int nr, const int64_t *offs,
                                                 GFrontEntry *out, GFrontEntry *ref)
{
    const int lane = __lane_id();
    const int k = uni((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    if (k >= nr) return;
    GDesc &D = *ro(run);
    const int r = r0 + k, s = D.s;
    int asz = uni((int)ro(D.st)[(size_t)r * kGWords + kGArch]);
    asz = asz < 0 ? 0 : (asz > s ? s : asz);
    const MDA_CONST int64_t *AE = ro(D.archE) + (size_t)r * s * K;
    const MDA_CONST uint8_t *nd = ro(D.nd) + (size_t)r * s;
    const int64_t base = offs[k], lim = offs[k + 1];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t run_n = 0;
    // key c = 0: energy sum; c = 1..K: objective c - 1
    int64_t bv[K + 1];
    int bslot[K + 1];
#pragma unroll
    for (int c = 0; c <= K; ++c) {
        bv[c] = INT64_MAX;
        bslot[c] = INT_MAX;
    }
    for (int b = 0; b < asz; b += 64) {
        const int e = b + lane;
        const bool flag = e < asz && nd[e] != 0;
        const uint64_t M = __ballot(flag);
        const int64_t pos = base + run_n + __popcll(M & below);
        if (flag) {
            int64_t sum = 0;
            GFrontEntry g;
#pragma unroll
            for (int q = 0; q < kMaxK; ++q) g.e[q] = 0;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                g.e[q] = AE[(size_t)e * K + q];
                sum += g.e[q];
                if (g.e[q] < bv[q + 1]) {
                    bv[q + 1] = g.e[q];
                    bslot[q + 1] = e;
                }
            }
            g.rep = r;
            g.slot = e;
            if (pos < lim) out[pos] = g;
            if (sum < bv[0]) {
                bv[0] = sum;
                bslot[0] = e;
            }
        }
        run_n += __popcll(M);
    }
    // least (value, slot) of each key over the wave
#pragma unroll
    for (int c = 0; c <= K; ++c) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const int64_t ov = __shfl_xor(bv[c], off);
            const int os = __shfl_xor(bslot[c], off);
            if (ov < bv[c] || (ov == bv[c] && os < bslot[c])) {
                bv[c] = ov;
                bslot[c] = os;
            }
        }
    }
    if (lane <= K) {
        int sl = bslot[0];
#pragma unroll
        for (int c = 1; c <= K; ++c) sl = (lane == c) ? bslot[c] : sl;
        GFrontEntry g;
#pragma unroll
        for (int q = 0; q < kMaxK; ++q) g.e[q] = INT64_MAX;
        if (sl != INT_MAX) {
#pragma unroll
            for (int q = 0; q < K; ++q) g.e[q] = AE[(size_t)sl * K + q];
        }
        g.rep = sl != INT_MAX ? r : -1;
        g.slot = sl != INT_MAX ? sl : -1;
        ref[(size_t)k * (K + 1) + lane] = g;
    }
}

// Pre-filter: candidates that a reference point dominates are dropped (a
// dominated entry is never in the merged front); the rest are appended to keep
// in arbitrary order.  One thread per candidate, reference points staged
// through LDS 256 at a time; the block stops once all its candidates are out.
template <int K>
__global__ void __launch_bounds__(256) k_gfilter(const GFrontEntry *cand, int64_t n, const GFrontEntry *ref, int nref,
                                                 GFrontEntry *keep, unsigned long long *nkeep)
{
    __shared__ int64_t tile[256 * K];
    const int tid = (int)threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    bool alive = i < n;
    int64_t c[K];
#pragma unroll
    for (int q = 0; q < K; ++q) c[q] = alive ? cand[i].e[q] : 0;
    for (int t0 = 0; t0 < nref; t0 += 256) {
        if (!__syncthreads_or(alive)) break;
        const int j = t0 + tid;
#pragma unroll
        for (int q = 0; q < K; ++q) tile[tid * K + q] = j < nref ? ref[j].e[q] : INT64_MAX;
        __syncthreads();
        const int cnt = min(256, nref - t0);
        if (alive) {
            for (int t = 0; t < cnt; ++t) {
                bool le = true, eq = true;
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    const int64_t v = tile[t * K + q];
                    le = le && v <= c[q];
                    eq = eq && v == c[q];
                }
                if (le && !eq) {
                    alive = false;
                    break;
                }
            }
        }
    }
    if (alive) {
        const unsigned long long at = atomicAdd(nkeep, 1ull);
        keep[at] = cand[i];
    }
}

// Exact pass over the survivors: an entry stays unless another survivor
// dominates it or has the same energies and a lower (replica, slot).
template <int K>
__global__ void __launch_bounds__(256) k_gexact(const GFrontEntry *cand, int64_t n, GFrontEntry *front,
                                                unsigned long long *nfront)
{
    __shared__ int64_t tile[256 * K];
    __shared__ int64_t tkey[256];
    const int tid = (int)threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 256 + tid;
    bool alive = i < n;
    int64_t c[K];
    int64_t ckey = 0;
    if (alive) {
#pragma unroll
        for (int q = 0; q < K; ++q) c[q] = cand[i].e[q];
        ckey = ((int64_t)cand[i].rep << 32) | (int64_t)(uint32_t)cand[i].slot;
    } else {
#pragma unroll
        for (int q = 0; q < K; ++q) c[q] = 0;
    }
    for (int64_t t0 = 0; t0 < n; t0 += 256) {
        if (!__syncthreads_or(alive)) break;
        const int64_t j = t0 + tid;
        if (j < n) {
#pragma unroll
            for (int q = 0; q < K; ++q) tile[tid * K + q] = cand[j].e[q];
            tkey[tid] = ((int64_t)cand[j].rep << 32) | (int64_t)(uint32_t)cand[j].slot;
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)256, n - t0);
        if (alive) {
            for (int t = 0; t < cnt; ++t) {
                bool le = true, eq = true;
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    const int64_t v = tile[t * K + q];
                    le = le && v <= c[q];
                    eq = eq && v == c[q];
                }
                if (le && (!eq || tkey[t] < ckey)) {
                    alive = false;
                    break;
                }
            }
        }
    }
    if (alive) {
        const unsigned long long at = atomicAdd(nfront, 1ull);
        front[at] = cand[i];
    }
}

// Stored solutions of n (replica, slot) pairs, packed (replica << 32 | slot),
// into out (n x nl words): one thread per word.
#ifdef MDA_GX_HOME
__global__ void __launch_bounds__(256) k_gxgather(const int64_t *at, int64_t n, const uint64_t *archX, int s, int nl,
                                                  uint64_t *out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n * nl) return;
    const int64_t i = t / nl;
    const int w = (int)(t - i * nl);
    const int64_t key = at[i];
    const int64_t rep = key >> 32, slot = key & 0xFFFFFFFFll;
    out[t] = archX[((size_t)rep * s + slot) * nl + w];
}

hipError_t launch_gxgather(const int64_t *at, int64_t n, const uint64_t *archX, int s, int nl, uint64_t *out,
                           hipStream_t stream)
{
    if (n > 0)
        hipLaunchKernelGGL(k_gxgather, dim3((unsigned)((n * nl + 255) / 256)), dim3(256), 0, stream, at, n, archX, s, nl,
                           out);
    return hipGetLastError();
}
#endif

}  // namespace mda
