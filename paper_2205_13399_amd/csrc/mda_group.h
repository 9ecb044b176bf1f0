// mda_group.h -- workgroup form of the multi-objective Digital Annealer
// (Ayodele et al., GECCO 2022, arXiv:2205.13399): one replica spread over the
// WR x WC waves of a workgroup, for instances whose n exceeds one wave's 64
// lanes (up to 128) or to put more waves behind one replica.
//
// Wave (p, c), p < WR, c < WC, holds facilities [p NS, p NS + NS) as register
// slots and locations [64 c, 64 c + 64) as lanes, with the same per-lane state
// as the one-wave form (the two energy differences with the sign folded in and
// a mask of its x bits).  The step is the same as the one-wave form's; the
// waves meet in LDS at most four times per step:
//   B1  "can any bit be accepted" flags (double-buffered by step parity);
//   B2  every lane's mask of accepted bits, from which each wave computes the
//       same uniform choice in ascending bit order a = i n + u;
//   B3  the chosen bit's differences and value, written by the wave holding it;
//   B4  the archive decision, taken identically by every wave, before the
//       archive is written.
// Energies and the offset are kept identically in every wave.  The operands
// are read with masks (facility and location below n), so dead slots and
// lanes read zeros as in the padded one-wave layout.
#pragma once

#include "mda_device.h"

namespace mda {

constexpr int kMaxGroupWaves = 8;

struct GroupLds {
    int32_t lnt[4096];
    int32_t flag[2][kMaxGroupWaves];
    uint64_t acc[kMaxGroupWaves][64];
    uint64_t xs[kMaxGroupWaves][64];
    int64_t part[kMaxGroupWaves][4];
    // per wave: the flipped facility's flow rows over this wave's slots
    // (four rows of 64), read back by the flip as uniform 16-byte loads
    int32_t stage[kMaxGroupWaves][256];
    int32_t pick[4];
};

struct Geo {
    int w, p, c, G, WC, i0, u, lane;
};

// Column masks of the whole solution in LDS (xs) -> this wave's fields and the
// energies, from scratch (as fields_from_scratch of the one-wave form).
template <int NS, int PV>
__device__ __forceinline__ void g_fields(Desc *Dp, Replica<NS> &S, const Geo &g, GroupLds &L)
{
    Desc &D = *cold(Dp);
    const int n = opaque(D.n);
    const int lane = opaque_lane(g.lane);
    const int ldk = D.ldk;
    const int u = g.u;
    const bool live = u < n;
    const int G = g.G, WC = g.WC;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        S.e1[s] = 0;
        S.e2[s] = 0;
    }
    const int fi = g.i0 + lane;   // facility of this lane's factor entry
    for (int w2 = 0; w2 < G; ++w2) {
        const int i02 = (w2 / WC) * NS, u02 = (w2 % WC) * 64;
        uint64_t todo = L.xs[w2][lane];
        for (;;) {
            const uint64_t bb = __ballot(todo != 0ull);
            if (bb == 0ull) break;
            const int bl = __ffsll((long long)bb) - 1;
            const int bs = uni(__ffsll((long long)rl64(todo, bl)) - 1);
            const int bi = i02 + bs, bu = u02 + bl;
            if (PV == kPvDense) {
                const size_t row = (size_t)(bi * n + bu) * (size_t)n * (size_t)D.pld;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const int i = g.i0 + s;
                    const bool ok = live && i < n;
                    S.e1[s] = (int32_t)((uint32_t)S.e1[s] + (ok ? (uint32_t)ro(D.P1)[row + (size_t)i * D.pld + u] : 0u));
                    S.e2[s] = (int32_t)((uint32_t)S.e2[s] + (ok ? (uint32_t)ro(D.P2)[row + (size_t)i * D.pld + u] : 0u));
                }
            } else {
                const int32_t dv = live ? ro(D.DA)[bu * ldk + u] : 0;
                const int32_t dw = (PV == kPvKronGen && live) ? ro(D.DB)[bu * ldk + u] : 0;
                const bool fok = fi < n;
                const int32_t fa1 = fok ? ro(D.KA1)[bi * ldk + fi] : 0;
                const int32_t fa2 = fok ? ro(D.KA2)[bi * ldk + fi] : 0;
                const int32_t fb1 = (PV == kPvKronGen && fok) ? ro(D.KB1)[bi * ldk + fi] : 0;
                const int32_t fb2 = (PV == kPvKronGen && fok) ? ro(D.KB2)[bi * ldk + fi] : 0;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    uint32_t t1 = (uint32_t)__mul24(rl(fa1, s), dv);
                    uint32_t t2 = (uint32_t)__mul24(rl(fa2, s), dv);
                    if (PV == kPvKronGen) {
                        t1 += (uint32_t)__mul24(rl(fb1, s), dw);
                        t2 += (uint32_t)__mul24(rl(fb2, s), dw);
                    }
                    S.e1[s] = (int32_t)((uint32_t)S.e1[s] + t1);
                    S.e2[s] = (int32_t)((uint32_t)S.e2[s] + t2);
                }
            }
            todo ^= (lane == bl) ? (1ull << bs) : 0ull;
        }
    }
    // Self term, penalty counts (row i over every column-wave of this wave's
    // row block, column u over every row block), diagonal, sign.
    const uint64_t xl = S.xm;
    uint32_t cu = 0;
    for (int p2 = 0; p2 * WC < G; ++p2) cu += (uint32_t)__popcll(L.xs[p2 * WC + g.c][lane]);
    const uint32_t ta1 = (uint32_t)D.two_alpha1, ta2 = (uint32_t)D.two_alpha2;
    int64_t acc1 = 0, acc2 = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = g.i0 + s;
        const bool on = (xl >> s) & 1ull;
        const bool ok = live && i < n;
        uint32_t ri = 0;
        for (int c2 = 0; c2 < WC; ++c2) ri += (uint32_t)__popcll(__ballot((L.xs[g.p * WC + c2][lane] >> s) & 1ull));
        const uint32_t dg1 = ok ? (uint32_t)ro(D.diag1)[i * ldk + u] : 0u;
        const uint32_t dg2 = ok ? (uint32_t)ro(D.diag2)[i * ldk + u] : 0u;
        uint32_t g1 = (uint32_t)S.e1[s] + dg1, g2 = (uint32_t)S.e2[s] + dg2;
        if (PV == kPvDense) {
            g1 -= on ? dg1 : 0u;
            g2 -= on ? dg2 : 0u;
        } else {
            g1 -= on ? 2u * (dg1 + ta1) : 0u;
            g2 -= on ? 2u * (dg2 + ta2) : 0u;
            const uint32_t cnt = ri + cu - (on ? 2u : 0u);
            g1 += cnt * ta1;
            g2 += cnt * ta2;
        }
        acc1 += (on && ok) ? (int64_t)(int32_t)g1 + (int32_t)dg1 : 0;
        acc2 += (on && ok) ? (int64_t)(int32_t)g2 + (int32_t)dg2 : 0;
        const int32_t s1 = on ? -(int32_t)g1 : (int32_t)g1;
        const int32_t s2 = on ? -(int32_t)g2 : (int32_t)g2;
        S.e1[s] = ok ? s1 : (live ? kDead : INT_MAX);
        S.e2[s] = ok ? s2 : (live ? kDead : INT_MAX);
    }
    const int64_t w1 = wave_sum64(acc1), w2s = wave_sum64(acc2);
    if (lane == 0) {
        L.part[g.w][0] = w1;
        L.part[g.w][1] = w2s;
    }
    __syncthreads();
    int64_t t1 = 0, t2 = 0;
    for (int w2 = 0; w2 < G; ++w2) {
        t1 += L.part[w2][0];
        t2 += L.part[w2][1];
    }
    S.E1 = D.q1 + t1 / 2;
    S.E2 = D.q2 + t2 / 2;
    __syncthreads();   // part[] is free again
}

// Random start: bit (i, u) is bit i of the 128-bit Philox block (0, u) with
// tag INIT (words x, y, z, w low to high), the same draw as the one-wave form;
// n <= 128.
template <int NS, int PV>
__device__ __forceinline__ void g_init(Desc *Dp, Replica<NS> &S, int r, const Geo &g, GroupLds &L)
{
    Desc &D = *cold(Dp);
    const int n = opaque(D.n);
    const U4 o = philox10((uint32_t)g.u, 0u, (uint32_t)r, kTagInit, D.key0, D.key1);
    const uint64_t lo = ((uint64_t)o.y << 32) | o.x, hi = ((uint64_t)o.w << 32) | o.z;
    const int i0 = g.i0;
    uint64_t v = (i0 == 0) ? lo : (i0 >= 64) ? (hi >> (i0 - 64)) : ((lo >> i0) | (hi << (64 - i0)));
    const int rows = n - i0;   // valid rows of this wave
    const uint64_t rmask = rows >= 64 ? ~0ull : (rows <= 0 ? 0ull : ((1ull << rows) - 1ull));
    const uint64_t smask = NS >= 64 ? ~0ull : ((1ull << NS) - 1ull);
    S.xm = (g.u < n) ? (v & rmask & smask) : 0ull;
    S.Eoff = 0;
    S.moves = S.scanned = S.rngb = S.detailed = 0;
    S.asize = 0;
    L.xs[g.w][g.lane] = S.xm;
    __syncthreads();
    g_fields<NS, PV>(Dp, S, g, L);
}

// Restart from archive member p: every wave loads its block of the solution.
template <int NS, int PV>
__device__ __forceinline__ void g_restart(Desc *Dp, Replica<NS> &S, int r, int pm, const Geo &g, GroupLds &L)
{
    Desc &D = *cold(Dp);
    S.xm = rw(D.archX)[((size_t)r * D.s + pm) * (size_t)D.xw + (size_t)g.w * 64 + g.lane];
    L.xs[g.w][g.lane] = S.xm;
    __syncthreads();
    g_fields<NS, PV>(Dp, S, g, L);
}

// Flip of bit (js, jl) (global facility and location) with differences d1, d2
// and value xj, in every wave's block.
template <int NS, int PV>
__device__ __forceinline__ void g_flip(Desc *Dp, Replica<NS> &S, const Geo &g, int js, int jl, int32_t d1,
                                       int32_t d2, uint32_t xj, GroupLds &L)
{
    Desc &D = *cold(Dp);
    const int n = opaque(D.n);
    const int lane = opaque_lane(g.lane);
    const int ldk = D.ldk;
    const int u = g.u;
    const bool live = u < n;
    const int jsl = js - g.i0;                    // slot of row js here, if in range
    const bool rowhere = jsl >= 0 && jsl < NS;
    const bool atj = u == jl;                     // this lane is location jl
    const uint64_t xmx = S.xm ^ (0ull - (uint64_t)xj);
    S.E1 += d1;
    S.E2 += d2;
    if (PV == kPvDense) {
        const int j = js * n + jl;
        const uint32_t c1 = (atj && rowhere) ? (uint32_t)(-2 * d1) - (uint32_t)ro(D.diag1)[js * ldk + jl] : 0u;
        const uint32_t c2 = (atj && rowhere) ? (uint32_t)(-2 * d2) - (uint32_t)ro(D.diag2)[js * ldk + jl] : 0u;
        const size_t row = (size_t)j * (size_t)n * (size_t)D.pld;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int i = g.i0 + s;
            const bool ok = live && i < n;
            const uint32_t t1 = ok ? (uint32_t)ro(D.P1)[row + (size_t)i * D.pld + u] : 0u;
            const uint32_t t2 = ok ? (uint32_t)ro(D.P2)[row + (size_t)i * D.pld + u] : 0u;
            const uint32_t b = (uint32_t)(xmx >> s) & 1u;
            const uint32_t m = 0u - b;
            S.e1[s] = (int32_t)((uint32_t)S.e1[s] + (t1 ^ m) + b);
            S.e2[s] = (int32_t)((uint32_t)S.e2[s] + (t2 ^ m) + b);
        }
        // bit j's own entry, in the wave that holds row js (jsl outside
        // [0, NS) elsewhere: no slot)
        add_to_slot<NS, int32_t>(S, uni(jsl), xmx, c1, c2);
    } else {
        const int fi = g.i0 + lane;
        const bool fok = fi < n;
        const int32_t dv = live ? ro(D.DA)[jl * ldk + u] : 0;
        const int32_t dw = (PV == kPvKronGen && live) ? ro(D.DB)[jl * ldk + u] : 0;
        const int32_t fa1 = fok ? ro(D.KA1)[js * ldk + fi] : 0;
        const int32_t fa2 = fok ? ro(D.KA2)[js * ldk + fi] : 0;
        const int32_t fb1 = (PV == kPvKronGen && fok) ? ro(D.KB1)[js * ldk + fi] : 0;
        const int32_t fb2 = (PV == kPvKronGen && fok) ? ro(D.KB2)[js * ldk + fi] : 0;
        // the wave's own staging words (no other wave reads them)
        int32_t *stage = L.stage[g.w];
        stage[lane] = fa1;
        stage[64 + lane] = fa2;
        if (PV == kPvKronGen) {
            stage[128 + lane] = fb1;
            stage[192 + lane] = fb2;
        }
        const MDA_LDS v4i32 *s4 = (const MDA_LDS v4i32 *)(MDA_LDS int32_t *)stage;
        const uint32_t ta1 = (uint32_t)D.two_alpha1, ta2 = (uint32_t)D.two_alpha2;
        const uint32_t q1 = atj ? ta1 : 0u, q2 = atj ? ta2 : 0u;
        // own column entry of bit j (only used in the wave holding it)
        const int jsc = rowhere ? jsl : 0;
        uint32_t own1 = (uint32_t)__mul24(rl(fa1, jsc), dv), own2 = (uint32_t)__mul24(rl(fa2, jsc), dv);
        if (PV == kPvKronGen) {
            own1 += (uint32_t)__mul24(rl(fb1, jsc), dw);
            own2 += (uint32_t)__mul24(rl(fb2, jsc), dw);
        }
        const uint32_t r1 = atj ? (uint32_t)(-2 * d1) - own1 : (live ? ta1 : 0u);
        const uint32_t r2 = atj ? (uint32_t)(-2 * d2) - own2 : (live ? ta2 : 0u);
#pragma unroll
        for (int g4 = 0; g4 < NS; g4 += 4) {
            const v4i32 a1 = s4[g4 / 4], a2 = s4[16 + g4 / 4];
            v4i32 b1 = a1, b2 = a2;
            if (PV == kPvKronGen) {
                b1 = s4[32 + g4 / 4];
                b2 = s4[48 + g4 / 4];
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int s = g4 + f;
                uint32_t t1 = (uint32_t)__mul24(a1[f], dv) + q1;
                uint32_t t2 = (uint32_t)__mul24(a2[f], dv) + q2;
                if (PV == kPvKronGen) {
                    t1 += (uint32_t)__mul24(b1[f], dw);
                    t2 += (uint32_t)__mul24(b2[f], dw);
                }
                const uint32_t b = (uint32_t)(xmx >> s) & 1u;
                const uint32_t m = 0u - b;
                S.e1[s] = (int32_t)((uint32_t)S.e1[s] + (t1 ^ m) + b);
                S.e2[s] = (int32_t)((uint32_t)S.e2[s] + (t2 ^ m) + b);
            }
        }
        // row js takes r_k in place of q_k (in the wave that holds it)
        add_to_slot<NS, int32_t>(S, uni(jsl), xmx, r1 - q1, r2 - q2);
    }
    S.xm ^= (atj && rowhere) ? (1ull << (jsl & 63)) : 0ull;
}

// Archive update (Algorithm 4 or 5): every wave scans the same energies and
// reaches the same decision; the writes wait for every wave's scan.
template <int NS>
__device__ __forceinline__ void g_archive(Desc *Dp, Replica<NS> &S, int r, uint32_t t, const Geo &g,
                                          uint32_t key0, uint32_t key1)
{
    Desc &D = *cold(Dp);
    const int lane = opaque_lane(g.lane);
    const int s = D.s;
    MDA_GLOBAL int64_t *AE = rw(D.archE) + (size_t)r * s * 2;
    const int asz = S.asize;
    const int64_t E1 = S.E1, E2 = S.E2;
    int slot = -1;
    if (D.archive == 0) {
        // first member that x dominates, 8 blocks of 64 members per round trip
        // (indices clamped into the archive, so every read is in bounds; all
        // loads of a trip are issued before any test, which takes lanes past
        // the end through a bitwise AND rather than a branch per block)
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
        if (!rejected && nb > 0) {
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
        if (rejected) slot = -2;
    }
    if (slot == -1 && asz < s) {
        slot = asz;
        S.asize = asz + 1;
    }
    slot = uni(slot);
    __syncthreads();   // B4: every wave has read the archive
    if (slot >= 0) {
        if (g.w == 0 && lane == 0) {
            AE[2 * slot] = E1;
            AE[2 * slot + 1] = E2;
        }
        rw(D.archX)[((size_t)r * s + slot) * (size_t)D.xw + (size_t)g.w * 64 + lane] = S.xm;
    }
}

// One annealing step of the workgroup form; true when a bit was flipped.
template <int NS, int PV, int AM>
__device__ __forceinline__ bool g_step(Desc *Dp, const Hot &H, Replica<NS> &S, int r, uint32_t t, const Geo &g,
                                       GroupLds &L, uint32_t thrmax)
{
    constexpr bool strict = AM == kAmStrict;
    const int n = H.n;
    const int lane = g.lane;
    const bool live = g.u < n;
    const uint32_t ti = table_index(t, H.ntab);
    const int32_t EoC = (int32_t)(S.Eoff < (int64_t)(INT_MAX - 1) ? S.Eoff : (int64_t)(INT_MAX - 1));
    const int64_t Xl = (int64_t)EoC + (int64_t)thrmax;
    const int32_t X = (int32_t)(Xl < (int64_t)(INT_MAX - 1) ? Xl : (int64_t)(INT_MAX - 1));

    // minimum per group of 8 slots: the exact test below passes over groups in
    // which no lane of this wave comes within reach
    int32_t gmin[NS / 8];
#pragma unroll
    for (int gg = 0; gg < NS; gg += 8) {
        int32_t gm = INT_MAX;
#pragma unroll
        for (int f = 0; f < 8; ++f)
            gm = min(gm, strict ? max(S.e1[gg + f], S.e2[gg + f]) : min(S.e1[gg + f], S.e2[gg + f]));
        gmin[gg >> 3] = gm;
    }
    int32_t mn = INT_MAX;
#pragma unroll
    for (int gg = 0; gg < NS / 8; ++gg) mn = min(mn, gmin[gg]);
    const uint64_t cand = __ballot(live && mn <= X);
    if (lane == 0) L.flag[t & 1u][g.w] = cand != 0ull ? 1 : 0;
    __syncthreads();   // B1
    int any = 0;
    for (int w2 = 0; w2 < g.G; ++w2) any |= L.flag[t & 1u][w2];
    any = uni(any);

    bool moved = false;
    if (any) {
        S.detailed++;
        const int64_t T = H.T[ti];
        const uint32_t Th = (uint32_t)((uint64_t)T >> 24), Tl = (uint32_t)T & 0xFFFFFFu;
        uint64_t acc = 0;
        const int rows = opaque(n - g.i0);   // facilities of this wave's block below n
#pragma unroll
        for (int gg = 0; gg < NS; gg += 8) {
            // dead lanes hold INT_MAX and never qualify; a group with no slot
            // within X on any lane has no acceptance and draws no random block
            if (gg < rows && __ballot(gmin[gg >> 3] <= X)) {
                const uint32_t slots = (rows - gg >= 8) ? 0xFFu : ((1u << (rows - gg)) - 1u);
                uint32_t certain = 0, maybe = 0;
#pragma unroll
                for (int f = 0; f < 8; ++f) {
                    const int s = gg + f;
                    const int32_t v = strict ? max(S.e1[s], S.e2[s]) : min(S.e1[s], S.e2[s]);
                    certain |= (v <= EoC) ? (1u << f) : 0u;
                    maybe |= (v <= X && v > EoC) ? (1u << f) : 0u;
                }
                certain &= slots;
                maybe &= slots;
                if (__ballot(maybe != 0u)) {
                    S.rngb++;
                    const U4 o = philox10(((uint32_t)((g.i0 + gg) >> 3) << 16) | (uint32_t)g.u, t, (uint32_t)r,
                                          kTagAcc, H.key0, H.key1);
                    // all eight lookups first, then every slot tested without a
                    // branch; slots that are not undecided keep their decision
                    uint32_t Lv[8];
#pragma unroll
                    for (int f = 0; f < 8; ++f) {
                        const uint32_t w = (f < 2) ? o.x : (f < 4) ? o.y : (f < 6) ? o.z : o.w;
                        Lv[f] = (uint32_t)L.lnt[(w >> (16 * (f & 1))) & 0xFFFu];
                    }
#pragma unroll
                    for (int f = 0; f < 8; ++f) {
                        const int s = gg + f;
                        const uint32_t u1 = (uint32_t)(max(S.e1[s], EoC) - EoC);
                        const uint32_t u2 = (uint32_t)(max(S.e2[s], EoC) - EoC);
                        const uint32_t Sx = strict ? (u1 + u2) : (u1 < u2 ? u1 : u2);
                        const uint32_t Lk = Lv[f] & 0xFFFFFu;
                        const uint64_t low = (uint64_t)Tl * (uint64_t)Lk;
                        // the exact threshold, compared in 64 bits
                        const uint64_t t64 = (uint64_t)Th * (uint64_t)Lk + (low >> 24);
                        const uint32_t ok = (uint64_t)Sx <= t64 ? 1u : 0u;
                        certain |= ((maybe >> f) & ok) << f;
                    }
                }
                acc |= (uint64_t)certain << gg;
            }
        }
        L.acc[g.w][lane] = acc;
        __syncthreads();   // B2
        int c = 0;
        for (int w2 = 0; w2 < g.G; ++w2) c += __popcll(L.acc[w2][lane]);
        const int cnt = wave_sum_dpp(c);
        if (cnt > 0) {
            const U4 o = philox10(0u, t, (uint32_t)r, kTagSel, H.key0, H.key1);
            int k = (int)scale32((uint32_t)uni((int)o.x), (uint32_t)cnt);
            // row (facility) of the k-th accepted bit: the largest row lo with
            // fewer than k + 1 accepted bits in the rows above it
            int lo = 0, hi = n;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                int b = 0;
                for (int w2 = 0; w2 < g.G; ++w2) {
                    const int i02 = (w2 / g.WC) * NS;
                    const int rr = mid - i02;
                    const uint64_t rm = rr <= 0 ? 0ull : (rr >= 64 ? ~0ull : ((1ull << rr) - 1ull));
                    b += __popcll(L.acc[w2][lane] & rm);
                }
                if (wave_sum_dpp(b) <= k) lo = mid;
                else hi = mid;
            }
            const int js = uni(lo);
            {
                int b = 0;
                for (int w2 = 0; w2 < g.G; ++w2) {
                    const int rr = js - (w2 / g.WC) * NS;
                    const uint64_t rm = rr <= 0 ? 0ull : (rr >= 64 ? ~0ull : ((1ull << rr) - 1ull));
                    b += __popcll(L.acc[w2][lane] & rm);
                }
                k -= wave_sum_dpp(b);
            }
            // location within row js: column-waves in order, lanes ascending
            const int pj = js / NS, sj = js - pj * NS;
            int jl = -1;
            for (int c2 = 0; c2 < g.WC; ++c2) {
                const uint64_t M = __ballot((L.acc[pj * g.WC + c2][lane] >> sj) & 1ull);
                const int pc = __popcll(M);
                if (jl < 0) {
                    if (k < pc) jl = c2 * 64 + kth_lane(M, k, lane);
                    else k -= pc;
                }
            }
            // the search and the ballots count the same bits, so jl was found;
            // kept inside [0, n) so that no read can leave the operands
            jl = uni(jl < 0 ? 0 : (jl >= n ? n - 1 : jl));
            const int owner = pj * g.WC + (jl >> 6);
            if (g.w == owner) {
                const int jll = jl & 63;
                int32_t d1 = 0, d2 = 0;
                pick_diffs<NS, int32_t>(S, uni(sj), jll, d1, d2);
                const uint32_t xj = (uint32_t)((rl64(S.xm, jll) >> sj) & 1ull);
                if (lane == 0) {
                    L.pick[0] = d1;
                    L.pick[1] = d2;
                    L.pick[2] = (int32_t)xj;
                }
            }
            __syncthreads();   // B3
            const int32_t d1 = uni(L.pick[0]), d2 = uni(L.pick[1]);
            const uint32_t xj = (uint32_t)uni(L.pick[2]);
            g_flip<NS, PV>(Dp, S, g, js, jl, d1, d2, xj, L);
            S.moves++;
            g_archive<NS>(Dp, S, r, t, g, H.key0, H.key1);
            moved = true;
            if (r < H.trace_R && g.w == 0 && lane == 0) rw(cold(Dp)->trace)[(size_t)r * H.steps + (t - 1u)] = js * n + jl;
        }
    }
    S.Eoff = moved ? 0 : ((H.escape == 0) ? S.Eoff + H.beta : S.Eoff);
    if (!moved) {
        if (r < H.trace_R && g.w == 0 && lane == 0) rw(cold(Dp)->trace)[(size_t)r * H.steps + (t - 1u)] = -1;
        if (H.escape != 0 && S.asize > 0) {
            const U4 o = philox10(0u, t, (uint32_t)r, kTagArc, H.key0, H.key1);
            const int pm = (int)scale32((uint32_t)uni((int)o.y), (uint32_t)S.asize);
            g_restart<NS, PV>(Dp, S, r, pm, g, L);
        }
    }
    return moved;
}

// Least combined difference over the whole replica (every wave, live lanes,
// all slots), the same in every wave: a step's cheap test passes exactly when
// it is within the step's reach.
template <int NS, int AM>
__device__ __forceinline__ int32_t g_least(const Replica<NS> &S, const Geo &g, GroupLds &L, int n)
{
    constexpr bool strict = AM == kAmStrict;
    int32_t mn = INT_MAX;
#pragma unroll
    for (int s = 0; s < NS; ++s) mn = min(mn, strict ? max(S.e1[s], S.e2[s]) : min(S.e1[s], S.e2[s]));
    mn = wave_min_dpp(g.u < n ? mn : INT_MAX);
    if (g.lane == 0) L.part[g.w][3] = mn;
    __syncthreads();
    int32_t least = INT_MAX;
    for (int w2 = 0; w2 < g.G; ++w2) least = min(least, (int32_t)L.part[w2][3]);
    __syncthreads();   // part[] is free again
    return uni(least);
}

// Final state: fields, solution block, statistics (random blocks summed over
// the waves).
template <int NS>
__device__ __forceinline__ void g_export(Desc *Dp, const Replica<NS> &S, int r, const Geo &g, GroupLds &L)
{
    Desc &D = *cold(Dp);
    const int n = opaque(D.n);
    const int m = D.m;
    const int u = g.u;
    rw(D.x)[(size_t)r * D.xrw + (size_t)g.w * 64 + g.lane] = S.xm;
    if (u < n) {
        MDA_GLOBAL int64_t *h1 = rw(D.h) + (size_t)r * 2 * m;
        MDA_GLOBAL int64_t *h2 = h1 + m;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int i = g.i0 + s;
            if (i < n) {
                const int a = i * n + u;
                const bool on = (S.xm >> s) & 1ull;
                const int32_t g1 = on ? -S.e1[s] : S.e1[s];
                const int32_t g2 = on ? -S.e2[s] : S.e2[s];
                h1[a] = (int64_t)(g1 - ro(D.diag1)[i * D.ldk + u]);
                h2[a] = (int64_t)(g2 - ro(D.diag2)[i * D.ldk + u]);
            }
        }
    }
    if (g.lane == 0) L.part[g.w][2] = S.rngb;
    __syncthreads();
    if (g.w == 0 && g.lane == 0) {
        int64_t rng = 0;
        for (int w2 = 0; w2 < g.G; ++w2) rng += L.part[w2][2];
        MDA_GLOBAL int64_t *st = rw(D.st) + (size_t)r * kStWords;
        st[kStE1] = S.E1;
        st[kStE2] = S.E2;
        st[kStEoff] = S.Eoff;
        st[kStMoves] = S.moves;
        st[kStScanned] = S.scanned;
        st[kStRng] = rng;
        st[kStArch] = S.asize;
        st[kStDetailed] = S.detailed;
    }
    __syncthreads();
}

template <int NS, int PV, int AM>
__device__ __forceinline__ void g_run(Desc *Dp, int r, const Geo &g, GroupLds &L)
{
    Replica<NS> S;
    g_init<NS, PV>(Dp, S, r, g, L);
    const Hot H = load_hot(Dp);
    // With the offset escape a step whose cheap test fails does nothing but
    // raise the offset: such steps are decided against the replica's least
    // combined difference (every wave holds the same value and takes the same
    // decision), with no barrier, one by one while the temperature changes and
    // a whole stretch at once (quiet_steps) after that.
    const bool skip = H.escape == 0;
    int32_t least = skip ? g_least<NS, AM>(S, g, L, H.n) : 0;
    uint32_t thr = H.thrmax[0];
    uint32_t t = 1;
    while (t <= H.steps) {
        uint32_t quiet = 0;
        if (skip) {
            if (t >= H.ntab) quiet = quiet_steps((int64_t)least, S.Eoff, (int64_t)thr, H.beta, H.steps - t + 1u);
            else quiet = (int64_t)least > (int64_t)step_reach<int32_t>(S.Eoff, (int64_t)thr) ? 1u : 0u;
        }
        if (quiet > 0u) {
            S.Eoff += (int64_t)quiet * H.beta;
            if (r < H.trace_R && g.w == 0) {
                MDA_GLOBAL int32_t *tr = rw(cold(Dp)->trace) + (size_t)r * H.steps + (t - 1u);
                for (uint32_t i = (uint32_t)g.lane; i < quiet; i += 64u) tr[i] = -1;
            }
        } else {
            quiet = 1u;
            if (g_step<NS, PV, AM>(Dp, H, S, r, t, g, L, thr) && skip) least = g_least<NS, AM>(S, g, L, H.n);
        }
        t += quiet;
        // threshold of step t: table entry min(t, ntab) - 1
        if (t <= H.steps) thr = H.thrmax[(t < H.ntab ? t : H.ntab) - 1u];
    }
    g_export<NS>(Dp, S, r, g, L);
}

// One replica per workgroup of WR x WC waves; workgroup b runs work items
// b, b + B, b + 2B, ... (B workgroups in the grid).
// Workgroups of up to 8 waves for small tiles; up to 4 (so that a wave may use
// the whole register file) from 24 slots up.
template <int NS>
constexpr int group_max_waves()
{
    return NS <= 16 ? kMaxGroupWaves : 4;
}

// OCC = 2 builds (from 24 slots up) keep cold-path state in scratch so that two
// workgroups share a CU; the host takes them when a launch has more replicas
// than one workgroup per CU can hold at once (n = 100, 2048 replicas: about a
// quarter faster; a single round of replicas is faster with OCC = 1).
template <int NS, int OCC>
__global__ void __launch_bounds__(64 * group_max_waves<NS>()) __attribute__((amdgpu_waves_per_eu(OCC))) k_group(const RunDesc *runs, const WorkItem *work, int nwork,
                                               const int32_t *lnt_, int WR, int WC)
{
    __shared__ GroupLds L;
    for (int k = (int)threadIdx.x; k < 4096; k += (int)blockDim.x) L.lnt[k] = ((const MDA_GLOBAL int32_t *)lnt_)[k];
    Geo g;
    g.lane = __lane_id();
    g.w = uni((int)(threadIdx.x >> 6));
    g.WC = WC;
    g.G = WR * WC;
    g.p = g.w / WC;
    g.c = g.w - g.p * WC;
    g.i0 = g.p * NS;
    g.u = g.c * 64 + g.lane;
    __syncthreads();
    for (int item = (int)blockIdx.x; item < nwork; item += (int)gridDim.x) {
        const WorkItem w = {ro(work)[item].run, ro(work)[item].replica};
        Desc *Dp = ro(runs) + uni(w.run);
        const int r = uni(w.replica);
        switch (path_variant(Dp) * 2 + (Dp->accept != 0 ? kAmLenient : kAmStrict)) {
#define X(PV, AM)                             \
    case PV * 2 + AM:                         \
        g_run<NS, PV, AM>(Dp, r, g, L); \
        break;
            X(kPvDense, kAmStrict) X(kPvDense, kAmLenient) X(kPvKronSym, kAmStrict) X(kPvKronSym, kAmLenient)
            X(kPvKronGen, kAmStrict) X(kPvKronGen, kAmLenient)
#undef X
        default: break;
        }
        __syncthreads();
    }
}

}  // namespace mda
