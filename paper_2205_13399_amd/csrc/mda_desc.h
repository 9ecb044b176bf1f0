// mda_desc.h -- device-visible description of one annealing run and the work
// items of a (batched) persistent launch.  Shared by the kernels and the host
// library of the MI355X multi-objective Digital Annealer.
#pragma once

#include <stdint.h>

namespace mda {

// Counter word 3 of every Philox call names what the draw is for.
enum : uint32_t { kTagAcc = 0, kTagSel = 1, kTagInit = 2, kTagArc = 3 };

enum : int32_t { kPathDense = 1, kPathKron = 2 };
enum : int32_t { kKronSym = 0, kKronGen = 1 };

// Per-replica scalar statistics/state block (int64 words).
enum : int32_t {
    kStE1 = 0, kStE2 = 1, kStEoff = 2, kStMoves = 3, kStScanned = 4, kStRng = 5,
    kStArch = 6, kStDetailed = 7, kStNd = 8, kStWords = 16
};

// Step variant of a run: update path (0 dense rows, 1 Kronecker with one
// product per objective, 2 with two) times 2 plus the acceptance rule (0
// strict, 1 lenient).  The one-wave persistent kernels are built per variant
// and a launch holds the items of one variant only.
constexpr int kStepVariants = 6;

// One non-dominated archive entry gathered for the host merge.
struct FrontEntry {
    int64_t e1, e2;
    int32_t replica, slot;
};

// Largest n of the one-replica-per-wave kernels (lane = location).
constexpr int kMaxWaveN = 64;

// Row stride of every per-lane operand on the device: rows of n entries are
// padded with zeros to kLD, so lanes beyond n always read zero.
constexpr int kLD = 64;

struct RunDesc {
    // problem
    int32_t n, m;              // facilities, bits
    int32_t s;                 // archive capacity
    int32_t path;              // kPathDense | kPathKron
    int32_t kform;             // kKronSym | kKronGen
    int32_t accept, archive, escape;
    int32_t two_alpha1, two_alpha2;
    int32_t R;                 // replicas
    int32_t trace_R;           // replicas [0, trace_R) record their flips
    uint32_t key0, key1;       // Philox key
    uint32_t steps;            // annealing steps
    uint32_t ntab;             // temperature-table entries; T_t = T[min(t, ntab) - 1]
    int32_t f64;               // 1: int64 energy differences (fields beyond the int32 bounds)
    int64_t beta;
    int64_t q1, q2;
    // schedule tables
    const int64_t *T;          // fixed-point temperature, 8 fractional bits
    const uint32_t *thrmax;    // (T * LNT[0]) >> 24, saturated at 2^32 - 2
    const int64_t *thrmax64;   // (T * LNT[0]) >> 24 (int64 runs)
    // Kronecker operands, n rows of kLD int32 (zero padded), row i' (or u'):
    //   P_k[(i,u)][(i',u')] = KA_k[i'][i] * DA[u'][u] (+ KB_k[i'][i] * DB[u'][u])
    //                         + 2 alpha_k [(i == i') != (u == u')]
    const int32_t *KA1, *KA2, *KB1, *KB2, *DA, *DB;
    // dense operands: symmetric P_k, m rows of n * pld int32, entry (j, v) of
    // row a at a * n * pld + j * pld + v (pld = n: no padding)
    const int32_t *P1, *P2;
    const int32_t *diag1, *diag2;   // d_k[(i,u)] = P_k[a][a] at i * kLD + u
    // outputs and archives
    uint64_t *x;               // [R][64] column masks: bit i of word u is x_{i,u}
    int64_t *h;                // [R][2][m] local fields (canonical order)
    int64_t *st;               // [R][kStWords]
    int64_t *archE;            // [R][s][2]
    uint64_t *archX;           // [R][s][n]
    uint8_t *nd;               // [R][s] 1 = not dominated within its archive
    int32_t *trace;            // [trace_R][steps]
    // plain-form state (one launch per step)
    int32_t *pe;               // [R][2][NS][64]
    int32_t ns_plain;          // NS of the plain state layout
    int32_t pad1;
    // layout of the replica over waves: wr x wc waves (1 x 1 = one wave per
    // replica, lane = location, slot = facility, n <= 64); in a workgroup run
    // wave (p, c) holds facilities [p gns, p gns + gns) and locations
    // [64 c, 64 c + 64), and solutions are stored as wr * wc * 64 words,
    // word (p wc + c) 64 + (u mod 64), bit i - p gns
    int32_t wr, wc, gns;
    int32_t ldk;               // row stride of KA, KB, DA, DB and the diagonals
    int32_t pld;               // dense P_k: entry (i, u) of row j at j * n * pld + i * pld + u
    int32_t xw;                // words per archived solution (n, or wr * wc * 64)
    int32_t xrw;               // words per replica in x (64, or wr * wc * 64)
    int32_t pad2;
};

inline __host__ __device__ int run_step_variant(int32_t path, int32_t kform, int32_t accept)
{
    return (path == kPathDense ? 0 : (kform == kKronGen ? 2 : 1)) * 2 + (accept != 0 ? 1 : 0);
}

struct WorkItem {
    int32_t run;      // index into the RunDesc array
    int32_t replica;
};

}  // namespace mda
