/*
 * mda_oracle.h -- CPU oracle of the multi-objective Digital Annealer (MDA) on the
 * bi-objective quadratic assignment problem (Ayodele, Allmendinger, Lopez-Ibanez,
 * Parizy, "Multi-objective QUBO Solver: Bi-objective Quadratic Assignment Problem",
 * GECCO 2022, arXiv:2205.13399).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation written from the paper's definitions.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the product
 * library shares no code, header, table or helper with it.
 *
 * Everything is integer arithmetic in int64 except the two host tables (the
 * geometric temperature schedule and the quantised -ln(u) table), which are
 * computed in IEEE double exactly as the readings below state.
 *
 * Readings of the paper taken here (each is repeated where it is used):
 *  R1 bit a = i*n + u means facility i sits at location u (row = facility,
 *     column = location), which reproduces the worked example of Section 2.2.
 *  R2 the energy difference of Eq. (cale) uses x_j inside the sum:
 *     dE_a = (1 - 2 x_a) (P_aa + sum_{b != a} P_ab x_b), P = Q + Q^T with the
 *     diagonal kept equal to Q_aa; this is the only reading that satisfies
 *     E(x with bit a flipped) = E(x) + dE_a.
 *  R3 acceptance: one uniform u per (bit, step); u is quantised to the
 *     midpoints (k + 1/2)/4096 and the test exp(-S/delta) >= u is done as
 *     S <= (T * LNT[k]) >> 24 with T = floor(delta * 2^8) and
 *     LNT[k] = round(-ln((k + 1/2)/4096) * 2^16).
 *  R4 strict rule (Eq. pacceptms): S = max(0, D1) + max(0, D2); lenient rule
 *     (Eq. pacceptml): S = min(max(0, D1), max(0, D2)); D_k = dE_k - E_offset.
 *  R5 the dynamic offset of Algorithm 1 (E_offset <- 0 on a move, += beta when
 *     nothing is accepted) is applied inside the MDA by default; the MDA's own
 *     escape (restart from a random archive member, Algorithm 3) is a switch.
 *  R6 the flip made among the accepted ones (Algorithm 3) is drawn uniformly
 *     over the accepted bits counted in ascending bit index,
 *     k = floor(w * c / 2^32) for a 32-bit random word w.
 *  R7 archive: fixed capacity s; the first dominated member is the lowest
 *     slot; equivalent points are appended while not full; dominance compares
 *     energies only.
 */
#ifndef MDA_ORACLE_H
#define MDA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- Section 2: QAP and its QUBO ---------------- */

/* Eq. (nqap): f(sigma) = sum_i sum_j H[i][j] * D[sigma_i][sigma_j]; perm is 0-based. */
int64_t orc_qap_cost(int32_t n, const int32_t *H, const int32_t *D, const int32_t *perm);

/* Eq. (cqap) evaluated directly on a 0/1 matrix x (x[i*n+u]). */
int64_t orc_cost_direct(int32_t n, const int32_t *H, const int32_t *D, const uint8_t *x);

/* Eq. (gqap) evaluated directly. */
int64_t orc_constraint_direct(int32_t n, const uint8_t *x);

/* Cost QUBO C of Eq. (cqap) in the upper-triangular form of the worked example
 * (Section 2.2): C[a][b] = H[i][j] D[u][v] + H[j][i] D[v][u] for a < b,
 * C[a][a] = H[i][i] D[u][u], zero below the diagonal; constant p_c = 0.
 * C has m*m entries, m = n*n. */
void orc_cost_qubo(int32_t n, const int32_t *H, const int32_t *D, int64_t *C);

/* Constraint QUBO G of Eq. (gqap), upper triangular: G[a][a] = -2,
 * G[a][b] = 2 for a < b when the two bits share a row or a column (not both),
 * constant p_g = 2n. */
void orc_constraint_qubo(int32_t n, int64_t *G, int64_t *pg);

/* Eq. (qubo): E(x) = x^T Q x + q for any m x m Q (not only triangular). */
int64_t orc_qubo_energy(int32_t m, const int64_t *Q, int64_t q, const uint8_t *x);

/* Eq. (cale) under reading R2: all m energy differences of Q at x. */
void orc_delta_energy(int32_t m, const int64_t *Q, const uint8_t *x, int64_t *dE);

/* Penalty weights.  2max: alpha = 2 * max_{a<=b} |C[a][b]| (the weight used by
 * the benchmark configurations).  Eq. (vermap) applied to the symmetric form of C
 * (each bit's full interaction row); returns w; Eq. (wvermaa) alpha = ceil(w/2). */
int64_t orc_penalty_2max(int32_t m, const int64_t *C);
int64_t orc_penalty_vl_w(int32_t m, const int64_t *C);

/* ---------------- random numbers and tables ---------------- */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Reading R3: LNT[k] = round(-ln((k + 0.5) / 4096) * 65536), k = 0..4095. */
void orc_lnt(int32_t *lnt);

/* Temperature T_t (fixed point, 8 fractional bits) for t = 1..steps: the
 * cooling test of Algorithm 3 at the top of each iteration, delta <- delta(1-xi)
 * while delta > delta_f, then T_t = floor(delta * 256).  T[t-1] holds T_t. */
void orc_temperature(double delta0, double deltaf, double xi, int64_t steps, int64_t *T);

/* Acceptance of one bit (readings R3, R4): dE_k are the two energy differences,
 * Eoff the current offset, T the fixed-point temperature and lnt_k = LNT[k] for
 * the bit's uniform index k; mode is ORC_STRICT or ORC_LENIENT.  Returns 0/1. */
int orc_accept(int64_t dE1, int64_t dE2, int64_t Eoff, int64_t T, int32_t lnt_k, int32_t mode);

/* ---------------- archive updates (Algorithms 4 and 5) ---------------- */

typedef struct {
    int32_t size, cap, m;
    int64_t *e1, *e2;   /* cap entries */
    uint8_t *x;         /* cap * m bits, one byte per bit */
} orc_archive;

/* p dominates q (Section 3.3): p.E <= q.E in both objectives and not equal in both. */
int orc_dominates(int64_t p1, int64_t p2, int64_t q1, int64_t q2);

/* Explorative update: returns the slot written, or -1 if the archive is unchanged. */
int32_t orc_archive_explore(orc_archive *A, int64_t e1, int64_t e2, const uint8_t *x);

/* Exploitative update; w is the 32-bit random word used to pick from B. */
int32_t orc_archive_exploit(orc_archive *A, int64_t e1, int64_t e2, const uint8_t *x, uint32_t w);

/* ---------------- the whole MDA (Algorithm 3) ---------------- */

enum { ORC_STRICT = 0, ORC_LENIENT = 1 };
enum { ORC_EXPLORE = 0, ORC_EXPLOIT = 1 };
enum { ORC_ESC_OFFSET = 0, ORC_ESC_ARCHIVE = 1 };
enum { ORC_PEN_2MAX = 0, ORC_PEN_VL = 1 };

/* Random-number tags: counter word 3 of every Philox call. */
enum { ORC_TAG_ACC = 0, ORC_TAG_SEL = 1, ORC_TAG_INIT = 2, ORC_TAG_ARC = 3 };

typedef struct {
    int32_t n, m;
    int64_t alpha1, alpha2, q1, q2;
    int64_t maxabs_c;       /* max(max|C1|, max|C2|), used by the default schedule */
    int64_t *P1, *P2;       /* m*m: P[a][b] = P[b][a] = Y[a][b] for a < b, P[a][a] = Y[a][a],
                               where Y_k = C_k + alpha_k G is Eq. (wqubom) */
    int32_t overflow;       /* 1 when some row bound exceeds 2^31 - 1 */
} orc_qubo;

/* Builds Y_k = C_k + alpha_k G (Eq. wqubom) from flows F1, F2 and distances D.
 * Returns 0, or -1 on allocation failure. */
int orc_build(int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D,
              int32_t penalty, orc_qubo *q);
void orc_free(orc_qubo *q);

typedef struct {
    int64_t steps;
    double delta0, deltaf, xi;
    int64_t beta;
    int32_t accept, archive, escape, archive_size;
    uint64_t seed;
    /* The schedule as input data: when not NULL, T_t = temp_table[t-1] for
     * t = 1..steps (fixed point, 8 fractional bits) replaces the geometric
     * cooling of delta0, deltaf and xi (Table param). */
    const int64_t *temp_table;
} orc_params;

typedef struct {
    uint8_t *x;          /* m */
    int64_t *h1, *h2;    /* m local fields h_k[a] = sum_{b != a} P_k[a][b] x_b */
    int64_t *state;      /* 4: E1, E2, E_offset, number of moves */
    int32_t *arch_size;  /* 1 */
    int64_t *arch_e;     /* 2 * archive_size: (E1, E2) per slot */
    uint8_t *arch_x;     /* archive_size * m */
    int32_t *trace;      /* steps entries (flipped bit or -1), may be NULL */
} orc_replica_out;

/* Runs replica r of one MDA run. Returns 0, or a negative value on bad input. */
int orc_mda_replica(const orc_qubo *q, const orc_params *p, int32_t r, orc_replica_out *out);

/* ---------------- K objectives on a generic QUBO ---------------- */
/*
 * The extension to more than two objectives named as future work in the
 * paper's Conclusion, on any QUBO (Eq. qubo), not only the bQAP's.  K
 * objectives x^T Q_k x + q_k (k = 1..K, K >= 1) over m bits, every other step
 * of Algorithm 3 as above, with readings:
 *  G1 acceptance with K objectives: strict S = sum_k max(0, D_k) (the product
 *     of the K probabilities of Eq. pacceptms), lenient S = min_k max(0, D_k)
 *     (the largest of them, Eq. pacceptml), D_k = dE_k - E_offset; accept iff
 *     S <= (T * LNT[idx]) >> 24 as in R3;
 *  G2 dominance: p dominates q when p_k <= q_k for every k and p != q
 *     (Section 3.3 with K objectives);
 *  G3 random numbers by bit index a, eight consecutive bits per block:
 *     start bit a = bit (a & 31) of word ((a >> 5) & 3) of the block
 *     (a >> 7, 0, r, INIT); acceptance index of bit a = bits 4..15 of the
 *     16-bit half (a & 1) of word (a & 7) >> 1 of the block (a >> 3, t, r, ACC);
 *     the choice, exploit and restart words as in R6 and Algorithm 5.
 */
typedef struct {
    int32_t m, K;
    int64_t *P;             /* K*m*m: P_k[a][b] = Q_k[a][b] + Q_k[b][a] (a != b), P_k[a][a] = Q_k[a][a] */
    int64_t *q;             /* K constants */
    int64_t maxabs_c;       /* max over k and a <= b of |C_k[a][b]|, C the upper-triangular form */
    int32_t overflow;       /* 1 when some row bound |P_aa| + sum_b |P_ab| exceeds 2^31 - 1 */
} orc_gqubo;

/* Q: K*m*m int32 row-major (Q_k[a][b] at (k*m + a)*m + b); q: K constants or
 * NULL for zeros.  Returns 0, or -1 on allocation failure. */
int orc_gbuild(int32_t m, int32_t K, const int32_t *Q, const int64_t *q, orc_gqubo *g);
void orc_gfree(orc_gqubo *g);

/* Reading G2. */
int orc_gdominates(int32_t K, const int64_t *p, const int64_t *q);

/* Reading G1 on the K differences dE. */
int orc_gaccept(int32_t K, const int64_t *dE, int64_t Eoff, int64_t T, int32_t lnt_k, int32_t mode);

typedef struct {
    int32_t size, cap, m, K;
    int64_t *e;         /* cap*K energies */
    uint8_t *x;         /* cap*m bits */
} orc_garchive;

/* Algorithms 4 and 5 with K-way dominance; same returns as the K = 2 forms. */
int32_t orc_garchive_explore(orc_garchive *A, const int64_t *e, const uint8_t *x);
int32_t orc_garchive_exploit(orc_garchive *A, const int64_t *e, const uint8_t *x, uint32_t w);

typedef struct {
    uint8_t *x;          /* m */
    int64_t *h;          /* K*m local fields h_k[a] = sum_{b != a} P_k[a][b] x_b */
    int64_t *state;      /* K + 2: E_1..E_K, E_offset, number of moves */
    int32_t *arch_size;  /* 1 */
    int64_t *arch_e;     /* archive_size * K */
    uint8_t *arch_x;     /* archive_size * m */
    int32_t *trace;      /* steps entries (flipped bit or -1), may be NULL */
} orc_greplica_out;

/* Replica r of the K-objective MDA (Algorithm 3, readings G1-G3).  Returns 0,
 * or a negative value on bad input. */
int orc_gmda_replica(const orc_gqubo *g, const orc_params *p, int32_t r, orc_greplica_out *out);

#ifdef __cplusplus
}
#endif
#endif
