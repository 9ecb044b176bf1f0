/*
 * mda_oracle.c -- CPU oracle of the multi-objective Digital Annealer on the
 * bi-objective QAP (arXiv:2205.13399).  TEST INFRASTRUCTURE ONLY: see the header
 * for who may use it and for the readings R1..R7 of the paper taken here.
 *
 * Plain scalar loops in the order the paper states them; int64 everywhere on the
 * integer side; no blocking, no fusion, no incremental tricks beyond the local
 * fields h that the paper's own energy-difference formula (Eq. cale) maintains.
 */
#include "mda_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define INT32_LIMIT 2147483647LL

/* ---------------- Section 2: QAP and its QUBO ---------------- */

int64_t orc_qap_cost(int32_t n, const int32_t *H, const int32_t *D, const int32_t *perm)
{
    /* Eq. (nqap): sum over facility pairs of flow times the distance between
     * their assigned locations. */
    int64_t f = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j)
            f += (int64_t)H[i * n + j] * D[perm[i] * n + perm[j]];
    return f;
}

int64_t orc_cost_direct(int32_t n, const int32_t *H, const int32_t *D, const uint8_t *x)
{
    /* Eq. (cqap): quadruple sum over (i, j, u, v). */
    int64_t c = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j)
            for (int32_t u = 0; u < n; ++u)
                for (int32_t v = 0; v < n; ++v)
                    c += (int64_t)H[i * n + j] * D[u * n + v] * x[i * n + u] * x[j * n + v];
    return c;
}

int64_t orc_constraint_direct(int32_t n, const uint8_t *x)
{
    /* Eq. (gqap): squared violation of every row sum and every column sum. */
    int64_t g = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t s = 0;
        for (int32_t u = 0; u < n; ++u) s += x[i * n + u];
        g += (1 - s) * (1 - s);
    }
    for (int32_t u = 0; u < n; ++u) {
        int64_t s = 0;
        for (int32_t i = 0; i < n; ++i) s += x[i * n + u];
        g += (1 - s) * (1 - s);
    }
    return g;
}

/* One entry of the upper-triangular cost QUBO (Section 2.2, reading R1). */
static int64_t cost_entry(int32_t n, const int32_t *H, const int32_t *D, int32_t a, int32_t b)
{
    int32_t i = a / n, u = a % n, j = b / n, v = b % n;
    if (a == b) return (int64_t)H[i * n + i] * D[u * n + u];
    if (a > b) return 0;
    return (int64_t)H[i * n + j] * D[u * n + v] + (int64_t)H[j * n + i] * D[v * n + u];
}

/* One entry of the upper-triangular constraint QUBO (Section 2.2). */
static int64_t constraint_entry(int32_t n, int32_t a, int32_t b)
{
    int32_t i = a / n, u = a % n, j = b / n, v = b % n;
    if (a == b) return -2;
    if (a > b) return 0;
    return ((i == j) != (u == v)) ? 2 : 0;
}

void orc_cost_qubo(int32_t n, const int32_t *H, const int32_t *D, int64_t *C)
{
    int32_t m = n * n;
    for (int32_t a = 0; a < m; ++a)
        for (int32_t b = 0; b < m; ++b)
            C[(int64_t)a * m + b] = cost_entry(n, H, D, a, b);
}

void orc_constraint_qubo(int32_t n, int64_t *G, int64_t *pg)
{
    int32_t m = n * n;
    for (int32_t a = 0; a < m; ++a)
        for (int32_t b = 0; b < m; ++b)
            G[(int64_t)a * m + b] = constraint_entry(n, a, b);
    *pg = 2 * (int64_t)n;
}

int64_t orc_qubo_energy(int32_t m, const int64_t *Q, int64_t q, const uint8_t *x)
{
    /* Eq. (qubo). */
    int64_t e = q;
    for (int32_t a = 0; a < m; ++a)
        for (int32_t b = 0; b < m; ++b)
            e += Q[(int64_t)a * m + b] * x[a] * x[b];
    return e;
}

void orc_delta_energy(int32_t m, const int64_t *Q, const uint8_t *x, int64_t *dE)
{
    /* Eq. (cale), reading R2: P = Q + Q^T with P_aa = Q_aa. */
    for (int32_t a = 0; a < m; ++a) {
        int64_t sum = Q[(int64_t)a * m + a];
        for (int32_t b = 0; b < m; ++b) {
            if (b == a) continue;
            int64_t pab = Q[(int64_t)a * m + b] + Q[(int64_t)b * m + a];
            sum += pab * x[b];
        }
        dE[a] = (1 - 2 * (int64_t)x[a]) * sum;
    }
}

int64_t orc_penalty_2max(int32_t m, const int64_t *C)
{
    int64_t mx = 0;
    for (int64_t k = 0; k < (int64_t)m * m; ++k) {
        int64_t v = C[k] < 0 ? -C[k] : C[k];
        if (v > mx) mx = v;
    }
    return 2 * mx;
}

int64_t orc_penalty_vl_w(int32_t m, const int64_t *C)
{
    /* Eq. (vermap) on the symmetric form S = C + C^T (diagonal C_aa), i.e. the
     * whole interaction of bit a: the largest change of C caused by turning one
     * bit off or on. */
    int64_t w = INT64_MIN;
    for (int32_t a = 0; a < m; ++a) {
        int64_t caa = C[(int64_t)a * m + a];
        int64_t neg = -caa, pos = caa;
        for (int32_t b = 0; b < m; ++b) {
            if (b == a) continue;
            int64_t sab = C[(int64_t)a * m + b] + C[(int64_t)b * m + a];
            if (sab < 0) neg -= sab;
            if (sab > 0) pos += sab;
        }
        if (neg > w) w = neg;
        if (pos > w) w = pos;
    }
    return w;
}

/* ---------------- random numbers and tables ---------------- */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    /* Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64
     * multiplications with the round constants below; the key is advanced by
     * the Weyl constants between rounds. */
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_lnt(int32_t *lnt)
{
    for (int k = 0; k < 4096; ++k)
        lnt[k] = (int32_t)llround(-log(((double)k + 0.5) / 4096.0) * 65536.0);
}

void orc_temperature(double delta0, double deltaf, double xi, int64_t steps, int64_t *T)
{
    double delta = delta0;
    for (int64_t t = 1; t <= steps; ++t) {
        if (delta > deltaf) delta = delta * (1.0 - xi);
        T[t - 1] = (int64_t)floor(delta * 256.0);
    }
}

/* ---------------- acceptance (Eqs. paccepts, pacceptms, pacceptml) ---------------- */

int orc_accept(int64_t dE1, int64_t dE2, int64_t Eoff, int64_t T, int32_t lnt_k, int32_t mode)
{
    /* Per objective Pr^k = exp(min{0, -(dE_k - E_offset)/delta}) = exp(-max(0, D_k)/delta).
     * Strict: the product, exp(-(max(0,D1) + max(0,D2))/delta).  Lenient: the
     * larger one, exp(-min(max(0,D1), max(0,D2))/delta).  Accept when the
     * probability is at least u, i.e. S <= delta * (-ln u), in fixed point. */
    int64_t d1 = dE1 - Eoff, d2 = dE2 - Eoff;
    int64_t p1 = d1 > 0 ? d1 : 0, p2 = d2 > 0 ? d2 : 0;
    int64_t S = (mode == ORC_LENIENT) ? (p1 < p2 ? p1 : p2) : (p1 + p2);
    int64_t thr = (T * (int64_t)lnt_k) >> 24;
    return S <= thr;
}

/* ---------------- archive (Algorithms 4 and 5) ---------------- */

int orc_dominates(int64_t p1, int64_t p2, int64_t q1, int64_t q2)
{
    int equivalent = (p1 == q1) && (p2 == q2);
    return (p1 <= q1) && (p2 <= q2) && !equivalent;
}

static void archive_put(orc_archive *A, int32_t slot, int64_t e1, int64_t e2, const uint8_t *x)
{
    A->e1[slot] = e1;
    A->e2[slot] = e2;
    memcpy(A->x + (int64_t)slot * A->m, x, (size_t)A->m);
}

static uint32_t mulhi32(uint32_t w, uint32_t c)
{
    return (uint32_t)(((uint64_t)w * c) >> 32);
}

int32_t orc_archive_explore(orc_archive *A, int64_t e1, int64_t e2, const uint8_t *x)
{
    /* Replace the first member that x dominates; otherwise append if not full. */
    for (int32_t i = 0; i < A->size; ++i) {
        if (orc_dominates(e1, e2, A->e1[i], A->e2[i])) {
            archive_put(A, i, e1, e2, x);
            return i;
        }
    }
    if (A->size < A->cap) {
        archive_put(A, A->size, e1, e2, x);
        return A->size++;
    }
    return -1;
}

int32_t orc_archive_exploit(orc_archive *A, int64_t e1, int64_t e2, const uint8_t *x, uint32_t w)
{
    /* Only when no member dominates x: replace a random member of
     * B = {y : x dominates y}, otherwise append if not full. */
    for (int32_t i = 0; i < A->size; ++i)
        if (orc_dominates(A->e1[i], A->e2[i], e1, e2)) return -1;
    int32_t nb = 0;
    for (int32_t i = 0; i < A->size; ++i)
        if (orc_dominates(e1, e2, A->e1[i], A->e2[i])) ++nb;
    if (nb > 0) {
        int32_t pick = (int32_t)mulhi32(w, (uint32_t)nb);
        for (int32_t i = 0; i < A->size; ++i) {
            if (orc_dominates(e1, e2, A->e1[i], A->e2[i])) {
                if (pick == 0) {
                    archive_put(A, i, e1, e2, x);
                    return i;
                }
                --pick;
            }
        }
    }
    if (A->size < A->cap) {
        archive_put(A, A->size, e1, e2, x);
        return A->size++;
    }
    return -1;
}

/* ---------------- QUBO of the bi-objective QAP (Eq. wqubom) ---------------- */

int orc_build(int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D,
              int32_t penalty, orc_qubo *q)
{
    int32_t m = n * n;
    int64_t mm = (int64_t)m * m;
    memset(q, 0, sizeof(*q));
    q->n = n;
    q->m = m;
    int64_t *C = (int64_t *)malloc((size_t)mm * sizeof(int64_t));
    q->P1 = (int64_t *)malloc((size_t)mm * sizeof(int64_t));
    q->P2 = (int64_t *)malloc((size_t)mm * sizeof(int64_t));
    if (!C || !q->P1 || !q->P2) {
        free(C);
        orc_free(q);
        return -1;
    }
    int64_t pg = 2 * (int64_t)n;
    for (int k = 0; k < 2; ++k) {
        const int32_t *F = k == 0 ? F1 : F2;
        int64_t *P = k == 0 ? q->P1 : q->P2;
        orc_cost_qubo(n, F, D, C);
        int64_t maxabs = orc_penalty_2max(m, C) / 2;
        if (maxabs > q->maxabs_c) q->maxabs_c = maxabs;
        int64_t alpha;
        if (penalty == ORC_PEN_VL) {
            int64_t w = orc_penalty_vl_w(m, C);
            alpha = (w + 1) / 2;   /* Eq. (wvermaa), rounded up to an integer */
        } else {
            alpha = 2 * maxabs;
        }
        /* Y = C + alpha G (upper triangular); P holds Y_ab in both (a,b) and
         * (b,a) off the diagonal and Y_aa on it. */
        for (int32_t a = 0; a < m; ++a) {
            for (int32_t b = a; b < m; ++b) {
                int64_t y = C[(int64_t)a * m + b] + alpha * constraint_entry(n, a, b);
                P[(int64_t)a * m + b] = y;
                P[(int64_t)b * m + a] = y;
            }
        }
        if (k == 0) { q->alpha1 = alpha; q->q1 = alpha * pg; }
        else        { q->alpha2 = alpha; q->q2 = alpha * pg; }
        /* Every local-field value |P_aa + sum_b P_ab x_b| must fit in int32. */
        for (int32_t a = 0; a < m; ++a) {
            int64_t s = 0;
            for (int32_t b = 0; b < m; ++b) {
                int64_t v = P[(int64_t)a * m + b];
                s += v < 0 ? -v : v;
            }
            if (s > INT32_LIMIT) q->overflow = 1;
        }
    }
    free(C);
    return 0;
}

void orc_free(orc_qubo *q)
{
    free(q->P1);
    free(q->P2);
    q->P1 = q->P2 = 0;
}

/* ---------------- the MDA, Algorithm 3 ---------------- */

static int64_t energy_of(const orc_qubo *q, const int64_t *P, int64_t qk, const uint8_t *x)
{
    /* Eq. (qubo) with Q = Y (upper triangle of P). */
    int32_t m = q->m;
    int64_t e = qk;
    for (int32_t a = 0; a < m; ++a) {
        if (!x[a]) continue;
        e += P[(int64_t)a * m + a];
        for (int32_t b = a + 1; b < m; ++b)
            if (x[b]) e += P[(int64_t)a * m + b];
    }
    return e;
}

static void fields_of(const orc_qubo *q, const int64_t *P, const uint8_t *x, int64_t *h)
{
    int32_t m = q->m;
    for (int32_t a = 0; a < m; ++a) {
        int64_t s = 0;
        for (int32_t b = 0; b < m; ++b)
            if (b != a && x[b]) s += P[(int64_t)a * m + b];
        h[a] = s;
    }
}

int orc_mda_replica(const orc_qubo *q, const orc_params *p, int32_t r, orc_replica_out *out)
{
    int32_t n = q->n, m = q->m;
    int32_t s = p->archive_size > 0 ? p->archive_size : m;
    if (p->steps < 0 || p->steps > 0xFFFFFFFFLL || r < 0) return -1;
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    int32_t lnt[4096];
    orc_lnt(lnt);

    uint8_t *x = out->x;
    int64_t *h1 = out->h1, *h2 = out->h2;
    int64_t *dE1 = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    int64_t *dE2 = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    uint8_t *acc = (uint8_t *)malloc((size_t)m);
    uint32_t *field = (uint32_t *)malloc((size_t)m * sizeof(uint32_t));
    if (!dE1 || !dE2 || !acc || !field) {
        free(dE1); free(dE2); free(acc); free(field);
        return -3;
    }

    /* Algorithm 3 starts from a random binary solution (reading: i.i.d. fair
     * bits).  Bit (i, u) is bit i%32 of word (i/32)%4 of the block (i/128, u). */
    for (int32_t a = 0; a < m; ++a) {
        int32_t i = a / n, u = a % n;
        uint32_t ctr[4] = {((uint32_t)(i >> 7) << 16) | (uint32_t)u, 0u, (uint32_t)r, ORC_TAG_INIT};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        x[a] = (uint8_t)((o[(i >> 5) & 3] >> (i & 31)) & 1u);
    }
    fields_of(q, q->P1, x, h1);
    fields_of(q, q->P2, x, h2);
    int64_t E1 = energy_of(q, q->P1, q->q1, x);
    int64_t E2 = energy_of(q, q->P2, q->q2, x);
    int64_t Eoff = 0, moves = 0;

    /* Algorithm 3: the archive starts empty, with capacity s. */
    orc_archive A;
    A.size = 0;
    A.cap = s;
    A.m = m;
    A.e1 = (int64_t *)malloc((size_t)s * sizeof(int64_t));
    A.e2 = (int64_t *)malloc((size_t)s * sizeof(int64_t));
    A.x = out->arch_x;
    if (!A.e1 || !A.e2) {
        free(dE1); free(dE2); free(acc); free(field); free(A.e1); free(A.e2);
        return -3;
    }

    double delta = p->delta0;
    for (int64_t t = 1; t <= p->steps; ++t) {
        /* Algorithm 3: geometric cooling at the top of each iteration, unless
         * the schedule is given as data. */
        int64_t T;
        if (p->temp_table) {
            T = p->temp_table[t - 1];
        } else {
            if (delta > p->deltaf) delta = delta * (1.0 - p->xi);
            T = (int64_t)floor(delta * 256.0);
        }

        /* Algorithm 3: energy differences of every neighbour, both objectives
         * (Eq. cale with Y and Z in place of Q). */
        for (int32_t a = 0; a < m; ++a) {
            int64_t sgn = 1 - 2 * (int64_t)x[a];
            dE1[a] = sgn * (q->P1[(int64_t)a * m + a] + h1[a]);
            dE2[a] = sgn * (q->P2[(int64_t)a * m + a] + h2[a]);
        }

        /* One 12-bit uniform index per bit (reading R3): the block of eight
         * facilities (i/8, u) shares one Philox call; facility i uses the
         * 16-bit half (i%8)%2 of word (i%8)/2, low 12 bits. */
        for (int32_t g = 0; g * 8 < n; ++g) {
            for (int32_t u = 0; u < n; ++u) {
                uint32_t ctr[4] = {((uint32_t)g << 16) | (uint32_t)u, (uint32_t)t, (uint32_t)r, ORC_TAG_ACC};
                uint32_t o[4];
                orc_philox4x32_10(ctr, key, o);
                for (int32_t f = 0; f < 8 && g * 8 + f < n; ++f) {
                    int32_t i = g * 8 + f;
                    field[i * n + u] = (o[f >> 1] >> (16 * (f & 1))) & 0xFFFu;
                }
            }
        }

        /* Algorithm 3: parallel acceptance test of every bit. */
        int64_t c = 0;
        for (int32_t a = 0; a < m; ++a) {
            acc[a] = (uint8_t)orc_accept(dE1[a], dE2[a], Eoff, T, lnt[field[a]], p->accept);
            c += acc[a];
        }

        if (c > 0) {
            /* Algorithm 3: uniform choice among the accepted flips, move, archive. */
            uint32_t ctr[4] = {0u, (uint32_t)t, (uint32_t)r, ORC_TAG_SEL};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            int64_t k = mulhi32(o[0], (uint32_t)c);
            int32_t j = -1;
            for (int32_t a = 0; a < m; ++a) {
                if (!acc[a]) continue;
                if (k == 0) { j = a; break; }
                --k;
            }
            int64_t sg = x[j] ? -1 : 1;
            E1 += dE1[j];
            E2 += dE2[j];
            x[j] ^= 1u;
            for (int32_t a = 0; a < m; ++a) {
                if (a == j) continue;
                h1[a] += sg * q->P1[(int64_t)a * m + j];
                h2[a] += sg * q->P2[(int64_t)a * m + j];
            }
            Eoff = 0;   /* Algorithm 1: the offset is cleared after a move */
            ++moves;
            if (p->archive == ORC_EXPLOIT) {
                uint32_t ca[4] = {0u, (uint32_t)t, (uint32_t)r, ORC_TAG_ARC};
                uint32_t oa[4];
                orc_philox4x32_10(ca, key, oa);
                orc_archive_exploit(&A, E1, E2, x, oa[0]);
            } else {
                orc_archive_explore(&A, E1, E2, x);
            }
            if (out->trace) out->trace[t - 1] = j;
        } else {
            if (out->trace) out->trace[t - 1] = -1;
            if (p->escape == ORC_ESC_OFFSET) {
                Eoff += p->beta;   /* Algorithm 1: raise the offset */
            } else if (A.size > 0) {
                /* Algorithm 3 (escape): continue from a random archive member. */
                uint32_t ca[4] = {0u, (uint32_t)t, (uint32_t)r, ORC_TAG_ARC};
                uint32_t oa[4];
                orc_philox4x32_10(ca, key, oa);
                int32_t pick = (int32_t)mulhi32(oa[1], (uint32_t)A.size);
                memcpy(x, A.x + (int64_t)pick * m, (size_t)m);
                fields_of(q, q->P1, x, h1);
                fields_of(q, q->P2, x, h2);
                E1 = energy_of(q, q->P1, q->q1, x);
                E2 = energy_of(q, q->P2, q->q2, x);
            }
        }
    }

    out->state[0] = E1;
    out->state[1] = E2;
    out->state[2] = Eoff;
    out->state[3] = moves;
    *out->arch_size = A.size;
    for (int32_t i = 0; i < A.size; ++i) {
        out->arch_e[2 * i] = A.e1[i];
        out->arch_e[2 * i + 1] = A.e2[i];
    }
    free(A.e1); free(A.e2);
    free(dE1); free(dE2); free(acc); free(field);
    return 0;
}

/* ---------------- K objectives on a generic QUBO (readings G1-G3) ---------------- */

int orc_gbuild(int32_t m, int32_t K, const int32_t *Q, const int64_t *q, orc_gqubo *g)
{
    int64_t mm = (int64_t)m * m;
    memset(g, 0, sizeof(*g));
    g->m = m;
    g->K = K;
    g->P = (int64_t *)malloc((size_t)(K * mm) * sizeof(int64_t));
    g->q = (int64_t *)malloc((size_t)K * sizeof(int64_t));
    if (!g->P || !g->q) {
        orc_gfree(g);
        return -1;
    }
    for (int32_t k = 0; k < K; ++k) {
        const int32_t *Qk = Q + k * mm;
        int64_t *Pk = g->P + k * mm;
        g->q[k] = q ? q[k] : 0;
        /* the symmetric form of Eq. (cale), reading R2 */
        for (int32_t a = 0; a < m; ++a) {
            for (int32_t b = 0; b < m; ++b) {
                int64_t v = (a == b) ? (int64_t)Qk[(int64_t)a * m + a]
                                     : (int64_t)Qk[(int64_t)a * m + b] + Qk[(int64_t)b * m + a];
                Pk[(int64_t)a * m + b] = v;
                if (a <= b) {
                    int64_t av = v < 0 ? -v : v;
                    if (av > g->maxabs_c) g->maxabs_c = av;
                }
            }
        }
        for (int32_t a = 0; a < m; ++a) {
            int64_t sum = 0;
            for (int32_t b = 0; b < m; ++b) {
                int64_t v = Pk[(int64_t)a * m + b];
                sum += v < 0 ? -v : v;
            }
            if (sum > INT32_LIMIT) g->overflow = 1;
        }
    }
    return 0;
}

void orc_gfree(orc_gqubo *g)
{
    free(g->P);
    free(g->q);
    g->P = 0;
    g->q = 0;
}

int orc_gdominates(int32_t K, const int64_t *p, const int64_t *q)
{
    int equal = 1;
    for (int32_t k = 0; k < K; ++k) {
        if (p[k] > q[k]) return 0;
        if (p[k] != q[k]) equal = 0;
    }
    return !equal;
}

int orc_gaccept(int32_t K, const int64_t *dE, int64_t Eoff, int64_t T, int32_t lnt_k, int32_t mode)
{
    /* Reading G1: per objective max(0, D_k); strict sums them (the product of
     * the K probabilities), lenient takes the least (the largest probability). */
    int64_t S = 0;
    for (int32_t k = 0; k < K; ++k) {
        int64_t d = dE[k] - Eoff;
        int64_t p = d > 0 ? d : 0;
        if (mode == ORC_LENIENT) S = (k == 0 || p < S) ? p : S;
        else S += p;
    }
    int64_t thr = (T * (int64_t)lnt_k) >> 24;
    return S <= thr;
}

static void garchive_put(orc_garchive *A, int32_t slot, const int64_t *e, const uint8_t *x)
{
    memcpy(A->e + (int64_t)slot * A->K, e, (size_t)A->K * sizeof(int64_t));
    memcpy(A->x + (int64_t)slot * A->m, x, (size_t)A->m);
}

int32_t orc_garchive_explore(orc_garchive *A, const int64_t *e, const uint8_t *x)
{
    /* Algorithm 4: replace the first member that x dominates, else append. */
    for (int32_t i = 0; i < A->size; ++i) {
        if (orc_gdominates(A->K, e, A->e + (int64_t)i * A->K)) {
            garchive_put(A, i, e, x);
            return i;
        }
    }
    if (A->size < A->cap) {
        garchive_put(A, A->size, e, x);
        return A->size++;
    }
    return -1;
}

int32_t orc_garchive_exploit(orc_garchive *A, const int64_t *e, const uint8_t *x, uint32_t w)
{
    /* Algorithm 5: only when no member dominates x; a random member of
     * B = {y : x dominates y} is replaced, else x is appended. */
    for (int32_t i = 0; i < A->size; ++i)
        if (orc_gdominates(A->K, A->e + (int64_t)i * A->K, e)) return -1;
    int32_t nb = 0;
    for (int32_t i = 0; i < A->size; ++i)
        if (orc_gdominates(A->K, e, A->e + (int64_t)i * A->K)) ++nb;
    if (nb > 0) {
        int32_t pick = (int32_t)mulhi32(w, (uint32_t)nb);
        for (int32_t i = 0; i < A->size; ++i) {
            if (orc_gdominates(A->K, e, A->e + (int64_t)i * A->K)) {
                if (pick == 0) {
                    garchive_put(A, i, e, x);
                    return i;
                }
                --pick;
            }
        }
    }
    if (A->size < A->cap) {
        garchive_put(A, A->size, e, x);
        return A->size++;
    }
    return -1;
}

/* Eq. (qubo) from the symmetric form: q + sum_{a in x} P_aa + sum_{a<b in x} P_ab. */
static int64_t genergy(int32_t m, const int64_t *P, int64_t q, const uint8_t *x)
{
    int64_t e = q;
    for (int32_t a = 0; a < m; ++a) {
        if (!x[a]) continue;
        e += P[(int64_t)a * m + a];
        for (int32_t b = a + 1; b < m; ++b)
            if (x[b]) e += P[(int64_t)a * m + b];
    }
    return e;
}

static void gfields(int32_t m, const int64_t *P, const uint8_t *x, int64_t *h)
{
    for (int32_t a = 0; a < m; ++a) {
        int64_t s = 0;
        for (int32_t b = 0; b < m; ++b)
            if (b != a && x[b]) s += P[(int64_t)a * m + b];
        h[a] = s;
    }
}

int orc_gmda_replica(const orc_gqubo *g, const orc_params *p, int32_t r, orc_greplica_out *out)
{
    int32_t m = g->m, K = g->K;
    int32_t s = p->archive_size > 0 ? p->archive_size : m;
    int64_t mm = (int64_t)m * m;
    if (p->steps < 0 || p->steps > 0xFFFFFFFFLL || r < 0 || K < 1) return -1;
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    int32_t lnt[4096];
    orc_lnt(lnt);

    uint8_t *x = out->x;
    int64_t *h = out->h;
    int64_t *dE = (int64_t *)malloc((size_t)(K * (int64_t)m) * sizeof(int64_t));
    int64_t *E = (int64_t *)malloc((size_t)K * sizeof(int64_t));
    int64_t *dEa = (int64_t *)malloc((size_t)K * sizeof(int64_t));
    uint8_t *acc = (uint8_t *)malloc((size_t)m);
    uint32_t *field = (uint32_t *)malloc((size_t)m * sizeof(uint32_t));
    orc_garchive A;
    A.size = 0;
    A.cap = s;
    A.m = m;
    A.K = K;
    A.e = (int64_t *)malloc((size_t)s * (size_t)K * sizeof(int64_t));
    A.x = out->arch_x;
    if (!dE || !E || !dEa || !acc || !field || !A.e) {
        free(dE); free(E); free(dEa); free(acc); free(field); free(A.e);
        return -3;
    }

    /* Algorithm 3 starts from a random binary solution (reading G3). */
    for (int32_t a = 0; a < m; ++a) {
        uint32_t ctr[4] = {(uint32_t)(a >> 7), 0u, (uint32_t)r, ORC_TAG_INIT};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        x[a] = (uint8_t)((o[(a >> 5) & 3] >> (a & 31)) & 1u);
    }
    for (int32_t k = 0; k < K; ++k) {
        gfields(m, g->P + k * mm, x, h + (int64_t)k * m);
        E[k] = genergy(m, g->P + k * mm, g->q[k], x);
    }
    int64_t Eoff = 0, moves = 0;

    double delta = p->delta0;
    for (int64_t t = 1; t <= p->steps; ++t) {
        /* Algorithm 3: cooling at the top of each iteration, unless the
         * schedule is given as data. */
        int64_t T;
        if (p->temp_table) {
            T = p->temp_table[t - 1];
        } else {
            if (delta > p->deltaf) delta = delta * (1.0 - p->xi);
            T = (int64_t)floor(delta * 256.0);
        }

        /* Eq. (cale) for every bit and objective. */
        for (int32_t k = 0; k < K; ++k) {
            const int64_t *Pk = g->P + k * mm;
            for (int32_t a = 0; a < m; ++a) {
                int64_t sgn = 1 - 2 * (int64_t)x[a];
                dE[(int64_t)k * m + a] = sgn * (Pk[(int64_t)a * m + a] + h[(int64_t)k * m + a]);
            }
        }

        /* One 12-bit index per bit (reading G3). */
        for (int32_t a = 0; a < m; ++a) {
            uint32_t ctr[4] = {(uint32_t)(a >> 3), (uint32_t)t, (uint32_t)r, ORC_TAG_ACC};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            int32_t f = a & 7;
            field[a] = (o[f >> 1] >> (16 * (f & 1) + 4)) & 0xFFFu;
        }

        /* Parallel acceptance test of every bit (reading G1). */
        int64_t c = 0;
        for (int32_t a = 0; a < m; ++a) {
            for (int32_t k = 0; k < K; ++k) dEa[k] = dE[(int64_t)k * m + a];
            acc[a] = (uint8_t)orc_gaccept(K, dEa, Eoff, T, lnt[field[a]], p->accept);
            c += acc[a];
        }

        if (c > 0) {
            /* Uniform choice among the accepted flips, move, archive. */
            uint32_t ctr[4] = {0u, (uint32_t)t, (uint32_t)r, ORC_TAG_SEL};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            int64_t kk = mulhi32(o[0], (uint32_t)c);
            int32_t j = -1;
            for (int32_t a = 0; a < m; ++a) {
                if (!acc[a]) continue;
                if (kk == 0) { j = a; break; }
                --kk;
            }
            int64_t sg = x[j] ? -1 : 1;
            for (int32_t k = 0; k < K; ++k) {
                const int64_t *Pk = g->P + k * mm;
                E[k] += dE[(int64_t)k * m + j];
                for (int32_t a = 0; a < m; ++a) {
                    if (a == j) continue;
                    h[(int64_t)k * m + a] += sg * Pk[(int64_t)a * m + j];
                }
            }
            x[j] ^= 1u;
            Eoff = 0;   /* Algorithm 1: the offset is cleared after a move */
            ++moves;
            if (p->archive == ORC_EXPLOIT) {
                uint32_t ca[4] = {0u, (uint32_t)t, (uint32_t)r, ORC_TAG_ARC};
                uint32_t oa[4];
                orc_philox4x32_10(ca, key, oa);
                orc_garchive_exploit(&A, E, x, oa[0]);
            } else {
                orc_garchive_explore(&A, E, x);
            }
            if (out->trace) out->trace[t - 1] = j;
        } else {
            if (out->trace) out->trace[t - 1] = -1;
            if (p->escape == ORC_ESC_OFFSET) {
                Eoff += p->beta;   /* Algorithm 1: raise the offset */
            } else if (A.size > 0) {
                /* Algorithm 3 (escape): continue from a random archive member. */
                uint32_t ca[4] = {0u, (uint32_t)t, (uint32_t)r, ORC_TAG_ARC};
                uint32_t oa[4];
                orc_philox4x32_10(ca, key, oa);
                int32_t pick = (int32_t)mulhi32(oa[1], (uint32_t)A.size);
                memcpy(x, A.x + (int64_t)pick * m, (size_t)m);
                for (int32_t k = 0; k < K; ++k) {
                    gfields(m, g->P + k * mm, x, h + (int64_t)k * m);
                    E[k] = genergy(m, g->P + k * mm, g->q[k], x);
                }
            }
        }
    }

    for (int32_t k = 0; k < K; ++k) out->state[k] = E[k];
    out->state[K] = Eoff;
    out->state[K + 1] = moves;
    *out->arch_size = A.size;
    memcpy(out->arch_e, A.e, (size_t)A.size * (size_t)K * sizeof(int64_t));
    free(A.e);
    free(dE); free(E); free(dEa); free(acc); free(field);
    return 0;
}
