// mda_host.cpp -- C ABI of the MI355X multi-objective Digital Annealer
// (declared and documented in include/mda.h).  Host side: QUBO operands of the
// bi-objective QAP (Sec. 2 of Ayodele et al., GECCO 2022), the fixed-point
// schedule and threshold tables, device memory, launches and result readout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "mda.h"
#include "mda_desc.h"
#include "mda_host_common.h"
#include "mda_internal.h"

namespace mda {
int ns_for(int n);
int group_waves_limit(int ns);
hipError_t launch_group(int ns, int occ, int wr, int wc, const RunDesc *runs, const WorkItem *work, int nwork,
                        const int32_t *lnt, int grid, hipStream_t stream);
hipError_t group_occupancy(int ns, int occ, int wr, int wc, int *blocks_per_cu);
hipError_t launch_persistent(int ns, int occ, int f64, int sv, const RunDesc *runs, const WorkItem *work, int nwork,
                             const int32_t *lnt, unsigned int *next, int grid, int block, hipStream_t stream);
hipError_t launch_plain(int ns, int sv, const RunDesc *run, int R, uint32_t steps, const int32_t *lnt, int block,
                        hipStream_t stream);
hipError_t launch_nondominated(const RunDesc *runs, const WorkItem *work, int nwork, hipStream_t stream);
hipError_t launch_best(const RunDesc *run, int R, int64_t *e1, int32_t *slot, hipStream_t stream);
size_t front_filter_scratch();
hipError_t launch_front_filter(const FrontEntry *ent, int64_t count, void *scratch, FrontEntry *out,
                               unsigned long long *nout, hipStream_t stream);
hipError_t launch_front_gather(const int64_t *archE, const uint8_t *nd, const int64_t *st, int s, int r0, int nr,
                               const int64_t *offs, FrontEntry *out, hipStream_t stream);
hipError_t launch_build_dense(int n, int ld, const int32_t *F, const int32_t *Dm, int32_t two_alpha, int32_t *P,
                              hipStream_t stream);
hipError_t persistent_occupancy(int ns, int occ, int f64, int sv, int block, int *blocks_per_cu);
}  // namespace mda

using namespace mda;

// ---------------------------------------------------------------- errors

static thread_local std::string g_err;

namespace mda {

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace mda

extern "C" const char *mda_last_error(void)
{
    return g_err.c_str();
}

// ---------------------------------------------------------------- device memory

static mda_alloc_fn g_alloc = nullptr;
static mda_free_fn g_release = nullptr;
static void *g_ctx = nullptr;

extern "C" int mda_set_allocator(mda_alloc_fn alloc, mda_free_fn release, void *ctx)
{
    if ((alloc == nullptr) != (release == nullptr)) return fail(MDA_EINVAL, "allocator and release must both be set");
    g_alloc = alloc;
    g_release = release;
    g_ctx = ctx;
    return MDA_OK;
}

// Allocation mode of the calling thread: the serving engine's scheduler
// allocates stream-ordered (hipMallocAsync), so that releasing one request's
// memory never waits for the other requests' work on the device.
static thread_local bool tl_stream_ordered = false;

namespace mda {

void *DevPool::alloc_bytes(size_t bytes, hipStream_t stream)
{
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    DevBuf b;
    if (tl_stream_ordered) {
        if (hipMallocAsync(&p, bytes, stream) != hipSuccess) p = nullptr;
        b.async = true;
    } else if (g_alloc) {
        p = g_alloc(bytes, (void *)stream, g_ctx);
        b.release = g_release;
        b.ctx = g_ctx;
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (!p) return nullptr;
    b.p = p;
    b.bytes = bytes;
    b.stream = stream;
    bufs.push_back(b);
    total += (int64_t)bytes;
    return p;
}

void DevPool::release_all()
{
    for (auto &b : bufs) {
        if (b.async) (void)hipFreeAsync(b.p, b.stream);
        else if (b.release) b.release(b.p, b.bytes, (void *)b.stream, b.ctx);
        else (void)hipFree(b.p);
    }
    bufs.clear();
    total = 0;
}

void threshold_table(int32_t *lnt)
{
    for (int k = 0; k < 4096; ++k) lnt[k] = (int32_t)std::llround(-std::log((k + 0.5) / 4096.0) * 65536.0);
}

int64_t temperature_table(double delta0, double deltaf, double xi, int64_t steps, std::vector<int64_t> &T)
{
    T.clear();
    double delta = delta0;
    for (int64_t t = 1; t <= steps; ++t) {
        bool cooled = false;
        if (delta > deltaf) {
            delta = delta * (1.0 - xi);
            cooled = true;
        }
        T.push_back((int64_t)std::floor(delta * 256.0));
        if (!cooled && t > 1) break;   // constant from here on
    }
    return (int64_t)T.size();
}

}  // namespace mda

extern "C" int mda_threshold_table(int32_t *lnt4096)
{
    if (!lnt4096) return fail(MDA_EINVAL, "null table");
    threshold_table(lnt4096);
    return MDA_OK;
}

extern "C" int mda_temperature_table(double delta0, double deltaf, double xi, int64_t steps, int64_t *T)
{
    if (!T || steps < 1) return fail(MDA_EINVAL, "bad arguments");
    if (!(delta0 * 256.0 <= kMaxTemp)) return fail(MDA_EOVERFLOW, "delta0 = %g exceeds 2^35", delta0);
    std::vector<int64_t> tab;
    temperature_table(delta0, deltaf, xi, steps, tab);
    for (int64_t t = 0; t < steps; ++t) T[t] = tab[std::min<int64_t>(t, (int64_t)tab.size() - 1)];
    return MDA_OK;
}

// ---------------------------------------------------------------- QUBO handle

struct mda_qubo {
    int32_t n = 0, m = 0;
    int32_t path = 0, kform = 0, symmetric = 0;
    int64_t alpha[2] = {0, 0}, q[2] = {0, 0};
    int64_t maxabs = 0;
    int32_t norm = 0;                  // normalisation 2^norm of both objectives (0: none)
    int32_t f64 = 0;                   // 1: energy differences in int64 (the int32 bounds fail)
    double scale[2] = {1.0, 1.0};      // s_k applied to F_k
    std::vector<int32_t> F1, F2, D, diag1, diag2;
    int32_t *dKA1 = nullptr, *dKA2 = nullptr, *dKB1 = nullptr, *dKB2 = nullptr, *dDA = nullptr, *dDB = nullptr;
    int32_t *dP1 = nullptr, *dP2 = nullptr, *ddiag1 = nullptr, *ddiag2 = nullptr;
    int32_t ldk = kLD;   // row stride of the per-lane operands and the diagonals
    int32_t pld = kLD;   // dense P_k: entry (i, u) of row j at j * n * pld + i * pld + u
    DevPool pool;
    int refs = 1;   // the owner plus every run that uses it
};

static void qubo_release(mda_qubo *q)
{
    // every run synchronises its stream before it drops its reference, and the
    // build waits for its uploads, so nothing on the device still reads q here
    if (--q->refs == 0) {
        q->pool.release_all();
        delete q;
    }
}

static bool is_symmetric(const std::vector<int32_t> &A, int n)
{
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (A[i * n + j] != A[j * n + i]) return false;
    return true;
}

// Entry (a, b), a <= b, of the upper-triangular cost QUBO C (Sec. 2.2).
static inline int64_t cost_upper(const int32_t *F, const int32_t *Dm, int n, int a, int b)
{
    const int i = a / n, u = a % n, j = b / n, v = b % n;
    if (a == b) return (int64_t)F[i * n + i] * Dm[u * n + u];
    return (int64_t)F[i * n + j] * Dm[u * n + v] + (int64_t)F[j * n + i] * Dm[v * n + u];
}

// Largest |entry| of the upper-triangular cost QUBO C of flows F (Sec. 2.2):
// F[i][i] D[u][u] on the diagonal, F[i][j] D[u][v] + F[j][i] D[v][u] off it.
// The off-diagonal form is unchanged by swapping (i, u) and (j, v), so a scan
// over all ordered pairs gives the maximum over the upper triangle.
static int64_t objective_maxabs(const int32_t *F, const int32_t *Dm, int n)
{
    int64_t mx = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int64_t fij = F[i * n + j], fji = F[j * n + i];
            for (int u = 0; u < n; ++u)
                for (int v = 0; v < n; ++v) {
                    const int64_t c = (i == j && u == v) ? fij * Dm[u * n + u]
                                                         : fij * Dm[u * n + v] + fji * Dm[v * n + u];
                    mx = std::max<int64_t>(mx, std::llabs(c));
                }
        }
    return mx;
}

// One build with the objectives normalised to 2^L (L = 0: as given); mxk[k]
// is max|C_k| of the given flows (only read when L > 0).
static int build_bqap(int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D, const mda_build_opts &o,
                      int L, const int64_t *mxk, hipStream_t stream, mda_qubo **out)
{
    // automatic path: dense rows only within an explicit budget (the Kronecker
    // update is the faster one at every size)
    const int64_t budget = o.dense_budget > 0 ? o.dense_budget : 0;

    std::unique_ptr<mda_qubo> q(new mda_qubo);
    const int m = n * n;
    q->n = n;
    q->m = m;
    const size_t nn = (size_t)n * n;
    q->F1.assign(F1, F1 + nn);
    q->F2.assign(F2, F2 + nn);
    q->D.assign(D, D + nn);

    // Objective normalisation (Sec. Parameter Settings): C_k is linear in F_k,
    // so scaling the flows by s_k = 2^L / max|C_k| scales C_k by s_k and keeps
    // its Kronecker form; the scaled flows are rounded to the nearest integer
    // (halves up).  An objective that vanishes is left as it is.
    q->norm = L;
    if (L > 0) {
        std::vector<int32_t> *Fv[2] = {&q->F1, &q->F2};
        for (int k = 0; k < 2; ++k) {
            const int64_t mx = mxk[k];
            if (mx == 0) continue;
            const double s = std::ldexp(1.0, L) / (double)mx;
            for (int32_t &f : *Fv[k]) {
                const double r = std::floor((double)f * s + 0.5);
                if (!(std::fabs(r) <= (double)INT32_MAX))
                    return fail(MDA_EOVERFLOW, "objective %d: scaled flow %g beyond int32", k + 1, r);
                f = (int32_t)r;
            }
            q->scale[k] = s;
        }
    }
    const int32_t *Fk[2] = {q->F1.data(), q->F2.data()};
    const int32_t *Dm = q->D.data();

    // Penalty weights (Eq. wqubom): 2 max|C_k|, or Eq. (vermap)/(wvermaa) on the
    // symmetric form of C_k; then the int32 bound on every bit's interactions.
    // Off the diagonal, entry (a, b) = ((i, u), (j, v)) of the symmetric form is
    // F[i][j] D[u][v] + F[j][i] D[v][u] (the same for (b, a)), so the scans run
    // over (i, j, u, v) without divisions; with non-negative F and D the row
    // sums have closed forms.
    std::vector<int32_t> DT(nn);
    for (int u = 0; u < n; ++u)
        for (int v = 0; v < n; ++v) DT[(size_t)v * n + u] = Dm[(size_t)u * n + v];
    bool nonneg = true;
    for (size_t e = 0; e < nn; ++e) nonneg &= q->D[e] >= 0 && q->F1[e] >= 0 && q->F2[e] >= 0;
    // why int32 differences cannot hold this instance (empty: they can)
    char why32[256] = "";
    const bool dsym_ = is_symmetric(q->D, n);
    for (int k = 0; k < 2; ++k) {
        const int32_t *F = Fk[k];
        int64_t mx = 0;
        for (int i = 0; i < n; ++i)
            for (int u = 0; u < n; ++u) mx = std::max<int64_t>(mx, std::llabs((int64_t)F[i * n + i] * Dm[u * n + u]));
        if (nonneg && dsym_ && is_symmetric(k == 0 ? q->F1 : q->F2, n)) {
            // off-diagonal entries are 2 F[i][j] D[u][v] over (i, u) != (j, v)
            int64_t fo = 0, fd = 0, da = 0, dof = 0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    (i == j ? fd : fo) = std::max<int64_t>(i == j ? fd : fo, F[i * n + j]);
                    da = std::max<int64_t>(da, Dm[i * n + j]);
                    if (i != j) dof = std::max<int64_t>(dof, Dm[i * n + j]);
                }
            mx = std::max(mx, 2 * std::max(fo * da, fd * dof));
        } else {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const int64_t fij = F[i * n + j], fji = F[j * n + i];
                for (int u = 0; u < n; ++u) {
                    const int32_t *dr = Dm + (size_t)u * n, *dc = DT.data() + (size_t)u * n;
                    for (int v = 0; v < n; ++v) {
                        if (i == j && u == v) continue;
                        mx = std::max<int64_t>(mx, std::llabs(fij * dr[v] + fji * dc[v]));
                    }
                }
            }
        }
        q->maxabs = std::max(q->maxabs, mx);
        // per-bit sums over b != a of the positive and negative parts of C_ab
        std::vector<int64_t> pos(m, 0), neg(m, 0);
        std::vector<int64_t> rowF(n, 0), colF(n, 0), rowD(n, 0), colD(n, 0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                rowF[i] += F[i * n + j];
                colF[j] += F[i * n + j];
                rowD[i] += Dm[i * n + j];
                colD[j] += Dm[i * n + j];
            }
        for (int i = 0; i < n; ++i)
            for (int u = 0; u < n; ++u) {
                const int a = i * n + u;
                const int64_t self = (int64_t)F[i * n + i] * Dm[u * n + u];
                if (nonneg) {
                    pos[a] = rowF[i] * rowD[u] + colF[i] * colD[u] - 2 * self;
                    continue;
                }
                int64_t pp = 0, nq = 0;
                for (int j = 0; j < n; ++j) {
                    const int64_t fij = F[i * n + j], fji = F[j * n + i];
                    const int32_t *dr = Dm + (size_t)u * n, *dc = DT.data() + (size_t)u * n;
                    for (int v = 0; v < n; ++v) {
                        if (j == i && v == u) continue;
                        const int64_t c = fij * dr[v] + fji * dc[v];
                        if (c > 0) pp += c;
                        else nq -= c;
                    }
                }
                pos[a] = pp;
                neg[a] = nq;
            }
        int64_t alpha = 2 * mx;
        if (o.penalty == MDA_PEN_VL) {
            int64_t w = INT64_MIN;
            for (int i = 0; i < n; ++i)
                for (int u = 0; u < n; ++u) {
                    const int a = i * n + u;
                    const int64_t caa = (int64_t)F[i * n + i] * Dm[u * n + u];
                    w = std::max(w, std::max(-caa + neg[a], caa + pos[a]));
                }
            alpha = (w + 1) / 2;
        }
        q->alpha[k] = alpha;
        q->q[k] = alpha * 2 * n;
        // the column entries (at most max|C| + 2 alpha) and the penalty 2 alpha
        // the kernels hold in 32 bits, at any difference width
        if (mx + 2 * alpha > INT32_MAX)
            return fail(MDA_EOVERFLOW, "objective %d: QUBO entries up to %lld exceed int32", k + 1,
                        (long long)(mx + 2 * alpha));
        // int32 differences: slots beyond n hold 2^30 and drift by at most
        // 2 alpha n; below 2^30 the drift keeps them positive and inside int32
        if (2 * alpha * n >= (int64_t)1 << 30 && !why32[0])
            snprintf(why32, sizeof why32, "penalty 2*alpha_%d*n = %lld exceeds 2^30", k + 1, (long long)(2 * alpha * n));
        // Every local field |P_aa + sum_b P_ab x_b| must fit int32: with the
        // penalty 2 alpha on the 2 (n - 1) bits sharing a's row or column,
        // sum_b |P_ab| <= |P_aa| + sum |C_ab| + 4 alpha (n - 1), exact when
        // no C_ab of those bits is below -2 alpha (always for non-negative
        // inputs); otherwise the exact sum is taken.
        for (int i = 0; i < n; ++i)
            for (int u = 0; u < n; ++u) {
                const int a = i * n + u;
                const int64_t self = (int64_t)F[i * n + i] * Dm[u * n + u];
                int64_t sum = std::llabs(self - 2 * alpha);
                if (nonneg) {
                    sum += pos[a] + 4 * alpha * (n - 1);
                } else {
                    for (int j = 0; j < n; ++j) {
                        const int64_t fij = F[i * n + j], fji = F[j * n + i];
                        const int32_t *dr = Dm + (size_t)u * n, *dc = DT.data() + (size_t)u * n;
                        for (int v = 0; v < n; ++v) {
                            if (j == i && v == u) continue;
                            int64_t c = fij * dr[v] + fji * dc[v];
                            if ((i == j) != (u == v)) c += 2 * alpha;
                            sum += std::llabs(c);
                        }
                    }
                }
                if (sum > INT32_MAX - 1 && !why32[0])
                    snprintf(why32, sizeof why32, "objective %d: bit %d has sum |P_ab| = %lld > 2^31-2", k + 1, a,
                             (long long)sum);
            }
    }
    q->diag1.resize(m);
    q->diag2.resize(m);
    for (int a = 0; a < m; ++a) {
        q->diag1[a] = (int32_t)(cost_upper(Fk[0], Dm, n, a, a) - 2 * q->alpha[0]);
        q->diag2[a] = (int32_t)(cost_upper(Fk[1], Dm, n, a, a) - 2 * q->alpha[1]);
    }

    // Kronecker operands.
    const bool dsym = is_symmetric(q->D, n);
    const bool fsym = is_symmetric(q->F1, n) && is_symmetric(q->F2, n);
    q->symmetric = (dsym || fsym) ? 1 : 0;
    std::vector<int32_t> KA[2], KB[2], DA, DB;
    int64_t maxop = 0;
    auto track = [&](const std::vector<int32_t> &v) {
        for (int32_t e : v) maxop = std::max<int64_t>(maxop, std::llabs((int64_t)e));
    };
    if (dsym || fsym) {
        q->kform = kKronSym;
        for (int k = 0; k < 2; ++k) {
            KA[k].resize(nn);
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b)
                    KA[k][a * n + b] = dsym ? Fk[k][a * n + b] + Fk[k][b * n + a] : Fk[k][a * n + b];
            track(KA[k]);
        }
        DA.resize(nn);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) DA[a * n + b] = dsym ? Dm[a * n + b] : Dm[a * n + b] + Dm[b * n + a];
        track(DA);
    } else {
        q->kform = kKronGen;
        for (int k = 0; k < 2; ++k) {
            KA[k].resize(nn);
            KB[k].assign(Fk[k], Fk[k] + nn);
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) KA[k][a * n + b] = Fk[k][b * n + a];
            track(KA[k]);
            track(KB[k]);
        }
        DA.resize(nn);
        DB.assign(Dm, Dm + nn);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) DA[a * n + b] = Dm[b * n + a];
        track(DA);
    }
    // 24-bit multiply-adds whose products (and, in the general form, their
    // sum) fit int32; the row bound implies it for int32 differences
    int64_t maxf = 0, maxd = 0;
    for (int k = 0; k < 2; ++k) {
        for (int32_t e : KA[k]) maxf = std::max<int64_t>(maxf, std::llabs((int64_t)e));
        for (int32_t e : KB[k]) maxf = std::max<int64_t>(maxf, std::llabs((int64_t)e));
    }
    for (int32_t e : DA) maxd = std::max<int64_t>(maxd, std::llabs((int64_t)e));
    for (int32_t e : DB) maxd = std::max<int64_t>(maxd, std::llabs((int64_t)e));
    const bool kron_ok = maxop < (1 << 23) && (q->kform == kKronGen ? 2 : 1) * maxf * maxd <= INT32_MAX;
    // width of the energy differences
    if (o.fields == 32 && why32[0]) return fail(MDA_EOVERFLOW, "%s (int32 fields requested)", why32);
    q->f64 = (o.fields == 64 || (o.fields == 0 && why32[0])) ? 1 : 0;
    if (q->f64 && n > kMaxWaveN)
        return fail(MDA_EOVERFLOW, "%s; int64 fields run one wave per replica (n <= %d), n = %d",
                    why32[0] ? why32 : "int64 fields requested", kMaxWaveN, n);
    // Operand layouts: up to 64 facilities every Kronecker row is padded to 64
    // entries (one wave per replica reads them unmasked), beyond to 128; the
    // dense rows are never padded (both forms mask their reads), so a move
    // streams 2 n^2 entries, the algorithmic amount.
    q->ldk = n <= kMaxWaveN ? kLD : 2 * kLD;
    q->pld = n;
    const bool dense_fits = 8 * (int64_t)m * n * q->pld <= budget;
    if (o.path == MDA_PATH_KRON) {
        if (!kron_ok) return fail(MDA_EOVERFLOW, "Kronecker operands exceed the 24-bit multiplier range");
        q->path = kPathKron;
    } else if (o.path == MDA_PATH_DENSE) {
        q->path = kPathDense;
    } else {
        q->path = (dense_fits || !kron_ok) ? kPathDense : kPathKron;
    }

    // Uploads.  Per-lane operands go up as rows of ldk entries, zero padded.
    auto up = [&](const std::vector<int32_t> &h) -> int32_t * {
        int32_t *d = q->pool.alloc<int32_t>(h.size(), stream);
        if (d && hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream) != hipSuccess)
            return nullptr;
        return d;
    };
    auto pad = [&](const std::vector<int32_t> &h, int rows) {
        const int ld = q->ldk;
        std::vector<int32_t> o((size_t)rows * ld, 0);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) o[(size_t)a * ld + b] = h[(size_t)a * n + b];
        return o;
    };
    // the one-wave form reads the diagonal for every register slot (up to
    // kMaxWaveN rows)
    q->ddiag1 = up(pad(q->diag1, std::max(n, kMaxWaveN)));
    q->ddiag2 = up(pad(q->diag2, std::max(n, kMaxWaveN)));
    if (!q->ddiag1 || !q->ddiag2) return fail(MDA_ENOMEM, "device allocation failed");
    if (q->path == kPathKron) {
        q->dKA1 = up(pad(KA[0], n));
        q->dKA2 = up(pad(KA[1], n));
        q->dDA = up(pad(DA, n));
        if (!q->dKA1 || !q->dKA2 || !q->dDA) return fail(MDA_ENOMEM, "device allocation failed");
        if (q->kform == kKronGen) {
            q->dKB1 = up(pad(KB[0], n));
            q->dKB2 = up(pad(KB[1], n));
            q->dDB = up(pad(DB, n));
            if (!q->dKB1 || !q->dKB2 || !q->dDB) return fail(MDA_ENOMEM, "device allocation failed");
        } else {
            q->dKB1 = q->dKA1;
            q->dKB2 = q->dKA2;
            q->dDB = q->dDA;
        }
    } else {
        int32_t *dF1 = up(q->F1), *dF2 = up(q->F2), *dD = up(q->D);
        q->dP1 = q->pool.alloc<int32_t>((size_t)m * n * q->pld, stream);
        q->dP2 = q->pool.alloc<int32_t>((size_t)m * n * q->pld, stream);
        if (!dF1 || !dF2 || !dD || !q->dP1 || !q->dP2) return fail(MDA_ENOMEM, "device allocation failed");
        HIP_TRY(launch_build_dense(n, q->pld, dF1, dD, (int32_t)(2 * q->alpha[0]), q->dP1, stream));
        HIP_TRY(launch_build_dense(n, q->pld, dF2, dD, (int32_t)(2 * q->alpha[1]), q->dP2, stream));
        q->dKA1 = q->dKA2 = q->dKB1 = q->dKB2 = q->dDA = q->dDB = dF1;   // unused on this path
    }
    HIP_TRY(hipStreamSynchronize(stream));
    *out = q.release();
    return MDA_OK;
}

extern "C" int qubo_build_bqap(int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D,
                               const mda_build_opts *opts, void *stream_, mda_qubo **out)
{
    if (!out) return fail(MDA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 2 || n > 100) return fail(MDA_EINVAL, "n = %d outside [2, 100]", n);
    if (!F1 || !F2 || !D) return fail(MDA_EINVAL, "F1, F2 and D must be non-NULL");
    mda_build_opts o{MDA_PEN_2MAX, MDA_PATH_AUTO, 0, 0, 0};
    if (opts) o = *opts;
    if (o.penalty != MDA_PEN_2MAX && o.penalty != MDA_PEN_VL) return fail(MDA_EINVAL, "unknown penalty %d", o.penalty);
    if (o.path < MDA_PATH_AUTO || o.path > MDA_PATH_KRON) return fail(MDA_EINVAL, "unknown path %d", o.path);
    if (o.normalise_log2 < -1 || o.normalise_log2 > 30)
        return fail(MDA_EINVAL, "normalise_log2 = %d outside [-1, 30]", o.normalise_log2);
    if (o.fields != 0 && o.fields != 32 && o.fields != 64)
        return fail(MDA_EINVAL, "fields = %d (0, 32 or 64)", o.fields);
    hipStream_t stream = (hipStream_t)stream_;
    int64_t mxk[2] = {0, 0};
    if (o.normalise_log2 != 0) {
        mxk[0] = objective_maxabs(F1, D, n);
        mxk[1] = objective_maxabs(F2, D, n);
    }
    if (o.normalise_log2 != -1) return build_bqap(n, F1, F2, D, o, o.normalise_log2, mxk, stream, out);
    // the paper's 2^23 where the int32 bounds allow it, else the largest power
    // below (int32 fields unless int64 ones were asked for)
    mda_build_opts o32 = o;
    if (o32.fields == 0) o32.fields = 32;
    for (int L = 23; L >= 1; --L) {
        const int rc = build_bqap(n, F1, F2, D, o32, L, mxk, stream, out);
        if (rc != MDA_EOVERFLOW) return rc;
    }
    return fail(MDA_EOVERFLOW, "no normalisation 2^L with 1 <= L <= 23 keeps every field within int32");
}

extern "C" int qubo_flows(const mda_qubo *q, int32_t *F1, int32_t *F2)
{
    if (!q) return fail(MDA_EINVAL, "NULL qubo");
    if (F1) std::memcpy(F1, q->F1.data(), q->F1.size() * sizeof(int32_t));
    if (F2) std::memcpy(F2, q->F2.data(), q->F2.size() * sizeof(int32_t));
    return MDA_OK;
}

extern "C" int qubo_info(const mda_qubo *q, mda_qubo_info *info)
{
    if (!q || !info) return fail(MDA_EINVAL, "NULL argument");
    info->n = q->n;
    info->m = q->m;
    info->path = q->path == kPathDense ? MDA_PATH_DENSE : MDA_PATH_KRON;
    info->symmetric = q->symmetric;
    info->alpha1 = q->alpha[0];
    info->alpha2 = q->alpha[1];
    info->q1 = q->q[0];
    info->q2 = q->q[1];
    info->maxabs_c = q->maxabs;
    info->device_bytes = q->pool.total;
    info->normalise_log2 = q->norm;
    info->fields = q->f64 ? 64 : 32;
    info->scale1 = q->scale[0];
    info->scale2 = q->scale[1];
    return MDA_OK;
}

extern "C" int qubo_build_scalarised(int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D, int32_t g10,
                                     const mda_build_opts *opts, void *stream, mda_qubo **out)
{
    if (!out) return fail(MDA_EINVAL, "out is NULL");
    *out = nullptr;
    if (g10 < 0 || g10 > 10) return fail(MDA_EINVAL, "g10 = %d outside [0, 10]", g10);
    if (n < 2 || n > 100) return fail(MDA_EINVAL, "n = %d outside [2, 100]", n);
    if (!F1 || !F2 || !D) return fail(MDA_EINVAL, "NULL input matrix");
    // C is linear in the flows: gamma R + (1 - gamma) S, times 10, is the cost
    // QUBO of g10 F1 + (10 - g10) F2 (Alg. SB-DA aggregation)
    const size_t nn = (size_t)n * n;
    std::vector<int32_t> F(nn), Z(nn, 0);
    for (size_t k = 0; k < nn; ++k) {
        const int64_t v = (int64_t)g10 * F1[k] + (int64_t)(10 - g10) * F2[k];
        if (v > INT32_MAX || v < INT32_MIN)
            return fail(MDA_EOVERFLOW, "scalarised flow %lld at (%zu, %zu) beyond int32", (long long)v, k / n, k % n);
        F[k] = (int32_t)v;
    }
    return qubo_build_bqap(n, F.data(), Z.data(), D, opts, stream, out);
}

extern "C" void qubo_free(mda_qubo *q)
{
    if (q) qubo_release(q);
}

// ---------------------------------------------------------------- runs

namespace {

// Device resources of one launch, shared by the runs it contains.
struct Launch {
    DevPool pool;
    RunDesc *ddesc = nullptr;
    WorkItem *dwork = nullptr;
    int nwork = 0;
    int32_t *dlnt = nullptr;
    unsigned int *dctr = nullptr;   // work-item counters, one per group
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // whole run
    hipEvent_t evk0 = nullptr, evk1 = nullptr; // annealing kernel(s) only
    hipGraph_t graph = nullptr;                // captured launch sequence, if any
    hipGraphExec_t graph_exec = nullptr;
    // streams on which further register-tile groups run beside the first
    // (default priority), with the fork and join events
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    ~Launch()
    {
        // wait for this launch only (its last event), not for later work on the stream
        if (ev1) (void)hipEventSynchronize(ev1);
        else if (stream || ev0) (void)hipStreamSynchronize(stream);
        for (hipStream_t st : side) (void)hipStreamSynchronize(st);
        for (hipStream_t st : side) (void)hipStreamDestroy(st);
        for (hipEvent_t e : join) (void)hipEventDestroy(e);
        if (fork) (void)hipEventDestroy(fork);
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (evk0) (void)hipEventDestroy(evk0);
        if (evk1) (void)hipEventDestroy(evk1);
        pool.release_all();
    }
};

}  // namespace

struct mda_run {
    mda_qubo *q = nullptr;
    mda_params p{};
    RunDesc h{};                       // host copy of this run's descriptor
    std::shared_ptr<Launch> launch;
    DevPool pool;                      // this run's outputs and tables
    std::vector<FrontEntry> merged;    // non-dominated union over replicas, once computed
    bool merged_ok = false;
    std::function<void()> on_release;  // set by the serving engine
    ~mda_run()
    {
        if (launch) {
            if (launch->ev1) (void)hipEventSynchronize(launch->ev1);
            else (void)hipStreamSynchronize(launch->stream);
        }
        pool.release_all();
        launch.reset();
        if (q) qubo_release(q);
        if (on_release) on_release();
    }
};

extern "C" void mda_params_default(mda_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->replicas = 1;
    p->archive_size = 0;
    p->steps = 0;
    p->delta0 = 0.0;
    p->deltaf = 0.0;
    p->xi = 0.001;
    p->beta = -1;
    p->accept = MDA_STRICT;
    p->archive = MDA_EXPLORE;
    p->escape = MDA_ESC_OFFSET;
    p->variant = MDA_VARIANT_AUTO;
}

// Host tables of a run: the fixed-point temperature T_t of each step and the
// largest threshold (T_t LNT[0]) >> 24, saturated at 2^32 - 2 for int32
// differences and as it is for int64 ones.
struct RunTables {
    std::vector<int64_t> T, thr64;
    std::vector<uint32_t> thr32;
};

// Checks p against q, resolves its defaults and fills the run descriptor d
// (every field but the device buffers of the run) and the host tables.
// Allocates nothing on the device.
static int resolve_run(const mda_qubo *q, const mda_params *pin, mda_params &p, RunDesc &d, RunTables &tab)
{
    std::vector<int64_t> &T = tab.T;
    std::vector<uint32_t> &thrmax = tab.thr32;
    p = *pin;
    if (p.replicas < 1) return fail(MDA_EINVAL, "replicas = %d", p.replicas);
    if (p.steps == 0) p.steps = (int64_t)std::llround(0.25 * (double)q->m * (double)q->m);
    // the kernels count steps t = 1..steps in 32 bits and stop after t == steps
    if (p.steps < 1 || p.steps > 0xFFFFFFFELL)
        return fail(MDA_EINVAL, "steps = %lld outside [1, 2^32 - 2]", (long long)p.steps);
    if (p.accept != MDA_STRICT && p.accept != MDA_LENIENT) return fail(MDA_EINVAL, "accept = %d", p.accept);
    if (p.archive != MDA_EXPLORE && p.archive != MDA_EXPLOIT) return fail(MDA_EINVAL, "archive = %d", p.archive);
    if (p.escape != MDA_ESC_OFFSET && p.escape != MDA_ESC_ARCHIVE) return fail(MDA_EINVAL, "escape = %d", p.escape);
    if (p.archive_size < 0) return fail(MDA_EINVAL, "archive_size = %d", p.archive_size);
    if (p.trace_replicas < 0 || p.trace_replicas > p.replicas) return fail(MDA_EINVAL, "trace_replicas = %d", p.trace_replicas);
    if (p.occupancy < 0 || p.occupancy > 2) return fail(MDA_EINVAL, "occupancy = %d outside [0, 2]", p.occupancy);
    if (p.delta0 <= 0.0) {
        p.delta0 = 1e9 * (double)q->maxabs / 8388608.0;
        p.deltaf = 1e4 * (double)q->maxabs / 8388608.0;
        if (p.xi <= 0.0) p.xi = 0.001;
    }
    if (!(p.xi >= 0.0 && p.xi < 1.0)) return fail(MDA_EINVAL, "xi = %g", p.xi);
    // every temperature is at most delta0 (the schedule only cools), so this
    // bound keeps each conversion of delta * 256 to an integer in range
    if (!(p.delta0 * 256.0 <= kMaxTemp)) return fail(MDA_EOVERFLOW, "delta0 = %g exceeds 2^35", p.delta0);
    if (p.beta < 0) p.beta = std::max<int64_t>(1, (int64_t)std::floor(p.delta0 / (double)p.steps));

    T.clear();
    if (p.temp_table) {
        // the schedule given as data: one entry per step, copied here
        T.assign(p.temp_table, p.temp_table + p.steps);
        p.temp_table = nullptr;
    } else {
        temperature_table(p.delta0, p.deltaf, p.xi, p.steps, T);
    }
    int32_t lnt[4096];
    threshold_table(lnt);
    thrmax.assign(T.size(), 0u);
    tab.thr64.assign(T.size(), 0);
    for (size_t t = 0; t < T.size(); ++t) {
        if (T[t] < 0 || (double)T[t] > kMaxTemp) return fail(MDA_EOVERFLOW, "temperature %lld out of range", (long long)T[t]);
        // saturated like the kernels' thresholds: 2^32 - 2 exceeds every statistic
        const uint64_t v = ((uint64_t)T[t] * (uint64_t)lnt[0]) >> 24;
        thrmax[t] = (uint32_t)std::min<uint64_t>(v, 0xFFFFFFFEull);
        tab.thr64[t] = (int64_t)v;
    }

    const int n = q->n, m = q->m, R = p.replicas;
    const int s = p.archive_size > 0 ? p.archive_size : m;
    std::memset(&d, 0, sizeof d);
    d.n = n;
    d.m = m;
    d.s = s;
    d.path = q->path;
    d.kform = q->kform;
    d.accept = p.accept;
    d.archive = p.archive;
    d.escape = p.escape;
    d.two_alpha1 = (int32_t)(2 * q->alpha[0]);
    d.two_alpha2 = (int32_t)(2 * q->alpha[1]);
    d.R = R;
    d.trace_R = p.trace_replicas;
    d.key0 = (uint32_t)p.seed;
    d.key1 = (uint32_t)(p.seed >> 32);
    d.steps = (uint32_t)p.steps;
    d.ntab = (uint32_t)T.size();
    d.beta = p.beta;
    d.q1 = q->q[0];
    d.q2 = q->q[1];
    d.f64 = q->f64;
    if (q->f64 && p.variant == MDA_VARIANT_PLAIN)
        return fail(MDA_EINVAL, "the plain form runs int32 energy differences only");
    // Layout of a replica over waves: one wave (n <= 64) or a workgroup of
    // wr x wc waves, wc = ceil(n / 64) location blocks and wr facility blocks of
    // gns = 8 ceil(ceil(n / wr) / 8) slots.
    {
        const int want = p.waves_per_replica;
        const int wc = (n + 63) / 64;
        if (want < 0 || want > 8) return fail(MDA_EINVAL, "waves_per_replica = %d outside [0, 8]", want);
        if (want == 1 && n > kMaxWaveN) return fail(MDA_EINVAL, "n = %d needs more than one wave per replica", n);
        if (q->f64 && want > 1)
            return fail(MDA_EINVAL, "int64 energy differences run one wave per replica (waves_per_replica = %d)", want);
        if ((want == 0 && n <= kMaxWaveN) || want == 1) {
            d.wr = d.wc = 1;
            d.gns = ns_for(n);
            d.xw = n;
            d.xrw = 64;
        } else {
            const int wr = want == 0 ? 2 : std::max(1, want / wc);
            const int per = (n + wr - 1) / wr;
            const int gns = ((per + 7) / 8) * 8;
            if (gns > 64 || wr * wc > group_waves_limit(gns) || wr * wc != (want == 0 ? 2 * wc : want))
                return fail(MDA_EINVAL, "no workgroup layout of %d waves for n = %d (%d location blocks)",
                            want == 0 ? 2 * wc : want, n, wc);
            if (p.variant == MDA_VARIANT_PLAIN) return fail(MDA_EINVAL, "the plain form runs one wave per replica");
            d.wr = wr;
            d.wc = wc;
            d.gns = gns;
            d.xw = wr * wc * 64;
            d.xrw = wr * wc * 64;
        }
    }
    d.ldk = q->ldk;
    d.pld = q->pld;
    d.KA1 = q->dKA1; d.KA2 = q->dKA2; d.KB1 = q->dKB1; d.KB2 = q->dKB2; d.DA = q->dDA; d.DB = q->dDB;
    d.P1 = q->dP1; d.P2 = q->dP2;
    d.diag1 = q->ddiag1; d.diag2 = q->ddiag2;
    d.ns_plain = ns_for(n);
    return MDA_OK;
}

static int prepare_run(mda_qubo *q, const mda_params *pin, hipStream_t stream, mda_run **out)
{
    std::unique_ptr<mda_run> r(new mda_run);
    RunTables tab;
    {
        const int rc = resolve_run(q, pin, r->p, r->h, tab);
        if (rc) return rc;
    }
    const std::vector<int64_t> &T = tab.T;
    const mda_params &p = r->p;
    RunDesc &d = r->h;
    const int m = q->m, R = p.replicas, s = d.s;
    DevPool &pool = r->pool;
    int64_t *dT = pool.alloc<int64_t>(T.size(), stream);
    uint32_t *dthr = pool.alloc<uint32_t>(T.size(), stream);
    int64_t *dthr64 = pool.alloc<int64_t>(T.size(), stream);
    d.x = pool.alloc<uint64_t>((size_t)R * d.xrw, stream);
    d.h = pool.alloc<int64_t>((size_t)R * 2 * m, stream);
    d.st = pool.alloc<int64_t>((size_t)R * kStWords, stream);
    d.archE = pool.alloc<int64_t>((size_t)R * s * 2, stream);
    d.archX = pool.alloc<uint64_t>((size_t)R * s * d.xw, stream);
    d.nd = pool.alloc<uint8_t>((size_t)R * s, stream);
    d.trace = pool.alloc<int32_t>((size_t)std::max(1, p.trace_replicas) * (size_t)(p.trace_replicas ? p.steps : 1), stream);
    if (p.variant == MDA_VARIANT_PLAIN) d.pe = pool.alloc<int32_t>((size_t)R * 2 * d.ns_plain * 64, stream);
    if (!dT || !dthr || !dthr64 || !d.x || !d.h || !d.st || !d.archE || !d.archX || !d.nd || !d.trace ||
        (p.variant == MDA_VARIANT_PLAIN && !d.pe))
        return fail(MDA_ENOMEM, "device allocation failed for the run (%lld bytes so far)", (long long)pool.total);
    HIP_TRY(hipMemcpyAsync(dT, T.data(), T.size() * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dthr, tab.thr32.data(), tab.thr32.size() * sizeof(uint32_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dthr64, tab.thr64.data(), tab.thr64.size() * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemsetAsync(d.nd, 0, (size_t)R * s, stream));
    d.T = dT;
    d.thrmax = dthr;
    d.thrmax64 = dthr64;
    q->refs++;
    r->q = q;
    *out = r.release();
    return MDA_OK;
}

// Threads per block: 1 to 4 waves (the kernels are built for at most 256).
static int default_block(int wpb)
{
    if (wpb <= 0) wpb = 4;
    if (wpb > 4) wpb = 4;
    return 64 * wpb;
}

namespace {

// One persistent launch: the work items [off, off + cnt) of one register tile,
// replica layout and field width, and (one wave per replica) step variant sv;
// the workgroup kernels take every variant (sv = -1).
struct Group {
    int ns, wr, wc, f64, sv, off, cnt;
};

// Work-item counters a launch holds: one per group (register tile, layout,
// field width and step variant; far fewer combinations occur).
constexpr int kMaxGroups = 128;

int group_variant(const RunDesc &d)
{
    return d.wr * d.wc == 1 ? run_step_variant(d.path, d.kform, d.accept) : -1;
}

// Work list of a launch: runs grouped by register tile, largest tile first
// (one persistent launch per tile, each with the occupancy of its own register
// budget); within a tile, largest instances first so that the items taken
// last, as waves become free, are the short ones.
void plan_work(const std::vector<RunDesc> &descs, std::vector<WorkItem> &work, std::vector<Group> &groups)
{
    const int count = (int)descs.size();
    // The 28- and 52-slot tiles pay only on their own: beside runs of 29 to
    // 32 (53 to 56) facilities of the same variant they would split that
    // launch in two (a longer tail), so runs of 25 to 28 (49 to 52)
    // facilities then join the 32-slot (56-slot) launch (the kernels read no
    // tile size from the descriptor).
    bool full[2][kStepVariants][2] = {};
    for (const RunDesc &d : descs)
        if (d.wr * d.wc == 1 && (d.gns == 32 || d.gns == 56)) full[d.f64 ? 1 : 0][group_variant(d)][d.gns == 56] = true;
    std::vector<int> tile(count);
    for (int i = 0; i < count; ++i) {
        const RunDesc &d = descs[i];
        const bool half = d.wr * d.wc == 1 && (d.gns == 28 || d.gns == 52);
        tile[i] = (half && full[d.f64 ? 1 : 0][group_variant(d)][d.gns == 52]) ? d.gns + 4 : d.gns;
    }
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const RunDesc &x = descs[a], &y = descs[b];
        if (x.wr * x.wc != y.wr * y.wc) return x.wr * x.wc > y.wr * y.wc;
        if (x.wc != y.wc) return x.wc > y.wc;
        if (x.f64 != y.f64) return x.f64 > y.f64;
        if (tile[a] != tile[b]) return tile[a] > tile[b];
        if (group_variant(x) != group_variant(y)) return group_variant(x) < group_variant(y);
        return (int64_t)x.m * x.steps > (int64_t)y.m * y.steps;
    });
    work.clear();
    groups.clear();
    for (int i : order) {
        const RunDesc &d = descs[i];
        const int sv = group_variant(d);
        if (groups.empty() || groups.back().ns != tile[i] || groups.back().wr != d.wr || groups.back().wc != d.wc ||
            groups.back().f64 != d.f64 || groups.back().sv != sv)
            groups.push_back(Group{tile[i], d.wr, d.wc, d.f64, sv, (int)work.size(), 0});
        for (int rr = 0; rr < d.R; ++rr) work.push_back(WorkItem{i, rr});
        groups.back().cnt += d.R;
    }
}

// Enqueues the annealing kernel(s) of a planned launch on stream: the plain
// form (one launch per step), or one persistent launch per group.  ddesc,
// dwork and dlnt are the device copies of the descriptors, the work list and
// the -ln table; cus is the device's compute-unit count.
int enqueue_anneal(const std::vector<Group> &groups, const RunDesc &first, bool plain, const RunDesc *ddesc,
                   const WorkItem *dwork, const int32_t *dlnt, unsigned int *dctr, int block, int cus,
                   hipStream_t stream, int occ_req = 0, const std::vector<hipStream_t> *side = nullptr,
                   hipEvent_t fork = nullptr, const std::vector<hipEvent_t> *join = nullptr)
{
    if (!plain && groups.size() > kMaxGroups)
        return fail(MDA_EINVAL, "%zu register tiles in one launch (at most %d)", groups.size(), kMaxGroups);
    int gi = 0;
    if (plain) {
        HIP_TRY(launch_plain(groups[0].ns, run_step_variant(first.path, first.kform, first.accept), ddesc, first.R,
                             first.steps, dlnt, block, stream));
        return MDA_OK;
    }
    // Several groups: group k goes to stream k mod (1 + side streams), so
    // that one group's tail overlaps the next group's work; the side streams
    // start after everything enqueued on stream so far and stream continues
    // after all of them (in a captured graph: parallel branches).
    const bool fan = side && !side->empty() && fork && join && join->size() == side->size() && groups.size() > 1;
    const int nstreams = fan ? 1 + (int)side->size() : 1;
    if (fan) {
        HIP_TRY(hipEventRecord(fork, stream));
        for (hipStream_t st : *side) HIP_TRY(hipStreamWaitEvent(st, fork, 0));
    }
    for (const Group &g : groups) {
        const hipStream_t gs = (gi % nstreams == 0) ? stream : (*side)[gi % nstreams - 1];
        int per_cu = 0;
        if (g.wr * g.wc == 1) {
            // one wave per SIMD when that holds every replica of the launch
            // at once, the two-wave build when more are waiting
            const int wpb = block / 64;
            HIP_TRY(persistent_occupancy(g.ns, 1, g.f64, g.sv, block, &per_cu));
            if (per_cu < 1) per_cu = 1;
            // (the int64 build has one register budget only); occ_req 1 or 2
            // overrides the rule
            int occ = !g.f64 && (int64_t)g.cnt > (int64_t)cus * per_cu * wpb ? 2 : 1;
            if (occ_req == 1 || occ_req == 2) occ = g.f64 ? 1 : occ_req;
            if (occ == 2) {
                HIP_TRY(persistent_occupancy(g.ns, 2, 0, g.sv, block, &per_cu));
                if (per_cu < 1) per_cu = 1;
            }
            int grid = cus * per_cu;
            const int need = (g.cnt + wpb - 1) / wpb;
            if (grid > need) grid = need;
            const hipError_t le = launch_persistent(g.ns, occ, g.f64, g.sv, ddesc, dwork + g.off, g.cnt, dlnt,
                                                    dctr + gi, grid, block, gs);
            if (le != hipSuccess)
                return fail(MDA_EDEVICE, "persistent launch (ns %d, grid %d, block %d, %d blocks/CU) failed: %s", g.ns,
                            grid, block, per_cu, hipGetErrorString(le));
        } else {
            // one replica per workgroup of wr x wc waves; the two-workgroups-per-CU
            // build when one per CU cannot hold every replica at once
            HIP_TRY(group_occupancy(g.ns, 1, g.wr, g.wc, &per_cu));
            if (per_cu < 1) per_cu = 1;
            const int occ = (int64_t)g.cnt > (int64_t)cus * per_cu ? 2 : 1;
            if (occ == 2) {
                HIP_TRY(group_occupancy(g.ns, 2, g.wr, g.wc, &per_cu));
                if (per_cu < 1) per_cu = 1;
            }
            int grid = cus * per_cu;
            if (grid > g.cnt) grid = g.cnt;
            const hipError_t le = launch_group(g.ns, occ, g.wr, g.wc, ddesc, dwork + g.off, g.cnt, dlnt, grid, gs);
            if (le != hipSuccess)
                return fail(MDA_EDEVICE, "workgroup launch (ns %d, %d x %d waves, grid %d, %d blocks/CU) failed: %s",
                            g.ns, g.wr, g.wc, grid, per_cu, hipGetErrorString(le));
        }
        ++gi;
    }
    if (fan) {
        for (size_t k = 0; k < side->size(); ++k) {
            HIP_TRY(hipEventRecord((*join)[k], (*side)[k]));
            HIP_TRY(hipStreamWaitEvent(stream, (*join)[k], 0));
        }
    }
    return MDA_OK;
}

}  // namespace

extern "C" int da_run_batch(const mda_qubo *const *qs, const mda_params *ps, int32_t count, mda_run **outs)
{
    if (!qs || !ps || !outs || count < 1) return fail(MDA_EINVAL, "bad batch arguments");
    for (int i = 0; i < count; ++i) outs[i] = nullptr;
    hipStream_t stream = (hipStream_t)ps[0].stream;
    {
        // an error left by earlier asynchronous work is reported as such
        const hipError_t pending = hipGetLastError();
        if (pending != hipSuccess)
            return fail(MDA_EDEVICE, "pending device error before the launch: %s", hipGetErrorString(pending));
    }
    const bool plain = ps[0].variant == MDA_VARIANT_PLAIN;
    if (plain && count != 1) return fail(MDA_EINVAL, "the plain form runs one instance per call");
    if (plain && ps[0].graph) return fail(MDA_EINVAL, "the plain form is launched step by step, not as a graph");
    std::vector<std::unique_ptr<mda_run>> runs;
    for (int i = 0; i < count; ++i) {
        if (!qs[i]) return fail(MDA_EINVAL, "qubo %d is NULL", i);
        if (ps[i].stream != ps[0].stream) return fail(MDA_EINVAL, "all runs of a batch share one stream");
        if ((ps[i].variant == MDA_VARIANT_PLAIN) != plain) return fail(MDA_EINVAL, "mixed variants in a batch");
        if ((ps[i].graph != 0) != (ps[0].graph != 0)) return fail(MDA_EINVAL, "mixed graph settings in a batch");
        mda_run *r = nullptr;
        const int rc = prepare_run(const_cast<mda_qubo *>(qs[i]), &ps[i], stream, &r);
        if (rc) return rc;
        runs.emplace_back(r);
    }
    auto L = std::make_shared<Launch>();
    L->stream = stream;
    const bool graph = ps[0].graph != 0;
    if (graph && !stream) return fail(MDA_EINVAL, "graph launches need a created stream, not the default one");
    std::vector<RunDesc> descs;
    for (int i = 0; i < count; ++i) descs.push_back(runs[i]->h);
    std::vector<Group> groups;
    std::vector<WorkItem> work;
    plan_work(descs, work, groups);
    if (plain && groups.size() != 1) return fail(MDA_EINVAL, "the plain form runs one instance per call");
    L->nwork = (int)work.size();
    L->ddesc = L->pool.alloc<RunDesc>(descs.size(), stream);
    L->dwork = L->pool.alloc<WorkItem>(work.size(), stream);
    L->dlnt = L->pool.alloc<int32_t>(4096, stream);
    L->dctr = L->pool.alloc<unsigned int>(kMaxGroups, stream);
    if (!L->ddesc || !L->dwork || !L->dlnt || !L->dctr) return fail(MDA_ENOMEM, "device allocation failed");
    if (!plain && groups.size() > 1) {
        // up to three more streams (four hardware queues per process)
        const size_t nside = std::min<size_t>(3, groups.size() - 1);
        HIP_TRY(hipEventCreateWithFlags(&L->fork, hipEventDisableTiming));
        for (size_t k = 0; k < nside; ++k) {
            hipStream_t st = nullptr;
            HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            L->side.push_back(st);
            hipEvent_t e = nullptr;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            L->join.push_back(e);
        }
    }
    int32_t lnt[4096];
    threshold_table(lnt);
    HIP_TRY(hipMemcpyAsync(L->ddesc, descs.data(), descs.size() * sizeof(RunDesc), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(L->dwork, work.data(), work.size() * sizeof(WorkItem), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(L->dlnt, lnt, sizeof lnt, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventCreate(&L->ev0));
    HIP_TRY(hipEventCreate(&L->ev1));
    HIP_TRY(hipEventCreate(&L->evk0));
    HIP_TRY(hipEventCreate(&L->evk1));
    const int block = default_block(ps[0].waves_per_block);
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));

    // The launch sequence: the annealing kernel(s), then the non-dominated
    // flags.  Either enqueued directly or captured into one graph.
    auto enqueue = [&](bool timed) -> int {
        if (timed) HIP_TRY(hipEventRecord(L->evk0, stream));
        const int rc = enqueue_anneal(groups, descs[0], plain, L->ddesc, L->dwork, L->dlnt, L->dctr, block, cus,
                                      stream, ps[0].occupancy, &L->side, L->fork, &L->join);
        if (rc) return rc;
        if (timed) HIP_TRY(hipEventRecord(L->evk1, stream));
        HIP_TRY(launch_nondominated(L->ddesc, L->dwork, L->nwork, stream));
        return MDA_OK;
    };
    HIP_TRY(hipEventRecord(L->ev0, stream));
    if (graph) {
        // captured on the caller's stream; no memset or event inside the graph
        HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue(false);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (ce != hipSuccess) return fail(MDA_EDEVICE, "graph capture failed: %s", hipGetErrorString(ce));
        L->graph = g;
        HIP_TRY(hipGraphInstantiate(&L->graph_exec, g, nullptr, nullptr, 0));
        HIP_TRY(hipEventRecord(L->evk0, stream));
        HIP_TRY(hipGraphLaunch(L->graph_exec, stream));
        HIP_TRY(hipEventRecord(L->evk1, stream));
    } else {
        const int rc = enqueue(true);
        if (rc) return rc;
    }
    HIP_TRY(hipEventRecord(L->ev1, stream));
    for (int i = 0; i < count; ++i) {
        runs[i]->launch = L;
        outs[i] = runs[i].release();
    }
    return MDA_OK;
}

extern "C" int da_run(const mda_qubo *q, const mda_params *p, mda_run **out)
{
    if (!out) return fail(MDA_EINVAL, "out is NULL");
    if (!q || !p) return fail(MDA_EINVAL, "NULL argument");
    return da_run_batch(&q, p, 1, out);
}

extern "C" int da_sync(mda_run *r)
{
    if (!r || !r->launch) return fail(MDA_EINVAL, "NULL run");
    HIP_TRY(hipStreamSynchronize(r->launch->stream));
    return MDA_OK;
}

extern "C" int da_elapsed_ms(mda_run *r, double *ms)
{
    if (!r || !r->launch || !ms) return fail(MDA_EINVAL, "NULL argument");
    HIP_TRY(hipEventSynchronize(r->launch->ev1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, r->launch->ev0, r->launch->ev1));
    *ms = f;
    return MDA_OK;
}

extern "C" int da_kernel_ms(mda_run *r, double *ms)
{
    if (!r || !r->launch || !ms) return fail(MDA_EINVAL, "NULL argument");
    HIP_TRY(hipEventSynchronize(r->launch->evk1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, r->launch->evk0, r->launch->evk1));
    *ms = f;
    return MDA_OK;
}

extern "C" void da_run_free(mda_run *r)
{
    delete r;
}

// ---------------------------------------------------------------- runs without allocation

namespace {

// The scratch area of da_run_noalloc: run descriptor, work list, -ln table and
// temperature tables of the latest call on this device.  Each device holds its
// own copy; host code only ever uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[MDA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch area, looked up once per
// device with that device current.
int scratch_address(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MDA_EDEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MDA_EDEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MDA_OK;
}

size_t align256(size_t b)
{
    return (b + 255) & ~(size_t)255;
}

// Byte offsets of the parts of the scratch area for R work items and ntab
// table entries; returns the total.
struct ScratchPlan {
    size_t desc, ctr, work, lnt, T, thr, thr64, total;
};

ScratchPlan scratch_plan(int64_t R, int64_t ntab)
{
    ScratchPlan sp;
    sp.desc = 0;
    sp.ctr = sp.desc + align256(sizeof(RunDesc));
    sp.work = sp.ctr + align256(kMaxGroups * sizeof(unsigned int));
    sp.lnt = sp.work + align256((size_t)R * sizeof(WorkItem));
    sp.T = sp.lnt + align256(4096 * sizeof(int32_t));
    sp.thr = sp.T + align256((size_t)ntab * sizeof(int64_t));
    sp.thr64 = sp.thr + align256((size_t)ntab * sizeof(uint32_t));
    sp.total = sp.thr64 + align256((size_t)ntab * sizeof(int64_t));
    return sp;
}

int fill_layout(const mda_params &p, const RunDesc &d, int64_t ntab, mda_run_layout *out)
{
    std::memset(out, 0, sizeof *out);
    const int64_t R = d.R, s = d.s, m = d.m;
    out->n = d.n;
    out->m = d.m;
    out->replicas = d.R;
    out->archive_size = d.s;
    out->steps = p.steps;
    out->trace_replicas = p.trace_replicas;
    out->wr = d.wr;
    out->wc = d.wc;
    out->gns = d.gns;
    out->x_words = d.xrw;
    out->arch_x_words = d.xw;
    out->n_x = R * d.xrw;
    out->n_h = R * 2 * m;
    out->n_st = R * kStWords;
    out->n_arch_e = R * s * 2;
    out->n_arch_x = R * s * d.xw;
    out->n_nd = R * s;
    out->n_trace = (int64_t)p.trace_replicas * p.steps;
    out->scratch_bytes = (int64_t)scratch_plan(R, ntab).total;
    if (out->scratch_bytes > MDA_NOALLOC_SCRATCH_BYTES)
        return fail(MDA_ERANGE, "the run needs %lld bytes of scratch (%d work items, %lld table entries); the "
                                "limit is %lld", (long long)out->scratch_bytes, d.R, (long long)ntab,
                    (long long)MDA_NOALLOC_SCRATCH_BYTES);
    return MDA_OK;
}

}  // namespace

extern "C" int da_run_layout(const mda_qubo *q, const mda_params *pin, mda_run_layout *out)
{
    if (!q || !pin || !out) return fail(MDA_EINVAL, "NULL argument");
    mda_params p;
    RunDesc d;
    RunTables tab;
    const int rc = resolve_run(q, pin, p, d, tab);
    if (rc) return rc;
    return fill_layout(p, d, (int64_t)tab.T.size(), out);
}

extern "C" int da_run_noalloc(const mda_qubo *q, const mda_params *pin, const mda_run_buffers *b)
{
    if (!q || !pin || !b) return fail(MDA_EINVAL, "NULL argument");
    if (pin->variant == MDA_VARIANT_PLAIN) return fail(MDA_EINVAL, "da_run_noalloc runs the persistent form only");
    if (pin->graph) return fail(MDA_EINVAL, "da_run_noalloc launches directly (graph must be 0)");
    if (!b->x || !b->h || !b->st || !b->arch_e || !b->arch_x || !b->nd)
        return fail(MDA_EINVAL, "a result buffer is NULL");
    if (pin->trace_replicas > 0 && !b->trace) return fail(MDA_EINVAL, "trace_replicas > 0 needs a trace buffer");
    hipStream_t stream = (hipStream_t)pin->stream;
    {
        const hipError_t pending = hipGetLastError();
        if (pending != hipSuccess)
            return fail(MDA_EDEVICE, "pending device error before the launch: %s", hipGetErrorString(pending));
    }
    mda_params p;
    RunDesc d;
    RunTables tab;
    int rc = resolve_run(q, pin, p, d, tab);
    if (rc) return rc;
    const std::vector<int64_t> &T = tab.T;
    mda_run_layout lay;
    rc = fill_layout(p, d, (int64_t)T.size(), &lay);
    if (rc) return rc;
    void *base = nullptr;
    rc = scratch_address(&base);
    if (rc) return rc;
    const ScratchPlan sp = scratch_plan(d.R, (int64_t)T.size());
    uint8_t *sb = static_cast<uint8_t *>(base);
    RunDesc *ddesc = reinterpret_cast<RunDesc *>(sb + sp.desc);
    WorkItem *dwork = reinterpret_cast<WorkItem *>(sb + sp.work);
    int32_t *dlnt = reinterpret_cast<int32_t *>(sb + sp.lnt);
    d.T = reinterpret_cast<const int64_t *>(sb + sp.T);
    d.thrmax = reinterpret_cast<const uint32_t *>(sb + sp.thr);
    d.thrmax64 = reinterpret_cast<const int64_t *>(sb + sp.thr64);
    d.x = b->x;
    d.h = b->h;
    d.st = b->st;
    d.archE = b->arch_e;
    d.archX = b->arch_x;
    d.nd = b->nd;
    d.trace = b->trace;
    d.pe = nullptr;
    std::vector<RunDesc> descs(1, d);
    std::vector<Group> groups;
    std::vector<WorkItem> work;
    plan_work(descs, work, groups);
    int32_t lnt[4096];
    threshold_table(lnt);
    // every part of the scratch area the kernels read is written here
    HIP_TRY(hipMemcpyAsync(ddesc, descs.data(), sizeof(RunDesc), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dwork, work.data(), work.size() * sizeof(WorkItem), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dlnt, lnt, sizeof lnt, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(sb + sp.T, T.data(), T.size() * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(sb + sp.thr, tab.thr32.data(), tab.thr32.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(hipMemcpyAsync(sb + sp.thr64, tab.thr64.data(), tab.thr64.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                           stream));
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    rc = enqueue_anneal(groups, d, false, ddesc, dwork, dlnt, reinterpret_cast<unsigned int *>(sb + sp.ctr),
                        default_block(p.waves_per_block), cus, stream, p.occupancy);
    if (rc) return rc;
    HIP_TRY(launch_nondominated(ddesc, dwork, (int)work.size(), stream));
    return MDA_OK;
}

// ---------------------------------------------------------------- readout

// Bit x_{i,u} of a stored solution (a row of x or an archive entry) in the run's
// layout over waves.
static inline bool sol_bit(const RunDesc &d, const uint64_t *words, int i, int u)
{
    if (d.wr * d.wc == 1) return (words[u] >> i) & 1ull;
    const int p = i / d.gns, c = u / 64;
    return (words[(size_t)(p * d.wc + c) * 64 + (u % 64)] >> (i - p * d.gns)) & 1ull;
}

static int copy_d2h(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MDA_OK;
}

extern "C" int da_params_get(const mda_run *r, mda_params *out)
{
    if (!r || !out) return fail(MDA_EINVAL, "NULL argument");
    *out = r->p;
    out->archive_size = r->h.s;
    out->waves_per_replica = r->h.wr * r->h.wc;
    return MDA_OK;
}

extern "C" int da_stats(mda_run *r, int64_t *moves, int64_t *scanned, int64_t *rng_blocks, int64_t *archived)
{
    if (!r) return fail(MDA_EINVAL, "NULL run");
    const RunDesc &d = r->h;
    std::vector<int64_t> st((size_t)d.R * kStWords);
    int rc = copy_d2h(st.data(), d.st, st.size() * sizeof(int64_t), r->launch->stream);
    if (rc) return rc;
    int64_t mv = 0, sc = 0, rb = 0, ar = 0;
    for (int i = 0; i < d.R; ++i) {
        mv += st[(size_t)i * kStWords + kStMoves];
        sc += st[(size_t)i * kStWords + kStScanned];
        rb += st[(size_t)i * kStWords + kStRng];
        ar += st[(size_t)i * kStWords + kStArch];
    }
    if (moves) *moves = mv;
    if (scanned) *scanned = sc;
    if (rng_blocks) *rng_blocks = rb;
    if (archived) *archived = ar;
    return MDA_OK;
}

extern "C" int da_state_get(mda_run *r, int32_t replica, mda_state *out)
{
    if (!r || !out) return fail(MDA_EINVAL, "NULL argument");
    const RunDesc &d = r->h;
    if (replica < 0 || replica >= d.R) return fail(MDA_EINVAL, "replica %d outside [0, %d)", replica, d.R);
    hipStream_t s = r->launch->stream;
    int64_t st[kStWords];
    int rc = copy_d2h(st, d.st + (size_t)replica * kStWords, sizeof st, s);
    if (rc) return rc;
    out->e1 = st[kStE1];
    out->e2 = st[kStE2];
    out->e_offset = st[kStEoff];
    out->moves = st[kStMoves];
    out->scanned = st[kStScanned];
    out->rng_blocks = st[kStRng];
    const int n = d.n, m = d.m;
    if (out->x) {
        std::vector<uint64_t> words((size_t)d.xrw);
        rc = copy_d2h(words.data(), d.x + (size_t)replica * d.xrw, words.size() * 8, s);
        if (rc) return rc;
        for (int i = 0; i < n; ++i)
            for (int u = 0; u < n; ++u) out->x[i * n + u] = sol_bit(d, words.data(), i, u) ? 1 : 0;
    }
    if (out->h1 && (rc = copy_d2h(out->h1, d.h + (size_t)replica * 2 * m, (size_t)m * 8, s))) return rc;
    if (out->h2 && (rc = copy_d2h(out->h2, d.h + (size_t)replica * 2 * m + m, (size_t)m * 8, s))) return rc;
    if (out->trace) {
        if (replica >= d.trace_R) return fail(MDA_EINVAL, "replica %d was not traced", replica);
        rc = copy_d2h(out->trace, d.trace + (size_t)replica * d.steps, (size_t)d.steps * 4, s);
        if (rc) return rc;
    }
    return MDA_OK;
}

namespace {

struct TmpPool {
    DevPool pool;
    ~TmpPool() { pool.release_all(); }
};

}  // namespace

// Flagged (non-dominated within their archive) entries of replicas
// [r0, r0 + nr), compacted on the device and copied back; st holds those
// replicas' statistics blocks.
static int gather_flagged(mda_run *r, int r0, int nr, const std::vector<int64_t> &st, std::vector<FrontEntry> &ent)
{
    const RunDesc &d = r->h;
    hipStream_t s = r->launch->stream;
    std::vector<int64_t> offs((size_t)nr);
    int64_t total = 0;
    for (int k = 0; k < nr; ++k) {
        offs[k] = total;
        total += std::max<int64_t>(0, st[(size_t)k * kStWords + kStNd]);
    }
    ent.clear();
    if (total == 0) return MDA_OK;
    TmpPool tmp;
    int64_t *doffs = tmp.pool.alloc<int64_t>((size_t)nr, s);
    FrontEntry *dout = tmp.pool.alloc<FrontEntry>((size_t)total, s);
    if (!doffs || !dout) return fail(MDA_ENOMEM, "device allocation failed for %lld front entries", (long long)total);
    HIP_TRY(hipMemcpyAsync(doffs, offs.data(), offs.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_front_gather(d.archE, d.nd, d.st, d.s, r0, nr, doffs, dout, s));
    if (total < 4096) {
        ent.resize((size_t)total);
        return copy_d2h(ent.data(), dout, ent.size() * sizeof(FrontEntry), s);
    }
    // many candidates: drop on the device those that an entry of strictly
    // smaller E1 dominates, copy the rest
    void *scratch = tmp.pool.alloc<char>(front_filter_scratch(), s);
    FrontEntry *dkeep = tmp.pool.alloc<FrontEntry>((size_t)total, s);
    unsigned long long *dn = tmp.pool.alloc<unsigned long long>(1, s);
    if (!scratch || !dkeep || !dn) return fail(MDA_ENOMEM, "device allocation failed for the front filter");
    HIP_TRY(launch_front_filter(dout, total, scratch, dkeep, dn, s));
    unsigned long long kept = 0;
    int rc = copy_d2h(&kept, dn, sizeof kept, s);
    if (rc) return rc;
    if ((int64_t)kept > total) return fail(MDA_EDEVICE, "front filter kept %llu of %lld", kept, (long long)total);
    ent.resize((size_t)kept);
    if (kept == 0) return MDA_OK;
    return copy_d2h(ent.data(), dkeep, ent.size() * sizeof(FrontEntry), s);
}

extern "C" int archive_get(mda_run *r, int32_t replica, int32_t raw, mda_archive_out *out, int64_t *count)
{
    if (!r || !count) return fail(MDA_EINVAL, "NULL argument");
    const RunDesc &d = r->h;
    if (replica < -1 || replica >= d.R) return fail(MDA_EINVAL, "replica %d outside [-1, %d)", replica, d.R);
    if (raw && replica < 0) return fail(MDA_EINVAL, "the raw archive is per replica");
    hipStream_t s = r->launch->stream;
    const int n = d.n, m = d.m, S = d.s;
    const int r0 = replica < 0 ? 0 : replica, r1 = replica < 0 ? d.R : replica + 1;
    const int nr = r1 - r0;
    int rc = MDA_OK;

    std::vector<FrontEntry> local;
    const std::vector<FrontEntry> *src = &local;
    if (replica < 0 && r->merged_ok) {
        src = &r->merged;
    } else {
        std::vector<int64_t> st((size_t)nr * kStWords);
        rc = copy_d2h(st.data(), d.st + (size_t)r0 * kStWords, st.size() * sizeof(int64_t), s);
        if (rc) return rc;
        if (raw) {
            // the ordered archive of one replica as stored
            const int asz = (int)std::min<int64_t>(std::max<int64_t>(0, st[kStArch]), S);
            std::vector<int64_t> E((size_t)asz * 2);
            if (asz && (rc = copy_d2h(E.data(), d.archE + (size_t)replica * S * 2, E.size() * sizeof(int64_t), s)))
                return rc;
            for (int e = 0; e < asz; ++e) local.push_back(FrontEntry{E[2 * (size_t)e], E[2 * (size_t)e + 1], replica, e});
        } else {
            rc = gather_flagged(r, r0, nr, st, local);
            if (rc) return rc;
            // Non-dominated union (Sec. 3.3): sort by (E1, E2, replica, slot) and keep
            // the strictly decreasing E2 staircase, so equal points reduce to the
            // lowest (replica, slot).
            std::sort(local.begin(), local.end(), [](const FrontEntry &a, const FrontEntry &b) {
                if (a.e1 != b.e1) return a.e1 < b.e1;
                if (a.e2 != b.e2) return a.e2 < b.e2;
                if (a.replica != b.replica) return a.replica < b.replica;
                return a.slot < b.slot;
            });
            std::vector<FrontEntry> keep;
            int64_t best2 = INT64_MAX;
            for (const FrontEntry &e : local) {
                if (e.e2 < best2) {
                    keep.push_back(e);
                    best2 = e.e2;
                }
            }
            local.swap(keep);
            if (replica < 0) {
                r->merged = local;
                r->merged_ok = true;
            }
        }
    }
    const std::vector<FrontEntry> &ent = *src;
    *count = (int64_t)ent.size();
    if (!out) return MDA_OK;
    if (out->cap < (int64_t)ent.size()) return fail(MDA_ERANGE, "capacity %lld < %lld entries", (long long)out->cap, (long long)ent.size());
    const size_t k_n = ent.size();
    const size_t xw = (size_t)d.xw;
    std::vector<uint64_t> cols;
    if (out->xbits || out->perm || out->feasible) {
        // stored solutions of every returned entry: one contiguous copy for a
        // raw archive, one copy per entry otherwise, then a single wait
        cols.resize(k_n * xw);
        if (raw) {
            if (k_n) HIP_TRY(hipMemcpyAsync(cols.data(), d.archX + (size_t)replica * S * xw, cols.size() * 8, hipMemcpyDeviceToHost, s));
        } else {
            for (size_t k = 0; k < k_n; ++k)
                HIP_TRY(hipMemcpyAsync(cols.data() + k * xw, d.archX + ((size_t)ent[k].replica * S + ent[k].slot) * xw,
                                       xw * 8, hipMemcpyDeviceToHost, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
    }
    const int words = (m + 31) / 32;
    std::vector<int> perm(n), colsum(n);
    for (size_t k = 0; k < k_n; ++k) {
        const FrontEntry &e = ent[k];
        if (out->e1) out->e1[k] = e.e1;
        if (out->e2) out->e2[k] = e.e2;
        if (out->replica) out->replica[k] = e.replica;
        if (out->slot) out->slot[k] = e.slot;
        if (cols.empty()) continue;
        const uint64_t *c = cols.data() + k * xw;
        bool feas = true;
        std::fill(perm.begin(), perm.end(), -1);
        std::fill(colsum.begin(), colsum.end(), 0);
        for (int i = 0; i < n; ++i) {
            int cnt = 0;
            for (int u = 0; u < n; ++u) {
                if (sol_bit(d, c, i, u)) {
                    ++cnt;
                    ++colsum[u];
                    perm[i] = u;
                }
            }
            if (cnt != 1) feas = false;
        }
        for (int u = 0; u < n; ++u)
            if (colsum[u] != 1) feas = false;
        if (out->feasible) out->feasible[k] = feas ? 1 : 0;
        if (out->perm)
            for (int i = 0; i < n; ++i) out->perm[k * n + i] = feas ? perm[i] : -1;
        if (out->xbits) {
            uint32_t *w = out->xbits + k * words;
            std::memset(w, 0, (size_t)words * 4);
            for (int i = 0; i < n; ++i)
                for (int u = 0; u < n; ++u)
                    if (sol_bit(d, c, i, u)) {
                        const int a = i * n + u;
                        w[a >> 5] |= 1u << (a & 31);
                    }
        }
    }
    return MDA_OK;
}

// ---------------------------------------------------------------- internal (serving engine)

namespace mda {

void set_stream_ordered_alloc(bool on)
{
    tl_stream_ordered = on;
}

int run_finished(mda_run *r)
{
    if (!r || !r->launch || !r->launch->ev1) return -1;
    const hipError_t e = hipEventQuery(r->launch->ev1);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return -1;
}

int set_error(int code, const char *msg)
{
    return fail(code, "%s", msg);
}

int64_t qubo_device_bytes(const mda_qubo *q)
{
    return q->pool.total;
}

void set_release_hook(mda_run *r, std::function<void()> hook)
{
    r->on_release = std::move(hook);
}

}  // namespace mda

extern "C" int64_t mda_footprint(int32_t n, const mda_params *p, const mda_build_opts *bo)
{
    if (n < 2 || n > 100 || !p) return fail(MDA_EINVAL, "bad footprint query");
    const int64_t m = (int64_t)n * n;
    const int64_t R = p->replicas > 0 ? p->replicas : 1;
    const int64_t s = p->archive_size > 0 ? p->archive_size : m;
    const int64_t steps = p->steps > 0 ? p->steps : (int64_t)std::llround(0.25 * (double)m * (double)m);
    const int wc = (n + 63) / 64;
    const bool group = p->waves_per_replica > 1 || (p->waves_per_replica == 0 && n > kMaxWaveN);
    const int G = group ? (p->waves_per_replica > 1 ? p->waves_per_replica : 2 * wc) : 1;
    const int64_t xw = group ? (int64_t)G * 64 : n, xrw = group ? (int64_t)G * 64 : 64;
    // run: x, fields, statistics, archive energies, solutions and flags, tables, trace
    int64_t b = R * (xrw * 8 + 2 * m * 8 + kStWords * 8) + R * s * (16 + xw * 8 + 1);
    b += steps * 20 + 65536;
    if (p->trace_replicas > 0) b += (int64_t)p->trace_replicas * steps * 4;
    // QUBO: dense rows when the build will pick them, the per-lane operands
    const mda_build_opts o = bo ? *bo : mda_build_opts{MDA_PEN_2MAX, MDA_PATH_AUTO, 0};
    const int64_t budget = o.dense_budget > 0 ? o.dense_budget : 0;
    const int64_t pld = n, ldk = n <= kMaxWaveN ? kLD : 2 * kLD;
    const int64_t dense = 8 * m * n * pld;
    const bool use_dense = o.path == MDA_PATH_DENSE || (o.path == MDA_PATH_AUTO && dense <= budget);
    b += (use_dense ? dense + 3 * m * 4 : 0) + 6 * (int64_t)n * ldk * 4 + 2 * std::max<int64_t>(n, kMaxWaveN) * ldk * 4;
    return b;
}

// ---------------------------------------------------------------- autotuner

namespace {

struct TuneKey {
    int32_t n, path, kform, accept, rbucket, f64;
    bool operator<(const TuneKey &o) const
    {
        if (f64 != o.f64) return f64 < o.f64;
        if (n != o.n) return n < o.n;
        if (path != o.path) return path < o.path;
        if (kform != o.kform) return kform < o.kform;
        if (accept != o.accept) return accept < o.accept;
        return rbucket < o.rbucket;
    }
};

std::mutex g_tune_mu;
std::map<TuneKey, mda_tuning> g_tune_cache;

}  // namespace

extern "C" int mda_autotune(const mda_qubo *q, const mda_params *pin, int64_t probe_steps, int32_t probe_replicas,
                            mda_tuning *out)
{
    if (!q || !pin || !out) return fail(MDA_EINVAL, "NULL argument");
    if (probe_steps < 1) probe_steps = 2000;
    const int n = q->n;
    int32_t R = pin->replicas;
    if (probe_replicas > 0 && probe_replicas < R) R = probe_replicas;
    int rb = 0;
    while ((1 << (rb + 1)) <= pin->replicas && rb < 30) ++rb;
    const TuneKey key{n, q->path, q->kform, pin->accept, rb, q->f64};
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second;
            out->cached = 1;
            return MDA_OK;
        }
    }
    std::memset(out, 0, sizeof *out);
    // candidates: one wave per replica (n <= 64) with 1, 2, 4 waves per block,
    // each with the one- and (from 32 slots, int32 differences) the
    // two-waves-per-SIMD build; workgroups of 2 and 4 waves where a layout
    // exists (their build by the host rule)
    struct Cand {
        int wpr, wpb, occ;
    };
    std::vector<Cand> cand;
    if (n <= kMaxWaveN)
        for (int wpb : {1, 2, 4}) {
            cand.push_back({1, wpb, 1});
            if (!q->f64 && ns_for(n) >= 32) cand.push_back({1, wpb, 2});
        }
    const int wc = (n + 63) / 64;
    for (int g : {2, 4}) {
        if (q->f64) break;   // int64 differences run one wave per replica
        const int wr = std::max(1, g / wc);
        if (wr * wc != g) continue;
        const int gns = (((n + wr - 1) / wr + 7) / 8) * 8;
        if (gns > 64 || g > group_waves_limit(gns)) continue;
        cand.push_back({g, 0, 0});
    }
    if (cand.size() > 16) cand.resize(16);
    mda_params p = *pin;
    p.replicas = R;
    p.steps = probe_steps;
    p.trace_replicas = 0;
    p.graph = 0;
    p.variant = MDA_VARIANT_PERSISTENT;
    // a first launch loads the code objects; it is not timed
    for (int pass = 0; pass < 2; ++pass) {
        for (size_t c = 0; c < cand.size(); ++c) {
            p.waves_per_replica = cand[c].wpr;
            p.waves_per_block = cand[c].wpb;
            p.occupancy = cand[c].occ;
            mda_run *r = nullptr;
            int rc = da_run(q, &p, &r);
            if (rc) return rc;
            double ms = 0;
            rc = da_kernel_ms(r, &ms);
            da_run_free(r);
            if (rc) return rc;
            if (pass == 1) {
                out->cand_wpr[c] = cand[c].wpr;
                out->cand_wpb[c] = cand[c].wpb;
                out->cand_occ[c] = cand[c].occ;
                out->probe_ms[c] = ms;
            }
            if (pass == 0) break;   // one warm-up launch is enough
        }
    }
    out->candidates = (int32_t)cand.size();
    int best = 0;
    for (int c = 1; c < out->candidates; ++c)
        if (out->probe_ms[c] < out->probe_ms[best]) best = c;
    out->waves_per_replica = out->cand_wpr[best];
    out->waves_per_block = out->cand_wpb[best];
    out->occupancy = out->cand_occ[best];
    out->best_ms = out->probe_ms[best];
    out->probe_steps = probe_steps;
    out->probe_replicas = R;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[key] = *out;
    return MDA_OK;
}

extern "C" int da_best(mda_run *r, int64_t *e1, int32_t *slot)
{
    if (!r || !e1 || !slot) return fail(MDA_EINVAL, "NULL argument");
    const RunDesc &d = r->h;
    hipStream_t s = r->launch->stream;
    TmpPool tmp;
    RunDesc *dd = tmp.pool.alloc<RunDesc>(1, s);
    int64_t *de = tmp.pool.alloc<int64_t>((size_t)d.R, s);
    int32_t *ds = tmp.pool.alloc<int32_t>((size_t)d.R, s);
    if (!dd || !de || !ds) return fail(MDA_ENOMEM, "device allocation failed for %d replicas", d.R);
    HIP_TRY(hipMemcpyAsync(dd, &d, sizeof d, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_best(dd, d.R, de, ds, s));
    int rc = copy_d2h(e1, de, (size_t)d.R * sizeof(int64_t), s);
    if (rc) return rc;
    return copy_d2h(slot, ds, (size_t)d.R * sizeof(int32_t), s);
}
