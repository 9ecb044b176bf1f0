// mda_generic_host.cpp -- C ABI of the K-objective annealer on a generic QUBO
// (declared and documented in include/mda.h): the symmetric rows of the K
// objectives on the device, run resolution, the persistent launch and the
// readout of states and archives.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "mda.h"
#include "mda_generic.h"
#include "mda_host_common.h"

namespace mda {
#define MDA_GK_DECL(K)                                                                                      \
    hipError_t launch_generic_k##K(int S, const GRunDesc *run, const int32_t *lnt, unsigned int *next,      \
                                   int grid, int block, size_t dyn_lds, hipStream_t stream, int R);         \
    hipError_t generic_occupancy_k##K(int S, int block, size_t dyn_lds, int *blocks_per_cu);
#define MDA_GF_DECL(K)                                                                                      \
    hipError_t launch_gfront_k##K(const GRunDesc *run, int r0, int nr, const int64_t *offs, int64_t total,      \
                                  GFrontEntry *cand, GFrontEntry *ref, GFrontEntry *keep, unsigned long long *nkeep, \
                                  hipStream_t stream);                                                          \
    hipError_t launch_gexact_k##K(const GFrontEntry *keep, int64_t n, GFrontEntry *front, unsigned long long *nfront, \
                                  hipStream_t stream);
MDA_GK_DECL(1) MDA_GK_DECL(2) MDA_GK_DECL(3) MDA_GK_DECL(4)
MDA_GF_DECL(1) MDA_GF_DECL(2) MDA_GF_DECL(3) MDA_GF_DECL(4)
#undef MDA_GF_DECL
hipError_t launch_zero_counter(unsigned int *p, hipStream_t stream);
hipError_t launch_gxgather(const int64_t *at, int64_t n, const uint64_t *archX, int s, int nl, uint64_t *out,
                           hipStream_t stream);
#undef MDA_GK_DECL
}  // namespace mda

using namespace mda;

// LDS of one workgroup on gfx950 and the part the two 4096-entry tables take
// (the -ln table and the thresholds at the final temperature)
constexpr size_t kLdsBytes = 160 * 1024, kLntBytes = 2 * 4096 * sizeof(int32_t);

struct mda_gqubo {
    int32_t m = 0, K = 0, S = 0, nl = 0;
    int64_t ld = 0;
    int64_t q[kMaxK] = {0, 0, 0, 0};
    int64_t maxabs = 0;
    int32_t *dP = nullptr;
    DevPool pool;
    int refs = 1;   // the owner plus every run that uses it
};

static void gqubo_release(mda_gqubo *g)
{
    if (g && --g->refs == 0) {
        g->pool.release_all();
        delete g;
    }
}

// Slots per lane: the smallest tile that holds m bits in 64 lanes and whose
// K * S differences fit the kernels' register budget; 0 if none does.
static int slots_for(int m, int K)
{
    for (int S : {8, 16, 32, 64})
        if (64 * S >= m && K * S <= 64) return S;
    return 0;
}

extern "C" int gqubo_build(int32_t m, int32_t K, const int32_t *Q, const int64_t *q, void *stream_, mda_gqubo **out)
{
    if (!out) return fail(MDA_EINVAL, "out is NULL");
    *out = nullptr;
    if (K < 1 || K > kMaxK) return fail(MDA_EINVAL, "K = %d outside [1, %d]", K, kMaxK);
    if (!Q) return fail(MDA_EINVAL, "Q is NULL");
    const int S = m >= 2 ? slots_for(m, K) : 0;
    if (S == 0) return fail(MDA_EINVAL, "m = %d outside [2, %d] for K = %d", m, K == 1 ? 4096 : K == 2 ? 2048 : 1024, K);
    hipStream_t stream = (hipStream_t)stream_;
    std::unique_ptr<mda_gqubo> g(new mda_gqubo);
    g->m = m;
    g->K = K;
    g->S = S;
    g->nl = (m + S - 1) / S;
    g->ld = 64 * (int64_t)S;
    const size_t mm = (size_t)m * m;
    // the symmetric form of Eq. (cale): P_ab = Q_ab + Q_ba off the diagonal,
    // P_aa = Q_aa; rows zero-padded to ld entries
    std::vector<int32_t> P((size_t)K * m * g->ld, 0);
    for (int k = 0; k < K; ++k) {
        const int32_t *Qk = Q + k * mm;
        g->q[k] = q ? q[k] : 0;
        for (int a = 0; a < m; ++a) {
            int64_t sum = 0;
            int32_t *row = P.data() + ((size_t)k * m + a) * g->ld;
            for (int b = 0; b < m; ++b) {
                const int64_t v = (a == b) ? (int64_t)Qk[(size_t)a * m + a]
                                           : (int64_t)Qk[(size_t)a * m + b] + Qk[(size_t)b * m + a];
                sum += std::llabs(v);
                if (a <= b) g->maxabs = std::max<int64_t>(g->maxabs, std::llabs(v));
                if (std::llabs(v) > INT32_MAX)
                    return fail(MDA_EOVERFLOW, "objective %d: P[%d][%d] = %lld beyond int32", k + 1, a, b, (long long)v);
                row[b] = (int32_t)v;
            }
            // every energy difference |P_aa + sum_b P_ab x_b| must fit int32
            // below INT_MAX, the value of bits beyond m
            if (sum > INT32_MAX - 1)
                return fail(MDA_EOVERFLOW, "objective %d: bit %d has sum |P_ab| = %lld > 2^31-2", k + 1, a,
                            (long long)sum);
        }
    }
    g->dP = g->pool.alloc<int32_t>(P.size(), stream);
    if (!g->dP) return fail(MDA_ENOMEM, "device allocation of %zu bytes failed", P.size() * sizeof(int32_t));
    HIP_TRY(hipMemcpyAsync(g->dP, P.data(), P.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    *out = g.release();
    return MDA_OK;
}

extern "C" int gqubo_info(const mda_gqubo *g, int32_t *m, int32_t *K, int64_t *maxabs_c)
{
    if (!g) return fail(MDA_EINVAL, "NULL qubo");
    if (m) *m = g->m;
    if (K) *K = g->K;
    if (maxabs_c) *maxabs_c = g->maxabs;
    return MDA_OK;
}

extern "C" void gqubo_free(mda_gqubo *g)
{
    gqubo_release(g);
}

struct GEntryH {
    int64_t e[kMaxK];
    int32_t rep, slot;
};

struct mda_grun {
    mda_gqubo *g = nullptr;
    mda_params p{};
    GRunDesc h{};
    GRunDesc *ddesc = nullptr;
    DevPool pool;
    std::vector<GEntryH> merged;   // merged front of all replicas, once computed
    bool merged_ok = false;
    hipStream_t stream = nullptr;
    hipEvent_t ek0 = nullptr, ek1 = nullptr;
    ~mda_grun()
    {
        if (ek1) (void)hipEventSynchronize(ek1);
        else (void)hipStreamSynchronize(stream);
        if (ek0) (void)hipEventDestroy(ek0);
        if (ek1) (void)hipEventDestroy(ek1);
        pool.release_all();
        gqubo_release(g);
    }
};

extern "C" int gda_run(const mda_gqubo *gc, const mda_params *pin, mda_grun **out)
{
    if (!out) return fail(MDA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!gc || !pin) return fail(MDA_EINVAL, "NULL argument");
    mda_gqubo *g = const_cast<mda_gqubo *>(gc);
    mda_params p = *pin;
    const int m = g->m, K = g->K;
    if (p.variant != MDA_VARIANT_AUTO && p.variant != MDA_VARIANT_PERSISTENT)
        return fail(MDA_EINVAL, "generic runs are persistent launches (variant = %d)", p.variant);
    if (p.graph || p.waves_per_replica < 0 || p.waves_per_replica > 1)
        return fail(MDA_EINVAL, "generic runs take no graph or workgroup layout");
    if (p.replicas < 1) return fail(MDA_EINVAL, "replicas = %d", p.replicas);
    if (p.steps == 0) p.steps = (int64_t)std::llround(0.25 * (double)m * (double)m);
    if (p.steps < 1 || p.steps > 0xFFFFFFFELL) return fail(MDA_EINVAL, "steps = %lld outside [1, 2^32 - 2]", (long long)p.steps);
    if (p.accept != MDA_STRICT && p.accept != MDA_LENIENT) return fail(MDA_EINVAL, "accept = %d", p.accept);
    if (p.archive != MDA_EXPLORE && p.archive != MDA_EXPLOIT) return fail(MDA_EINVAL, "archive = %d", p.archive);
    if (p.escape != MDA_ESC_OFFSET && p.escape != MDA_ESC_ARCHIVE) return fail(MDA_EINVAL, "escape = %d", p.escape);
    if (p.archive_size < 0) return fail(MDA_EINVAL, "archive_size = %d", p.archive_size);
    {
        const int64_t s_ = p.archive_size > 0 ? p.archive_size : m;
        if (s_ * K * (int64_t)sizeof(int64_t) > (int64_t)(kLdsBytes - kLntBytes))
            return fail(MDA_EINVAL, "archive_size %lld x %d objectives exceeds the %d entries a wave keeps in LDS",
                        (long long)s_, K, (int)((kLdsBytes - kLntBytes) / sizeof(int64_t)));
    }
    if (p.trace_replicas < 0 || p.trace_replicas > p.replicas)
        return fail(MDA_EINVAL, "trace_replicas = %d", p.trace_replicas);
    if (p.delta0 <= 0.0) {
        // Table param's schedule on coefficients scaled to 2^23, scaled to max|C|
        p.delta0 = 1e9 * (double)g->maxabs / 8388608.0;
        p.deltaf = 1e4 * (double)g->maxabs / 8388608.0;
        if (p.xi <= 0.0) p.xi = 0.001;
    }
    if (!(p.xi >= 0.0 && p.xi < 1.0)) return fail(MDA_EINVAL, "xi = %g", p.xi);
    if (!(p.delta0 * 256.0 <= kMaxTemp)) return fail(MDA_EOVERFLOW, "delta0 = %g exceeds 2^35", p.delta0);
    if (p.beta < 0) p.beta = std::max<int64_t>(1, (int64_t)std::floor(p.delta0 / (double)p.steps));
    std::vector<int64_t> T;
    if (p.temp_table) {
        T.assign(p.temp_table, p.temp_table + p.steps);
        p.temp_table = nullptr;
    } else {
        temperature_table(p.delta0, p.deltaf, p.xi, p.steps, T);
    }
    int32_t lnt[4096];
    threshold_table(lnt);
    std::vector<int64_t> thr(T.size());
    for (size_t t = 0; t < T.size(); ++t) {
        if (T[t] < 0 || (double)T[t] > kMaxTemp) return fail(MDA_EOVERFLOW, "temperature %lld out of range", (long long)T[t]);
        thr[t] = (int64_t)(((uint64_t)T[t] * (uint64_t)lnt[0]) >> 24);
    }

    std::unique_ptr<mda_grun> r(new mda_grun);
    r->stream = (hipStream_t)p.stream;
    hipStream_t stream = r->stream;
    r->p = p;
    const int R = p.replicas, s = p.archive_size > 0 ? p.archive_size : m;
    GRunDesc &d = r->h;
    std::memset(&d, 0, sizeof d);
    d.m = m;
    d.K = K;
    d.S = g->S;
    d.nl = g->nl;
    d.s = s;
    d.accept = p.accept;
    d.archive = p.archive;
    d.escape = p.escape;
    d.R = R;
    d.trace_R = p.trace_replicas;
    d.key0 = (uint32_t)p.seed;
    d.key1 = (uint32_t)(p.seed >> 32);
    d.steps = (uint32_t)p.steps;
    d.ntab = (uint32_t)T.size();
    d.beta = p.beta;
    for (int k = 0; k < K; ++k) d.q[k] = g->q[k];
    d.ld = g->ld;
    d.P = g->dP;
    DevPool &pool = r->pool;
    GRunDesc *ddesc = pool.alloc<GRunDesc>(1, stream);
    int32_t *dlnt = pool.alloc<int32_t>(4096, stream);
    unsigned int *dnext = pool.alloc<unsigned int>(1, stream);
    int64_t *dT = pool.alloc<int64_t>(T.size(), stream);
    int64_t *dthr = pool.alloc<int64_t>(T.size(), stream);
    d.x = pool.alloc<uint64_t>((size_t)R * 64, stream);
    d.h = pool.alloc<int64_t>((size_t)R * K * m, stream);
    d.st = pool.alloc<int64_t>((size_t)R * kGWords, stream);
    d.archE = pool.alloc<int64_t>((size_t)R * s * K, stream);
    d.archX = pool.alloc<uint64_t>((size_t)R * s * d.nl, stream);
    d.nd = pool.alloc<uint8_t>((size_t)R * s, stream);
    d.trace = pool.alloc<int32_t>((size_t)std::max(1, p.trace_replicas) * (size_t)(p.trace_replicas ? p.steps : 1), stream);
    if (!ddesc || !dlnt || !dnext || !dT || !dthr || !d.x || !d.h || !d.st || !d.archE || !d.archX || !d.nd || !d.trace)
        return fail(MDA_ENOMEM, "device allocation failed for the run (%lld bytes so far)", (long long)pool.total);
    d.T = dT;
    d.thrmax = dthr;
    r->ddesc = ddesc;
    HIP_TRY(hipMemcpyAsync(dT, T.data(), T.size() * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dthr, thr.data(), thr.size() * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(dlnt, lnt, sizeof lnt, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ddesc, &d, sizeof d, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemsetAsync(d.nd, 0, (size_t)R * s, stream));
    HIP_TRY(hipEventCreate(&r->ek0));
    HIP_TRY(hipEventCreate(&r->ek1));
    int dev = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // each wave keeps its replica's archive energies in LDS beside the two
    // 16 KB tables: as many waves per block as fit (up to the requested count)
    const size_t per_wave = (size_t)s * K * sizeof(int64_t);
    int wpb = (p.waves_per_block >= 1 && p.waves_per_block <= 4) ? p.waves_per_block : 4;
    while (wpb > 1 && kLdsBytes - kLntBytes < wpb * per_wave) --wpb;
    const int block = 64 * wpb;
    const size_t dyn = wpb * per_wave;
    hipError_t oe = hipErrorInvalidValue;
    switch (K) {
    case 1: oe = generic_occupancy_k1(g->S, block, dyn, &per_cu); break;
    case 2: oe = generic_occupancy_k2(g->S, block, dyn, &per_cu); break;
    case 3: oe = generic_occupancy_k3(g->S, block, dyn, &per_cu); break;
    default: oe = generic_occupancy_k4(g->S, block, dyn, &per_cu); break;
    }
    if (oe != hipSuccess) return fail(MDA_EDEVICE, "occupancy query failed: %s", hipGetErrorString(oe));
    if (per_cu < 1) per_cu = 1;
    int grid = cus * per_cu;
    const int need = (R + block / 64 - 1) / (block / 64);
    if (grid > need) grid = need;
    HIP_TRY(launch_zero_counter(dnext, stream));
    HIP_TRY(hipEventRecord(r->ek0, stream));
    hipError_t le = hipErrorInvalidValue;
    switch (K) {
    case 1: le = launch_generic_k1(g->S, ddesc, dlnt, dnext, grid, block, dyn, stream, R); break;
    case 2: le = launch_generic_k2(g->S, ddesc, dlnt, dnext, grid, block, dyn, stream, R); break;
    case 3: le = launch_generic_k3(g->S, ddesc, dlnt, dnext, grid, block, dyn, stream, R); break;
    default: le = launch_generic_k4(g->S, ddesc, dlnt, dnext, grid, block, dyn, stream, R); break;
    }
    if (le != hipSuccess)
        return fail(MDA_EDEVICE, "generic launch (K %d, S %d, grid %d) failed: %s", K, g->S, grid, hipGetErrorString(le));
    HIP_TRY(hipEventRecord(r->ek1, stream));
    g->refs++;
    r->g = g;
    *out = r.release();
    return MDA_OK;
}

extern "C" int gda_params_get(const mda_grun *r, mda_params *out)
{
    if (!r || !out) return fail(MDA_EINVAL, "NULL argument");
    *out = r->p;
    out->archive_size = r->h.s;
    return MDA_OK;
}

extern "C" int gda_kernel_ms(mda_grun *r, double *ms)
{
    if (!r || !ms) return fail(MDA_EINVAL, "NULL argument");
    HIP_TRY(hipEventSynchronize(r->ek1));
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, r->ek0, r->ek1));
    *ms = f;
    return MDA_OK;
}

static int gcopy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return MDA_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MDA_OK;
}

extern "C" int gda_state_get(mda_grun *r, int32_t replica, uint8_t *x, int64_t *h, int64_t *E, int64_t *e_offset,
                             int64_t *moves, int32_t *trace)
{
    if (!r) return fail(MDA_EINVAL, "NULL run");
    const GRunDesc &d = r->h;
    if (replica < 0 || replica >= d.R) return fail(MDA_EINVAL, "replica %d outside [0, %d)", replica, d.R);
    if (trace && replica >= d.trace_R) return fail(MDA_EINVAL, "replica %d was not traced", replica);
    hipStream_t s = r->stream;
    int rc;
    int64_t st[kGWords];
    if ((rc = gcopy(st, d.st + (size_t)replica * kGWords, sizeof st, s))) return rc;
    if (E)
        for (int k = 0; k < d.K; ++k) E[k] = st[kGE + k];
    if (e_offset) *e_offset = st[kGEoff];
    if (moves) *moves = st[kGMoves];
    if (x) {
        uint64_t w[64];
        if ((rc = gcopy(w, d.x + (size_t)replica * 64, sizeof w, s))) return rc;
        for (int a = 0; a < d.m; ++a) x[a] = (uint8_t)((w[a / d.S] >> (a % d.S)) & 1ull);
    }
    if (h && (rc = gcopy(h, d.h + (size_t)replica * d.K * d.m, (size_t)d.K * d.m * 8, s))) return rc;
    if (trace && (rc = gcopy(trace, d.trace + (size_t)replica * d.steps, (size_t)d.steps * 4, s))) return rc;
    return MDA_OK;
}

namespace {

struct TmpPool {
    DevPool pool;
    ~TmpPool() { pool.release_all(); }
};

bool lex_less(const GEntryH &a, const GEntryH &b, int K)
{
    for (int k = 0; k < K; ++k)
        if (a.e[k] != b.e[k]) return a.e[k] < b.e[k];
    if (a.rep != b.rep) return a.rep < b.rep;
    return a.slot < b.slot;
}

// Non-dominated entries of the archives of replicas [r0, r0 + nr) (Section
// 3.3), equal energy vectors reduced to the lowest (replica, slot), sorted by
// (E, replica, slot).  The device gathers the flagged entries, drops those
// that one of each replica's K + 1 reference entries (least energy sum, least
// energy per objective) dominates, and keeps the survivors that no other
// survivor dominates; the host sorts what is left.
int merged_front(mda_grun *r, int r0, int nr, const std::vector<int64_t> &st, std::vector<GEntryH> &out)
{
    const GRunDesc &d = r->h;
    const int K = d.K;
    hipStream_t s = r->stream;
    out.clear();
    std::vector<int64_t> offs((size_t)nr + 1, 0);
    for (int k = 0; k < nr; ++k) offs[k + 1] = offs[k] + std::max<int64_t>(0, st[(size_t)k * kGWords + kGNd]);
    const int64_t total = offs[nr];
    if (total == 0) return MDA_OK;
    TmpPool tmp;
    int64_t *doffs = tmp.pool.alloc<int64_t>(offs.size(), s);
    GFrontEntry *cand = tmp.pool.alloc<GFrontEntry>((size_t)total, s);
    GFrontEntry *ref = tmp.pool.alloc<GFrontEntry>((size_t)nr * (K + 1), s);
    GFrontEntry *keep = tmp.pool.alloc<GFrontEntry>((size_t)total, s);
    GFrontEntry *front = tmp.pool.alloc<GFrontEntry>((size_t)total, s);
    unsigned long long *cnt = tmp.pool.alloc<unsigned long long>(2, s);
    if (!doffs || !cand || !ref || !keep || !front || !cnt)
        return fail(MDA_ENOMEM, "device allocation failed for %lld front candidates", (long long)total);
    HIP_TRY(hipMemcpyAsync(doffs, offs.data(), offs.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned long long), s));
    hipError_t e = hipErrorInvalidValue;
    switch (K) {
    case 1: e = launch_gfront_k1(r->ddesc, r0, nr, doffs, total, cand, ref, keep, cnt, s); break;
    case 2: e = launch_gfront_k2(r->ddesc, r0, nr, doffs, total, cand, ref, keep, cnt, s); break;
    case 3: e = launch_gfront_k3(r->ddesc, r0, nr, doffs, total, cand, ref, keep, cnt, s); break;
    default: e = launch_gfront_k4(r->ddesc, r0, nr, doffs, total, cand, ref, keep, cnt, s); break;
    }
    if (e != hipSuccess) return fail(MDA_EDEVICE, "front gather failed: %s", hipGetErrorString(e));
    unsigned long long nk = 0, nf = 0;
    int rc = gcopy(&nk, cnt, sizeof nk, s);
    if (rc) return rc;
    if ((int64_t)nk > total) return fail(MDA_EDEVICE, "front filter kept %llu of %lld", nk, (long long)total);
    switch (K) {
    case 1: e = launch_gexact_k1(keep, (int64_t)nk, front, cnt + 1, s); break;
    case 2: e = launch_gexact_k2(keep, (int64_t)nk, front, cnt + 1, s); break;
    case 3: e = launch_gexact_k3(keep, (int64_t)nk, front, cnt + 1, s); break;
    default: e = launch_gexact_k4(keep, (int64_t)nk, front, cnt + 1, s); break;
    }
    if (e != hipSuccess) return fail(MDA_EDEVICE, "front pass failed: %s", hipGetErrorString(e));
    if ((rc = gcopy(&nf, cnt + 1, sizeof nf, s))) return rc;
    if (nf > nk) return fail(MDA_EDEVICE, "front pass kept %llu of %llu", nf, nk);
    std::vector<GFrontEntry> fe((size_t)nf);
    if ((rc = gcopy(fe.data(), front, fe.size() * sizeof(GFrontEntry), s))) return rc;
    out.resize(fe.size());
    for (size_t i = 0; i < fe.size(); ++i) {
        std::memcpy(out[i].e, fe[i].e, sizeof out[i].e);
        out[i].rep = fe[i].rep;
        out[i].slot = fe[i].slot;
    }
    std::sort(out.begin(), out.end(), [K](const GEntryH &a, const GEntryH &b) { return lex_less(a, b, K); });
    return MDA_OK;
}

}  // namespace

extern "C" int garchive_get(mda_grun *r, int32_t replica, int32_t raw, int64_t cap, int64_t *e, int32_t *rep,
                            int32_t *slot, uint32_t *xbits, int64_t *count)
{
    if (!r || !count) return fail(MDA_EINVAL, "NULL argument");
    const GRunDesc &d = r->h;
    const int K = d.K, s = d.s;
    if (replica < -1 || replica >= d.R) return fail(MDA_EINVAL, "replica %d outside [-1, %d)", replica, d.R);
    if (replica < 0 && raw) return fail(MDA_EINVAL, "the raw archive is per replica");
    hipStream_t st_ = r->stream;
    HIP_TRY(hipEventSynchronize(r->ek1));
    int rc;
    std::vector<GEntryH> local;
    const std::vector<GEntryH> *src = &local;
    if (replica < 0 && r->merged_ok) {
        src = &r->merged;
    } else {
        const int r0 = replica < 0 ? 0 : replica, nr = replica < 0 ? d.R : 1;
        std::vector<int64_t> st((size_t)nr * kGWords);
        if ((rc = gcopy(st.data(), d.st + (size_t)r0 * kGWords, st.size() * 8, st_))) return rc;
        if (raw) {
            const int asz = (int)std::min<int64_t>(std::max<int64_t>(st[kGArch], 0), s);
            std::vector<int64_t> E((size_t)asz * K);
            if ((rc = gcopy(E.data(), d.archE + (size_t)replica * s * K, E.size() * 8, st_))) return rc;
            local.resize((size_t)asz);
            for (int q = 0; q < asz; ++q) {
                GEntryH g{};
                for (int kk = 0; kk < K; ++kk) g.e[kk] = E[(size_t)q * K + kk];
                g.rep = replica;
                g.slot = q;
                local[q] = g;
            }
        } else {
            if ((rc = merged_front(r, r0, nr, st, local))) return rc;
            if (replica < 0) {
                r->merged = local;
                r->merged_ok = true;
                src = &r->merged;
            }
        }
    }
    const std::vector<GEntryH> &ent = *src;
    *count = (int64_t)ent.size();
    if (!e) return MDA_OK;
    if (cap < (int64_t)ent.size()) return fail(MDA_ERANGE, "capacity %lld < %zu entries", (long long)cap, ent.size());
    const int words = (d.m + 31) / 32;
    std::vector<uint64_t> xw;
    if (xbits && !ent.empty()) {
        // stored solutions of the returned entries: one contiguous copy of a
        // raw archive, else gathered on the device and copied once
        xw.resize(ent.size() * (size_t)d.nl);
        if (raw) {
            if ((rc = gcopy(xw.data(), d.archX + (size_t)replica * s * d.nl, xw.size() * 8, st_))) return rc;
        } else {
            std::vector<int64_t> at(ent.size());
            for (size_t i = 0; i < ent.size(); ++i) at[i] = ((int64_t)ent[i].rep << 32) | (int64_t)ent[i].slot;
            TmpPool tmp;
            int64_t *dat = tmp.pool.alloc<int64_t>(at.size(), st_);
            uint64_t *dx = tmp.pool.alloc<uint64_t>(xw.size(), st_);
            if (!dat || !dx) return fail(MDA_ENOMEM, "device allocation failed for %zu solutions", ent.size());
            HIP_TRY(hipMemcpyAsync(dat, at.data(), at.size() * 8, hipMemcpyHostToDevice, st_));
            HIP_TRY(launch_gxgather(dat, (int64_t)at.size(), d.archX, s, d.nl, dx, st_));
            if ((rc = gcopy(xw.data(), dx, xw.size() * 8, st_))) return rc;
        }
    }
    for (size_t i = 0; i < ent.size(); ++i) {
        for (int k = 0; k < K; ++k) e[i * K + k] = ent[i].e[k];
        if (rep) rep[i] = ent[i].rep;
        if (slot) slot[i] = ent[i].slot;
        if (xbits) {
            const uint64_t *xs = xw.data() + i * d.nl;
            uint32_t *o = xbits + i * words;
            std::memset(o, 0, (size_t)words * 4);
            for (int a = 0; a < d.m; ++a)
                if ((xs[a / d.S] >> (a % d.S)) & 1ull) o[a >> 5] |= 1u << (a & 31);
        }
    }
    return MDA_OK;
}

extern "C" int gda_stats(mda_grun *r, int64_t *moves, int64_t *scanned, int64_t *rng_blocks, int64_t *archived)
{
    if (!r) return fail(MDA_EINVAL, "NULL run");
    const GRunDesc &d = r->h;
    std::vector<int64_t> st((size_t)d.R * kGWords);
    int rc = gcopy(st.data(), d.st, st.size() * sizeof(int64_t), r->stream);
    if (rc) return rc;
    int64_t mv = 0, sc = 0, rb = 0, ar = 0;
    for (int i = 0; i < d.R; ++i) {
        mv += st[(size_t)i * kGWords + kGMoves];
        sc += st[(size_t)i * kGWords + kGScanned];
        rb += st[(size_t)i * kGWords + kGRng];
        ar += st[(size_t)i * kGWords + kGArch];
    }
    if (moves) *moves = mv;
    if (scanned) *scanned = sc;
    if (rng_blocks) *rng_blocks = rb;
    if (archived) *archived = ar;
    return MDA_OK;
}

extern "C" void gda_run_free(mda_grun *r)
{
    delete r;
}
