/*
 * mda.h -- C ABI of the MI355X multi-objective Digital Annealer (MDA) for the
 * bi-objective quadratic assignment problem (bQAP).
 *
 * Method: Ayodele, Allmendinger, Lopez-Ibanez, Parizy, "Multi-objective QUBO
 * Solver: Bi-objective Quadratic Assignment Problem", GECCO 2022
 * (arXiv:2205.13399).  Section 2 defines the QUBO of the bQAP, Section 3.1 the
 * parallel-trial annealing step (Algorithm 1, Eqs. cale and paccepts),
 * Section 3.3 the multi-objective annealer (Algorithm 3, Eqs. wqubom,
 * pacceptms, pacceptml) and its archive updates (Algorithms 4 and 5).
 *
 * Conventions shared by every call:
 *  - Every function returns MDA_OK (0) or a negative MDA_E* code and never
 *    aborts or throws across the ABI; mda_last_error() gives a thread-local
 *    message for the last failure.
 *  - Bit a = i*n + u of a solution means "facility i is at location u"
 *    (row = facility, column = location, as in the worked example of Sec. 2.2).
 *  - Host arrays passed in are owned by the caller and copied before return.
 *    Handles are owned by the library and released with the matching *_free
 *    (NULL is a no-op).  A run keeps its QUBO referenced: free runs first.
 *  - Device memory is obtained through the allocator installed with
 *    mda_set_allocator (default: hipMalloc / hipFree).  Work is enqueued on the
 *    HIP stream given in the parameters; da_run returns before the device is
 *    done, archive_get and da_state_get synchronise that stream.
 *  - A handle is not thread-safe; distinct handles may be used from distinct
 *    threads.  Runs sharing a stream execute in submission order.
 */
#ifndef MDA_H
#define MDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MDA_OK = 0,
    MDA_EINVAL = -1,     /* bad argument (size, NULL pointer, unknown option) */
    MDA_EOVERFLOW = -2,  /* a local field or threshold would not fit its integer type */
    MDA_ENOMEM = -3,     /* host or device allocation failed */
    MDA_EDEVICE = -4,    /* a HIP call failed */
    MDA_ERANGE = -5,     /* output capacity too small (count holds the size needed) */
    MDA_EBUSY = -6       /* the run is still referenced or in use */
};

/* Penalty weight alpha_k of the one-hot constraint QUBO G (Eq. wqubom). */
enum { MDA_PEN_2MAX = 0,   /* alpha_k = 2 * max |C_k| (the benchmark setting) */
       MDA_PEN_VL = 1 };   /* Eq. (vermap) on the symmetric form, alpha = ceil(w/2), Eq. (wvermaa) */

/* How the local fields are updated after a flip. */
enum { MDA_PATH_AUTO = 0,  /* Kronecker; dense when the rows fit a positive dense_budget, or when the
                              Kronecker operands exceed the 24-bit multiplier range */
       MDA_PATH_DENSE = 1, /* stream int32 rows of the symmetric P_1, P_2 from HBM */
       MDA_PATH_KRON = 2 };/* regenerate the column from F_k, D and alpha_k */

enum { MDA_STRICT = 0, MDA_LENIENT = 1 };        /* Eq. (pacceptms) / Eq. (pacceptml) */
enum { MDA_EXPLORE = 0, MDA_EXPLOIT = 1 };       /* Algorithm 4 / Algorithm 5 */
enum { MDA_ESC_OFFSET = 0,                       /* Algorithm 1: E_offset += beta when stuck */
       MDA_ESC_ARCHIVE = 1 };                    /* Algorithm 3: restart from a random archive member */
enum { MDA_VARIANT_AUTO = 0,                     /* persistent launch */
       MDA_VARIANT_PERSISTENT = 1,               /* all steps in one launch, state on chip */
       MDA_VARIANT_PLAIN = 2 };                  /* one launch per annealing step, state in HBM */

typedef struct mda_qubo mda_qubo;  /* one bQAP instance: host copies + device operands */
typedef struct mda_run mda_run;    /* one run: device replica state and archives */

typedef struct {
    int32_t penalty;         /* MDA_PEN_* */
    int32_t path;            /* MDA_PATH_* */
    int64_t dense_budget;    /* bytes of dense rows MDA_PATH_AUTO may take; <= 0: none (the Kronecker
                                update is the faster one at every size) */
    int32_t normalise_log2;  /* objective normalisation (Sec. Parameter Settings, which
                                sets the largest coefficient of each C_k to 2^23):
                                0 = none; L in [1, 30] = each F_k is scaled by
                                s_k = 2^L / max|C_k| and rounded to the nearest integer
                                (halves up), so max|C_k| is 2^L up to that rounding
                                (an objective with C_k = 0 is left as it is);
                                -1 = the largest L <= 23 for which the int32 bounds of
                                qubo_build_bqap hold */
    int32_t fields;          /* width of the energy differences (local fields) the runs keep:
                                0 = int32 when every bit's |P_aa| + sum_b |P_ab| <= 2^31 - 2 and
                                2 alpha_k n < 2^30, else int64 (n <= 64 only); 32 = int32 only;
                                64 = int64 (n <= 64) */
} mda_build_opts;

typedef struct {
    int32_t n, m;            /* facilities, bits (m = n*n) */
    int32_t path;            /* MDA_PATH_DENSE or MDA_PATH_KRON as chosen */
    int32_t symmetric;       /* 1 when D (or F1 and F2) is symmetric */
    int64_t alpha1, alpha2;  /* penalty weights */
    int64_t q1, q2;          /* constant terms alpha_k * 2n of Y and Z */
    int64_t maxabs_c;        /* max(max|C_1|, max|C_2|), after normalisation */
    int64_t device_bytes;    /* device memory held by the handle */
    int32_t normalise_log2;  /* L applied (0 = none) */
    int32_t fields;          /* 32 or 64: width of the energy differences */
    double scale1, scale2;   /* s_k applied to F_k (1 when none; energies are in scaled units) */
} mda_qubo_info;

/*
 * Builds the two penalised objective QUBOs of Eq. (wqubom) for one bQAP
 * instance (Sec. 2.2-2.3): C_k from flows F_k and distances D (Eq. cqap), G
 * from the two-way one-hot constraint (Eq. gqap), Y = C_1 + alpha_1 G,
 * Z = C_2 + alpha_2 G, and uploads what the chosen update path needs.
 *   n            2 <= n <= 100 (m = n*n <= 10000)
 *   F1, F2, D    host, row-major n*n int32: F_k[i*n+j] flow from facility i to j
 *                in objective k, D[u*n+v] distance from location u to v
 *   opts         NULL for defaults (MDA_PEN_2MAX, MDA_PATH_AUTO, no dense budget)
 *   stream       hipStream_t for the uploads (NULL = default stream)
 *   out          receives the handle
 * Errors: MDA_EINVAL (n outside [2, 100], a NULL array, an unknown option),
 * MDA_EOVERFLOW (a QUBO entry max|C_k| + 2 alpha_k beyond int32; a scaled flow
 * beyond int32; int32 fields requested where some bit's |P_aa| + sum_b |P_ab|
 * exceeds 2^31-2 or 2 alpha_k n >= 2^30; int64 fields needed or requested with
 * n > 64; with normalise_log2 = -1: no L in [1, 23] fits int32 fields),
 * MDA_ENOMEM, MDA_EDEVICE.
 */
int qubo_build_bqap(int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D,
                    const mda_build_opts *opts, void *stream, mda_qubo **out);

/*
 * SB-DA (Alg. SB-DA, Sec. 3.2) on the same kernels: the QUBO of the
 * scalarised cost gamma R + (1 - gamma) S with gamma = g10 / 10, scaled by 10
 * to stay integer -- C is linear in the flows, so this is the cost QUBO of the
 * flows g10 F1 + (10 - g10) F2 -- with its own penalty (opts->penalty; the
 * paper's is MDA_PEN_VL) and a second objective identically zero, under which
 * the strict rule is the single-objective DA's (Eq. paccepts).  Arguments as
 * qubo_build_bqap; F1, F2 are the flows as given (normalise them first with
 * qubo_build_bqap + qubo_flows for the normalised variant).
 * Errors: as qubo_build_bqap; MDA_EINVAL for g10 outside [0, 10];
 * MDA_EOVERFLOW when a scalarised flow exceeds int32.
 */
int qubo_build_scalarised(int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D, int32_t g10,
                          const mda_build_opts *opts, void *stream, mda_qubo **out);

/* The flows q was built from, after normalisation: host, row-major n*n int32
 * each (either may be NULL).  Errors: MDA_EINVAL (NULL q). */
int qubo_flows(const mda_qubo *q, int32_t *F1, int32_t *F2);
/* Sizes, chosen path, penalty weights, normalisation and device bytes of q.
 * Errors: MDA_EINVAL (NULL argument). */
int qubo_info(const mda_qubo *q, mda_qubo_info *info);
void qubo_free(mda_qubo *q);

typedef struct {
    int32_t replicas;         /* independent annealing chains, >= 1 */
    int32_t archive_size;     /* s; 0 = m (Table param) */
    int64_t steps;            /* I_max, 1 <= steps <= 2^32 - 2; 0 = 0.25 * m^2 (Table param) */
    double delta0, deltaf, xi;/* geometric schedule; delta0 <= 0 selects 1e9*M/2^23, 1e4*M/2^23, 1e-3
                                 where M = max|C| (the paper's values on coefficients scaled to 2^23) */
    int64_t beta;             /* E_offset increment; < 0 selects max(1, floor(delta0/steps)) */
    int32_t accept;           /* MDA_STRICT | MDA_LENIENT */
    int32_t archive;          /* MDA_EXPLORE | MDA_EXPLOIT */
    int32_t escape;           /* MDA_ESC_OFFSET | MDA_ESC_ARCHIVE */
    int32_t variant;          /* MDA_VARIANT_* */
    uint64_t seed;            /* Philox key of this run */
    int32_t trace_replicas;   /* record the flipped bit of every step for replicas [0, k) */
    int32_t waves_per_block;  /* launch shape hint, 1..4 (larger is clamped); 0 = default; results do not depend on it */
    void *stream;             /* hipStream_t; NULL = default stream */
    int32_t graph;            /* 1: capture the launch sequence (one persistent launch per register tile, then the
                                 non-dominated flags) into a HIP graph and launch it; needs a created stream;
                                 da_kernel_ms then times the whole graph.  0: launch directly */
    int32_t waves_per_replica;/* 0: one wave for n <= 64, else a workgroup of 2 * ceil(n / 64) waves;
                                 1: one wave (n <= 64); 2..8: a workgroup of that many waves, split into
                                 ceil(n / 64) location blocks and facility blocks of equal size */
    const int64_t *temp_table;/* optional host array of the resolved step count's entries: T_t of step t
                                 (t = 1..steps) at index t - 1, the temperature delta_t in fixed point with
                                 8 fractional bits (floor(256 delta_t)), each in [0, 2^43]; it replaces the
                                 geometric schedule of delta0, deltaf and xi (Table param) as input data.
                                 Copied before da_run returns.  delta0 still sets the default beta.
                                 NULL: the geometric schedule */
    int32_t occupancy;        /* one-wave form, int32 differences: 0 = automatic (the build holding two waves
                                 per SIMD when a launch has more replicas than one wave per SIMD holds at
                                 once); 1 or 2: that build (2 exists from 32 register slots, i.e. n > 28;
                                 smaller tiles take 1).  In a batch the first block's value applies.
                                 Results do not depend on it */
} mda_params;

/* Fills p with the defaults of Table (param) and the benchmark settings. */
void mda_params_default(mda_params *p);

/*
 * Runs Algorithm 3 (MDA) for p->replicas independent replicas of q: random
 * start, per-step energy differences of both objectives for all m bits from
 * maintained local fields, parallel acceptance with the dynamic offset,
 * uniform choice of one accepted flip, field update, archive update.
 * Asynchronous on p->stream.  Errors: MDA_EINVAL, MDA_EOVERFLOW (delta0 above
 * 2^35, or a temp_table entry outside [0, 2^43]), MDA_ENOMEM, MDA_EDEVICE.
 */
int da_run(const mda_qubo *q, const mda_params *p, mda_run **out);

/*
 * Runs several independent MDA runs (instances of any size, each with its own
 * parameters and seed) together on ps[0].stream: the replicas of all runs form
 * one work list, grouped by register tile (slots per lane: 8 * ceil(n / 8),
 * or 28 for n of 25 to 28 and 52 for n of 49 to 52 unless the batch holds
 * runs of 29 to 32, or 53 to 56, with the same step variant, which they then
 * join), and each group is one persistent
 * launch; with ps[0].graph the launches are
 * one HIP graph.  Each result is identical to the corresponding da_run.  outs
 * receives one handle per run.  All runs share the stream, variant and graph
 * setting.
 */
int da_run_batch(const mda_qubo *const *qs, const mda_params *ps, int32_t count, mda_run **outs);

/* Waits for the run's device work. */
int da_sync(mda_run *r);

/* Device time of the run's launch in milliseconds (HIP events; synchronises). */
int da_elapsed_ms(mda_run *r, double *ms);

/* Device time of the annealing kernel(s) alone: initial state, all steps and
 * the final state of every replica, without the non-dominated filter. */
int da_kernel_ms(mda_run *r, double *ms);

typedef struct {
    int64_t cap;          /* entries the arrays below can hold */
    int64_t *e1, *e2;     /* energies E_1, E_2 (Eq. mqap) */
    int32_t *replica;     /* replica the entry comes from */
    int32_t *slot;        /* archive slot within that replica */
    uint8_t *feasible;    /* 1 when x is a permutation matrix (g(x) = 0), may be NULL */
    uint32_t *xbits;      /* cap * ceil(m/32) words, bit a of word a/32, may be NULL */
    int32_t *perm;        /* cap * n, location of each facility (-1 if infeasible), may be NULL */
} mda_archive_out;

/*
 * Copies archives to the host.  replica >= 0: that replica's archive; -1: the
 * union over all replicas.  raw = 1: the ordered archive as stored (one replica
 * only); raw = 0: its non-dominated entries (Sec. 3.3), equal-energy duplicates
 * reduced to the lowest (replica, slot), sorted by (E1, E2, replica, slot).
 * out == NULL is a size query.  *count receives the number of entries.
 * Synchronises the run's stream.  Errors: MDA_EINVAL, MDA_ERANGE, MDA_EDEVICE.
 */
int archive_get(mda_run *r, int32_t replica, int32_t raw, mda_archive_out *out, int64_t *count);

typedef struct {
    uint8_t *x;             /* m bits, one byte each, may be NULL */
    int64_t *h1, *h2;       /* local fields h_k[a] = sum_{b != a} P_k[a][b] x_b, may be NULL */
    int64_t e1, e2;         /* energies of x */
    int64_t e_offset;       /* current offset */
    int64_t moves;          /* accepted flips */
    int64_t scanned;        /* archive entries compared */
    int64_t rng_blocks;     /* acceptance random blocks drawn */
    int32_t *trace;         /* resolved-steps entries (bit index or -1), may be NULL; needs trace_replicas */
} mda_state;

/* Final state of one replica (synchronises).  st->trace receives as many
 * entries as the run's resolved step count (da_params_get), which differs from
 * the steps passed in when those were 0. */
int da_state_get(mda_run *r, int32_t replica, mda_state *st);

/* The parameters run r uses, each default resolved: steps (0 -> m^2 / 4, Table
 * param), delta0, deltaf, xi and beta (the schedule of Table param scaled by
 * max |C| / 2^23 when delta0 <= 0; beta < 0 -> max(1, floor(delta0 / steps))),
 * archive_size (0 -> m) and waves_per_replica (0 -> the layout chosen).
 * temp_table is returned as NULL (the run keeps its own copy).  The other
 * fields are returned as given.  Does not synchronise.
 * Errors: MDA_EINVAL (NULL argument). */
int da_params_get(const mda_run *r, mda_params *out);

/* Run statistics summed over replicas: moves, archive entries compared, random
 * blocks drawn, total archive entries (synchronises). */
int da_stats(mda_run *r, int64_t *moves, int64_t *scanned, int64_t *rng_blocks, int64_t *archived);

/* Each replica's best solution, the state Algorithm 1 returns: the archive
 * entry of least E_1 (the first slot among equal ones) of replicas [0, R),
 * found on the device.  e1 and slot receive R entries each (INT64_MAX and -1
 * for an empty archive); synchronises.  With a second objective identically
 * zero (SB-DA) the archive keeps the lowest-energy states the replica
 * visited, so this is its least-energy state.  Errors: MDA_EINVAL (NULL
 * argument), MDA_ENOMEM, MDA_EDEVICE. */
int da_best(mda_run *r, int64_t *e1, int32_t *slot);

void da_run_free(mda_run *r);

/* Installs the device allocator (NULL alloc restores hipMalloc/hipFree). */
typedef void *(*mda_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*mda_free_fn)(void *ptr, size_t bytes, void *stream, void *ctx);
int mda_set_allocator(mda_alloc_fn alloc, mda_free_fn release, void *ctx);

const char *mda_last_error(void);

/*
 * Device bytes a run of an n-facility instance with parameters p (and the QUBO
 * built with opts) holds: replica state, archives (Table param size s = m by
 * default), tables and operands.  Host only.  Negative MDA_E* on bad input.
 */
int64_t mda_footprint(int32_t n, const mda_params *p, const mda_build_opts *opts);

/*
 * Launch-shape autotuner.  Times probe runs (probe_steps steps of at most
 * probe_replicas replicas, q's update path and p's acceptance rule) for each
 * shape: one wave per replica (n <= 64) with 1, 2 or 4 waves per block, and
 * workgroups of 2 or 4 waves per replica where a layout exists; returns the
 * fastest.  Results are remembered per (n, update path, acceptance rule,
 * replica count rounded down to a power of two) for the life of the process
 * (cached = 1 when answered from there).  Launch shapes never change results.
 * probe_steps < 1: 2000; probe_replicas < 1: all of p->replicas.
 */
typedef struct {
    int32_t waves_per_block;     /* chosen: set in mda_params */
    int32_t waves_per_replica;   /* chosen: set in mda_params */
    int32_t candidates;          /* shapes timed */
    int32_t cached;
    double best_ms;
    int64_t probe_steps;
    int32_t probe_replicas;
    int32_t occupancy;           /* chosen: set in mda_params (0 = automatic, for workgroup layouts) */
    int32_t cand_wpb[16], cand_wpr[16];
    double probe_ms[16];         /* persistent-kernel time of each candidate */
    int32_t cand_occ[16];
} mda_tuning;

int mda_autotune(const mda_qubo *q, const mda_params *p, int64_t probe_steps, int32_t probe_replicas,
                 mda_tuning *out);

/* ---------------- serving engine ----------------
 *
 * Clients submit bQAP solves (the problem statement of Sec. 2.1: F1, F2, D)
 * at any time.  A scheduler thread admits pending requests in arrival order
 * while their footprint (mda_footprint) fits the memory budget, and packs
 * every admitted request -- any mix of n -- into one batched launch on one of
 * max_inflight streams, so requests arriving while others run are launched
 * beside them.  A result stays on the device until collected with
 * mda_server_wait; it is identical to da_run of the same instance,
 * parameters and seed.  The server allocates stream-ordered device memory of
 * its own (not through mda_set_allocator).  Runs handed to the client may be
 * freed before or after mda_server_destroy: the server's streams stay valid
 * for the life of the process.
 */
typedef struct mda_server mda_server;

typedef struct {
    int64_t hbm_budget;      /* device bytes admitted requests may hold; <= 0: half the free memory */
    int32_t max_inflight;    /* launches (streams) in flight, 1..8; 0 = 4 */
    int32_t max_batch;       /* requests per launch; 0 = 64 */
    int32_t device;          /* HIP device; < 0 = the current one */
    int32_t reserved;        /* 0 */
} mda_server_opts;

typedef struct {
    int64_t ticket;
    int32_t n;
    int32_t status;          /* 2 = done, negative MDA_E* = failed */
    double t_submit, t_admit, t_launch, t_done;   /* seconds since the server started */
    int64_t bit_trials;      /* replicas * n^2 * steps */
    int64_t footprint;       /* device bytes accounted to the request */
    int32_t batch;           /* requests in its launch */
    int32_t slot;            /* server stream (0 .. max_inflight - 1) its launch ran on */
} mda_request_info;

typedef struct {
    int64_t launches, completed, bit_trials;
    int64_t pending, in_flight;
    int64_t hbm_used, hbm_budget;
    double now, first_launch, last_done;   /* seconds since the server started */
} mda_server_counters;

int mda_server_create(const mda_server_opts *opts, mda_server **out);
/* Copies the instance (and p->temp_table, if given); p->stream and p->graph are ignored; steps and
 * replicas must be set. */
int mda_server_submit(mda_server *s, int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D,
                      const mda_build_opts *opts, const mda_params *p, int64_t *ticket);
/* Waits up to timeout_s (< 0: no limit) for the request; on success hands its run to the caller
 * (NULL run: freed at once) and fills info.  The request's footprint counts against the budget
 * until its run is freed (da_run_free), also after the run has been handed over.  MDA_EBUSY on timeout (the ticket stays valid); the
 * request's own error code if it failed.  A ticket is collected once. */
int mda_server_wait(mda_server *s, int64_t ticket, double timeout_s, mda_run **run, mda_request_info *info);
int mda_server_stats(mda_server *s, mda_server_counters *st);
/* Fails requests not yet admitted, waits for launched ones, frees uncollected results. */
void mda_server_destroy(mda_server *s);

/* ---------------- runs into caller-owned buffers, allocating nothing ----------------
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The
 * variant of da_run below writes every result into device buffers the caller
 * owns and keeps the launch's own data (run descriptor, work list, -ln table,
 * temperature tables) in a fixed scratch area of MDA_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it has run on until the process ends.
 * It calls no hipMalloc, hipFree or allocator callback.
 *
 * Every call on one device shares that device's scratch area and overwrites
 * it (nothing in it has to start at zero): calls on the same stream run in
 * order, calls that overlap on one device (different streams, other threads)
 * race and must not be made.
 */
#define MDA_NOALLOC_SCRATCH_BYTES ((int64_t)4 << 20)

typedef struct {
    int32_t n, m, replicas;
    int32_t archive_size;      /* s, resolved */
    int64_t steps;             /* resolved step count */
    int32_t trace_replicas;
    int32_t wr, wc, gns;       /* layout over waves: wr x wc waves per replica (1 x 1: one wave), gns
                                  facilities per wave row */
    int64_t x_words;           /* uint64 words of x per replica: 64 (one wave) or wr * wc * 64 */
    int64_t arch_x_words;      /* uint64 words per archived solution: n (one wave) or wr * wc * 64 */
    /* element counts of the buffers of mda_run_buffers */
    int64_t n_x, n_h, n_st, n_arch_e, n_arch_x, n_nd, n_trace;
    int64_t scratch_bytes;     /* of the scratch area this run needs (<= MDA_NOALLOC_SCRATCH_BYTES) */
} mda_run_layout;

/* Sizes of the buffers da_run_noalloc writes for q and p (host only; the
 * checks of da_run are applied).  Errors: those of da_run's argument checks,
 * MDA_ERANGE when the run's work list and tables need more scratch than
 * MDA_NOALLOC_SCRATCH_BYTES (layout still filled). */
int da_run_layout(const mda_qubo *q, const mda_params *p, mda_run_layout *out);

/* Device buffers of one run, owned by the caller, sized by da_run_layout.
 * Solution words: with one wave per replica, word u (u < n) holds location u's
 * column, bit i = x_{i,u}; with a workgroup, word (p*wc + c)*64 + (u mod 64)
 * with c = u / 64 holds bit i - p*gns = x_{i,u} for facilities
 * i in [p*gns, p*gns + gns). */
typedef struct {
    uint64_t *x;       /* [R][x_words] final solution */
    int64_t *h;        /* [R][2][m] final local fields h_1, h_2 at bit a = i*n + u */
    int64_t *st;       /* [R][16] E_1, E_2, E_offset, moves, archive entries compared, random blocks drawn,
                          archive size, steps with an exact acceptance test, non-dominated count; rest unused */
    int64_t *arch_e;   /* [R][s][2] archive energies (E_1, E_2) in slot order; slots [0, size) are defined */
    uint64_t *arch_x;  /* [R][s][arch_x_words] archived solutions */
    uint8_t *nd;       /* [R][s] 1 = not dominated within its archive; slots [0, size) are defined */
    int32_t *trace;    /* [trace_replicas][steps] flipped bit or -1; NULL when trace_replicas = 0 */
} mda_run_buffers;

/* da_run of q with parameters p, results in b instead of a run handle: the
 * same trajectories, states, archives and flags as da_run.  Asynchronous on
 * p->stream; the caller synchronises before reading b.  Host arrays (p and
 * p->temp_table) may be released when it returns.  p->variant must not be
 * MDA_VARIANT_PLAIN and p->graph must be 0.  Errors: MDA_EINVAL (a NULL
 * argument or buffer, the plain form, the graph flag, and the argument checks
 * of da_run), MDA_ERANGE (more than MDA_NOALLOC_SCRATCH_BYTES of scratch
 * needed: replicas * 8 + steps * 20 bytes, roughly, with a temp_table or a
 * schedule that keeps cooling), MDA_EOVERFLOW, MDA_EDEVICE. */
int da_run_noalloc(const mda_qubo *q, const mda_params *p, const mda_run_buffers *b);

/* ---------------- K objectives on a generic QUBO ----------------
 *
 * The extension beyond two objectives that the paper's Conclusion names, on any
 * QUBO (Eq. qubo): K objectives E_k(x) = x^T Q_k x + q_k over m bits, the MDA of
 * Algorithm 3 with the strict rule (Eq. pacceptms) summing max(0, dE_k -
 * E_offset) over the K objectives and the lenient rule (Eq. pacceptml) taking
 * their least, and K-way dominance (Section 3.3) in the archive updates
 * (Algorithms 4 and 5).  Bits carry no (facility, location) structure: the
 * random numbers go by bit index, eight consecutive bits per Philox block (bit
 * a: start bit (a & 31) of word (a >> 5) & 3 of block (a >> 7, 0, replica,
 * INIT); acceptance index bits 4..15 of half (a & 1) of word (a & 7) >> 1 of
 * block (a >> 3, step, replica, ACC)).  Dense rows of the symmetric form only.
 */
typedef struct mda_gqubo mda_gqubo;   /* K generic objective QUBOs on the device */
typedef struct mda_grun mda_grun;     /* one K-objective run: replica state and archives */

/*
 * Builds the K objectives.
 *   m      bits, 2 <= m <= 4096 / K rounded down to 1024, 2048 or 4096
 *          (K = 1: 4096, K = 2: 2048, K = 3 or 4: 1024): a replica's K m
 *          differences stay in one wave's registers
 *   K      objectives, 1 <= K <= 4
 *   Q      host int32, K * m * m, row-major: Q_k[a][b] at (k * m + a) * m + b;
 *          any matrix (only Q + Q^T off the diagonal and Q_aa on it matter)
 *   q      host int64 constants q_k, K of them, or NULL for zeros
 *   stream hipStream_t for the uploads (NULL = default stream)
 * Errors: MDA_EINVAL (sizes, NULL arrays), MDA_EOVERFLOW (some bit's
 * |P_aa| + sum_b |P_ab| beyond 2^31 - 2, P = the symmetric form), MDA_ENOMEM,
 * MDA_EDEVICE.
 */
int gqubo_build(int32_t m, int32_t K, const int32_t *Q, const int64_t *q, void *stream, mda_gqubo **out);
/* Sizes and the largest |C_k[a][b]| over k and a <= b (C the upper-triangular
 * form; the default schedule scales with it). */
int gqubo_info(const mda_gqubo *g, int32_t *m, int32_t *K, int64_t *maxabs_c);
void gqubo_free(mda_gqubo *g);

/* Runs p->replicas replicas, one wave each (asynchronous on p->stream; the
 * run holds a reference to g, which may be freed before the run).  The fields
 * of p are those of da_run, with variant MDA_VARIANT_AUTO or
 * MDA_VARIANT_PERSISTENT, graph 0 and waves_per_replica 0 or 1.  Each wave
 * keeps its replica's archive energies in LDS: archive_size * K is at most
 * 16384 (the default archive_size = m always fits; waves_per_block shrinks
 * until the block's archives fit).  Errors: as da_run, and MDA_EINVAL for the
 * unsupported fields and a larger archive. */
int gda_run(const mda_gqubo *g, const mda_params *p, mda_grun **out);
/* p as resolved (steps, schedule, beta, archive size). */
int gda_params_get(const mda_grun *r, mda_params *out);
/* Device time of the annealing kernel (synchronises). */
int gda_kernel_ms(mda_grun *r, double *ms);
/* Final state of one replica (synchronises): x (m bytes), h (K * m fields,
 * objective-major), E (K energies), offset, moves, trace (resolved steps,
 * needs trace_replicas); each may be NULL. */
int gda_state_get(mda_grun *r, int32_t replica, uint8_t *x, int64_t *h, int64_t *E, int64_t *e_offset,
                  int64_t *moves, int32_t *trace);
/*
 * Archives (synchronises).  replica >= 0 with raw = 1: that replica's archive
 * in slot order; raw = 0: the non-dominated entries of that replica's archive
 * (replica >= 0) or of the union over all replicas (replica = -1), equal
 * energy vectors reduced to the lowest (replica, slot), sorted
 * lexicographically by (E_1, ..., E_K, replica, slot).  e receives cap * K
 * energies; rep, slot and xbits (cap * ceil(m / 32) words, bit a of word
 * a / 32) may be NULL; e == NULL is a size query; *count gets the entries.
 * Errors: MDA_EINVAL, MDA_ERANGE (cap too small), MDA_EDEVICE.
 */
int garchive_get(mda_grun *r, int32_t replica, int32_t raw, int64_t cap, int64_t *e, int32_t *rep, int32_t *slot,
                 uint32_t *xbits, int64_t *count);
/* Run statistics summed over replicas, as da_stats: moves, archive entries
 * compared, random blocks drawn (one per wave-level draw), archive entries
 * (synchronises); each may be NULL. */
int gda_stats(mda_grun *r, int64_t *moves, int64_t *scanned, int64_t *rng_blocks, int64_t *archived);
void gda_run_free(mda_grun *r);

/* Debug/verification exports: the library's own host tables.
 * mda_temperature_table errors: MDA_EINVAL (NULL T, steps < 1), MDA_EOVERFLOW
 * (delta0 above 2^35, the largest starting temperature a run accepts). */
int mda_threshold_table(int32_t *lnt4096);
int mda_temperature_table(double delta0, double deltaf, double xi, int64_t steps, int64_t *T);

#ifdef __cplusplus
}
#endif
#endif
