// mda_server.cpp -- serving engine of the MI355X multi-objective Digital
// Annealer: bQAP solve requests arrive at any time and are admitted by device
// memory footprint; every scheduling round packs the admitted requests (any
// mix of n) into one batched launch on a free stream, so requests that arrive
// while others are on the GPU run alongside them.  Results stay on the device
// until the client collects them.  Each result is identical to a da_run of
// the same instance, parameters and seed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mda.h"
#include "mda_internal.h"

namespace {

int sfail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return mda::set_error(code, buf);
}

struct Request {
    int64_t id = 0;
    int32_t n = 0;
    std::vector<int32_t> F1, F2, D;
    mda_build_opts bo{};
    mda_params p{};
    std::vector<int64_t> T;   // the request's own copy of p.temp_table, if given
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    int64_t footprint = 0;
    int32_t batch = 0;
    int32_t slot = -1;
    mda_qubo *q = nullptr;
    mda_run *run = nullptr;
    int status = 0;   // 0 pending, 1 on the device, 2 done, < 0 failed (an MDA_E* code)
    std::string msg;
};

struct Flight {
    int slot = 0;
    std::vector<std::shared_ptr<Request>> reqs;
};

}  // namespace

struct mda_server {
    mda_server_opts o{};
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<char> busy;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> pending;
    std::map<int64_t, std::shared_ptr<Request>> live;   // submitted and not yet collected
    std::vector<Flight> flights;
    // device bytes of admitted requests whose runs still hold their memory: a
    // run's footprint is returned when its device memory is freed (da_run_free,
    // by the server or by the client that collected it, before or after
    // mda_server_destroy), so the counter outlives the server
    std::shared_ptr<std::atomic<int64_t>> used = std::make_shared<std::atomic<int64_t>>(0);
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    std::chrono::steady_clock::time_point t0;
    // statistics
    int64_t launches = 0, completed = 0, bit_trials = 0;
    double first_launch = -1, last_done = 0;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void run_worker();
};

void mda_server::run_worker()
{
    (void)hipSetDevice(device);
    mda::set_stream_ordered_alloc(true);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // 1. completed launches
        for (size_t f = 0; f < flights.size();) {
            bool done = true;
            for (auto &r : flights[f].reqs)
                if (r->run && mda::run_finished(r->run) == 0) done = false;
            if (!done) {
                ++f;
                continue;
            }
            const double t = now();
            for (auto &r : flights[f].reqs) {
                if (r->status == 1) {
                    r->status = 2;
                    r->t_done = t;
                    ++completed;
                    bit_trials += (int64_t)r->n * r->n * (int64_t)r->p.replicas * r->p.steps;
                }
                qubo_free(r->q);   // the run keeps its own reference
                r->q = nullptr;
            }
            last_done = t;
            busy[flights[f].slot] = 0;
            flights.erase(flights.begin() + (long)f);
            cv_done.notify_all();
        }
        if (stop && pending.empty() && flights.empty()) break;
        // 2. admission: FIFO, by footprint, into one launch per free stream
        int slot = -1;
        for (size_t k = 0; k < busy.size(); ++k)
            if (!busy[k]) {
                slot = (int)k;
                break;
            }
        if (slot >= 0 && !pending.empty()) {
            std::vector<std::shared_ptr<Request>> batch;
            int64_t left = o.hbm_budget - used->load();
            while (!pending.empty() && (int)batch.size() < o.max_batch) {
                auto r = pending.front();
                if (r->footprint > o.hbm_budget) {
                    pending.pop_front();
                    r->status = MDA_ENOMEM;
                    r->msg = "request needs more device memory than the server's budget";
                    cv_done.notify_all();
                    continue;
                }
                if (r->footprint > left) break;
                left -= r->footprint;
                pending.pop_front();
                batch.push_back(r);
            }
            if (!batch.empty()) {
                for (auto &r : batch) used->fetch_add(r->footprint);
                busy[slot] = 1;
                hipStream_t st = streams[slot];
                const double ta = now();
                lk.unlock();
                // build and launch outside the lock
                std::vector<const mda_qubo *> qs;
                std::vector<mda_params> ps;
                std::vector<std::shared_ptr<Request>> ok;
                for (auto &r : batch) {
                    r->t_admit = ta;
                    const int rc = qubo_build_bqap(r->n, r->F1.data(), r->F2.data(), r->D.data(), &r->bo, st, &r->q);
                    if (rc) {
                        r->status = rc;
                        r->msg = mda_last_error();
                        continue;
                    }
                    mda_params p = r->p;
                    p.stream = st;
                    p.graph = 0;
                    qs.push_back(r->q);
                    ps.push_back(p);
                    ok.push_back(r);
                }
                std::vector<mda_run *> outs(ok.size(), nullptr);
                int rc = MDA_OK;
                if (!ok.empty()) rc = da_run_batch(qs.data(), ps.data(), (int32_t)ok.size(), outs.data());
                const double tl = now();
                lk.lock();
                if (rc) {
                    for (auto &r : ok) {
                        r->status = rc;
                        r->msg = mda_last_error();
                    }
                }
                for (auto &r : batch) {
                    if (r->status < 0) {
                        used->fetch_sub(r->footprint);
                        if (r->q) qubo_free(r->q);
                        r->q = nullptr;
                    }
                }
                Flight fl;
                fl.slot = slot;
                for (size_t k = 0; k < ok.size(); ++k) {
                    if (rc) continue;
                    const int64_t fp = ok[k]->footprint;
                    std::shared_ptr<std::atomic<int64_t>> ctr = used;
                    mda::set_release_hook(outs[k], [ctr, fp] { ctr->fetch_sub(fp); });
                    ok[k]->run = outs[k];
                    ok[k]->status = 1;
                    ok[k]->t_launch = tl;
                    ok[k]->batch = (int32_t)ok.size();
                    ok[k]->slot = slot;
                    fl.reqs.push_back(ok[k]);
                }
                if (!fl.reqs.empty()) {
                    ++launches;
                    if (first_launch < 0) first_launch = tl;
                    flights.push_back(std::move(fl));
                } else {
                    busy[slot] = 0;
                }
                cv_done.notify_all();
                continue;   // look again at once: more may fit on another stream
            }
        }
        // 3. wait for work, for the device, or (requests waiting for memory
        // that collected runs still hold) for a release
        if (flights.empty() && pending.empty()) cv_work.wait(lk);
        else if (flights.empty()) cv_work.wait_for(lk, std::chrono::milliseconds(1));
        else cv_work.wait_for(lk, std::chrono::microseconds(200));
    }
}

extern "C" int mda_server_create(const mda_server_opts *opts, mda_server **out)
{
    if (!out) return sfail(MDA_EINVAL, "out is NULL");
    *out = nullptr;
    std::unique_ptr<mda_server> s(new mda_server);
    if (opts) s->o = *opts;
    if (s->o.max_inflight <= 0) s->o.max_inflight = 4;
    if (s->o.max_inflight > 8) return sfail(MDA_EINVAL, "max_inflight = %d outside [1, 8]", s->o.max_inflight);
    if (s->o.max_batch <= 0) s->o.max_batch = 64;
    if (s->o.device < 0) {
        if (hipGetDevice(&s->device) != hipSuccess) return sfail(MDA_EDEVICE, "no HIP device");
    } else {
        s->device = s->o.device;
    }
    if (hipSetDevice(s->device) != hipSuccess) return sfail(MDA_EDEVICE, "hipSetDevice(%d) failed", s->device);
    if (s->o.hbm_budget <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return sfail(MDA_EDEVICE, "hipMemGetInfo failed");
        s->o.hbm_budget = (int64_t)(fr / 2);
    }
    // keep freed stream-ordered memory in the pool between requests
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess && pool) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    for (int k = 0; k < s->o.max_inflight; ++k) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return sfail(MDA_EDEVICE, "stream creation failed");
        s->streams.push_back(st);
        s->busy.push_back(0);
    }
    s->t0 = std::chrono::steady_clock::now();
    mda_server *raw = s.get();
    raw->worker = std::thread([raw] { raw->run_worker(); });
    *out = s.release();
    return MDA_OK;
}

extern "C" int mda_server_submit(mda_server *s, int32_t n, const int32_t *F1, const int32_t *F2, const int32_t *D,
                                 const mda_build_opts *bo, const mda_params *p, int64_t *ticket)
{
    if (!s || !F1 || !F2 || !D || !p || !ticket) return sfail(MDA_EINVAL, "NULL argument");
    if (n < 2 || n > 100) return sfail(MDA_EINVAL, "n = %d outside [2, 100]", n);
    if (p->variant == MDA_VARIANT_PLAIN) return sfail(MDA_EINVAL, "the server runs the persistent form");
    if (p->replicas < 1 || p->steps < 1) return sfail(MDA_EINVAL, "replicas and steps must be set");
    auto r = std::make_shared<Request>();
    const size_t nn = (size_t)n * n;
    r->n = n;
    r->F1.assign(F1, F1 + nn);
    r->F2.assign(F2, F2 + nn);
    r->D.assign(D, D + nn);
    r->bo = bo ? *bo : mda_build_opts{MDA_PEN_2MAX, MDA_PATH_AUTO, 0};
    r->p = *p;
    if (p->temp_table) {
        r->T.assign(p->temp_table, p->temp_table + p->steps);
        r->p.temp_table = r->T.data();
    }
    r->footprint = mda_footprint(n, p, &r->bo);
    if (r->footprint < 0) return (int)r->footprint;
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return sfail(MDA_EBUSY, "server is stopping");
    r->id = s->next_id++;
    r->t_submit = s->now();
    s->pending.push_back(r);
    s->live[r->id] = r;
    *ticket = r->id;
    s->cv_work.notify_all();
    return MDA_OK;
}

extern "C" int mda_server_wait(mda_server *s, int64_t ticket, double timeout_s, mda_run **run, mda_request_info *info)
{
    if (!s) return sfail(MDA_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->live.find(ticket);
    if (it == s->live.end()) return sfail(MDA_EINVAL, "unknown ticket %lld", (long long)ticket);
    auto r = it->second;
    auto ready = [&] { return r->status == 2 || r->status < 0; };
    if (timeout_s < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
        return sfail(MDA_EBUSY, "request %lld not finished", (long long)ticket);
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->ticket = r->id;
        info->n = r->n;
        info->status = r->status;
        info->t_submit = r->t_submit;
        info->t_admit = r->t_admit;
        info->t_launch = r->t_launch;
        info->t_done = r->t_done;
        info->bit_trials = (int64_t)r->n * r->n * (int64_t)r->p.replicas * r->p.steps;
        info->footprint = r->footprint;
        info->batch = r->batch;
        info->slot = r->slot;
    }
    const int st = r->status;
    const std::string msg = r->msg;
    if (st == 2) {
        // the footprint is returned when the run is freed (its release hook)
        if (run) *run = r->run;
        else da_run_free(r->run);
        r->run = nullptr;
    }
    s->live.erase(it);
    s->cv_work.notify_all();
    if (st < 0) return sfail(st, "request %lld failed: %s", (long long)ticket, msg.c_str());
    return MDA_OK;
}

extern "C" int mda_server_stats(mda_server *s, mda_server_counters *out)
{
    if (!s || !out) return sfail(MDA_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    std::memset(out, 0, sizeof *out);
    out->launches = s->launches;
    out->completed = s->completed;
    out->bit_trials = s->bit_trials;
    out->pending = (int64_t)s->pending.size();
    out->in_flight = (int64_t)s->flights.size();
    out->hbm_used = s->used->load();
    out->hbm_budget = s->o.hbm_budget;
    out->now = s->now();
    out->first_launch = s->first_launch;
    out->last_done = s->last_done;
    return MDA_OK;
}

extern "C" void mda_server_destroy(mda_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        for (auto &r : s->pending) {
            r->status = MDA_EBUSY;
            r->msg = "server stopped before the request was admitted";
        }
        s->pending.clear();
        s->cv_work.notify_all();
        s->cv_done.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->live)
        if (kv.second->run) da_run_free(kv.second->run);
    // streams stay alive: runs handed to the client keep using them
    delete s;
}
