// da_server.cpp -- continuous-batching solve server.
//
// Jobs are submitted from any thread.  Three kinds of work overlap:
//   * host preparation (two prep threads): the device image of the coupling
//     matrix and the host image of the level tables of each submitted job;
//   * admission (the device worker): prepared jobs are admitted first-fit, in
//     submission order (never ahead of an earlier job still being prepared),
//     while their device footprint (da_job_footprint) fits the free budget; an admitted job's matrix, tables and initial state are
//     uploaded on an upload stream while the current epoch runs;
//   * epochs: every resident job advances by up to epoch_steps Monte Carlo
//     steps, all of them together in one persistent launch of the batched
//     step kernel (replayed from a captured graph);
//   * retirement: after an epoch, jobs that reached their step count are
//     copied to host buffers and their device memory is released, which lets
//     waiting jobs in;
//   * preemption: when the highest-priority waiting job does not fit, resident
//     jobs of lower priority are snapshotted to host memory between epochs and
//     released; they queue again and resume from the snapshot when re-admitted.
// The step kernel resumes exactly where an epoch stopped and every random
// number is keyed by (seed, job-local replica id, global step), so a job's
// results are the same alone, in any mix, and as a plain da_anneal call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "da_runtime.h"

using namespace dapt;

namespace {

constexpr int64_t kDefaultEpochSteps = 8192;
constexpr int kPrepThreads = 2;

struct Job {
    uint64_t ticket = 0;
    std::vector<int32_t> Q;           // until prepared
    da_job spec{};
    int32_t dtype = 0, wscale = 1;
    int64_t footprint = 0;
    HostMatrix hm;                    // prepared, until uploaded
    std::unique_ptr<HostTables> ht;   // prepared, until uploaded
    da_ctx *ctx = nullptr;
    std::shared_ptr<LevelTables> tables;
    JobDesc J{};
    std::atomic<int64_t> done_steps{0};   // written by the worker, read by status queries
    int32_t priority = 0;
    // a preempted job's replica state (host), restored when it is re-admitted
    bool preempted = false;
    std::vector<uint8_t> snap_x, snap_bx;
    std::vector<int32_t> snap_h, snap_eoff;
    std::vector<int64_t> snap_E, snap_bE, snap_nacc;
    int status = DA_OK;
    std::string err;
    // results
    std::vector<uint8_t> best_x, final_x;
    std::vector<int64_t> best_E, final_E, n_accept;
    da_job_stats stats{};
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct da_server {
    size_t budget = 0;
    int64_t epoch_steps = kDefaultEpochSteps;
    int32_t max_resident = 0;
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_prep, cv_work, cv_done;
    std::deque<std::unique_ptr<Job>> incoming;        // submitted, not yet prepared
    std::set<uint64_t> preparing;                     // taken by a prep thread
    std::deque<std::unique_ptr<Job>> queue;           // prepared, in ticket order
    std::vector<std::unique_ptr<Job>> resident;
    std::map<uint64_t, std::unique_ptr<Job>> finished;
    std::set<uint64_t> retiring;   // left `resident`, results being copied out
    std::set<uint64_t> preempting; // left `resident`, state being copied out
    uint64_t next_ticket = 1;
    int64_t used = 0;
    bool stop = false;
    std::vector<std::thread> prep;
    std::thread worker;
    hipStream_t stream = nullptr;   // epochs and result copies
    hipStream_t upload = nullptr;   // admission uploads and state initialisation
    BatchRunner runner;

    void prep_loop();
    void run();
    bool admit_locked(std::vector<Job *> &admitted);
    int start_job(Job &j);
    void retire(std::unique_ptr<Job> &j);
    void pick_victims_locked(std::vector<std::unique_ptr<Job>> &victims);
    void preempt(Job &j);
    void enqueue_locked(std::unique_ptr<Job> jp);
    bool known_locked(uint64_t ticket) const;
    uint64_t first_unprepared_locked() const {
        uint64_t t = UINT64_MAX;
        for (auto &q : incoming) t = std::min(t, q->ticket);
        for (uint64_t p : preparing) t = std::min(t, p);
        return t;
    }
    // something the device worker can do now
    bool has_work_locked() const {
        if (stop || !resident.empty()) return true;
        const uint64_t fu = first_unprepared_locked();
        for (auto &q : queue)
            if (q->ticket < fu) return true;
        return false;
    }
    // queue order: higher priority first, then submission order
    static bool before(const Job &a, const Job &b) {
        return a.priority != b.priority ? a.priority > b.priority : a.ticket < b.ticket;
    }
};

extern "C" int64_t da_job_footprint(int32_t N, int32_t dtype_bytes, int32_t replicas,
                                    int32_t n_levels) {
    if (N < 1 || replicas < 1 || n_levels < 1 || (dtype_bytes != 1 && dtype_bytes != 2 &&
                                                   dtype_bytes != 4))
        return -1;
    const int64_t ld = ((int64_t)N + 63) / 64 * 64;
    const int64_t w = ld * ld * dtype_bytes + ld * 4;
    const int64_t state = StateBuf::bytes_for(replicas, (int32_t)ld);
    const int64_t tables = level_table_bytes(n_levels, (int64_t)n_levels * kMaxBuckets);
    const int64_t out = (int64_t)replicas * N * 2 + (int64_t)replicas * 8 * 3;
    return w + state + tables + out;
}

// Host preparation of submitted jobs, off the submitting and device threads.
void da_server::prep_loop() {
    for (;;) {
        std::unique_ptr<Job> jp;
        {
            std::unique_lock<std::mutex> lock(mu);
            cv_prep.wait(lock, [&] { return stop || !incoming.empty(); });
            if (stop) return;
            jp = std::move(incoming.front());
            incoming.pop_front();
            preparing.insert(jp->ticket);
        }
        Job &j = *jp;
        prepare_matrix(j.Q.data(), j.spec.N, j.dtype, j.wscale, j.hm);
        std::vector<int32_t>().swap(j.Q);
        j.ht.reset(new HostTables());
        build_host_tables(schedule_temps(j.spec.schedule), *j.ht);
        {
            std::lock_guard<std::mutex> lock(mu);
            preparing.erase(j.ticket);
            enqueue_locked(std::move(jp));
        }
        cv_work.notify_one();
    }
}

void da_server::enqueue_locked(std::unique_ptr<Job> jp) {
    auto pos = std::upper_bound(queue.begin(), queue.end(), jp,
                                [](const std::unique_ptr<Job> &a, const std::unique_ptr<Job> &b) {
                                    return before(*a, *b);
                                });
    queue.insert(pos, std::move(jp));
}

// Device context, tables and initial state of an admitted job, on the upload
// stream (the caller synchronises it before the job's first epoch).
int da_server::start_job(Job &j) {
    da_ctx *ctx = nullptr;
    int rc = create_ctx(j.hm, upload, &ctx, j.err);
    HostMatrix().W.swap(j.hm.W);
    if (rc) return rc;
    j.ctx = ctx;
    // (a re-admitted job's tables come from the cache, or are built again)
    j.tables = get_level_tables(schedule_temps(j.spec.schedule), j.err, j.ht.get());
    j.ht.reset();
    if (!j.tables) return DA_ENOMEM;
    ctx->keep_tables = j.tables;
    if (!ctx->st.ensure(j.spec.replicas, ctx->ld, j.err)) return DA_ENOMEM;
    const LaunchShape sh = batch_shape(ctx);
    j.J = make_job(ctx, *j.tables, j.spec.replicas, 0u, j.spec.seed, j.spec.steps,
                   j.spec.schedule, sh);
    if (const char *why = job_range_error(j.J)) {
        j.err = why;
        return DA_EINVAL;
    }
    if (!j.preempted) {
        rc = init_state(ctx, j.J, j.spec.schedule.init, upload);
        if (rc) j.err = ctx->err;
        return rc;
    }
    // continue from the snapshot (the host copies live until the upload
    // stream is synchronised, before the job's next epoch)
    const size_t R = (size_t)j.spec.replicas, rows = R * (size_t)j.J.ld;
    hipError_t e = hipMemcpyAsync(j.J.x, j.snap_x.data(), rows, hipMemcpyHostToDevice, upload);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.J.bx, j.snap_bx.data(), rows, hipMemcpyHostToDevice, upload);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.J.h, j.snap_h.data(), rows * 4, hipMemcpyHostToDevice, upload);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.J.E, j.snap_E.data(), R * 8, hipMemcpyHostToDevice, upload);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.J.bE, j.snap_bE.data(), R * 8, hipMemcpyHostToDevice, upload);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.J.nacc, j.snap_nacc.data(), R * 8, hipMemcpyHostToDevice, upload);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.J.eoff, j.snap_eoff.data(), R * 4, hipMemcpyHostToDevice, upload);
    if (e != hipSuccess) {
        j.err = std::string("snapshot upload: ") + hipGetErrorString(e);
        return DA_EDEVICE;
    }
    return DA_OK;
}

// Resident jobs to send back to the queue so that the highest-priority
// waiting job fits: strictly lower priority only, lowest priority and then
// latest admitted first, and only if enough of them free enough room.
void da_server::pick_victims_locked(std::vector<std::unique_ptr<Job>> &victims) {
    const uint64_t fu = first_unprepared_locked();
    Job *head = nullptr;
    for (auto &q : queue)
        if (q->ticket < fu) {
            head = q.get();
            break;
        }
    if (!head) return;
    auto fits = [&](int64_t freed, size_t leaving) {
        const bool mem = head->footprint <= (int64_t)budget - used + freed;
        const bool slots = max_resident <= 0 ||
                           (int64_t)resident.size() - (int64_t)leaving < (int64_t)max_resident;
        return mem && slots;
    };
    if (fits(0, 0)) return;   // it is admitted on the next pass
    std::vector<size_t> cand;
    for (size_t i = 0; i < resident.size(); ++i)
        if (resident[i]->priority < head->priority && resident[i]->status == DA_OK &&
            resident[i]->done_steps < resident[i]->spec.steps)
            cand.push_back(i);
    std::stable_sort(cand.begin(), cand.end(), [&](size_t a, size_t b) {
        const Job &x = *resident[a], &y = *resident[b];
        if (x.priority != y.priority) return x.priority < y.priority;
        return x.stats.t_admit > y.stats.t_admit;
    });
    int64_t freed = 0;
    size_t n = 0;
    while (n < cand.size() && !fits(freed, n)) freed += resident[cand[n++]]->footprint;
    if (!fits(freed, n)) return;   // even all of them would not make room
    std::vector<size_t> take(cand.begin(), cand.begin() + (ptrdiff_t)n);
    std::sort(take.rbegin(), take.rend());   // erase from the back
    for (size_t i : take) {
        preempting.insert(resident[i]->ticket);
        victims.push_back(std::move(resident[i]));
        resident.erase(resident.begin() + (ptrdiff_t)i);
    }
}

// Copies a resident job's replica state and coupling matrix to host memory
// and frees its device memory (no epoch is in flight when this runs).
void da_server::preempt(Job &j) {
    da_ctx *ctx = j.ctx;
    const size_t R = (size_t)j.spec.replicas, ld = (size_t)j.J.ld, rows = R * ld;
    j.snap_x.resize(rows);
    j.snap_bx.resize(rows);
    j.snap_h.resize(rows);
    j.snap_E.resize(R);
    j.snap_bE.resize(R);
    j.snap_nacc.resize(R);
    j.snap_eoff.resize(R);
    j.hm.W.resize(ld * ld * (size_t)ctx->dtype);
    hipError_t e = hipMemcpyAsync(j.snap_x.data(), j.J.x, rows, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.snap_bx.data(), j.J.bx, rows, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.snap_h.data(), j.J.h, rows * 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.snap_E.data(), j.J.E, R * 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.snap_bE.data(), j.J.bE, R * 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.snap_nacc.data(), j.J.nacc, R * 8, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.snap_eoff.data(), j.J.eoff, R * 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(j.hm.W.data(), ctx->d_W, j.hm.W.size(), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        j.status = DA_EDEVICE;
        j.err = std::string("preemption snapshot: ") + hipGetErrorString(e);
    }
    da_destroy(ctx);
    j.ctx = nullptr;
    j.tables.reset();
    j.preempted = true;
    j.stats.preemptions += 1;
}

bool da_server::admit_locked(std::vector<Job *> &admitted) {
    bool any = false;
    // submission order: a job never overtakes an earlier one still being prepared
    const uint64_t first_unprepared = first_unprepared_locked();
    for (auto it = queue.begin(); it != queue.end();) {
        if ((*it)->ticket > first_unprepared) {
            ++it;
            continue;
        }
        if (max_resident > 0 && (int32_t)(resident.size() + admitted.size()) >= max_resident) break;
        if ((*it)->footprint <= (int64_t)budget - used) {
            used += (*it)->footprint;
            (*it)->stats.t_admit = now_s(t0);
            admitted.push_back(it->get());
            resident.push_back(std::move(*it));
            it = queue.erase(it);
            any = true;
        } else {
            ++it;
        }
    }
    return any;
}

void da_server::retire(std::unique_ptr<Job> &jp) {
    Job &j = *jp;
    if (j.status == DA_OK && j.ctx) {
        const size_t R = (size_t)j.spec.replicas, N = (size_t)j.spec.N, ld = (size_t)j.J.ld;
        j.best_x.resize(R * N);
        j.final_x.resize(R * N);
        j.best_E.resize(R);
        j.final_E.resize(R);
        j.n_accept.resize(R);
        hipError_t e = hipMemcpy2DAsync(j.best_x.data(), N, j.J.bx, ld, N, R,
                                        hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(j.final_x.data(), N, j.J.x, ld, N, R, hipMemcpyDeviceToHost,
                                 stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(j.best_E.data(), j.J.bE, R * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(j.final_E.data(), j.J.E, R * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(j.n_accept.data(), j.J.nacc, R * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            j.status = DA_EDEVICE;
            j.err = hipGetErrorString(e);
        }
    }
    if (j.ctx) da_destroy(j.ctx);
    j.ctx = nullptr;
    j.tables.reset();
    for (auto *v : {&j.snap_x, &j.snap_bx}) std::vector<uint8_t>().swap(*v);
    for (auto *v : {&j.snap_h, &j.snap_eoff}) std::vector<int32_t>().swap(*v);
    for (auto *v : {&j.snap_E, &j.snap_bE, &j.snap_nacc}) std::vector<int64_t>().swap(*v);
    j.stats.t_done = now_s(t0);
}

// The device worker.  Each pass: admit and upload new jobs (overlapping the
// epoch in flight), finish that epoch, retire, then launch the next epoch
// without waiting for it.
void da_server::run() {
    // every launch and copy of this thread goes to the server's device; if it
    // cannot be selected, every job fails with that error instead of running
    const hipError_t dev_err = hipSetDevice(device);
    std::vector<Job *> in_epoch;
    std::vector<JobDesc> jobs;
    bool inflight = false;
    for (;;) {
        std::vector<Job *> admitted;
        {
            std::unique_lock<std::mutex> lock(mu);
            if (!inflight) cv_work.wait(lock, [&] { return has_work_locked(); });
            if (stop) {
                for (auto *dq : {&incoming, &queue})
                    for (auto &q : *dq) {
                        q->status = DA_ENOTFOUND;
                        q->err = "server shut down before the job was admitted";
                    }
                incoming.clear();
                queue.clear();
                if (resident.empty() && !inflight) break;
            } else {
                admit_locked(admitted);
            }
        }
        for (Job *j : admitted) {
            if (dev_err != hipSuccess) {
                j->status = DA_EDEVICE;
                j->err = std::string("server device selection failed: ") +
                         hipGetErrorString(dev_err);
            } else {
                j->status = start_job(*j);
            }
            j->stats.device_bytes = j->footprint;
        }
        if (inflight) {
            std::string err;
            int rc = DA_OK;
            const hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) {
                rc = DA_EDEVICE;
                err = hipGetErrorString(e);
            }
            for (size_t a = 0; a < in_epoch.size(); ++a) {
                Job &j = *in_epoch[a];
                if (rc) {
                    j.status = rc;
                    j.err = err;
                } else {
                    j.done_steps = jobs[a].s1;
                    j.stats.epochs += 1;
                }
            }
            inflight = false;
        }
        if (!admitted.empty()) {
            const hipError_t e = hipStreamSynchronize(upload);
            for (Job *j : admitted) {
                if (e != hipSuccess && j->status == DA_OK) {
                    j->status = DA_EDEVICE;
                    j->err = hipGetErrorString(e);
                }
                // a re-admitted job's snapshot is on the device now
                for (auto *v : {&j->snap_x, &j->snap_bx}) std::vector<uint8_t>().swap(*v);
                for (auto *v : {&j->snap_h, &j->snap_eoff}) std::vector<int32_t>().swap(*v);
                for (auto *v : {&j->snap_E, &j->snap_bE, &j->snap_nacc})
                    std::vector<int64_t>().swap(*v);
                j->preempted = false;
            }
        }
        // retire finished (or failed) jobs and wake their waiters
        std::vector<std::unique_ptr<Job>> leaving;
        {
            std::lock_guard<std::mutex> lock(mu);
            for (auto it = resident.begin(); it != resident.end();) {
                if ((*it)->status != DA_OK || (*it)->done_steps >= (*it)->spec.steps) {
                    retiring.insert((*it)->ticket);
                    leaving.push_back(std::move(*it));
                    it = resident.erase(it);
                } else {
                    ++it;
                }
            }
        }
        for (auto &jp : leaving) retire(jp);
        if (!leaving.empty()) {
            {
                std::lock_guard<std::mutex> lock(mu);
                for (auto &jp : leaving) {
                    used -= jp->footprint;
                    const uint64_t t = jp->ticket;
                    retiring.erase(t);
                    finished[t] = std::move(jp);
                }
            }
            cv_done.notify_all();
        }
        // preemption (no epoch in flight here): lower-priority resident jobs
        // make room for the highest-priority waiting job that does not fit;
        // it is admitted on the next pass, while the next epoch runs
        std::vector<std::unique_ptr<Job>> victims;
        if (!stop) {
            std::lock_guard<std::mutex> lock(mu);
            pick_victims_locked(victims);
        }
        for (auto &vp : victims) preempt(*vp);
        if (!victims.empty()) {
            {
                std::lock_guard<std::mutex> lock(mu);
                for (auto &vp : victims) {
                    used -= vp->footprint;
                    preempting.erase(vp->ticket);
                    if (vp->status != DA_OK) {
                        vp->stats.t_done = now_s(t0);
                        const uint64_t t = vp->ticket;
                        finished[t] = std::move(vp);
                    } else {
                        enqueue_locked(std::move(vp));
                    }
                }
            }
            cv_done.notify_all();
        }
        // next epoch over every resident job, launched without waiting
        in_epoch.clear();
        jobs.clear();
        std::vector<BatchItem> items;
        {
            std::lock_guard<std::mutex> lock(mu);
            for (auto &jp : resident) {
                Job &j = *jp;
                JobDesc J = j.J;
                J.s0 = j.done_steps;
                J.s1 = std::min(j.spec.steps, j.done_steps + epoch_steps);
                append_batch_items(J, (int)jobs.size(), items);
                jobs.push_back(J);
                in_epoch.push_back(&j);
            }
        }
        if (!jobs.empty()) {
            std::string err;
            const int rc = runner.run(jobs, items, stream, err);
            if (rc) {
                for (Job *j : in_epoch) {
                    j->status = rc;
                    j->err = err;
                }
            } else {
                inflight = true;
            }
        }
    }
    cv_done.notify_all();
}

bool da_server::known_locked(uint64_t ticket) const {
    if (finished.count(ticket) || retiring.count(ticket) || preparing.count(ticket) ||
        preempting.count(ticket))
        return true;
    for (auto *dq : {&incoming, &queue})
        for (auto &q : *dq)
            if (q->ticket == ticket) return true;
    for (auto &q : resident)
        if (q->ticket == ticket) return true;
    return false;
}

extern "C" {

int da_server_create(size_t hbm_budget, const da_server_opts *opts, da_server **out) {
    if (!out) return fail(nullptr, DA_EINVAL, "out is null");
    *out = nullptr;
    if (hbm_budget == 0) return fail(nullptr, DA_EINVAL, "hbm_budget must be > 0");
    auto *srv = new (std::nothrow) da_server();
    if (!srv) return fail(nullptr, DA_ENOMEM, "host allocation failed");
    srv->budget = hbm_budget;
    if (opts && opts->epoch_steps > 0) srv->epoch_steps = opts->epoch_steps;
    srv->max_resident = BatchRunner::kCapJobs;
    if (opts && opts->max_resident > 0)
        srv->max_resident = std::min<int32_t>(opts->max_resident, BatchRunner::kCapJobs);
    srv->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&srv->device) != hipSuccess) {
        delete srv;
        return fail(nullptr, DA_EDEVICE, "no current HIP device");
    }
    if (hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&srv->upload, hipStreamNonBlocking) != hipSuccess) {
        if (srv->stream) (void)hipStreamDestroy(srv->stream);
        delete srv;
        return fail(nullptr, DA_EDEVICE, "server stream creation failed");
    }
    std::string err;
    const int rc = srv->runner.prepare(err);
    if (rc) {
        (void)hipStreamDestroy(srv->stream);
        (void)hipStreamDestroy(srv->upload);
        delete srv;
        return fail(nullptr, rc, err);
    }
    for (int t = 0; t < kPrepThreads; ++t) srv->prep.emplace_back([srv] { srv->prep_loop(); });
    srv->worker = std::thread([srv] { srv->run(); });
    *out = srv;
    return DA_OK;
}

int da_submit(da_server *srv, const da_job *job, uint64_t *ticket) {
    if (!srv || !job || !ticket || !job->Q) return fail(nullptr, DA_EINVAL, "null argument");
    if (job->N < 1 || job->N > DA_MAX_N) return fail(nullptr, DA_EINVAL, "N must be in [1, 8192]");
    if (job->replicas < 1 || job->steps < 0 || job->steps >= (int64_t(1) << 31))
        return fail(nullptr, DA_EINVAL, "bad replicas or steps");
    const double t_submit = now_s(srv->t0);
    std::string err;
    int rc = validate_schedule(&job->schedule, err);
    if (rc) return fail(nullptr, rc, err);
    if (job->schedule.n_levels == 0)
        return fail(nullptr, DA_EINVAL, "per-step schedules are run by da_anneal*, not served");
    auto j = std::make_unique<Job>();
    // the server keeps jobs in dense storage (sparse row lists are a da_create option)
    rc = derive_storage(job->Q, job->N, job->dtype_hint & ~DA_STORE_SPARSE, j->dtype, j->wscale,
                        err);
    if (rc) return fail(nullptr, rc, err);
    j->footprint = da_job_footprint(job->N, j->dtype, job->replicas, job->schedule.n_levels);
    if (j->footprint > (int64_t)srv->budget)
        return fail(nullptr, DA_ENOMEM, "job alone exceeds the server's device budget");
    j->spec = *job;
    j->priority = job->priority;
    j->Q.assign(job->Q, job->Q + (size_t)job->N * job->N);
    j->spec.Q = j->Q.data();
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        j->ticket = srv->next_ticket++;
        j->stats.t_submit = t_submit;
        *ticket = j->ticket;
        srv->incoming.push_back(std::move(j));
    }
    srv->cv_prep.notify_one();
    return DA_OK;
}

static int collect(da_server *srv, uint64_t ticket, da_result *out, da_job_stats *stats,
                   bool wait) {
    if (!srv) return fail(nullptr, DA_EINVAL, "server is null");
    std::unique_ptr<Job> j;
    {
        std::unique_lock<std::mutex> lock(srv->mu);
        auto known = [&] { return srv->known_locked(ticket); };
        if (!known()) return fail(nullptr, DA_ENOTFOUND, "unknown or already collected ticket");
        if (wait) {
            srv->cv_done.wait(lock, [&] { return srv->finished.count(ticket) > 0 || !known(); });
        }
        auto it = srv->finished.find(ticket);
        if (it == srv->finished.end()) {
            if (!known()) return fail(nullptr, DA_ENOTFOUND, "job was dropped");
            return DA_ENOTREADY;
        }
        j = std::move(it->second);
        srv->finished.erase(it);
    }
    if (stats) *stats = j->stats;
    if (j->status != DA_OK) return fail(nullptr, j->status, j->err);
    if (out) {
        if (out->best_x) std::memcpy(out->best_x, j->best_x.data(), j->best_x.size());
        if (out->final_x) std::memcpy(out->final_x, j->final_x.data(), j->final_x.size());
        if (out->best_E) std::memcpy(out->best_E, j->best_E.data(), j->best_E.size() * 8);
        if (out->final_E) std::memcpy(out->final_E, j->final_E.data(), j->final_E.size() * 8);
        if (out->n_accept) std::memcpy(out->n_accept, j->n_accept.data(), j->n_accept.size() * 8);
    }
    return DA_OK;
}

int da_job_status(da_server *srv, uint64_t ticket, int32_t *state, int64_t *done_steps) {
    if (!srv) return fail(nullptr, DA_EINVAL, "server is null");
    std::lock_guard<std::mutex> lock(srv->mu);
    int32_t st = -1;
    int64_t done = 0;
    auto f = srv->finished.find(ticket);
    if (f != srv->finished.end()) {
        st = 2;
        done = f->second->done_steps;
    } else if (srv->retiring.count(ticket)) {
        st = 2;
    } else {
        for (auto &q : srv->resident)
            if (q->ticket == ticket) {
                st = 1;
                done = q->done_steps;
            }
        if (st < 0 && srv->known_locked(ticket)) {
            st = 0;
            for (auto &q : srv->queue)
                if (q->ticket == ticket) done = q->done_steps;
        }
    }
    if (st < 0) return fail(nullptr, DA_ENOTFOUND, "unknown or already collected ticket");
    if (state) *state = st;
    if (done_steps) *done_steps = done;
    return DA_OK;
}

int da_poll(da_server *srv, uint64_t ticket, da_result *out, da_job_stats *stats) {
    return collect(srv, ticket, out, stats, false);
}

int da_wait(da_server *srv, uint64_t ticket, da_result *out, da_job_stats *stats) {
    return collect(srv, ticket, out, stats, true);
}

void da_server_destroy(da_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stop = true;
    }
    srv->cv_prep.notify_all();
    srv->cv_work.notify_all();
    for (auto &t : srv->prep)
        if (t.joinable()) t.join();
    if (srv->worker.joinable()) srv->worker.join();
    {
        // jobs a prep thread finished after the worker stopped admitting
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->queue.clear();
        srv->incoming.clear();
    }
    srv->cv_done.notify_all();
    srv->runner.release();
    if (srv->stream) (void)hipStreamDestroy(srv->stream);
    if (srv->upload) (void)hipStreamDestroy(srv->upload);
    delete srv;
}

}  // extern "C"
