// server.hip -- continuous-batching search service (labs_server_* / labs_search_*).
//
// The server owns one HIP stream, a pool of walk slots carved out of a device-memory budget
// (each slot = one resident walk state plus its visited table) and a scheduler thread.  Every
// tick the scheduler admits queued jobs whose walks fit in the free slots, advances every
// resident walk by steps_per_tick logical steps in one launch of the walk kernel (mixed lengths
// in one grid), reads the walk states back into one of two pinned snapshots, and retires jobs
// that reached their budget or saw a target hit.  Ticks overlap: tick k is enqueued before the
// host summarises the snapshot of tick k-1, so the GPU does not wait for the host.  A job that
// stopped at tick k-1 may still be advanced by tick k (its walks are already done, or the extra
// steps are discarded); its result comes from the snapshot of the tick it stopped at.  Because
// all walks of a job start together and advance in lockstep of steps_per_tick logical steps, and a
// job can only stop at those boundaries, its result is a function of the request alone, whatever
// else shares the GPU.

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace liblabs {
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int check_device();
} // namespace liblabs

using namespace liblabs;

namespace {

struct Job {
    uint64_t id = 0;
    labs_search_req req{};
    int32_t n = 0;
    int64_t steps = 0;   // per-walk step budget
    int64_t isl_t = -1;  // integer target, -1 = none
    int32_t state = LABS_JOB_QUEUED;
    bool cancel = false;
    int64_t first_tick = -1; // the first tick that advanced its walks
    std::vector<int32_t> slots;
    labs_search_status st{};
};

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

} // namespace

struct labs_server {
    labs_server_opts opts{};
    std::chrono::steady_clock::time_point t0;
    hipStream_t stream = nullptr;
    int32_t max_slots = 0;
    int64_t table_words = 0;
    WalkState *d_states = nullptr;
    uint64_t *d_tables = nullptr;
    int32_t *d_order = nullptr;
    WalkState *h_states = nullptr;   // pinned: fresh states uploaded at admission
    WalkState *h_snap[2] = {};       // pinned: walk states read back after ticks (alternating)
    int32_t *h_order[2] = {};        // pinned: active slot lists of the ticks (alternating)
    hipEvent_t ev[2] = {};           // end of each alternating tick's readback
    std::vector<int32_t> free_slots;

    std::mutex mu;
    std::condition_variable cv_work;  // scheduler waits for work
    std::condition_variable cv_done;  // waiters wait for job completion
    std::deque<uint64_t> queue;
    std::map<uint64_t, Job> jobs;
    uint64_t next_id = 1;
    bool stop = false;
    int device_error = LABS_OK;
    std::thread worker;

    std::atomic<int64_t> ticks{0};
    std::atomic<int32_t> resident{0};
    std::atomic<int32_t> peak{0};
    std::atomic<int64_t> flips{0};
};

namespace {

void finish_job(labs_server *S, Job &j, int32_t state)
{
    j.state = state;
    j.st.state = state;
    j.st.t_done = now_s(S->t0);
    for (int32_t s : j.slots)
        S->free_slots.push_back(s);
    j.slots.clear();
}

// Summarise a job from its walks' states in a tick's snapshot.
void summarise(const WalkState *snap, Job &j)
{
    int64_t best = INT64_MAX, hit = -1, steps_done = INT64_MAX, fl = 0;
    int32_t best_w = -1, hit_w = -1;
    const WalkState *best_ws = nullptr;
    for (int32_t w = 0; w < (int32_t)j.slots.size(); w++) {
        const WalkState &ws = snap[j.slots[(size_t)w]];
        if (ws.best_isl < best) {
            best = ws.best_isl;
            best_w = w;
            best_ws = &ws;
        }
        if (ws.watch_step >= 0 && (hit < 0 || ws.watch_step < hit)) {
            hit = ws.watch_step;
            hit_w = w;
        }
        steps_done = std::min(steps_done, ws.t);
        fl += ws.flips;
    }
    j.st.best_isl = best;
    j.st.best_walk = best_w;
    j.st.best_F = best > 0 ? ((double)j.req.L * j.req.L) / (2.0 * (double)best) : -1.0;
    j.st.hit_step = hit;
    j.st.hit_walk = hit_w;
    j.st.steps_done = steps_done == INT64_MAX ? 0 : steps_done;
    j.st.flip_evals = fl;
    if (best_ws)
        memcpy(j.st.best_bits, best_ws->best_x, sizeof j.st.best_bits);
}

void cancel_all(labs_server *S)
{
    for (auto &kv : S->jobs)
        if (kv.second.state == LABS_JOB_RUNNING || kv.second.state == LABS_JOB_QUEUED)
            finish_job(S, kv.second, LABS_JOB_CANCELLED);
    S->queue.clear();
    S->cv_done.notify_all();
}

void scheduler(labs_server *S)
{
    WalkLaunch lp{};
    // the mixed-length matrix-core kernel serves every length (measured faster than the
    // bit-sliced one on mixed batches of L = 201..303)
    lp.variant = LABS_VARIANT_MFMA;
    lp.waves_per_block = 1;
    lp.probe_width = 2;
    lp.shape = -1;
    lp.chunk = S->opts.steps_per_tick;
    lp.persistent = 0;
    std::vector<int32_t> fresh;
    int64_t tick = 0;         // ticks enqueued so far
    bool in_flight = false;   // tick - 1 is enqueued and not summarised yet
    hipError_t e = hipSuccess;
    while (true) {
        int32_t n_active = 0;
        const int cur = (int)(tick & 1);
        bool idle = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // retire cancelled running jobs
            for (auto &kv : S->jobs) {
                Job &j = kv.second;
                if (j.state == LABS_JOB_RUNNING && j.cancel)
                    finish_job(S, j, LABS_JOB_CANCELLED);
            }
            // admit queued jobs in arrival order while their walks fit (slots freed by the last
            // summary are free on the GPU once the ticks already enqueued have run: the uploads
            // below follow them on the stream)
            fresh.clear();
            while (!S->stop && !S->queue.empty()) {
                Job &j = S->jobs[S->queue.front()];
                if (j.cancel) {
                    S->queue.pop_front();
                    continue;
                }
                if ((int32_t)S->free_slots.size() < j.req.n_walks)
                    break;
                S->queue.pop_front();
                j.state = LABS_JOB_RUNNING;
                j.st.state = LABS_JOB_RUNNING;
                j.st.t_admit = now_s(S->t0);
                j.first_tick = tick;
                for (int32_t w = 0; w < j.req.n_walks; w++) {
                    const int32_t slot = S->free_slots.back();
                    S->free_slots.pop_back();
                    j.slots.push_back(slot);
                    WalkState &ws = S->h_states[slot];
                    memset(&ws, 0, sizeof ws);
                    ws.L = j.req.L;
                    ws.table_log2 = S->opts.table_log2;
                    ws.seed = j.req.seed;
                    ws.walk_id = (uint32_t)w;
                    ws.steps = j.steps;
                    ws.restart_period = 0;
                    ws.target_isl = -1;       // walks run to the tick boundary ...
                    ws.watch_isl = j.isl_t;   // ... and record their first hit
                    ws.table_offset = (int64_t)slot * S->table_words;
                    ws.trace_offset = -1;
                    ws.score_offset = -1;
                    ws.step_cap = INT64_MAX;
                    ws.hit_step = -1;
                    ws.watch_step = -1;
                    ws.status = kFresh;
                    fresh.push_back(slot);
                }
            }
            // active list: every slot of a running job
            for (auto &kv : S->jobs) {
                const Job &j = kv.second;
                if (j.state != LABS_JOB_RUNNING)
                    continue;
                for (int32_t s : j.slots)
                    S->h_order[cur][n_active++] = s;
            }
            S->resident.store(n_active);
            if (n_active > S->peak.load())
                S->peak.store(n_active);
            if (n_active == 0 && !in_flight) {
                if (S->stop)
                    break;
                S->cv_work.wait_for(lk, std::chrono::milliseconds(50));
                continue;
            }
            idle = n_active == 0;
        }
        // enqueue tick `tick`: upload fresh states and the active list, advance, read back into
        // this tick's snapshot (the span of slots in use)
        if (!idle) {
            for (int32_t slot : fresh) {
                if (e == hipSuccess)
                    e = hipMemcpyAsync(S->d_states + slot, S->h_states + slot, sizeof(WalkState),
                                       hipMemcpyHostToDevice, S->stream);
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(S->d_order, S->h_order[cur], sizeof(int32_t) * (size_t)n_active,
                                   hipMemcpyHostToDevice, S->stream);
            if (e == hipSuccess)
                e = launch_walk(lp, S->d_states, n_active, S->d_order, S->d_tables, nullptr, nullptr, nullptr,
                                S->stream);
            if (e == hipSuccess) {
                int32_t lo = INT32_MAX, hi = -1;
                for (int32_t i = 0; i < n_active; i++) {
                    lo = std::min(lo, S->h_order[cur][i]);
                    hi = std::max(hi, S->h_order[cur][i]);
                }
                e = hipMemcpyAsync(S->h_snap[cur] + lo, S->d_states + lo, sizeof(WalkState) * (size_t)(hi - lo + 1),
                                   hipMemcpyDeviceToHost, S->stream);
            }
            if (e == hipSuccess)
                e = hipEventRecord(S->ev[cur], S->stream);
        }
        // summarise the previous tick while this one runs
        if (e == hipSuccess && in_flight)
            e = hipEventSynchronize(S->ev[cur ^ 1]);
        std::unique_lock<std::mutex> lk(S->mu);
        if (e != hipSuccess) {
            S->device_error = hip_fail(e, "server tick");
            cancel_all(S);
            break;
        }
        if (in_flight) {
            S->ticks.fetch_add(1);
            const WalkState *snap = S->h_snap[cur ^ 1];
            int64_t tick_flips = 0;
            for (auto &kv : S->jobs) {
                Job &j = kv.second;
                // jobs admitted after the summarised tick have no state in its snapshot
                if (j.state != LABS_JOB_RUNNING || j.first_tick > tick - 1)
                    continue;
                const int64_t before = j.st.flip_evals;
                summarise(snap, j);
                tick_flips += j.st.flip_evals - before;
                bool all_done = true;
                for (int32_t s : j.slots)
                    all_done = all_done && snap[s].status == kDone;
                if (all_done || j.st.hit_step >= 0 || j.cancel)
                    finish_job(S, j, j.cancel ? LABS_JOB_CANCELLED : LABS_JOB_DONE);
            }
            S->flips.fetch_add(tick_flips);
            S->cv_done.notify_all();
        }
        in_flight = !idle;
        if (!idle)
            tick++;
        if (S->stop && !in_flight)
            break;
    }
    // a stopped server leaves no tick in flight
    if (in_flight)
        (void)hipEventSynchronize(S->ev[(tick - 1) & 1]);
}

} // namespace

namespace {

void free_server_memory(labs_server *S)
{
    if (S->d_states) (void)hipFree(S->d_states);
    if (S->d_tables) (void)hipFree(S->d_tables);
    if (S->d_order) (void)hipFree(S->d_order);
    if (S->h_states) (void)hipHostFree(S->h_states);
    for (int b = 0; b < 2; b++) {
        if (S->h_snap[b]) (void)hipHostFree(S->h_snap[b]);
        if (S->h_order[b]) (void)hipHostFree(S->h_order[b]);
        if (S->ev[b]) (void)hipEventDestroy(S->ev[b]);
    }
    if (S->stream) (void)hipStreamDestroy(S->stream);
}

} // namespace

extern "C" int labs_server_create(const labs_server_opts *opts, labs_server **srv)
{
    if (!srv)
        return fail(LABS_EINVAL, "NULL srv");
    *srv = nullptr;
    labs_server_opts o{};
    if (opts)
        o = *opts;
    if (o.table_log2 == 0)
        o.table_log2 = 16;
    if (o.steps_per_tick == 0)
        o.steps_per_tick = 256;
    if (o.device_mem_bytes == 0)
        o.device_mem_bytes = (int64_t)8 << 30;
    if (o.table_log2 < 1 || o.table_log2 > 30 || o.steps_per_tick < 1 || o.device_mem_bytes < 0 || o.max_walks < 0)
        return fail(LABS_EINVAL, "bad server options");
    int rc = check_device();
    if (rc)
        return rc;
    labs_server *S = new labs_server();
    S->opts = o;
    S->t0 = std::chrono::steady_clock::now();
    S->table_words = (int64_t)1 << o.table_log2;
    const int64_t per_walk = S->table_words * 8 + (int64_t)sizeof(WalkState) + 4;
    int64_t slots = o.device_mem_bytes / per_walk;
    if (o.max_walks > 0)
        slots = std::min<int64_t>(slots, o.max_walks);
    slots = std::min<int64_t>(slots, 1 << 20);
    if (slots < 1) {
        delete S;
        return fail(LABS_ENOMEM, "device_mem_bytes holds no walk (%lld bytes per walk)", (long long)per_walk);
    }
    S->max_slots = (int32_t)slots;
    hipError_t e = hipStreamCreate(&S->stream);
    if (e == hipSuccess) e = hipMalloc(&S->d_states, sizeof(WalkState) * (size_t)slots);
    if (e == hipSuccess) e = hipMalloc(&S->d_tables, sizeof(uint64_t) * (size_t)(slots * S->table_words));
    if (e == hipSuccess) e = hipMalloc(&S->d_order, sizeof(int32_t) * (size_t)slots);
    if (e == hipSuccess) e = hipHostMalloc((void **)&S->h_states, sizeof(WalkState) * (size_t)slots, hipHostMallocDefault);
    for (int b = 0; b < 2; b++) {
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&S->h_snap[b], sizeof(WalkState) * (size_t)slots, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&S->h_order[b], sizeof(int32_t) * (size_t)slots, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&S->ev[b], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        free_server_memory(S);
        delete S;
        return hip_fail(e, "labs_server_create");
    }
    memset(S->h_states, 0, sizeof(WalkState) * (size_t)slots);
    for (int b = 0; b < 2; b++)
        memset(S->h_snap[b], 0, sizeof(WalkState) * (size_t)slots);
    for (int32_t s = (int32_t)slots - 1; s >= 0; s--)
        S->free_slots.push_back(s);
    S->worker = std::thread(scheduler, S);
    *srv = S;
    return LABS_OK;
}

extern "C" int labs_search_submit(labs_server *S, const labs_search_req *r, uint64_t *job_id)
{
    if (!S || !r || !job_id)
        return fail(LABS_EINVAL, "NULL argument");
    if (r->L < 3 || r->L > LABS_WALK_L_MAX || (r->L % 2) == 0)
        return fail(LABS_EINVAL, "L = %d must be odd in [3, %d]", r->L, LABS_WALK_L_MAX);
    if (r->n_walks < 1 || r->flip_budget < 0)
        return fail(LABS_EINVAL, "n_walks >= 1 and flip_budget >= 0 required");
    if (r->target_F_num > 0 && r->target_F_den <= 0)
        return fail(LABS_EINVAL, "target_F_den must be > 0");
    if (r->n_walks > S->max_slots)
        return fail(LABS_ENOMEM, "job needs %d walk slots, the budget holds %d", r->n_walks, S->max_slots);
    Job j;
    j.req = *r;
    j.n = (r->L + 1) / 2;
    j.steps = r->flip_budget / ((int64_t)r->n_walks * j.n);
    j.isl_t = -1;
    if (r->target_F_num > 0) {
        const int rc = labs_isl_threshold(r->L, r->target_F_num, r->target_F_den, &j.isl_t);
        if (rc)
            return rc;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->device_error)
        return fail(S->device_error, "server stopped after a device error");
    j.id = S->next_id++;
    j.st.state = LABS_JOB_QUEUED;
    j.st.best_walk = -1;
    j.st.hit_step = -1;
    j.st.hit_walk = -1;
    j.st.t_submit = now_s(S->t0);
    S->jobs[j.id] = j;
    S->queue.push_back(j.id);
    *job_id = j.id;
    S->cv_work.notify_one();
    return LABS_OK;
}

extern "C" int labs_search_poll(labs_server *S, uint64_t job_id, labs_search_status *st)
{
    if (!S || !st)
        return fail(LABS_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(job_id);
    if (it == S->jobs.end())
        return fail(LABS_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    *st = it->second.st;
    const int32_t s = it->second.state;
    return (s == LABS_JOB_DONE || s == LABS_JOB_CANCELLED) ? LABS_OK : LABS_EPENDING;
}

extern "C" int labs_search_wait(labs_server *S, uint64_t job_id, int64_t timeout_ms, labs_search_status *st)
{
    if (!S || !st)
        return fail(LABS_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms < 0 ? 0 : timeout_ms);
    while (true) {
        auto it = S->jobs.find(job_id);
        if (it == S->jobs.end())
            return fail(LABS_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
        const int32_t s = it->second.state;
        if (s == LABS_JOB_DONE || s == LABS_JOB_CANCELLED) {
            *st = it->second.st;
            return LABS_OK;
        }
        if (timeout_ms >= 0) {
            if (S->cv_done.wait_until(lk, deadline) == std::cv_status::timeout) {
                auto it2 = S->jobs.find(job_id);
                if (it2 == S->jobs.end())
                    return fail(LABS_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
                *st = it2->second.st;
                const int32_t s2 = it2->second.state;
                return (s2 == LABS_JOB_DONE || s2 == LABS_JOB_CANCELLED) ? LABS_OK : LABS_EPENDING;
            }
        } else {
            S->cv_done.wait(lk);
        }
    }
}

extern "C" int labs_search_cancel(labs_server *S, uint64_t job_id)
{
    if (!S)
        return fail(LABS_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(job_id);
    if (it == S->jobs.end())
        return fail(LABS_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    Job &j = it->second;
    if (j.state == LABS_JOB_QUEUED) {
        j.cancel = true;
        j.state = LABS_JOB_CANCELLED;
        j.st.state = LABS_JOB_CANCELLED;
        j.st.t_done = now_s(S->t0);
        S->cv_done.notify_all();
    } else if (j.state == LABS_JOB_RUNNING) {
        j.cancel = true;
    }
    S->cv_work.notify_one();
    return LABS_OK;
}

extern "C" int labs_server_stats(labs_server *S, int64_t *ticks, int32_t *resident_walks, int32_t *peak_walks,
                                 int64_t *flip_evals)
{
    if (!S)
        return fail(LABS_EINVAL, "NULL server");
    if (ticks) *ticks = S->ticks.load();
    if (resident_walks) *resident_walks = S->resident.load();
    if (peak_walks) *peak_walks = S->peak.load();
    if (flip_evals) *flip_evals = S->flips.load();
    return LABS_OK;
}

extern "C" int labs_search_release(labs_server *S, uint64_t job_id)
{
    if (!S)
        return fail(LABS_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(job_id);
    if (it == S->jobs.end())
        return fail(LABS_ENOTFOUND, "unknown job %llu", (unsigned long long)job_id);
    const int32_t st = it->second.state;
    if (st != LABS_JOB_DONE && st != LABS_JOB_CANCELLED)
        return fail(LABS_EPENDING, "job %llu is not finished", (unsigned long long)job_id);
    S->jobs.erase(it);
    return LABS_OK;
}

extern "C" void labs_server_destroy(labs_server *S)
{
    if (!S)
        return;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->stop = true;
        for (auto &kv : S->jobs)
            if (kv.second.state == LABS_JOB_RUNNING || kv.second.state == LABS_JOB_QUEUED)
                kv.second.cancel = true;
        S->cv_work.notify_all();
    }
    if (S->worker.joinable())
        S->worker.join();
    {
        // every job still queued or running ends cancelled (and its waiters wake up)
        std::unique_lock<std::mutex> lk(S->mu);
        cancel_all(S);
    }
    (void)hipStreamSynchronize(S->stream);
    free_server_memory(S);
    delete S;
}
