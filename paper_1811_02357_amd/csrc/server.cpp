// server.cpp -- continuous batching of IRT-PS reconstructions.
//
// A scheduler thread owns one HIP stream and a device memory budget handed in
// by the caller.  Submitted jobs wait in FIFO order; a job is admitted when a
// region of its workspace footprint fits in the budget (first fit).  Newly
// admitted jobs get their t = 0 steps (PS of the inputs, cold integration);
// then every resident job advances by one IRT iteration in the same set of
// launches (the multi-job engine), so jobs that arrive while others run join
// at the next iteration boundary and leave when their own T is reached.  Each
// job's arithmetic depends only on its own inputs and seed, so its result is
// the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "host.hpp"
#include "irtps.h"

using namespace irtps;
using namespace irtps::host;

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Job {
    uint64_t id = 0;
    irtps_problem pr{};
    irtps_params pa{};
    irtps_outputs out{};
    std::vector<float> lights, intens;  // host copies of the calibration
    size_t bytes = 0;                   // workspace footprint
    size_t offset = 0;                  // region in the budget once admitted
    int state = IRTPS_JOB_QUEUED;
    int status = IRTPS_OK;
    int t = 0;
    int t_last = 0;                     // iterations to run: T, lowered by the stop rule
    int tiles = 0;                      // tracer tiles (table space while resident)
    bool admitted = false;
    bool initialised = false;
    bool cancel = false;
    double t_submit = 0, t_start = 0, t_end = 0;
};

// First-fit allocator over [0, size) with 256-byte granularity.
struct Regions {
    std::map<size_t, size_t> free;  // offset -> length
    void reset(size_t size) {
        free.clear();
        if (size) free[0] = size;
    }
    bool take(size_t bytes, size_t* off) {
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t next = it->first + bytes;
                free.erase(it);
                if (rest) free[next] = rest;
                return true;
            }
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        auto it = free.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

}  // namespace

struct irtps_server {
    irtps_server_cfg cfg{};
    char* base = nullptr;   // caller's device memory
    size_t table_bytes = 0; // head of the budget: job table and tile lists
    size_t pool_bytes = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::thread worker;
    bool stop = false;
    uint64_t next_id = 1;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Job> jobs;
    std::vector<uint64_t> resident;
    Regions regions;
    size_t in_use = 0;
    long long resident_tiles = 0;
    // statistics
    uint64_t submitted = 0, completed = 0, failed = 0, cancelled = 0;
    std::vector<double> latencies;
    double first_submit = 0, last_end = 0;
    uint64_t iterations = 0, segments_budget = 0;

    void run();
    bool step();  // one scheduling round; false when idle
};

namespace {

void finish(irtps_server* s, Job& J, int state, int status) {
    J.state = state;
    J.status = status;
    J.t_end = now_s();
    if (J.admitted) {
        s->regions.give(J.offset, J.bytes);
        s->in_use -= J.bytes;
        s->resident_tiles -= J.tiles;
        J.admitted = false;
    }
    if (state == IRTPS_JOB_DONE) {
        ++s->completed;
        s->latencies.push_back(J.t_end - J.t_submit);
        s->last_end = J.t_end;
    } else if (state == IRTPS_JOB_CANCELLED) {
        ++s->cancelled;
    } else {
        ++s->failed;
    }
}

}  // namespace

bool irtps_server::step() {
    std::vector<kern::JobDesc> fresh, running;
    std::vector<uint64_t> fresh_ids, running_ids;
    std::vector<int> running_T;  // each running job's T after its iteration
    {
        std::unique_lock<std::mutex> lock(mu);
        // cancellations take effect at the iteration boundary; a job whose state
        // changes here wakes its waiters even if nothing else runs this round
        bool changed = false;
        for (auto it = resident.begin(); it != resident.end();) {
            Job& J = jobs[*it];
            if (J.cancel) {
                finish(this, J, IRTPS_JOB_CANCELLED, IRTPS_ERR_CANCELLED);
                it = resident.erase(it);
                changed = true;
            } else {
                ++it;
            }
        }
        // admission, FIFO, by footprint
        while (!queue.empty()) {
            Job& J = jobs[queue.front()];
            if (J.cancel) {
                J.state = IRTPS_JOB_CANCELLED;
                J.status = IRTPS_ERR_CANCELLED;
                J.t_end = now_s();
                ++cancelled;
                queue.pop_front();
                changed = true;
                continue;
            }
            if (cfg.max_resident_jobs > 0 && (int)resident.size() >= cfg.max_resident_jobs) break;
            // the resident set's descriptors and tile lists must fit the table area
            if (eng::table_bytes((int)resident.size() + 1, (int)(resident_tiles + J.tiles)) > table_bytes) break;
            size_t off = 0;
            if (!regions.take(J.bytes, &off)) break;
            J.offset = off;
            J.admitted = true;
            in_use += J.bytes;
            resident_tiles += J.tiles;
            J.state = IRTPS_JOB_RUNNING;
            J.t_start = now_s();
            resident.push_back(J.id);
            queue.pop_front();
        }
        // Which resident jobs advance this round: all of them, or (fill policy)
        // the oldest one and then those with the least remaining work, in that
        // order, until their pixels reach cfg.fill_pixels, so that a round is no
        // longer than it must be to fill the GPU, short jobs are not held behind
        // the iterations of long ones, and no job waits for ever.
        std::vector<uint64_t> order(resident.begin(), resident.end());
        if (cfg.fill_pixels > 0 && !order.empty()) {
            auto remaining = [&](uint64_t id) {
                const Job& J = jobs[id];
                return (double)(J.t_last - J.t) * J.pr.width * J.pr.height * J.pa.spp * std::max(J.pa.bounces, 1);
            };
            auto oldest = std::min_element(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
                return jobs[a].t_submit < jobs[b].t_submit;
            });
            std::iter_swap(order.begin(), oldest);
            std::stable_sort(order.begin() + 1, order.end(),
                             [&](uint64_t a, uint64_t b) { return remaining(a) < remaining(b); });
        }
        long long picked_px = 0;
        for (uint64_t id : order) {
            Job& J = jobs[id];
            kern::JobDesc D;
            const int rc = eng::fill_job(D, J.pr, J.pa, J.out, base + table_bytes + J.offset);
            if (rc != IRTPS_OK) {
                J.status = rc;
                continue;
            }
            if (!J.initialised) {
                fresh.push_back(D);
                fresh_ids.push_back(id);
            }
            const bool room = cfg.fill_pixels <= 0 || running.empty() || picked_px < cfg.fill_pixels;
            if (J.t < J.t_last && room) {
                D.t = J.t;
                running.push_back(D);
                running_ids.push_back(id);
                picked_px += (long long)J.pr.width * J.pr.height;
            }
        }
        if (fresh.empty() && running.empty()) {
            // jobs with T = 0 that are initialised, or nothing resident
            bool any = changed;
            for (auto it = resident.begin(); it != resident.end();) {
                Job& J = jobs[*it];
                if (J.status != IRTPS_OK) {
                    finish(this, J, IRTPS_JOB_FAILED, J.status);
                    it = resident.erase(it);
                    any = true;
                } else if (J.initialised && J.t >= J.t_last) {
                    finish(this, J, IRTPS_JOB_DONE, IRTPS_OK);
                    it = resident.erase(it);
                    any = true;
                } else {
                    ++it;
                }
            }
            if (any) cv.notify_all();
            return any;
        }
    }
    int rc = IRTPS_OK;
    // the job table after the iteration (the stop rule may lower a job's T on the
    // device); read only once the stream has been synchronised
    std::vector<kern::JobDesc> after;
    if (cfg.dry_run == 0) {
        if (!fresh.empty()) {
            eng::Batch b;
            b.build(fresh);
            rc = b.place(base, table_bytes);
            if (rc == IRTPS_OK) rc = b.upload_tables(stream);
            if (rc == IRTPS_OK) rc = b.run_init(stream);
        }
        // jobs admitted this round also run their first iteration now
        if (rc == IRTPS_OK && !running.empty()) {
            eng::Batch b;
            b.build(running);
            rc = b.place(base, table_bytes);
            if (rc == IRTPS_OK) rc = b.upload_tables(stream);
            if (rc == IRTPS_OK) rc = b.run_iteration(stream);
            // the stop rule may have lowered a job's T on the device
            if (rc == IRTPS_OK) {
                after.resize(running.size());
                const hipError_t e = hipMemcpyAsync(after.data(), b.d_jobs, sizeof(kern::JobDesc) * after.size(),
                                                    hipMemcpyDeviceToHost, stream);
                if (e != hipSuccess) {
                    rc = hip_fail(e);
                    after.clear();
                }
            }
        }
        if (rc == IRTPS_OK) {
            const hipError_t e = hipStreamSynchronize(stream);
            if (e != hipSuccess) rc = hip_fail(e);
        }
        if (rc == IRTPS_OK)
            for (size_t k = 0; k < after.size(); ++k) running_T.push_back(after[k].T);
    } else {
        // scheduler-only mode: no kernel runs, no output is written
        std::this_thread::sleep_for(std::chrono::microseconds(200 * (int)(fresh.size() + running.size())));
    }
    std::unique_lock<std::mutex> lock(mu);
    ++iterations;
    for (uint64_t id : fresh_ids) jobs[id].initialised = true;
    for (size_t k = 0; k < running_ids.size(); ++k) {
        Job& J = jobs[running_ids[k]];
        J.t += 1;
        if (k < running_T.size() && running_T[k] < J.t_last) J.t_last = running_T[k];
    }
    for (auto it = resident.begin(); it != resident.end();) {
        Job& J = jobs[*it];
        if (rc != IRTPS_OK || J.status != IRTPS_OK) {
            finish(this, J, IRTPS_JOB_FAILED, rc != IRTPS_OK ? rc : J.status);
            it = resident.erase(it);
        } else if (J.initialised && J.t >= J.t_last) {
            finish(this, J, IRTPS_JOB_DONE, IRTPS_OK);
            it = resident.erase(it);
        } else {
            ++it;
        }
    }
    cv.notify_all();
    return true;
}

void irtps_server::run() {
    for (;;) {
        {
            std::unique_lock<std::mutex> lock(mu);
            cv.wait(lock, [&] { return stop || !queue.empty() || !resident.empty(); });
            if (stop) return;
        }
        step();
    }
}

extern "C" {

int irtps_server_create(const irtps_server_cfg* cfg, void* ws_dev, size_t ws_bytes, irtps_server** out) {
    if (!cfg || !out || cfg->max_resident_jobs < 0 || cfg->reserved != 0 || cfg->fill_pixels < 0 ||
        (cfg->dry_run != 0 && cfg->dry_run != 1))
        return IRTPS_ERR_INVALID_ARG;
    if (cfg->dry_run == 0 && (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) % kAlign))) return IRTPS_ERR_WORKSPACE;
    const size_t tables = cfg->table_bytes ? align_up(cfg->table_bytes) : align_up(std::max<size_t>(ws_bytes / 64, 1 << 20));
    if (ws_bytes <= tables) return IRTPS_ERR_WORKSPACE;
    irtps_server* s = new irtps_server();
    s->cfg = *cfg;
    s->base = static_cast<char*>(ws_dev);
    s->table_bytes = tables;
    s->pool_bytes = (ws_bytes - tables) / kAlign * kAlign;
    s->regions.reset(s->pool_bytes);
    if (cfg->dry_run == 0) {
        const hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete s;
            return hip_fail(e);
        }
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return IRTPS_OK;
}

int irtps_server_submit(irtps_server* s, const irtps_problem* problem, const irtps_params* params,
                        const irtps_outputs* outputs, uint64_t* job_id) {
    if (!s || !problem || !params || !outputs || !job_id) return IRTPS_ERR_INVALID_ARG;
    STATUS_TRY(check_problem(problem, params));
    if (!outputs->normals_dev || !outputs->albedo_dev || !outputs->depth_dev) return IRTPS_ERR_INVALID_ARG;
    // what the batched kernels do not run is refused here, not when the job starts
    if (problem->box || (params->flags & (IRTPS_FLAG_ROBUST_INTEGRATION | IRTPS_FLAG_EXACT_R_MASK)))
        return IRTPS_ERR_INVALID_ARG;
    Job J;
    J.pr = *problem;
    J.pa = *params;
    J.t_last = params->iterations;
    J.out = *outputs;
    const int K = problem->num_lights;
    J.lights.assign(problem->light_dirs_host, problem->light_dirs_host + 3 * K);
    if (problem->light_intensity_host)
        J.intens.assign(problem->light_intensity_host, problem->light_intensity_host + K);
    J.pr.light_dirs_host = J.lights.data();
    J.pr.light_intensity_host = J.intens.empty() ? nullptr : J.intens.data();
    {
        kern::PsMatrix M;
        STATUS_TRY(make_psmatrix(K, J.pr.light_dirs_host, J.pr.light_intensity_host, M));
    }
    J.bytes = align_up(eng::job_region_bytes(J.pr));
    J.tiles = eng::max_tracer_tiles(problem->width, problem->height);
    // a job that could never be resident, even alone, is refused now
    if (J.bytes > s->pool_bytes || eng::table_bytes(1, J.tiles) > s->table_bytes) return IRTPS_ERR_OOM;
    std::lock_guard<std::mutex> lock(s->mu);
    J.id = s->next_id++;
    J.t_submit = now_s();
    if (s->submitted == 0) s->first_submit = J.t_submit;
    ++s->submitted;
    *job_id = J.id;
    s->queue.push_back(J.id);
    s->jobs.emplace(J.id, std::move(J));
    s->jobs[*job_id].pr.light_dirs_host = s->jobs[*job_id].lights.data();
    s->jobs[*job_id].pr.light_intensity_host =
        s->jobs[*job_id].intens.empty() ? nullptr : s->jobs[*job_id].intens.data();
    s->cv.notify_all();
    return IRTPS_OK;
}

int irtps_server_poll(irtps_server* s, uint64_t job_id, irtps_job_status* st) {
    if (!s || !st) return IRTPS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return IRTPS_ERR_NOT_FOUND;
    const Job& J = it->second;
    st->state = J.state;
    st->status = J.status;
    st->iteration = J.t;
    st->reserved = 0;
    st->submit_s = J.t_submit;
    st->start_s = J.t_start;
    st->end_s = J.t_end;
    return IRTPS_OK;
}

int irtps_server_wait(irtps_server* s, uint64_t job_id, double timeout_s, irtps_job_status* st) {
    if (!s || !st) return IRTPS_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lock(s->mu);
    auto done = [&] {
        auto it = s->jobs.find(job_id);
        return it == s->jobs.end() || it->second.state >= IRTPS_JOB_DONE;
    };
    if (timeout_s < 0) s->cv.wait(lock, done);
    else s->cv.wait_for(lock, std::chrono::duration<double>(timeout_s), done);
    lock.unlock();
    const int rc = irtps_server_poll(s, job_id, st);
    if (rc != IRTPS_OK) return rc;
    return st->state >= IRTPS_JOB_DONE ? IRTPS_OK : IRTPS_ERR_BUSY;
}

int irtps_server_cancel(irtps_server* s, uint64_t job_id) {
    if (!s) return IRTPS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return IRTPS_ERR_NOT_FOUND;
    if (it->second.state >= IRTPS_JOB_DONE) return IRTPS_OK;
    it->second.cancel = true;
    s->cv.notify_all();
    return IRTPS_OK;
}

int irtps_server_stats(irtps_server* s, irtps_server_statistics* out) {
    if (!s || !out) return IRTPS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->cancelled = s->cancelled;
    out->resident = (int32_t)s->resident.size();
    out->queued = (int32_t)s->queue.size();
    out->bytes_in_use = s->in_use;
    out->bytes_budget = s->pool_bytes;
    out->iterations = s->iterations;
    if (!s->latencies.empty()) {
        std::vector<double> v(s->latencies);
        std::sort(v.begin(), v.end());
        auto q = [&](double f) {
            const double pos = f * (double)(v.size() - 1);
            const size_t i = (size_t)pos;
            const double w = pos - (double)i;
            return i + 1 < v.size() ? v[i] * (1 - w) + v[i + 1] * w : v[i];
        };
        out->p50_latency_s = q(0.50);
        out->p99_latency_s = q(0.99);
        const double span = s->last_end - s->first_submit;
        out->jobs_per_s = span > 0 ? (double)s->completed / span : 0.0;
    }
    return IRTPS_OK;
}

int irtps_server_destroy(irtps_server* s) {
    if (!s) return IRTPS_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    int rc = IRTPS_OK;
    if (s->stream) {
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e == hipSuccess) e = hipStreamDestroy(s->stream);
        if (e != hipSuccess) rc = hip_fail(e);
    }
    delete s;
    return rc;
}

}  // extern "C"
