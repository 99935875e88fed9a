// Continuous-batching server for invasion jobs (ibip_server_* in ibip.h).
//
// Jobs arrive at any time (ibip_server_submit). A worker thread admits a
// pending job as soon as an execution slot is free and the job's scratch
// fits in the server's HBM pool (first fit over one device allocation,
// looking past a job that does not fit yet to smaller ones behind it, within
// a bounded window, so a huge job does not block the queue). An admitted job
// runs entirely stream-ordered on its slot's stream: setup, the step loop in
// one workgroup, sphere insertion and finalisation, with no host
// synchronisation; jobs on different slots overlap on the device. The worker
// polls each slot's completion event, returns the job's scratch to the pool
// and records its latency from submission to completion.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ibip_internal.h"

namespace ibip {
namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Pool {
  public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

enum JobState { J_PENDING = 0, J_RUNNING = 1, J_DONE = 2 };

struct Job {
    ibip_job job{};
    size_t bytes = 0, off = 0;
    int slot = -1;
    int state = J_PENDING;
    bool cancel = false;  // cancellation requested while it ran
    Clock::time_point t_submit, t_done;
};

constexpr size_t kSlotSmall = 4096;  // LoopState + loop arguments of one slot

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint8_t* dev_small = nullptr;   // device: LoopState at 0, loop arguments at 512
    uint8_t* host_small = nullptr;  // pinned: LoopState copy at 0, loop-argument staging at 512
    int64_t ticket = -1;
    bool broken = false;            // its stream failed; no job is admitted to it again
    int phase = 0;                  // 1: the job's step loop, 2: its post-processing
    uint32_t* cancel_host = nullptr;  // coherent pinned word the job's loop reads every 1024 steps
    uint32_t* cancel_dev = nullptr;   // its device address
};

}  // namespace
}  // namespace ibip

struct ibip_server {
    int device = 0;
    size_t budget = 0;
    int max_inflight = 0;
    int lookahead = 0;
    uint8_t* pool_base = nullptr;
    ibip::Pool pool;
    std::vector<ibip::Slot> slots;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, ibip::Job> jobs;
    int64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::string err;
    ibip_tuning tuning{};  // launch parameters of the jobs admitted from now on
    ibip_server_stats stats{};
};

namespace ibip {
namespace {

void set_err(ibip_server* S, const std::string& m) { S->err = m; }

// Start job `t` on slot `si` (mu held). Returns false if a HIP call failed.
bool start_job(ibip_server* S, int64_t t, int si) {
    Job& J = S->jobs[t];
    Slot& sl = S->slots[si];
    const ibip_job& jb = J.job;
    JobBufs b = carve(S->pool_base + J.off, jb.dims, jb.centre_step, false);
    LoopState* st = (LoopState*)sl.dev_small;
    void* dargs = sl.dev_small + 512;
    hipError_t e = job_setup(b, st, jb.image, jb.inlets, jb.dims, jb.max_steps, jb.seq, sl.stream,
                             edt_tiles(S->tuning));
    // a step with more centres than the threshold stops the loop; the worker
    // then runs that step over the whole GPU and resumes the loop (advance())
    fill_loop_args(sl.host_small + 512, b, st, jb.dims, wide_threshold(S->tuning.batch_wide));
    __atomic_store_n(sl.cancel_host, 0u, __ATOMIC_RELEASE);
    set_loop_cancel(sl.host_small + 512, sl.cancel_dev);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dargs, sl.host_small + 512, loop_args_bytes(), hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess) e = launch_loop_jobs(dargs, 1, sl.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sl.host_small, st, sizeof(LoopState), hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) {
        set_err(S, std::string("server: launch failed: ") + hipGetErrorString(e));
        // work queued before the failure may still write into the job's
        // region: wait for it before the caller returns the region to the
        // pool, and retire the slot if its stream is in an error state
        if (hipStreamSynchronize(sl.stream) != hipSuccess) {
            (void)hipGetLastError();
            sl.broken = true;
        }
        return false;
    }
    J.slot = si;
    J.state = J_RUNNING;
    sl.ticket = t;
    sl.phase = 1;
    S->stats.running++;
    S->stats.pending--;
    if (S->stats.running > S->stats.peak_running) S->stats.peak_running = S->stats.running;
    return true;
}

// The slot's queued work ended (mu held). After a loop segment that stopped
// at a wide step: queue that step over the whole GPU and the next loop
// segment; after the last segment: queue the post-processing. Returns false
// when the job is finished (or a launch failed: *e holds the error).
bool advance(ibip_server* S, int si, hipError_t* e) {
    Slot& sl = S->slots[si];
    if (sl.phase != 1 || *e != hipSuccess) return false;
    Job& J = S->jobs[sl.ticket];
    const ibip_job& jb = J.job;
    const LoopState* hs = (const LoopState*)sl.host_small;
    if (J.cancel || hs->status == LS_CANCEL) return false;  // finish_job reports the cancellation
    LoopState* st = (LoopState*)sl.dev_small;
    hipError_t r = hipSuccess;
    if (hs->status == LS_WIDE && hs->err == 0) {
        r = launch_wide_and_loop_host(sl.host_small + 512, (int64_t)jb.dims.X * jb.dims.Y * jb.dims.Z, sl.stream);
    } else {
        JobBufs b = carve(S->pool_base + J.off, jb.dims, jb.centre_step, false);
        r = job_post_devk(b, st, jb.dims, jb.seq, jb.rad2, jb.M, sl.stream);
        sl.phase = 2;
    }
    if (r == hipSuccess) r = hipMemcpyAsync(sl.host_small, st, sizeof(LoopState), hipMemcpyDeviceToHost, sl.stream);
    if (r == hipSuccess) r = hipEventRecord(sl.done, sl.stream);
    if (r != hipSuccess) {
        set_err(S, std::string("server: launch failed: ") + hipGetErrorString(r));
        if (hipStreamSynchronize(sl.stream) != hipSuccess) {
            (void)hipGetLastError();
            sl.broken = true;
        }
        *e = r;
        return false;
    }
    return true;
}

void finish_job(ibip_server* S, int si, hipError_t e) {
    Slot& sl = S->slots[si];
    Job& J = S->jobs[sl.ticket];
    const LoopState* hs = (const LoopState*)sl.host_small;
    J.job.status = IBIP_OK;
    J.job.n_steps = 0;
    const bool cancelled = sl.phase == 1 && (J.cancel || hs->status == LS_CANCEL);
    if (e != hipSuccess) J.job.status = IBIP_EDEVICE;
    else if (cancelled) J.job.status = IBIP_ECANCELLED;
    else if (hs->err == 2) J.job.status = IBIP_ENOSOLID;
    else if (hs->err == 3) J.job.status = IBIP_ECAPACITY;
    else if (hs->err) J.job.status = IBIP_EDEVICE;
    else J.job.n_steps = (int64_t)hs->k - 1;
    J.state = J_DONE;
    J.t_done = Clock::now();
    S->pool.release(J.off, J.bytes);
    S->stats.bytes_in_use -= (int64_t)J.bytes;
    S->stats.running--;
    S->stats.completed++;
    if (cancelled && e == hipSuccess) S->stats.cancelled++;
    sl.ticket = -1;
}

void worker_main(ibip_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progressed = false;
        // completions
        for (size_t si = 0; si < S->slots.size(); si++) {
            Slot& sl = S->slots[si];
            if (sl.ticket < 0) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            hipError_t e = q == hipSuccess ? hipSuccess : q;
            progressed = true;
            if (advance(S, (int)si, &e)) continue;
            finish_job(S, (int)si, e);
        }
        if (progressed) S->cv_done.notify_all();
        // admissions: first pending job (within the window) whose scratch fits
        for (;;) {
            int free_slot = -1;
            for (size_t si = 0; si < S->slots.size(); si++)
                if (S->slots[si].ticket < 0 && !S->slots[si].broken) {
                    free_slot = (int)si;
                    break;
                }
            if (free_slot < 0 || S->pending.empty()) break;
            bool started = false;
            const size_t window = std::min<size_t>(S->pending.size(), (size_t)S->lookahead);
            for (size_t w = 0; w < window; w++) {
                const int64_t t = S->pending[w];
                Job& J = S->jobs[t];
                size_t off = 0;
                if (!S->pool.alloc(J.bytes, &off)) continue;
                J.off = off;
                S->stats.bytes_in_use += (int64_t)J.bytes;
                if (S->stats.bytes_in_use > S->stats.peak_bytes) S->stats.peak_bytes = S->stats.bytes_in_use;
                S->pending.erase(S->pending.begin() + (long)w);
                if (!start_job(S, t, free_slot)) {
                    // the job could not be launched: report it failed
                    J.job.status = IBIP_EDEVICE;
                    J.state = J_DONE;
                    J.t_done = Clock::now();
                    S->pool.release(J.off, J.bytes);
                    S->stats.bytes_in_use -= (int64_t)J.bytes;
                    S->stats.pending--;
                    S->stats.completed++;
                    S->cv_done.notify_all();
                }
                started = true;
                progressed = true;
                break;
            }
            if (!started) break;
        }
        // with every slot retired no pending job can run: report them failed
        if (!S->pending.empty() &&
            std::all_of(S->slots.begin(), S->slots.end(), [](const Slot& x) { return x.broken; })) {
            for (const int64_t t : S->pending) {
                Job& J = S->jobs[t];
                J.job.status = IBIP_EDEVICE;
                J.state = J_DONE;
                J.t_done = Clock::now();
                S->stats.pending--;
                S->stats.completed++;
            }
            S->pending.clear();
            S->cv_done.notify_all();
        }
        const bool idle = S->stats.running == 0;
        if (S->stop && idle && S->pending.empty()) break;
        if (!progressed) {
            if (idle && S->pending.empty()) {
                S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
            } else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            }
        }
    }
}

}  // namespace
}  // namespace ibip

using namespace ibip;

extern "C" {

ibip_status ibip_server_create(ibip_server** out, int32_t device, const ibip_server_opts* opts) {
    if (!out) return IBIP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return IBIP_EDEVICE;
    const int64_t budget = opts && opts->hbm_budget_bytes > 0 ? opts->hbm_budget_bytes : ((int64_t)8 << 30);
    const int inflight = opts && opts->max_inflight > 0 ? opts->max_inflight : 16;
    const int lookahead = opts && opts->lookahead > 0 ? opts->lookahead : 8;
    ibip_server* S = new (std::nothrow) ibip_server();
    if (!S) return IBIP_ENOMEM;
    S->device = device;
    S->budget = (size_t)budget;
    S->max_inflight = inflight;
    S->lookahead = lookahead;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(device);
    bool ok = hipMalloc(&S->pool_base, S->budget) == hipSuccess;
    S->slots.resize(inflight);
    for (auto& sl : S->slots) {
        if (!ok) break;
        ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
             hipMalloc(&sl.dev_small, kSlotSmall) == hipSuccess &&
             hipHostMalloc(&sl.host_small, kSlotSmall, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&sl.cancel_host, 64, hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess &&
             hipHostGetDevicePointer((void**)&sl.cancel_dev, sl.cancel_host, 0) == hipSuccess;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    if (!ok) {
        (void)hipGetLastError();
        for (auto& sl : S->slots) {
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.dev_small) (void)hipFree(sl.dev_small);
            if (sl.host_small) (void)hipHostFree(sl.host_small);
            if (sl.cancel_host) (void)hipHostFree(sl.cancel_host);
        }
        if (S->pool_base) (void)hipFree(S->pool_base);
        delete S;
        return IBIP_ENOMEM;
    }
    S->pool.init(S->budget);
    S->worker = std::thread(worker_main, S);
    *out = S;
    return IBIP_OK;
}

ibip_status ibip_server_submit(ibip_server* S, const ibip_job* job, int64_t* ticket) {
    if (!S || !job || !ticket) return IBIP_EINVAL;
    if (!job->image || !job->inlets || !job->seq || !dims_ok(job->dims) || job->max_steps < 0) {
        std::lock_guard<std::mutex> g(S->mu);
        set_err(S, "server_submit: bad job");
        return IBIP_EINVAL;
    }
    const size_t bytes = align256(job_bytes(job->dims, job->centre_step == nullptr, false));
    std::lock_guard<std::mutex> g(S->mu);
    if (bytes > S->budget) {
        set_err(S, "server_submit: the job's scratch exceeds the server's HBM budget");
        return IBIP_ECAPACITY;
    }
    const int64_t t = S->next_ticket++;
    Job& J = S->jobs[t];
    J.job = *job;
    J.job.status = 0;
    J.job.n_steps = 0;
    J.bytes = bytes;
    J.t_submit = Clock::now();
    S->pending.push_back(t);
    S->stats.submitted++;
    S->stats.pending++;
    *ticket = t;
    S->cv_work.notify_one();
    return IBIP_OK;
}

ibip_status ibip_server_poll(ibip_server* S, int64_t ticket, int32_t* done) {
    if (!S || !done) return IBIP_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return IBIP_EINVAL;
    *done = it->second.state == J_DONE ? 1 : 0;
    return IBIP_OK;
}

ibip_status ibip_server_wait(ibip_server* S, int64_t ticket, ibip_job* result, double* latency_ms) {
    if (!S) return IBIP_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return IBIP_EINVAL;
    S->cv_done.wait(lk, [&] { return S->jobs[ticket].state == J_DONE; });
    Job& J = S->jobs[ticket];
    if (result) *result = J.job;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(J.t_done - J.t_submit).count();
    const ibip_status st = (ibip_status)J.job.status;
    S->jobs.erase(ticket);
    return st;
}

ibip_status ibip_server_cancel(ibip_server* S, int64_t ticket) {
    if (!S) return IBIP_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->jobs.find(ticket);
    if (it != S->jobs.end() && it->second.state == J_RUNNING) {
        // a running job: its loop stops at its next check (every 1024 steps)
        // and the worker queues nothing more for it
        Job& J = it->second;
        J.cancel = true;
        __atomic_store_n(S->slots[J.slot].cancel_host, 1u, __ATOMIC_RELEASE);
        return IBIP_OK;
    }
    if (it == S->jobs.end() || it->second.state != J_PENDING) {
        set_err(S, "server_cancel: the job is done or unknown");
        return IBIP_EINVAL;
    }
    for (auto p = S->pending.begin(); p != S->pending.end(); ++p)
        if (*p == ticket) {
            S->pending.erase(p);
            break;
        }
    Job& J = it->second;
    J.job.status = IBIP_ECANCELLED;
    J.state = J_DONE;
    J.t_done = Clock::now();
    S->stats.pending--;
    S->stats.cancelled++;
    S->cv_done.notify_all();
    return IBIP_OK;
}

ibip_status ibip_server_stats_get(ibip_server* S, ibip_server_stats* out) {
    if (!S || !out) return IBIP_EINVAL;
    std::lock_guard<std::mutex> g(S->mu);
    *out = S->stats;
    return IBIP_OK;
}

ibip_status ibip_server_set_tuning(ibip_server* S, const ibip_tuning* t) {
    if (!S) return IBIP_EINVAL;
    if (t && !tuning_ok(*t)) return IBIP_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    S->tuning = t ? *t : ibip_tuning{};
    return IBIP_OK;
}

const char* ibip_server_last_error(const ibip_server* S) { return S ? S->err.c_str() : "null server"; }

ibip_status ibip_server_destroy(ibip_server* S) {
    if (!S) return IBIP_EINVAL;
    {
        std::lock_guard<std::mutex> g(S->mu);
        // pending jobs are cancelled; running ones finish
        for (int64_t t : S->pending) {
            Job& J = S->jobs[t];
            J.job.status = IBIP_ECANCELLED;
            J.state = J_DONE;
            S->stats.cancelled++;
        }
        S->pending.clear();
        S->stats.pending = 0;
        S->stop = true;
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
    if (S->worker.joinable()) S->worker.join();
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    for (auto& sl : S->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipStreamDestroy(sl.stream);
        (void)hipEventDestroy(sl.done);
        (void)hipFree(sl.dev_small);
        (void)hipHostFree(sl.host_small);
        (void)hipHostFree(sl.cancel_host);
    }
    (void)hipFree(S->pool_base);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete S;
    return IBIP_OK;
}

}  // extern "C"
