// sr_server.hip -- continuous-batching sort server on top of libsortrace.
//
// Requests (keys already resident in device memory) arrive with a timestamp.
// One worker thread:
//   1. makes a request visible once its arrival time has passed (FIFO);
//   2. admits requests in FIFO order while the HBM footprint of admitted,
//      unfinished requests (their keys plus the scratch their sort needs,
//      2 x n x element size) stays within the budget;
//   3. whenever one of its streams is idle, groups admitted requests of the
//      oldest request's dtype (up to max_batch_requests / max_batch_keys) into
//      one batch and enqueues it on that stream: sr_sort_batch (every request
//      sorted in its own buffer, one set of launches for the batch), or
//      sr_sort_keys for a batch of one; an event marks its completion;
//   4. polls the events; a finished batch releases its footprint and stream.
// Requests arriving while batches run are admitted as memory frees up and go
// into the next batch on the next idle stream, so work from different
// arrivals overlaps on the device.  With streams = 1 and
// max_batch_requests = 1 the same loop is a plain one-at-a-time FIFO server.
// Streams are created with the default priority.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sortrace.h"

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

int es_of(sr_dtype dt) { return dt == SR_UINT64 ? 8 : 4; }

struct Req {
    uint64_t tag;
    sr_dtype dt;
    void* keys;
    size_t n;
    size_t foot;
    hipEvent_t ready = nullptr;  // producer's event; the batch's stream waits for it
    double t_arrive, t_admit = -1, t_launch = -1, t_done = -1;
    int batch = -1;
    sr_status status = SR_OK;
};

struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    void** h_ptrs = nullptr;    // pinned staging
    int64_t* h_lens = nullptr;
    void** d_ptrs = nullptr;    // device copies read by sr_sort_batch
    int64_t* d_lens = nullptr;
    bool busy = false;
    std::vector<size_t> reqs;
    size_t foot = 0;
};

}  // namespace

struct sr_server {
    sr_server_config cfg;
    std::chrono::steady_clock::time_point t0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::vector<Req> reqs;           // every request ever submitted
    std::deque<size_t> arriving;     // submitted, ordered by arrival time
    std::deque<size_t> admitted;     // admitted, not yet launched
    std::vector<size_t> finished;    // completed, not yet collected
    size_t foot_in_use = 0;
    size_t unfinished = 0;
    int next_batch = 0;
    std::atomic<bool> stop{false};
    std::thread worker;
    std::string error;
    std::condition_variable idle_cv;

    void loop();
};

void sr_server::loop() {
    while (!stop.load()) {
        bool progress = false;
        std::unique_lock<std::mutex> lk(mu);
        const double t = now_s(t0);
        // arrivals in time order, then FIFO admission under the footprint budget
        while (!arriving.empty() && reqs[arriving.front()].t_arrive <= t) {
            Req& r = reqs[arriving.front()];
            const bool fits = foot_in_use + r.foot <= cfg.hbm_budget_bytes;
            if (!fits) break;
            foot_in_use += r.foot;
            r.t_admit = t;
            admitted.push_back(arriving.front());
            arriving.pop_front();
            progress = true;
        }
        // launch on idle streams
        for (auto& sl : slots) {
            if (sl.busy || admitted.empty()) continue;
            const sr_dtype dt = reqs[admitted.front()].dt;
            sl.reqs.clear();
            size_t keys = 0;
            for (auto it = admitted.begin(); it != admitted.end() && (int)sl.reqs.size() < cfg.max_batch_requests;) {
                Req& r = reqs[*it];
                if (r.dt == dt && (sl.reqs.empty() || keys + r.n <= cfg.max_batch_keys)) {
                    sl.reqs.push_back(*it);
                    keys += r.n;
                    it = admitted.erase(it);
                } else {
                    ++it;
                }
            }
            const int bid = next_batch++;
            sl.foot = 0;
            for (size_t q = 0; q < sl.reqs.size(); ++q) {
                Req& r = reqs[sl.reqs[q]];
                r.batch = bid;
                r.t_launch = now_s(t0);
                sl.foot += r.foot;
                sl.h_ptrs[q] = r.keys;
                sl.h_lens[q] = (int64_t)r.n;
            }
            std::vector<hipEvent_t> waits;
            for (size_t q : sl.reqs)
                if (reqs[q].ready) waits.push_back(reqs[q].ready);
            lk.unlock();
            sr_status s = SR_OK;
            std::string msg;
            for (hipEvent_t ev : waits) {
                if (hipStreamWaitEvent(sl.st, ev, 0) != hipSuccess) {
                    s = SR_ERR_DEVICE;
                    msg = std::string("waiting for a request's ready event: ") + hipGetErrorString(hipGetLastError());
                    break;
                }
            }
            if (s != SR_OK) {
                // nothing enqueued for this batch; it finishes with the error below
            } else if (sl.reqs.size() == 1) {
                s = sr_sort_keys(dt, sl.h_ptrs[0], (size_t)sl.h_lens[0], sl.st);
            } else if (hipMemcpyAsync(sl.d_ptrs, sl.h_ptrs, sizeof(void*) * sl.reqs.size(), hipMemcpyHostToDevice,
                                      sl.st) != hipSuccess ||
                       hipMemcpyAsync(sl.d_lens, sl.h_lens, sizeof(int64_t) * sl.reqs.size(), hipMemcpyHostToDevice,
                                      sl.st) != hipSuccess) {
                s = SR_ERR_DEVICE;
                msg = std::string("staging the batch: ") + hipGetErrorString(hipGetLastError());
            } else {
                s = sr_sort_batch(dt, sl.d_ptrs, sl.d_lens, sl.reqs.size(), keys, sl.st);
            }
            if (s != SR_OK && msg.empty()) msg = sr_last_error_message();
            // the completion event is recorded even after a failed enqueue, so
            // the batch still finishes (with its error status)
            if (hipEventRecord(sl.done, sl.st) != hipSuccess) {
                msg = std::string("completion event: ") + hipGetErrorString(hipGetLastError());
                s = SR_ERR_DEVICE;
                (void)hipStreamSynchronize(sl.st);  // an event never recorded again reads as complete
                (void)hipGetLastError();
            }
            lk.lock();
            for (size_t q : sl.reqs) reqs[q].status = s;
            if (s != SR_OK && error.empty()) error = msg;
            sl.busy = true;
            progress = true;
        }
        // completions
        for (auto& sl : slots) {
            if (!sl.busy) continue;
            if (hipEventQuery(sl.done) != hipSuccess) continue;
            const double td = now_s(t0);
            for (size_t q : sl.reqs) {
                reqs[q].t_done = td;
                finished.push_back(q);
            }
            foot_in_use -= sl.foot;
            unfinished -= sl.reqs.size();
            sl.busy = false;
            sl.reqs.clear();
            progress = true;
        }
        if (unfinished == 0) idle_cv.notify_all();
        lk.unlock();
        if (!progress) std::this_thread::yield();
    }
}

extern "C" {

sr_status sr_server_create(const sr_server_config* cfg, sr_server** out) {
    if (!cfg || !out || cfg->streams < 1 || cfg->streams > 16 || cfg->max_batch_requests < 1 ||
        cfg->hbm_budget_bytes == 0 || cfg->max_batch_keys == 0)
        return SR_ERR_INVALID_ARGUMENT;
    sr_server* s = new sr_server();
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    s->slots.resize(cfg->streams);
    for (auto& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&sl.h_ptrs, sizeof(void*) * cfg->max_batch_requests, 0) != hipSuccess ||
            hipHostMalloc((void**)&sl.h_lens, sizeof(int64_t) * cfg->max_batch_requests, 0) != hipSuccess ||
            hipMalloc((void**)&sl.d_ptrs, sizeof(void*) * cfg->max_batch_requests) != hipSuccess ||
            hipMalloc((void**)&sl.d_lens, sizeof(int64_t) * cfg->max_batch_requests) != hipSuccess) {
            (void)hipGetLastError();
            sr_server_destroy(s);
            return SR_ERR_OUT_OF_MEMORY;
        }
        // size every stream's scratch for the largest batch of every dtype up
        // front, so the worker loop never allocates
        for (sr_dtype dt : {SR_INT32, SR_FLOAT32, SR_UINT64}) {
            if (sr_reserve(dt, cfg->max_batch_keys, (size_t)cfg->max_batch_requests, sl.st) != SR_OK) {
                sr_server_destroy(s);
                return SR_ERR_OUT_OF_MEMORY;
            }
        }
        if (hipStreamSynchronize(sl.st) != hipSuccess) {
            (void)hipGetLastError();
            sr_server_destroy(s);
            return SR_ERR_DEVICE;
        }
    }
    s->worker = std::thread([s]() { s->loop(); });
    *out = s;
    return SR_OK;
}

sr_status sr_server_submit(sr_server* s, sr_dtype dt, void* keys, size_t n, uint64_t tag, double t_arrive,
                           void* ready_event) {
    if (!s || (dt != SR_INT32 && dt != SR_FLOAT32 && dt != SR_UINT64) || (n > 0 && !keys)) return SR_ERR_INVALID_ARGUMENT;
    Req r;
    r.tag = tag;
    r.dt = dt;
    r.keys = keys;
    r.n = n;
    r.foot = 2 * n * (size_t)es_of(dt);
    r.t_arrive = t_arrive;
    r.ready = (hipEvent_t)ready_event;
    if (r.foot > s->cfg.hbm_budget_bytes || n > s->cfg.max_batch_keys) return SR_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->arriving.empty() && s->reqs[s->arriving.back()].t_arrive > t_arrive)
        return SR_ERR_INVALID_ARGUMENT;  // arrivals must be submitted in time order
    s->reqs.push_back(r);
    s->arriving.push_back(s->reqs.size() - 1);
    s->unfinished++;
    return SR_OK;
}

double sr_server_now(sr_server* s) { return s ? now_s(s->t0) : 0.0; }

sr_status sr_server_wait_idle(sr_server* s, double timeout_s) {
    if (!s) return SR_ERR_INVALID_ARGUMENT;
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->idle_cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                        [s]() { return s->unfinished == 0; });
    if (!ok) return SR_ERR_INTERNAL;
    return s->error.empty() ? SR_OK : SR_ERR_DEVICE;
}

sr_status sr_server_records(sr_server* s, sr_request_record* out, size_t cap, size_t* count) {
    if (!s || !count || (cap > 0 && !out)) return SR_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(s->mu);
    size_t k = 0;
    while (k < cap && k < s->finished.size()) {
        const Req& r = s->reqs[s->finished[k]];
        out[k].tag = r.tag;
        out[k].dtype = (int32_t)r.dt;
        out[k].batch = r.batch;
        out[k].n = (int64_t)r.n;
        out[k].status = (int32_t)r.status;
        out[k].t_arrive = r.t_arrive;
        out[k].t_admit = r.t_admit;
        out[k].t_launch = r.t_launch;
        out[k].t_done = r.t_done;
        ++k;
    }
    s->finished.erase(s->finished.begin(), s->finished.begin() + (long)k);
    *count = k;
    return SR_OK;
}

sr_status sr_server_destroy(sr_server* s) {
    if (!s) return SR_ERR_INVALID_ARGUMENT;
    s->stop.store(true);
    if (s->worker.joinable()) s->worker.join();
    for (auto& sl : s->slots) {
        // teardown: failures here leave nothing to recover
        if (sl.st) (void)hipStreamSynchronize(sl.st);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_ptrs) (void)hipHostFree(sl.h_ptrs);
        if (sl.h_lens) (void)hipHostFree(sl.h_lens);
        if (sl.d_ptrs) (void)hipFree(sl.d_ptrs);
        if (sl.d_lens) (void)hipFree(sl.d_lens);
        if (sl.st) {
            sr_release_stream(sl.st);
            (void)hipStreamDestroy(sl.st);
        }
    }
    delete s;
    return SR_OK;
}

}  // extern "C"
