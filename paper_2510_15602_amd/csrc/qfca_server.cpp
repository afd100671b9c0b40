// Serving loop: continuous batching of single-image requests over resident
// models.  A dispatcher thread owns all device work: it admits pending
// requests into a launch whenever one of its slots (a stream with its own
// context, staging buffers and graphs) is free and the requests' working
// memory fits in the budget (serve_policy.h), issues the launch through the
// batched path, and retires it when the slot's end event has completed.
// Launches on different slots overlap on the device.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include <hip/hip_ext.h>

#include "qfca_internal.h"
#include "serve_policy.h"

using namespace qfca;

namespace {

struct Request {
    uint64_t ticket = 0;
    qfca_model model = nullptr;
    const float* X = nullptr;
    int H = 0, W = 0, C = 0;
    float* score = nullptr;
    double t_submit = 0.0;
    int group = 0;
    size_t bytes = 0, off = 0;
};

struct LaunchSlot {
    qfca_ctx ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int32_t* h_err = nullptr;  // pinned: the launch's wait-failure flag
    bool busy = false;
    double t_launch = 0.0;
    std::vector<Request> reqs;
};

double mono_now() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

}  // namespace

struct qfca_server_s {
    int device = 0;
    qfca_server_config cfg{};
    char* base = nullptr;  // device budget
    serve::Arena arena;
    std::vector<LaunchSlot> slots;
    hipEvent_t t0 = nullptr;  // origin of device intervals

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> incoming;           // submitted, not yet seen by the dispatcher
    std::deque<qfca_completion> finished;   // completed, not yet polled
    std::vector<qfca_params> groups;        // parameter sets seen (group ids)
    uint64_t next_ticket = 1;
    qfca_server_counters st{};
    std::vector<std::pair<double, double>> intervals;  // device intervals of retired launches (s)
    bool stop = false;
    std::thread th;

    std::deque<Request> pending;  // dispatcher only
};

namespace {

bool same_group(const qfca_params& a, const qfca_params& b) {
    return a.C == b.C && a.k == b.k && a.B == b.B && a.T == b.T && a.sigma_s == b.sigma_s &&
           a.preproc == b.preproc && a.proj_prec == b.proj_prec;
}

// Retires a launch: completions, memory, statistics.  Called with mu held.
void retire(qfca_server s, LaunchSlot& L, int32_t status) {
    const double now = mono_now();
    float ms0 = 0.f, ms1 = 0.f;
    if (status == QFCA_OK && hipEventElapsedTime(&ms0, s->t0, L.ev0) == hipSuccess &&
        hipEventElapsedTime(&ms1, s->t0, L.ev1) == hipSuccess)
        s->intervals.push_back({1e-3 * ms0, 1e-3 * ms1});
    for (const Request& r : L.reqs) {
        s->arena.release(r.off, r.bytes);
        qfca_completion c{};
        c.ticket = r.ticket;
        c.status = status;
        c.batch_size = (int32_t)L.reqs.size();
        c.t_submit = r.t_submit;
        c.t_launch = L.t_launch;
        c.t_done = now;
        s->finished.push_back(c);
        ++s->st.completed;
        if (status != QFCA_OK) ++s->st.failed;
    }
    L.reqs.clear();
    L.busy = false;
}

// Issues one launch of `reqs` on slot L.  Returns the launch status.
qfca_status issue(qfca_server s, LaunchSlot& L, std::vector<Request>& reqs) {
    const size_t n = reqs.size();
    std::vector<qfca_job> jobs(n);
    std::vector<long long*> asum(n);
    for (size_t i = 0; i < n; ++i) {
        const Request& r = reqs[i];
        const size_t N = (size_t)r.H * r.W;
        char* p = s->base + r.off;
        const size_t ob = serve::align_up((size_t)r.C * N);
        jobs[i] = qfca_job{};
        jobs[i].model = r.model;
        jobs[i].X = r.X;
        jobs[i].H = r.H;
        jobs[i].W = r.W;
        jobs[i].score = r.score;
        jobs[i].bins = (uint8_t*)p;
        asum[i] = (long long*)(p + ob);
    }
    if (hipEventRecord(L.ev0, L.stream) != hipSuccess) return QFCA_E_DEVICE;
    *L.h_err = 0;
    qfca_status st = score_batch_ext(L.ctx, jobs.data(), (int32_t)n, asum.data(), L.h_err);
    if (st != QFCA_OK) return st;
    if (hipEventRecord(L.ev1, L.stream) != hipSuccess) return QFCA_E_DEVICE;
    return QFCA_OK;
}

void dispatcher(qfca_server s) {
    (void)hipSetDevice(s->device);
    std::vector<Request> batch;
    uint64_t last_blocked = 0;  // a request waiting for memory is counted once
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        while (!s->incoming.empty()) {
            s->pending.push_back(s->incoming.front());
            s->incoming.pop_front();
        }
        bool progress = false, any_busy = false;
        // retire finished launches
        for (LaunchSlot& L : s->slots) {
            if (!L.busy) continue;
            const hipError_t e = hipEventQuery(L.ev1);
            if (e == hipSuccess) {
                retire(s, L, *L.h_err ? QFCA_E_DEVICE : QFCA_OK);
                progress = true;
            } else if (e != hipErrorNotReady) {
                retire(s, L, QFCA_E_DEVICE);
                progress = true;
            } else {
                any_busy = true;
            }
        }
        if (progress) s->cv_done.notify_all();
        // admit and launch while a slot is free
        for (LaunchSlot& L : s->slots) {
            if (L.busy || s->pending.empty()) continue;
            uint64_t blocked = 0;
            serve::form_batch(s->pending, s->arena, s->cfg.max_batch, batch, &blocked);
            if (blocked && blocked != last_blocked) ++s->st.deferred_memory;
            last_blocked = blocked ? blocked : last_blocked;
            if (batch.empty()) break;  // the head's memory does not fit yet
            L.t_launch = mono_now();
            L.reqs = batch;
            L.busy = true;
            ++s->st.launches;
            s->st.max_batch_seen = std::max(s->st.max_batch_seen, (int32_t)batch.size());
            lk.unlock();
            const qfca_status st = issue(s, L, L.reqs);
            lk.lock();
            if (st != QFCA_OK) {
                // work the failed call did enqueue may still use the memory
                (void)hipStreamSynchronize(L.stream);
                retire(s, L, st);
                s->cv_done.notify_all();
            } else {
                any_busy = true;
            }
            int inflight = 0;
            for (const LaunchSlot& M : s->slots) inflight += M.busy ? 1 : 0;
            s->st.max_inflight_seen = std::max(s->st.max_inflight_seen, (int32_t)inflight);
            progress = true;
        }
        if (s->stop && s->pending.empty() && s->incoming.empty() && !any_busy) break;
        if (!progress) {
            if (any_busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
    }
}

qfca_status srv_fail(qfca_status st, const char* msg) {
    set_error(msg);
    return st;
}

void teardown(qfca_server s) {
    for (LaunchSlot& L : s->slots) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.ctx) (void)qfca_ctx_destroy(L.ctx);
        if (L.ev0) (void)hipEventDestroy(L.ev0);
        if (L.ev1) (void)hipEventDestroy(L.ev1);
        if (L.h_err) (void)hipHostFree(L.h_err);
        if (L.stream) (void)hipStreamDestroy(L.stream);
    }
    if (s->t0) (void)hipEventDestroy(s->t0);
    if (s->base) (void)hipFree(s->base);
    delete s;
}

}  // namespace

extern "C" {

double qfca_clock(void) { return mono_now(); }

qfca_status qfca_server_create(int32_t device, const qfca_server_config* cfg, qfca_server* out) {
    if (!cfg || !out) return srv_fail(QFCA_E_ARG, "NULL argument");
    *out = nullptr;
    if (cfg->max_inflight < 1 || cfg->max_inflight > 8) return srv_fail(QFCA_E_ARG, "max_inflight must be 1..8");
    if (cfg->max_batch < 1 || cfg->max_batch > BATCH_MAXJ) return srv_fail(QFCA_E_ARG, "max_batch must be 1..256");
    if (cfg->hbm_budget < serve::kAlign) return srv_fail(QFCA_E_ARG, "hbm_budget too small");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return srv_fail(QFCA_E_ARG, "no such device");
    if (hipSetDevice(device) != hipSuccess) return srv_fail(QFCA_E_DEVICE, "hipSetDevice failed");
    qfca_server s = new (std::nothrow) qfca_server_s();
    if (!s) return srv_fail(QFCA_E_NOMEM, "server allocation failed");
    s->device = device;
    s->cfg = *cfg;
    const size_t budget = (size_t)cfg->hbm_budget / serve::kAlign * serve::kAlign;
    if (hipMalloc((void**)&s->base, budget) != hipSuccess) {
        (void)hipGetLastError();
        teardown(s);
        return srv_fail(QFCA_E_NOMEM, "could not allocate the server's memory budget");
    }
    s->arena.reset(budget);
    s->st.arena_bytes = budget;
    // Each slot's stream is created with a CU mask covering every compute
    // unit: such a stream gets a hardware queue of its own, so launches of
    // different slots are never serialised behind one another in a shared
    // queue (ordinary streams are spread over a small pool of queues).
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 1) {
        teardown(s);
        return srv_fail(QFCA_E_DEVICE, "could not read the compute-unit count");
    }
    std::vector<uint32_t> cu_mask((size_t)(ncu + 31) / 32, 0xFFFFFFFFu);
    if (ncu % 32) cu_mask.back() = (1u << (ncu % 32)) - 1u;
    s->slots.resize(cfg->max_inflight);
    for (LaunchSlot& L : s->slots) {
        if (hipExtStreamCreateWithCUMask(&L.stream, (uint32_t)cu_mask.size(), cu_mask.data()) != hipSuccess ||
            hipEventCreate(&L.ev0) != hipSuccess || hipEventCreate(&L.ev1) != hipSuccess ||
            hipHostMalloc((void**)&L.h_err, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
            teardown(s);
            return srv_fail(QFCA_E_DEVICE, "could not create the server's streams");
        }
        qfca_status st = qfca_ctx_create(device, L.stream, &L.ctx);
        if (st != QFCA_OK) {
            teardown(s);
            return st;
        }
        if (cfg->Ws > 0) {
            st = qfca_ctx_set_tile(L.ctx, cfg->Ws, cfg->Hb > 0 ? cfg->Hb : 128, 64, 1);
            if (st != QFCA_OK) {
                teardown(s);
                return st;
            }
        }
    }
    if (hipEventCreate(&s->t0) != hipSuccess || hipEventRecord(s->t0, s->slots[0].stream) != hipSuccess ||
        hipEventSynchronize(s->t0) != hipSuccess) {
        teardown(s);
        return srv_fail(QFCA_E_DEVICE, "could not record the server's time origin");
    }
    try {
        s->th = std::thread(dispatcher, s);
    } catch (...) {
        teardown(s);
        return srv_fail(QFCA_E_NOMEM, "could not start the dispatcher thread");
    }
    *out = s;
    return QFCA_OK;
}

qfca_status qfca_server_submit(qfca_server s, qfca_model model, const float* X, int32_t H, int32_t W,
                               float* score, uint64_t* ticket) {
    if (!s || !model || !X || !score || !ticket) return srv_fail(QFCA_E_ARG, "NULL argument");
    qfca_params p{};
    qfca_status st = qfca_model_params(model, &p);
    if (st != QFCA_OK) return st;
    qfca_job J{};
    J.model = model;
    J.X = X;
    J.H = H;
    J.W = W;
    J.score = score;
    st = batch_job_check(s->slots[0].ctx, J, p);
    if (st != QFCA_OK) return st;
    Request r;
    r.model = model;
    r.X = X;
    r.H = H;
    r.W = W;
    r.C = p.C;
    r.score = score;
    r.bytes = serve::request_bytes(p.C, H, W);
    if (r.bytes > s->arena.size()) return srv_fail(QFCA_E_NOMEM, "request exceeds the server's memory budget");
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return srv_fail(QFCA_E_STATE, "server is shutting down");
        int gid = -1;
        for (size_t i = 0; i < s->groups.size(); ++i)
            if (same_group(s->groups[i], p)) gid = (int)i;
        if (gid < 0) {
            s->groups.push_back(p);
            gid = (int)s->groups.size() - 1;
        }
        r.group = gid;
        r.ticket = s->next_ticket++;
        r.t_submit = mono_now();
        s->incoming.push_back(r);
        ++s->st.submitted;
        *ticket = r.ticket;
    }
    s->cv_work.notify_one();
    return QFCA_OK;
}

qfca_status qfca_server_poll(qfca_server s, qfca_completion* out, int32_t cap, int32_t* n) {
    if (!s || !n || (cap > 0 && !out)) return srv_fail(QFCA_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    int32_t k = 0;
    while (k < cap && !s->finished.empty()) {
        out[k++] = s->finished.front();
        s->finished.pop_front();
    }
    *n = k;
    return QFCA_OK;
}

qfca_status qfca_server_drain(qfca_server s) {
    if (!s) return srv_fail(QFCA_E_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_work.notify_one();
    s->cv_done.wait(lk, [s] { return s->st.completed == s->st.submitted; });
    return QFCA_OK;
}

qfca_status qfca_server_stats(qfca_server s, qfca_server_counters* out) {
    if (!s || !out) return srv_fail(QFCA_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    qfca_server_counters r = s->st;
    r.arena_peak = s->arena.peak();
    std::vector<std::pair<double, double>> iv = s->intervals;
    std::sort(iv.begin(), iv.end());
    double busy = 0.0, cur0 = 0.0, cur1 = -1.0;
    uint64_t ov = 0;
    for (size_t i = 0; i < iv.size(); ++i) {
        // overlap with any other interval: with the running union of earlier
        // starts, or with the next interval's start
        const bool meets_prev = i > 0 && iv[i].first < cur1;
        const bool meets_next = i + 1 < iv.size() && iv[i + 1].first < iv[i].second;
        if (meets_prev || meets_next) ++ov;
        if (iv[i].first > cur1) {
            if (cur1 > cur0) busy += cur1 - cur0;
            cur0 = iv[i].first;
            cur1 = iv[i].second;
        } else {
            cur1 = std::max(cur1, iv[i].second);
        }
    }
    if (cur1 > cur0) busy += cur1 - cur0;
    r.device_busy_s = busy;
    r.device_span_s = iv.empty() ? 0.0 : std::max_element(iv.begin(), iv.end(), [](auto& a, auto& b) {
                                              return a.second < b.second;
                                          })->second - iv.front().first;
    r.overlapped = ov;
    *out = r;
    return QFCA_OK;
}

qfca_status qfca_server_destroy(qfca_server s) {
    if (!s) return srv_fail(QFCA_E_ARG, "NULL argument");
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_one();
    if (s->th.joinable()) s->th.join();
    teardown(s);
    return QFCA_OK;
}

}  // extern "C"
