// conv_serve.cpp -- continuous-batching server for the width-5 separable
// convolution.
//
// Requests (device-resident images of any size, each with its own taps) are
// submitted without blocking.  One scheduler thread per server loops over:
//   1. retire: launches whose completion event has fired free their slots and
//      HBM budget and stamp their tickets done;
//   2. admit: while a launch stream is idle, queued requests are taken in
//      arrival order as long as a slot is free and their footprint (input +
//      output bytes) fits the budget, up to max_batch requests of one dtype
//      and max_batch_bytes per launch (so large frames run alone and small
//      ones share launches);
//   3. launch: each admitted group becomes ONE batch launch on its stream (a
//      group of one the single-image kernel), after a wait on the producers'
//      events, followed by a completion event;
//   4. poll the in-flight events, or spin briefly and then sleep when idle;
//      while nothing was submitted or finished the loop skips the lock.
// A submit that finds nothing queued and a stream idle, arriving at least
// 10 us after the previous one, launches its request itself (unless
// queue_only is set): at sparse arrivals there is nothing to batch with and
// the hop to the scheduler only adds latency.  It hands the in-flight launch
// to the scheduler, which retires it like its own.
// Requests that arrive while a launch runs go into the next launch on another
// stream, so their work overlaps on the device.  A request's result is the
// same tile code on the same values as a lone call, so it is bitwise
// identical.
//
// Locking: the mutex guards what submitters and pollers touch (queue, ticket
// table, event pool, statistics) and the budget counters.  Streams and the
// list of in-flight launches belong to the scheduler thread, and every HIP
// call of the scheduler runs without the lock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "conv_common.h"

using namespace convsep5;

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum ReqState { QUEUED = 0, INFLIGHT = 1, DONE = 2, FAILED = 3 };

constexpr uint64_t kSpinIdleNs = 2000000;  // scheduler spins 2 ms after going idle
// A submit launches its request itself only if the previous submit was at
// least this long ago (longer than a launch takes to enqueue).
constexpr uint64_t kDirectGapNs = 10000;

struct Req {
    uint64_t ticket = 0;
    const void *in = nullptr;
    void *out = nullptr;
    float k[5] = {0, 0, 0, 0, 0};
    conv_image img{};
    uint64_t footprint = 0;
    conv_req_times t{};
    int state = QUEUED;
    hipEvent_t ready = nullptr;  // recorded on the producer stream at submit
    hipStream_t producer = nullptr;
};

struct Launch {
    std::vector<Req *> reqs;
    uint64_t bytes = 0;
    hipEvent_t ev = nullptr;
    int stream = 0;
};

}  // namespace

struct conv_server {
    // fixed after creation
    conv_serve_cfg cfg{};
    int device = 0;
    std::vector<hipStream_t> streams;
    // scheduler thread only
    std::vector<Launch> inflight;
    // shared, guarded by mu
    std::mutex mu;
    std::condition_variable cv;       // new work or stop
    std::condition_variable idle_cv;  // nothing queued or in flight
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, Req *> reqs;
    std::vector<hipEvent_t> ready_pool;  // producer-stream events
    std::vector<hipEvent_t> event_pool;  // launch-completion events
    std::vector<char> stream_busy;
    std::vector<Launch> handoff;         // launched by a submitter, not yet polled
    uint64_t last_submit_ns = 0;
    uint64_t bytes_in_flight = 0;
    int slots_in_flight = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool idle = true;
    // Bumped (under mu) whenever a submit or destroy changes what the
    // scheduler must look at, so that its polling loop can skip the lock
    // while nothing changed: a submitter then rarely finds mu held.
    std::atomic<uint64_t> seq{0};
    conv_serve_stats stats{};
    std::thread th;

    void run();
    std::vector<Launch> admit_locked();
    conv_status enqueue(Launch &L, hipEvent_t done_ev);
    bool launched_locked(Launch &L, conv_status rc, uint64_t t_launch);
};

// Takes admissible requests off the queue (caller holds mu).
std::vector<Launch> conv_server::admit_locked() {
    std::vector<Launch> out;
    while (!queue.empty()) {
        int s = -1;
        for (int i = 0; i < (int)streams.size(); ++i)
            if (!stream_busy[i]) {
                s = i;
                break;
            }
        if (s < 0) break;
        Launch L;
        L.stream = s;
        const int dtype = queue.front()->img.dtype;
        const uint64_t cap = cfg.max_batch_bytes ? cfg.max_batch_bytes : ~(uint64_t)0;
        while (!queue.empty() && (int)L.reqs.size() < cfg.max_batch &&
               slots_in_flight + 1 <= cfg.max_slots &&
               bytes_in_flight + queue.front()->footprint <= cfg.hbm_budget_bytes &&
               queue.front()->img.dtype == dtype &&
               (L.reqs.empty() || L.bytes + queue.front()->footprint <= cap)) {
            Req *r = queue.front();
            queue.pop_front();
            L.reqs.push_back(r);
            L.bytes += r->footprint;
            bytes_in_flight += r->footprint;
            slots_in_flight += 1;
        }
        if (L.reqs.empty()) break;  // the head does not fit yet: wait for a retirement
        stream_busy[s] = 1;
        const uint64_t t = now_ns();
        for (Req *r : L.reqs) {
            r->t.admit_ns = t;
            r->t.batch_size = (int32_t)L.reqs.size();
            r->t.stream = s;
            r->state = INFLIGHT;
        }
        if (event_pool.empty()) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess)
                event_pool.push_back(e);
        }
        if (!event_pool.empty()) {
            L.ev = event_pool.back();
            event_pool.pop_back();
        }
        stats.max_bytes_in_flight = std::max<uint64_t>(stats.max_bytes_in_flight, bytes_in_flight);
        stats.max_slots_in_flight = std::max(stats.max_slots_in_flight, slots_in_flight);
        stats.max_batch = std::max(stats.max_batch, (int32_t)L.reqs.size());
        out.push_back(std::move(L));
    }
    return out;
}

// Enqueues one admitted group on its stream (no lock held).
conv_status conv_server::enqueue(Launch &L, hipEvent_t done_ev) {
    if (!done_ev) return CONV_EHIP;
    const int n = (int)L.reqs.size();
    const int dtype = L.reqs[0]->img.dtype;
    std::vector<const void *> ins(n);
    std::vector<void *> outs(n);
    std::vector<float> ks(5 * n);
    std::vector<conv_image> imgs(n);
    for (int i = 0; i < n; ++i) {
        const Req *r = L.reqs[i];
        ins[i] = r->in;
        outs[i] = r->out;
        for (int j = 0; j < 5; ++j) ks[5 * i + j] = r->k[j];
        imgs[i] = r->img;
    }
    hipStream_t s = streams[L.stream];
    const conv_tile_cfg tc = get_cfg(dtype, 1);
    std::vector<ImgDev> descs;
    int64_t total = 0;
    int dt = 0;
    // a group of one runs the single-image kernel (same tiles, same bits,
    // less to marshal); larger groups one batch launch
    conv_status st = n == 1 ? CONV_OK
                            : build_batch(n, ins.data(), outs.data(), ks.data(), imgs.data(),
                                          CONV_1PASS_FUSED, tc, &descs, &total, &dt);
    // The launch starts only after each request's producer work.  Events
    // recorded on one stream complete in order, so waiting on the latest
    // request of each producer stream covers the earlier ones.
    std::vector<std::pair<hipStream_t, hipEvent_t>> last;
    for (Req *r : L.reqs) {
        if (!r->ready) continue;  // producer_wait = 0
        bool found = false;
        for (auto &pe : last)
            if (pe.first == r->producer) {
                pe.second = r->ready;
                found = true;
            }
        if (!found) last.emplace_back(r->producer, r->ready);
    }
    for (auto &pe : last)
        if (st == CONV_OK && hipStreamWaitEvent(s, pe.second, 0) != hipSuccess) st = CONV_EHIP;
    if (st == CONV_OK)
        st = n == 1 ? conv_sep5_1pass(ins[0], outs[0], ks.data(), &imgs[0], CONV_1PASS_FUSED, s)
                    : enqueue_batch(descs, total, dtype, MODE_FUSED, tc, s);
    if (st == CONV_OK && hipEventRecord(done_ev, s) != hipSuccess) st = CONV_EHIP;
    return st;
}

// Bookkeeping after a launch attempt (caller holds mu): stamps the launch
// time and returns the ready events; a failed launch fails its requests and
// frees what admission took.  True if the launch is in flight.
bool conv_server::launched_locked(Launch &L, conv_status rc, uint64_t t_launch) {
    for (Req *r : L.reqs) {
        if (r->ready) ready_pool.push_back(r->ready);
        r->ready = nullptr;
        r->t.launch_ns = t_launch;
    }
    if (rc != CONV_OK) {
        for (Req *r : L.reqs) {
            r->t.done_ns = t_launch;
            r->state = FAILED;
        }
        stats.failed += L.reqs.size();
        bytes_in_flight -= L.bytes;
        slots_in_flight -= (int)L.reqs.size();
        stream_busy[L.stream] = 0;
        if (L.ev) event_pool.push_back(L.ev);
        return false;
    }
    stats.launches += 1;
    int busy = 0;
    for (char b : stream_busy) busy += b != 0;
    stats.max_streams_busy = std::max(stats.max_streams_busy, (int32_t)busy);
    return true;
}

void conv_server::run() {
    hipSetDevice(device);
    uint64_t seen = ~0ull;  // seq when the locked part last ran
    for (;;) {
        // 1. retire finished launches (event queries without the lock)
        std::vector<std::pair<Launch, hipError_t>> finished;
        for (size_t i = 0; i < inflight.size();) {
            const hipError_t q = hipEventQuery(inflight[i].ev);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            finished.emplace_back(std::move(inflight[i]), q);
            inflight.erase(inflight.begin() + i);
        }
        const uint64_t t_done = now_ns();
        // Nothing finished and nothing submitted since the last look: the
        // queue cannot have become admissible, so poll again without mu.
        const uint64_t s_now = seq.load(std::memory_order_acquire);
        if (finished.empty() && s_now == seen && !inflight.empty()) {
            std::this_thread::yield();
            continue;
        }
        seen = s_now;
        std::vector<Launch> admitted;
        {
            std::lock_guard<std::mutex> g(mu);
            for (auto &fq : finished) {
                Launch &L = fq.first;
                for (Req *r : L.reqs) {
                    r->t.done_ns = t_done;
                    r->state = fq.second == hipSuccess ? DONE : FAILED;
                }
                if (fq.second == hipSuccess) stats.completed += L.reqs.size();
                else stats.failed += L.reqs.size();
                bytes_in_flight -= L.bytes;
                slots_in_flight -= (int)L.reqs.size();
                stream_busy[L.stream] = 0;
                event_pool.push_back(L.ev);
            }
            // launches made by submitters join the polled set
            for (Launch &L : handoff) inflight.push_back(std::move(L));
            handoff.clear();
            // 2. admit
            admitted = admit_locked();
        }
        // 3. launch (no lock)
        if (!admitted.empty()) {
            std::vector<conv_status> rc(admitted.size());
            for (size_t i = 0; i < admitted.size(); ++i) rc[i] = enqueue(admitted[i], admitted[i].ev);
            const uint64_t t_launch = now_ns();
            std::lock_guard<std::mutex> g(mu);
            for (size_t i = 0; i < admitted.size(); ++i)
                if (launched_locked(admitted[i], rc[i], t_launch))
                    inflight.push_back(std::move(admitted[i]));
        }
        // 4. wait
        if (!inflight.empty()) {
            std::this_thread::yield();
            continue;
        }
        std::unique_lock<std::mutex> lk(mu);
        // (slots still in flight here belong to a launch a submitter is making)
        if (!queue.empty() || !handoff.empty() || slots_in_flight > 0) continue;
        idle = true;
        idle_cv.notify_all();
        if (stop) break;
        // Stay awake a little for the next arrival (a futex wake-up costs tens
        // of microseconds), then sleep until a submit.
        const uint64_t idle_from = now_ns();
        const uint64_t s_idle = seq.load(std::memory_order_relaxed);
        lk.unlock();
        while (seq.load(std::memory_order_acquire) == s_idle && now_ns() - idle_from < kSpinIdleNs)
            std::this_thread::yield();
        lk.lock();
        if (queue.empty() && handoff.empty() && !stop) cv.wait(lk);
    }
}

extern "C" {

conv_status conv_serve_create(const conv_serve_cfg *cfg, conv_server **srv) {
    clear_error();
    if (!cfg || !srv) return set_error(CONV_EINVAL, "NULL argument");
    *srv = nullptr;
    if (cfg->hbm_budget_bytes == 0 || cfg->max_slots < 1 || cfg->n_streams < 1 ||
        cfg->n_streams > 16 || cfg->max_batch < 1 ||
        (cfg->producer_wait != 0 && cfg->producer_wait != 1) ||
        (cfg->queue_only != 0 && cfg->queue_only != 1))
        return set_error(CONV_EINVAL, "bad server configuration");
    int prev = 0;
    hipGetDevice(&prev);
    int dev = cfg->device < 0 ? prev : cfg->device;
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_error(e, "hipSetDevice");
    auto *s = new conv_server();
    s->cfg = *cfg;
    s->device = dev;
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t x : s->streams) hipStreamDestroy(x);
            delete s;
            hipSetDevice(prev);
            return hip_error(e, "hipStreamCreate");
        }
        s->streams.push_back(st);
        s->stream_busy.push_back(0);
    }
    hipSetDevice(prev);
    s->th = std::thread([s] { s->run(); });
    *srv = s;
    return CONV_OK;
}

conv_status conv_serve_submit(conv_server *srv, const void *d_in, void *d_out, const float k[5],
                              const conv_image *img, hipStream_t stream, uint64_t *ticket) {
    const uint64_t t_submit = now_ns();
    clear_error();
    if (!srv || !ticket || !k) return set_error(CONV_EINVAL, "NULL argument");
    Layout L;
    conv_status st = check_image(img, &L);
    if (st != CONV_OK) return st;
    if ((st = reject_hwc(L, "the server")) != CONV_OK) return st;
    if (!L.empty) {
        if (!d_in || !d_out) return set_error(CONV_EINVAL, "NULL device pointer");
        if (overlaps(d_in, L.extent_bytes, d_out, L.extent_bytes))
            return set_error(CONV_EALIAS, "input and output overlap");
    }
    const uint64_t fp = 2 * (uint64_t)L.extent_bytes;
    if (fp > srv->cfg.hbm_budget_bytes)
        return set_error(CONV_ENOMEM, "footprint %llu exceeds the budget %llu",
                         (unsigned long long)fp, (unsigned long long)srv->cfg.hbm_budget_bytes);
    hipEvent_t ready = nullptr;
    if (!L.empty && srv->cfg.producer_wait) {
        {
            std::lock_guard<std::mutex> g(srv->mu);
            if (!srv->ready_pool.empty()) {
                ready = srv->ready_pool.back();
                srv->ready_pool.pop_back();
            }
        }
        hipError_t e = hipSuccess;
        if (!ready) e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(ready, stream);
        if (e != hipSuccess) {
            if (ready) {
                std::lock_guard<std::mutex> g(srv->mu);
                srv->ready_pool.push_back(ready);
            }
            return hip_error(e, "recording the request's ready event");
        }
    }
    auto *r = new Req();
    r->ready = ready;
    r->producer = stream;
    r->in = d_in;
    r->out = d_out;
    for (int i = 0; i < 5; ++i) r->k[i] = k[i];
    r->img = *img;
    r->footprint = fp;
    r->t.submit_ns = t_submit;
    // the direct launch runs on this thread: its current device must be the
    // server's (descriptors and the CU count follow the current device)
    int cur = -1;
    const bool on_device = hipGetDevice(&cur) == hipSuccess && cur == srv->device;
    Launch direct;
    bool have_direct = false;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        if (srv->stop) {
            if (r->ready) srv->ready_pool.push_back(r->ready);
            delete r;
            return set_error(CONV_EINVAL, "server is shutting down");
        }
        r->ticket = srv->next_ticket++;
        srv->stats.submitted += 1;
        srv->reqs[r->ticket] = r;
        if (L.empty) {
            r->t.admit_ns = r->t.launch_ns = r->t.done_ns = r->t.submit_ns;
            r->state = DONE;
            srv->stats.completed += 1;
        } else {
            // Nothing is queued and the previous request came long enough ago
            // that this thread can spend a launch (~6 us) without falling
            // behind its arrivals: there is nothing to batch this request
            // with, so admit and launch it here (if a stream is idle) rather
            // than wake the scheduler.  Dense arrivals stay with the
            // scheduler, which batches them.
            const bool try_direct = !srv->cfg.queue_only && srv->queue.empty() &&
                                    t_submit - srv->last_submit_ns >= kDirectGapNs;
            srv->last_submit_ns = t_submit;
            srv->queue.push_back(r);
            srv->idle = false;
            srv->seq.fetch_add(1, std::memory_order_release);
            if (try_direct && on_device) {
                std::vector<Launch> now = srv->admit_locked();
                if (!now.empty()) {
                    direct = std::move(now[0]);
                    have_direct = true;
                }
            }
        }
        *ticket = r->ticket;
    }
    if (have_direct) {
        const conv_status rc = srv->enqueue(direct, direct.ev);
        const uint64_t t_launch = now_ns();
        std::lock_guard<std::mutex> g(srv->mu);
        if (srv->launched_locked(direct, rc, t_launch)) {
            if (srv->stats.direct_launches < INT32_MAX) srv->stats.direct_launches += 1;
            srv->handoff.push_back(std::move(direct));
        }
        srv->seq.fetch_add(1, std::memory_order_release);
    }
    srv->cv.notify_one();
    return CONV_OK;
}

conv_status conv_serve_poll(conv_server *srv, uint64_t ticket, conv_req_times *t) {
    clear_error();
    if (!srv) return set_error(CONV_EINVAL, "NULL server");
    std::lock_guard<std::mutex> g(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return set_error(CONV_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second;
    if (r->state == QUEUED || r->state == INFLIGHT) return CONV_EAGAIN;
    if (t) *t = r->t;
    const int state = r->state;
    srv->reqs.erase(it);
    delete r;
    if (state == FAILED)
        return set_error(CONV_EHIP, "the launch of ticket %llu failed", (unsigned long long)ticket);
    return CONV_OK;
}

conv_status conv_serve_drain(conv_server *srv) {
    clear_error();
    if (!srv) return set_error(CONV_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv.notify_one();
    srv->idle_cv.wait(lk, [srv] { return srv->idle; });
    return CONV_OK;
}

conv_status conv_serve_get_stats(conv_server *srv, conv_serve_stats *stats) {
    clear_error();
    if (!srv || !stats) return set_error(CONV_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(srv->mu);
    *stats = srv->stats;
    return CONV_OK;
}

conv_status conv_serve_destroy(conv_server *srv) {
    clear_error();
    if (!srv) return CONV_OK;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
        srv->seq.fetch_add(1, std::memory_order_release);
    }
    srv->cv.notify_one();
    if (srv->th.joinable()) srv->th.join();
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(srv->device);
    for (hipEvent_t e : srv->event_pool) hipEventDestroy(e);
    for (hipEvent_t e : srv->ready_pool) hipEventDestroy(e);
    for (hipStream_t s : srv->streams) hipStreamDestroy(s);
    hipSetDevice(prev);
    for (auto &kv : srv->reqs) delete kv.second;
    delete srv;
    return CONV_OK;
}

}  // extern "C"
