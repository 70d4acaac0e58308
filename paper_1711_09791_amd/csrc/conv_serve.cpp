// conv_serve.cpp -- continuous-batching server for the width-5 separable
// convolution.
//
// Requests (device-resident images of any size, each with its own taps) are
// submitted without blocking into a host-side queue; the images stay in
// device memory and only their descriptors pass through the queue.  One
// scheduler thread per server loops over:
//   1. retire: launches whose completion word holds their token free their
//      slots and HBM budget and stamp their tickets done;
//   2. admit: while a launch stream has room (no launch, or with
//      launch_depth > 1 fewer than that many, the last one already
//      enqueued), queued requests are taken in arrival order as long as a
//      slot is free and their footprint (input + output bytes) fits the
//      budget, up to max_batch requests of one dtype
//      and max_batch_bytes per launch (so large frames run alone and small
//      ones share launches).  A request whose buffers overlap those of a
//      request admitted before it and not yet retired (it reads what that one
//      writes, or writes what that one reads or writes) stops admission until
//      that request retires, so such requests run in submission order and
//      never share a launch;
//   3. launch: each admitted group becomes ONE batch launch on its stream (a
//      group of one the single-image kernel), after a wait on the producers'
//      events, followed by a one-lane kernel that writes the launch's token
//      into that stream's completion word in pinned host memory;
//   4. poll the completion words without pausing (plain loads of host
//      memory, no HIP call, so the polling never contends with a launch in
//      the HIP runtime; a launch not confirmed after 2 ms is checked with
//      hipStreamQuery, which reports a failed stream), or spin 2 ms and then
//      sleep when idle; while nothing was submitted or finished the loop
//      skips the lock.
// A submit that finds nothing queued and a stream idle launches its request
// itself (unless queue_only is set) when submits arrive sparsely: the running
// mean gap between submits, and the gap before this one, are at least the
// time a launch takes to enqueue, so there is nothing to batch with and the
// hop to the scheduler would only add latency.  It hands the in-flight launch
// to the scheduler, which writes its completion token (with one launch per
// stream) and retires it like its own.  Dense arrivals go to the scheduler,
// which batches them.
// Requests that arrive while a launch runs go into the next launch on another
// stream, so their work overlaps on the device.  A request's result is the
// same tile code on the same values as a lone call, so it is bitwise
// identical.
//
// Locking: the mutex guards what submitters and pollers touch (queue, ticket
// table, request pool, producer-event pool, statistics) and the budget
// counters.  Streams and the list of in-flight launches belong to the
// scheduler thread, and every HIP call of the scheduler runs without the lock.
// Requests live in a pool of fixed blocks and are found by ticket in a
// power-of-two table: no heap allocation per request and no hashing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <memory>
#include <thread>
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

// Writes a launch's token into its stream's completion word: launched right
// after the launch's kernel, so it runs once that kernel is complete.  One
// lane stores it.  Against the runtime's stream write (hipStreamWriteValue64)
// this costs the scheduler less host time per launch and the completion is
// seen sooner: on the mixed serving stream at half load, launch-to-seen fell
// from 27 to 24 us at the median and the 640x480 capacity rose from 805k to
// 855k requests/s.
__global__ __launch_bounds__(64) void k_token(uint64_t *word, uint64_t token) {
    // a system-scope store goes through to host memory (no cache keeps it)
    if (threadIdx.x == 0) __hip_atomic_store(word, token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t write_done_token(hipStream_t s, uint64_t *word, uint64_t token) {
    hipLaunchKernelGGL(k_token, dim3(1), dim3(64), 0, s, word, token);
    return hipGetLastError();
}

enum ReqState { QUEUED = 0, INFLIGHT = 1, DONE = 2, FAILED = 3 };

constexpr uint64_t kSpinIdleNs = 2000000;  // scheduler spins 2 ms after going idle
// A submit launches its request itself only while the running mean gap
// between submits, and the gap before this submit, are at least this long
// (about what a launch takes to enqueue): then the submitting thread keeps up
// with its arrivals.
constexpr uint64_t kDirectGapNs = 8000;
// The running mean: gap_mean += (gap - gap_mean) / 4, each gap clamped to
// kGapClampNs so that a burst after an idle spell is seen within a few submits.
constexpr uint64_t kGapClampNs = 100000;
constexpr int kPoolBlock = 256;         // requests per pool block
// A launch whose completion word has not shown its token this long after the
// launch is checked with hipStreamQuery (a failed launch never writes it).
constexpr uint64_t kStreamCheckNs = 2000000;
// Completion words are one 64-byte line apart (in 8-byte words).
constexpr int kDoneStride = 8;
constexpr size_t kTicketTable0 = 1024;  // initial ticket table size (power of two)

struct Req {
    uint64_t ticket = 0;
    const void *in = nullptr;
    void *out = nullptr;
    int64_t bytes = 0;           // extent of the input (and of the output) in bytes
    float k[5] = {0, 0, 0, 0, 0};
    conv_image img{};
    uint64_t footprint = 0;
    conv_req_times t{};
    int state = QUEUED;
    int active_idx = -1;         // position in the server's admitted list
    hipEvent_t ready = nullptr;  // recorded on the producer stream at submit
    hipStream_t producer = nullptr;
};

// Whether b, submitted after a, must wait for a: b reads what a writes, or
// writes what a reads or writes.
bool conflicts(const Req *a, const Req *b) {
    return overlaps(b->in, b->bytes, a->out, a->bytes) ||
           overlaps(b->out, b->bytes, a->in, a->bytes) ||
           overlaps(b->out, b->bytes, a->out, a->bytes);
}

struct Launch {
    std::vector<Req *> reqs;
    uint64_t bytes = 0;
    uint64_t token = 0;    // written to its stream's completion word after the kernel
    uint64_t check_ns = 0; // next time to ask hipStreamQuery about it
    int stream = 0;
    bool token_pending = false;  // launched by a submitter: the scheduler writes its token
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
    std::vector<Req *> active;           // admitted, not yet retired
    // requests: fixed blocks, a free list, and the ticket table
    std::vector<std::unique_ptr<Req[]>> blocks;
    std::vector<Req *> free_reqs;
    std::vector<Req *> table;            // ticket & (size - 1) -> live request
    std::vector<hipEvent_t> ready_pool;  // producer-stream events
    // Completion words, one per stream, in pinned host memory: the stream
    // writes a launch's token after its kernel; the scheduler reads them with
    // plain loads.  Tokens grow in admission order and a stream's launches
    // are enqueued in that order, so a word at or past a launch's token
    // means that launch and every earlier one on the stream are done.
    uint64_t *done_host = nullptr;
    uint64_t *done_dev = nullptr;
    uint64_t next_token = 1;
    int depth = 1;                       // launches in flight per stream, at most
    std::vector<int> stream_load;        // launches admitted, not yet retired
    std::vector<char> stream_pending;    // one of them not yet enqueued
    std::vector<uint64_t> stream_bytes;  // their footprint
    std::vector<Launch> handoff;         // launched by a submitter, not yet polled
    uint64_t last_submit_ns = 0;
    uint64_t gap_mean_ns = kGapClampNs;  // running mean gap between submits
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
    std::vector<Launch> admit_locked(bool idle_only);
    bool blocked_locked(const Req *r, const Launch &L) const;
    void retire_locked(Req *r, int state, uint64_t t_done);
    conv_status enqueue(Launch &L, bool write_token = true);
    bool launched_locked(Launch &L, conv_status rc, uint64_t t_launch);
    Req *new_req_locked();
    void put_ticket_locked(Req *r);
    Req *find_ticket_locked(uint64_t ticket) const;
    void free_req_locked(Req *r);
};

Req *conv_server::new_req_locked() {
    if (free_reqs.empty()) {
        blocks.emplace_back(new Req[kPoolBlock]);
        Req *b = blocks.back().get();
        free_reqs.reserve(blocks.size() * kPoolBlock);
        for (int i = kPoolBlock - 1; i >= 0; --i) free_reqs.push_back(&b[i]);
    }
    Req *r = free_reqs.back();
    free_reqs.pop_back();
    *r = Req();
    return r;
}

// Tickets are consecutive, so live tickets collide in the table only when
// more of them are unpolled than it has entries: then it doubles.
void conv_server::put_ticket_locked(Req *r) {
    if (table.empty()) table.assign(kTicketTable0, nullptr);
    while (table[r->ticket & (table.size() - 1)]) {
        std::vector<Req *> old;
        old.swap(table);
        for (size_t n = old.size() * 2;; n *= 2) {
            table.assign(n, nullptr);
            bool ok = true;
            for (Req *e : old) {
                if (!e) continue;
                Req *&slot = table[e->ticket & (n - 1)];
                if (slot) {
                    ok = false;
                    break;
                }
                slot = e;
            }
            if (ok) break;
        }
    }
    table[r->ticket & (table.size() - 1)] = r;
}

Req *conv_server::find_ticket_locked(uint64_t ticket) const {
    if (table.empty()) return nullptr;
    Req *r = table[ticket & (table.size() - 1)];
    return r && r->ticket == ticket ? r : nullptr;
}

void conv_server::free_req_locked(Req *r) {
    table[r->ticket & (table.size() - 1)] = nullptr;
    free_reqs.push_back(r);
}

// The request leaves the admitted list with its final state.
void conv_server::retire_locked(Req *r, int state, uint64_t t_done) {
    r->t.done_ns = t_done;
    r->state = state;
    if (r->active_idx >= 0) {
        Req *last = active.back();
        active[r->active_idx] = last;
        last->active_idx = r->active_idx;
        active.pop_back();
        r->active_idx = -1;
    }
}

// r must wait: it conflicts with an admitted request not yet retired, or with
// one already in the group being formed.
bool conv_server::blocked_locked(const Req *r, const Launch &L) const {
    for (const Req *a : active)
        if (conflicts(a, r)) return true;
    for (const Req *a : L.reqs)
        if (conflicts(a, r)) return true;
    return false;
}

// Takes admissible requests off the queue (caller holds mu).  A group goes
// to an idle stream, else (idle_only false, launch_depth > 1) behind the
// launch with the fewest bytes on a stream with room whose launches are all
// enqueued already, so that each stream receives its launches in token order.
std::vector<Launch> conv_server::admit_locked(bool idle_only) {
    std::vector<Launch> out;
    const int room = idle_only ? 1 : depth;
    while (!queue.empty()) {
        int s = -1;
        for (int i = 0; i < (int)streams.size(); ++i) {
            if (stream_pending[i] || stream_load[i] >= room) continue;
            if (s < 0 || stream_load[i] < stream_load[s] ||
                (stream_load[i] == stream_load[s] && stream_bytes[i] < stream_bytes[s]))
                s = i;
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
               (L.reqs.empty() || L.bytes + queue.front()->footprint <= cap) &&
               !blocked_locked(queue.front(), L)) {
            Req *r = queue.front();
            queue.pop_front();
            L.reqs.push_back(r);
            L.bytes += r->footprint;
            bytes_in_flight += r->footprint;
            slots_in_flight += 1;
        }
        // the head does not fit yet, or must wait for an earlier request:
        // wait for a retirement
        if (L.reqs.empty()) break;
        stream_load[s] += 1;
        stream_pending[s] = 1;
        stream_bytes[s] += L.bytes;
        const uint64_t t = now_ns();
        for (Req *r : L.reqs) {
            r->t.admit_ns = t;
            r->t.batch_size = (int32_t)L.reqs.size();
            r->t.stream = s;
            r->state = INFLIGHT;
            r->active_idx = (int)active.size();
            active.push_back(r);
        }
        L.token = next_token++;
        stats.max_bytes_in_flight = std::max<uint64_t>(stats.max_bytes_in_flight, bytes_in_flight);
        stats.max_slots_in_flight = std::max(stats.max_slots_in_flight, slots_in_flight);
        stats.max_batch = std::max(stats.max_batch, (int32_t)L.reqs.size());
        out.push_back(std::move(L));
    }
    return out;
}

// Enqueues one admitted group on its stream (no lock held).
conv_status conv_server::enqueue(Launch &L, bool write_token) {
    const int n = (int)L.reqs.size();
    hipStream_t s = streams[L.stream];
    if (n == 1) {
        // a group of one runs the single-image kernel (same tiles, same bits)
        const Req *r = L.reqs[0];
        conv_status st = CONV_OK;
        if (r->ready && hipStreamWaitEvent(s, r->ready, 0) != hipSuccess) st = CONV_EHIP;
        if (st == CONV_OK) st = conv_sep5_1pass(r->in, r->out, r->k, &r->img, CONV_1PASS_FUSED, s);
        if (st == CONV_OK && !write_token) L.token_pending = true;
        else if (st == CONV_OK && write_done_token(s, &done_dev[L.stream * kDoneStride], L.token) != hipSuccess)
            st = CONV_EHIP;
        return st;
    }
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
    const conv_tile_cfg tc = get_cfg(dtype, 1);
    std::vector<ImgDev> descs;
    int64_t total = 0;
    int dt = 0;
    conv_status st = build_batch(n, ins.data(), outs.data(), ks.data(), imgs.data(),
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
    if (st == CONV_OK) st = enqueue_batch(descs, total, dtype, MODE_FUSED, tc, s);
    if (st == CONV_OK && !write_token) L.token_pending = true;
    else if (st == CONV_OK && write_done_token(s, &done_dev[L.stream * kDoneStride], L.token) != hipSuccess)
        st = CONV_EHIP;
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
    stream_pending[L.stream] = 0;
    if (rc != CONV_OK) {
        for (Req *r : L.reqs) retire_locked(r, FAILED, t_launch);
        stats.failed += L.reqs.size();
        bytes_in_flight -= L.bytes;
        slots_in_flight -= (int)L.reqs.size();
        stream_load[L.stream] -= 1;
        stream_bytes[L.stream] -= L.bytes;
        return false;
    }
    L.check_ns = t_launch + kStreamCheckNs;
    stats.launches += 1;
    int busy = 0;
    for (int b : stream_load) busy += b;
    stats.max_streams_busy = std::max(stats.max_streams_busy, (int32_t)busy);
    return true;
}

void conv_server::run() {
    hipSetDevice(device);
    uint64_t seen = ~0ull;  // seq when the locked part last ran
    for (;;) {
        // 1. retire finished launches (completion words, without the lock)
        std::vector<std::pair<Launch, hipError_t>> finished;
        for (size_t i = 0; i < inflight.size();) {
            Launch &L = inflight[i];
            hipError_t q = __atomic_load_n(&done_host[L.stream * kDoneStride], __ATOMIC_ACQUIRE) >= L.token
                               ? hipSuccess
                               : hipErrorNotReady;
            if (q == hipErrorNotReady) {
                const uint64_t t = now_ns();
                if (t >= L.check_ns) {
                    // slow path: a failed launch never writes its token
                    q = hipStreamQuery(streams[L.stream]);
                    L.check_ns = t + kStreamCheckNs;
                }
            }
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            finished.emplace_back(std::move(L), q);
            inflight.erase(inflight.begin() + i);
        }
        const uint64_t t_done = now_ns();
        // Nothing finished and nothing submitted since the last look: the
        // queue cannot have become admissible, so poll again without mu.
        // Every stream full of launches this thread polls: nothing can be
        // admitted (and no submitter launch is pending) until one finishes.
        const uint64_t s_now = seq.load(std::memory_order_acquire);
        if (finished.empty() && !inflight.empty() &&
            (s_now == seen || inflight.size() >= streams.size() * (size_t)depth))
            continue;
        seen = s_now;
        std::vector<Launch> admitted;
        {
            std::lock_guard<std::mutex> g(mu);
            for (auto &fq : finished) {
                Launch &L = fq.first;
                for (Req *r : L.reqs) retire_locked(r, fq.second == hipSuccess ? DONE : FAILED, t_done);
                if (fq.second == hipSuccess) stats.completed += L.reqs.size();
                else stats.failed += L.reqs.size();
                bytes_in_flight -= L.bytes;
                slots_in_flight -= (int)L.reqs.size();
                stream_load[L.stream] -= 1;
                stream_bytes[L.stream] -= L.bytes;
            }
            // launches made by submitters join the polled set
            for (Launch &L : handoff) inflight.push_back(std::move(L));
            handoff.clear();
            // 2. admit
            admitted = admit_locked(false);
        }
        // A submitter's launch leaves its token to this thread (the submitting
        // thread then spends only the kernel launch).  Its stream takes no
        // other launch before this one retires (one launch per stream), and
        // the kernel outlasts the hand-off, so the token still follows it.
        for (Launch &L : inflight)
            if (L.token_pending) {
                (void)write_done_token(streams[L.stream], &done_dev[L.stream * kDoneStride], L.token);
                L.token_pending = false;
            }
        // 3. launch (no lock)
        if (!admitted.empty()) {
            std::vector<conv_status> rc(admitted.size());
            for (size_t i = 0; i < admitted.size(); ++i) rc[i] = enqueue(admitted[i]);
            const uint64_t t_launch = now_ns();
            std::lock_guard<std::mutex> g(mu);
            for (size_t i = 0; i < admitted.size(); ++i)
                if (launched_locked(admitted[i], rc[i], t_launch))
                    inflight.push_back(std::move(admitted[i]));
        }
        // 4. wait: while launches are in flight the thread polls without
        // pausing (a yield costs a system call and delays the next admission
        // and retirement by a few microseconds, measured)
        if (!inflight.empty()) continue;
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
        while (seq.load(std::memory_order_acquire) == s_idle && now_ns() - idle_from < kSpinIdleNs) {
        }
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
        (cfg->queue_only != 0 && cfg->queue_only != 1) || cfg->launch_depth < 0 ||
        cfg->launch_depth > 4)
        return set_error(CONV_EINVAL, "bad server configuration");
    int prev = 0;
    hipGetDevice(&prev);
    int dev = cfg->device < 0 ? prev : cfg->device;
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_error(e, "hipSetDevice");
    auto *s = new conv_server();
    s->cfg = *cfg;
    s->depth = cfg->launch_depth > 1 ? cfg->launch_depth : 1;
    s->device = dev;
    // one 64-byte line per stream's completion word
    const size_t done_bytes = (size_t)cfg->n_streams * kDoneStride * sizeof(uint64_t);
    e = hipHostMalloc((void **)&s->done_host, done_bytes, hipHostMallocDefault);
    if (e == hipSuccess) {
        std::memset(s->done_host, 0, done_bytes);
        e = hipHostGetDevicePointer((void **)&s->done_dev, s->done_host, 0);
    }
    if (e != hipSuccess) {
        if (s->done_host) hipHostFree(s->done_host);
        delete s;
        hipSetDevice(prev);
        return hip_error(e, "allocating the completion words");
    }
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t x : s->streams) hipStreamDestroy(x);
            hipHostFree(s->done_host);
            delete s;
            hipSetDevice(prev);
            return hip_error(e, "hipStreamCreate");
        }
        s->streams.push_back(st);
        s->stream_load.push_back(0);
        s->stream_pending.push_back(0);
        s->stream_bytes.push_back(0);
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
    // the direct launch runs on this thread: its current device must be the
    // server's (descriptors and the CU count follow the current device)
    int cur = -1;
    const bool on_device = hipGetDevice(&cur) == hipSuccess && cur == srv->device;
    Launch direct;
    bool have_direct = false;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        if (srv->stop) {
            if (ready) srv->ready_pool.push_back(ready);
            return set_error(CONV_EINVAL, "server is shutting down");
        }
        Req *r = srv->new_req_locked();
        r->ready = ready;
        r->producer = stream;
        r->in = d_in;
        r->out = d_out;
        r->bytes = L.extent_bytes;
        for (int i = 0; i < 5; ++i) r->k[i] = k[i];
        r->img = *img;
        r->footprint = fp;
        r->t.submit_ns = t_submit;
        r->ticket = srv->next_ticket++;
        srv->put_ticket_locked(r);
        srv->stats.submitted += 1;
        if (L.empty) {
            r->t.admit_ns = r->t.launch_ns = r->t.done_ns = r->t.submit_ns;
            r->state = DONE;
            srv->stats.completed += 1;
        } else {
            // Nothing is queued and submits arrive sparsely enough that this
            // thread can spend a launch (~5 us) without falling behind its
            // arrivals: there is nothing to batch this request with, so admit
            // and launch it here (if a stream is idle and no earlier request
            // holds its buffers) rather than wake the scheduler.  Dense
            // arrivals stay with the scheduler, which batches them.
            const uint64_t gap = std::min<uint64_t>(t_submit - srv->last_submit_ns, kGapClampNs);
            srv->gap_mean_ns = srv->gap_mean_ns - srv->gap_mean_ns / 4 + gap / 4;
            // sparse on average and not inside a burst
            const bool try_direct = !srv->cfg.queue_only && srv->queue.empty() &&
                                    srv->gap_mean_ns >= kDirectGapNs && gap >= kDirectGapNs;
            srv->last_submit_ns = t_submit;
            srv->queue.push_back(r);
            srv->idle = false;
            srv->seq.fetch_add(1, std::memory_order_release);
            if (try_direct && on_device) {
                std::vector<Launch> now = srv->admit_locked(true);
                if (!now.empty()) {
                    direct = std::move(now[0]);
                    have_direct = true;
                }
            }
        }
        *ticket = r->ticket;
    }
    if (have_direct) {
        // with one launch per stream the scheduler writes the launch's token
        const conv_status rc = srv->enqueue(direct, /*write_token=*/srv->depth > 1);
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
    Req *r = srv->find_ticket_locked(ticket);
    if (!r) return set_error(CONV_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (r->state == QUEUED || r->state == INFLIGHT) return CONV_EAGAIN;
    if (t) *t = r->t;
    const int state = r->state;
    srv->free_req_locked(r);
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
    for (hipEvent_t e : srv->ready_pool) hipEventDestroy(e);
    for (hipStream_t s : srv->streams) {
        hipStreamSynchronize(s);
        hipStreamDestroy(s);
    }
    hipHostFree(srv->done_host);
    hipSetDevice(prev);
    delete srv;  // the request pool's blocks go with it
    return CONV_OK;
}

}  // extern "C"
