// conv_loadgen.cpp -- open-loop request generator used to measure serving
// latency (see conv_loadgen.h).  Built into libconvsep5_loadgen.so, which
// calls libconvsep5 only through its public C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <vector>

#include "conv_loadgen.h"

namespace {

using Clock = std::chrono::steady_clock;

uint64_t ns_of(Clock::time_point t) {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(t.time_since_epoch())
        .count();
}

// Busy-waits until t0 + offset_s; returns how late it is (s, >= 0).
double wait_until(Clock::time_point t0, double offset_s) {
    const auto target = t0 + std::chrono::duration_cast<Clock::duration>(
                                 std::chrono::duration<double>(offset_s));
    Clock::time_point now;
    while ((now = Clock::now()) < target) {
    }
    return std::chrono::duration<double>(now - target).count();
}

bool args_ok(int32_t n, const double *arr, const void *const *in, void *const *out,
             const float *k, const conv_image *imgs) {
    if (n < 0) return false;
    if (n == 0) return true;
    return arr && in && out && k && imgs;
}

// A kernel with no work: what a launch costs by itself.
__global__ void k_empty() {}

conv_status one_call(int32_t form, const void *in, void *out, float *tmp, const float *k,
                     const conv_image *img, hipStream_t s) {
    switch (form) {
        case 0:
            hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s);
            return hipGetLastError() == hipSuccess ? CONV_OK : CONV_EHIP;
        case 1: return conv_sep5_1pass(in, out, k, img, CONV_1PASS_FUSED, s);
        case 2: return conv_sep5_1pass(in, out, k, img, CONV_1PASS_DIRECT25, s);
        default: return conv_sep5_2pass(in, out, tmp, k, img, s);
    }
}

}  // namespace

extern "C" {

conv_status conv_loadgen_serve(conv_server *srv, int32_t n, const double *arrival_s,
                               const void *const *d_in, void *const *d_out, const float *k,
                               const conv_image *imgs, hipStream_t stream, uint64_t *tickets,
                               double *lag_s) {
    if (!srv || !tickets || !args_ok(n, arrival_s, d_in, d_out, k, imgs)) return CONV_EINVAL;
    const auto t0 = Clock::now() + std::chrono::milliseconds(1);
    for (int32_t i = 0; i < n; ++i) {
        const double lag = wait_until(t0, arrival_s[i]);
        if (lag_s) lag_s[i] = lag;
        const conv_status st =
            conv_serve_submit(srv, d_in[i], d_out[i], k + 5 * i, &imgs[i], stream, &tickets[i]);
        if (st != CONV_OK) return st;
    }
    return CONV_OK;
}

conv_status conv_loadgen_direct(int32_t n, const double *arrival_s, const void *const *d_in,
                                void *const *d_out, const float *k, const conv_image *imgs,
                                int32_t n_streams, uint64_t *submit_ns, uint64_t *done_ns,
                                double *lag_s) {
    if (!submit_ns || !done_ns || n_streams < 1 || n_streams > 16 ||
        !args_ok(n, arrival_s, d_in, d_out, k, imgs))
        return CONV_EINVAL;
    std::vector<hipStream_t> streams(n_streams, nullptr);
    std::vector<hipEvent_t> events(n, nullptr);
    conv_status rc = CONV_OK;
    for (auto &s : streams)
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) rc = CONV_EHIP;
    for (auto &e : events)
        if (rc == CONV_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            rc = CONV_EHIP;
    // the watcher stamps completions of the requests enqueued so far
    std::atomic<int32_t> enqueued{0};
    std::atomic<bool> abort{false};
    std::thread watcher([&] {
        std::vector<int32_t> pending;
        int32_t seen = 0, completed = 0;
        while (completed < n && !abort.load()) {
            const int32_t e = enqueued.load(std::memory_order_acquire);
            for (; seen < e; ++seen) pending.push_back(seen);
            for (size_t j = 0; j < pending.size();) {
                const hipError_t q = hipEventQuery(events[pending[j]]);
                if (q == hipErrorNotReady) {
                    ++j;
                    continue;
                }
                done_ns[pending[j]] = ns_of(Clock::now());
                ++completed;
                pending[j] = pending.back();
                pending.pop_back();
            }
            if (pending.empty()) std::this_thread::yield();
        }
    });
    const auto t0 = Clock::now() + std::chrono::milliseconds(1);
    for (int32_t i = 0; i < n && rc == CONV_OK; ++i) {
        const double lag = wait_until(t0, arrival_s[i]);
        if (lag_s) lag_s[i] = lag;
        hipStream_t s = streams[i % n_streams];
        submit_ns[i] = ns_of(Clock::now());
        rc = conv_sep5_1pass(d_in[i], d_out[i], k + 5 * i, &imgs[i], CONV_1PASS_FUSED, s);
        if (rc == CONV_OK && hipEventRecord(events[i], s) != hipSuccess) rc = CONV_EHIP;
        if (rc == CONV_OK) enqueued.store(i + 1, std::memory_order_release);
    }
    if (rc != CONV_OK) abort.store(true);
    watcher.join();
    for (auto s : streams)
        if (s) hipStreamSynchronize(s);
    for (auto e : events)
        if (e) hipEventDestroy(e);
    for (auto s : streams)
        if (s) hipStreamDestroy(s);
    return rc;
}

conv_status conv_loadgen_call_latency(int32_t form, int32_t n, const void *d_in, void *d_out,
                                      float *d_tmp, const float *k, const conv_image *img,
                                      hipStream_t stream, double *gpu_us, double *host_us) {
    if (form < 0 || form > 3 || n < 1 || n > 100000 || !gpu_us || !host_us) return CONV_EINVAL;
    if (form != 0 && (!d_in || !d_out || !k || !img)) return CONV_EINVAL;
    conv_status rc = one_call(form, d_in, d_out, d_tmp, k, img, stream);
    if (rc != CONV_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = CONV_EHIP;
    if (rc == CONV_OK && hipStreamSynchronize(stream) != hipSuccess) rc = CONV_EHIP;
    if (rc == CONV_OK && hipEventRecord(e0, stream) != hipSuccess) rc = CONV_EHIP;
    for (int32_t i = 0; i < n && rc == CONV_OK; ++i)
        rc = one_call(form, d_in, d_out, d_tmp, k, img, stream);
    if (rc == CONV_OK && hipEventRecord(e1, stream) != hipSuccess) rc = CONV_EHIP;
    if (rc == CONV_OK && hipEventSynchronize(e1) != hipSuccess) rc = CONV_EHIP;
    float ms = 0.f;
    if (rc == CONV_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = CONV_EHIP;
    if (rc == CONV_OK) *gpu_us = 1e3 * ms / n;
    std::vector<double> lat;
    lat.reserve(n);
    for (int32_t i = 0; i < n && rc == CONV_OK; ++i) {
        const auto t = Clock::now();
        rc = one_call(form, d_in, d_out, d_tmp, k, img, stream);
        if (rc == CONV_OK && hipStreamSynchronize(stream) != hipSuccess) rc = CONV_EHIP;
        lat.push_back(std::chrono::duration<double, std::micro>(Clock::now() - t).count());
    }
    if (rc == CONV_OK) {
        std::nth_element(lat.begin(), lat.begin() + n / 2, lat.end());
        *host_us = lat[n / 2];
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
