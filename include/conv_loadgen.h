/*
 * conv_loadgen.h -- open-loop load generator for measuring the serving path of
 * libconvsep5 (libconvsep5_loadgen.so).  Not needed to use the library; it
 * exists so that request arrival times are kept by native code with a busy
 * wait on the steady clock, not by an interpreter.
 *
 * Both entry points submit request i at t0 + arrival_s[i] (t0 = the call time
 * plus 1 ms), in index order, from the calling thread, and return when every
 * request has been submitted (conv_loadgen_serve) or has completed
 * (conv_loadgen_direct).  Timestamps are CLOCK_MONOTONIC nanoseconds, the
 * clock of conv_req_times.  Arguments per request follow conv_sep5_1pass:
 * d_in[i], d_out[i] device images described by imgs[i], taps k[5i .. 5i+4].
 * lag_s[i] (optional) receives how late submission i was against its
 * schedule.  Errors: a conv_status (CONV_EINVAL for bad arguments; the first
 * failing submission's status otherwise).
 */
#ifndef CONV_LOADGEN_H
#define CONV_LOADGEN_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "conv_sep5.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Submits every request to `srv` (conv_serve_submit with producer `stream`);
 * tickets[i] receives request i's ticket.  Completion is then read with
 * conv_serve_drain / conv_serve_poll. */
conv_status conv_loadgen_serve(conv_server *srv, int32_t n, const double *arrival_s,
                               const void *const *d_in, void *const *d_out,
                               const float *k, const conv_image *imgs,
                               hipStream_t stream, uint64_t *tickets,
                               double *lag_s);

/* The per-image-launch baseline without a server: request i is one
 * conv_sep5_1pass (fused) launch on stream i % n_streams of n_streams
 * library-created streams, then an event; a watcher thread polls the events
 * and stamps done_ns[i] when request i's event completes.  submit_ns[i] is
 * taken right before the launch.  Returns after every request completed. */
conv_status conv_loadgen_direct(int32_t n, const double *arrival_s,
                                const void *const *d_in, void *const *d_out,
                                const float *k, const conv_image *imgs,
                                int32_t n_streams, uint64_t *submit_ns,
                                uint64_t *done_ns, double *lag_s);

/* Launch-overhead probe, the GPU counterpart of the paper's empty tasks and
 * empty OpenCL kernels (Section 6, Table 2): what one call costs apart from
 * the pixels.  form 0 launches a kernel that does nothing (one wavefront);
 * form 1 / 2 call conv_sep5_1pass (fused / direct 25-tap) and form 3
 * conv_sep5_2pass on the image d_in -> d_out described by img, with taps
 * k[0..4] and workspace d_tmp; form 0 reads none of them.  After one warm-up
 * call the probe makes n calls back to back on `stream` between two timing
 * events (gpu_us receives the elapsed time / n: the GPU's time per call with
 * the launches queued ahead), then n calls one at a time, each followed by
 * hipStreamSynchronize, timed on the host's steady clock (host_us receives
 * the median: submit-to-completion latency of a lone call).  Synchronises
 * `stream`.  n must be 1..100000; errors as conv_sep5_1pass / 2pass, or
 * CONV_EHIP for the empty kernel's launch. */
conv_status conv_loadgen_call_latency(int32_t form, int32_t n, const void *d_in, void *d_out,
                                      float *d_tmp, const float *k, const conv_image *img,
                                      hipStream_t stream, double *gpu_us, double *host_us);

#ifdef __cplusplus
}
#endif

#endif /* CONV_LOADGEN_H */
