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

#ifdef __cplusplus
}
#endif

#endif /* CONV_LOADGEN_H */
