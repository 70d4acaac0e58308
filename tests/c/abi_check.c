/*
 * abi_check.c -- the C ABI of libconvsep5 used from plain C with HIP device
 * memory (no Python, no torch): fused, direct and two-pass forms, the
 * single pass with copy-back, a two-image batch (eager and as a captured
 * plan), tile configurations and the tuner, the two-pass form with a
 * 16-bit intermediate, the continuous-batching server, width 7 in every
 * form, one pyramid level, and the error path, on a
 * 3 x 97 x 333 image, each compared with the FP64 oracle of Eq. 1 (arXiv
 * 1711.09791, Section 1; zero border, Section 5), which this test links as
 * test infrastructure.
 *
 * Pixels are m/256 (m from a 32-bit LCG) and the taps the binomial
 * [1,4,6,4,1]/16, so every FP32 operation is exact and every form must equal
 * the oracle rounded to FP32 bit for bit; a second pass with unnormalised
 * positive taps checks the 1e-6 relative bound.
 * Prints "abi_check OK" and exits 0 on success; prints the failure and exits 1
 * otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "conv_sep5.h"

/* the oracle (oracle/conv5_oracle.c) */
void oracle_conv5_direct(const double *A, double *B, const double *k, int64_t planes,
                         int64_t rows, int64_t cols, int nthreads);
void oracle_conv5_twopass_q(const double *A, double *B, double *aux, const double *k,
                            int64_t planes, int64_t rows, int64_t cols, int tfmt);
void oracle_conv_direct_n(const double *A, double *B, const double *K, int n, int64_t planes,
                          int64_t rows, int64_t cols, int nthreads);

#define P 3
#define R 97
#define C 333
#define N (P * R * C)

static int fail(const char *what) {
    printf("abi_check FAILED: %s (%s)\n", what, conv_last_error());
    return 1;
}

#define HIPCHECK(x)                                                      \
    do {                                                                 \
        hipError_t e_ = (x);                                             \
        if (e_ != hipSuccess) {                                          \
            printf("abi_check FAILED: %s: %s\n", #x, hipGetErrorString(e_)); \
            return 1;                                                    \
        }                                                                \
    } while (0)

/* max relative error of got vs ref; zero references must be exactly +0 */
static double compare(const float *got, const double *ref, int exact) {
    double worst = 0.0;
    for (int i = 0; i < N; ++i) {
        if (ref[i] == 0.0) {
            if (got[i] != 0.0f || signbit(got[i])) return INFINITY;
            continue;
        }
        if (exact && got[i] != (float)ref[i]) return INFINITY;
        const double e = fabs((double)got[i] - ref[i]) / fabs(ref[i]);
        if (e > worst) worst = e;
    }
    return worst;
}

int main(void) {
    static float host[N], out[N];
    static double a64[N], ref[N];
    uint32_t s = 12345u;
    for (int i = 0; i < N; ++i) {
        s = s * 1664525u + 1013904223u;
        host[i] = (float)(s >> 24) / 256.0f;
        a64[i] = host[i];
    }
    const conv_image img = {P, R, C, CONV_F32, 0, 0};
    const size_t bytes = sizeof(float) * N;
    void *d_in, *d_out, *d_cb;
    HIPCHECK(hipMalloc(&d_in, bytes));
    HIPCHECK(hipMalloc(&d_out, bytes));
    HIPCHECK(hipMalloc(&d_cb, bytes));
    hipStream_t st;
    HIPCHECK(hipStreamCreate(&st));
    HIPCHECK(hipMemcpy(d_in, host, bytes, hipMemcpyHostToDevice));

    const float tap_sets[2][5] = {{1.0f / 16, 4.0f / 16, 6.0f / 16, 4.0f / 16, 1.0f / 16},
                                  {0.3f, 1.7f, 0.9f, 2.25f, 0.05f}};
    for (int t = 0; t < 2; ++t) {
        const float *k = tap_sets[t];
        const double k64[5] = {k[0], k[1], k[2], k[3], k[4]};
        oracle_conv5_direct(a64, ref, k64, P, R, C, 1);
        const int exact = t == 0;
        const char *names[5] = {"fused", "direct25", "2pass", "copy-back", "2pass-noalloc"};
        for (int form = 0; form < 5; ++form) {
            HIPCHECK(hipMemsetAsync(d_out, 0xff, bytes, st)); /* NaN pattern */
            conv_status rc;
            void *dst = d_out;
            if (form == 0) rc = conv_sep5_1pass(d_in, d_out, k, &img, CONV_1PASS_FUSED, st);
            else if (form == 1) rc = conv_sep5_1pass(d_in, d_out, k, &img, CONV_1PASS_DIRECT25, st);
            else if (form == 2) rc = conv_sep5_2pass(d_in, d_out, NULL, k, &img, st);
            else if (form == 4) rc = conv_sep5_2pass_noalloc(d_in, d_out, k, &img, CONV_F32, st);
            else {
                HIPCHECK(hipMemcpyAsync(d_cb, d_in, bytes, hipMemcpyDeviceToDevice, st));
                rc = conv_sep5_1pass(d_cb, d_cb, k, &img, CONV_1PASS_FUSED, st);
                dst = d_cb;
            }
            if (rc != CONV_OK) return fail(names[form]);
            HIPCHECK(hipStreamSynchronize(st));
            HIPCHECK(hipMemcpy(out, dst, bytes, hipMemcpyDeviceToHost));
            /* the direct form rounds K = k k^T once, so it is exact only for dyadic products */
            const double e = compare(out, ref, exact);
            printf("%-9s taps %d: max rel err %.3e\n", names[form], t, e);
            if (!(e <= 1e-6)) return fail(names[form]);
        }
    }

    /* the library's image copy moves every element unchanged */
    {
        HIPCHECK(hipMemsetAsync(d_out, 0xff, bytes, st));
        if (conv_image_copy(d_in, d_out, &img, st) != CONV_OK) return fail("image copy");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(out, d_out, bytes, hipMemcpyDeviceToHost));
        if (memcmp(out, host, bytes) != 0) return fail("image copy differs from its input");
        printf("image copy: OK\n");
    }

    /* the direct form's own tile configuration (kind 2): another band height
       gives the same bits */
    {
        const float *k = tap_sets[1];
        static float want[N];
        conv_tile_cfg d0, c16 = {16, 1, 0, 8, 0};
        if (conv_get_tile_cfg(CONV_F32, 2, &d0) != CONV_OK) return fail("get kind 2");
        if (conv_sep5_1pass(d_in, d_out, k, &img, CONV_1PASS_DIRECT25, st) != CONV_OK)
            return fail("direct25 default tiles");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(want, d_out, bytes, hipMemcpyDeviceToHost));
        if (conv_set_tile_cfg(CONV_F32, 2, &c16) != CONV_OK) return fail("set kind 2");
        HIPCHECK(hipMemsetAsync(d_out, 0xff, bytes, st));
        if (conv_sep5_1pass(d_in, d_out, k, &img, CONV_1PASS_DIRECT25, st) != CONV_OK)
            return fail("direct25 16-row bands");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(out, d_out, bytes, hipMemcpyDeviceToHost));
        if (conv_set_tile_cfg(CONV_F32, 2, &d0) != CONV_OK) return fail("restore kind 2");
        if (memcmp(out, want, bytes) != 0) return fail("direct25 bits depend on the band height");
        printf("direct25 with its own tiles: bitwise equal\n");
    }

    /* two images in one batch launch: the image and its first plane alone */
    {
        const float *k = tap_sets[1];
        const double k64[5] = {k[0], k[1], k[2], k[3], k[4]};
        static float out2[R * C];
        static double ref2[R * C];
        void *d_out2;
        HIPCHECK(hipMalloc(&d_out2, sizeof(float) * R * C));
        const void *ins[2] = {d_in, d_in};
        void *outs[2] = {d_out, d_out2};
        const conv_image imgs[2] = {img, {1, R, C, CONV_F32, 0, 0}};
        float kk[10];
        memcpy(kk, k, sizeof(float) * 5);
        memcpy(kk + 5, k, sizeof(float) * 5);
        if (conv_sep5_batch(2, ins, outs, kk, imgs, CONV_1PASS_FUSED, st) != CONV_OK)
            return fail("batch");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(out, d_out, bytes, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(out2, d_out2, sizeof(float) * R * C, hipMemcpyDeviceToHost));
        oracle_conv5_direct(a64, ref, k64, P, R, C, 1);
        oracle_conv5_direct(a64, ref2, k64, 1, R, C, 1);
        if (!(compare(out, ref, 0) <= 1e-6)) return fail("batch image 0");
        for (int i = 0; i < R * C; ++i)
            if (out2[i] != out[i]) return fail("batch image 1 differs from plane 0 of image 0");
        HIPCHECK(hipFree(d_out2));
        printf("batch: OK\n");
    }

    /* the batch captured as a plan and replayed twice, with eager work in
     * between; a changed tile configuration and the tuner's pick: every
     * result equals the default eager one bit for bit */
    {
        const float *k = tap_sets[1];
        static float want[N], want2[R * C], got2[R * C];
        void *d_o2;
        HIPCHECK(hipMalloc(&d_o2, sizeof(float) * R * C));
        const void *ins[2] = {d_in, d_in};
        void *outs[2] = {d_out, d_o2};
        const conv_image imgs[2] = {img, {1, R, C, CONV_F32, 0, 0}};
        float kk[10];
        memcpy(kk, k, sizeof(float) * 5);
        memcpy(kk + 5, k, sizeof(float) * 5);
        if (conv_sep5_batch(2, ins, outs, kk, imgs, CONV_1PASS_FUSED, st) != CONV_OK)
            return fail("batch (plan reference)");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(want, d_out, bytes, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(want2, d_o2, sizeof(float) * R * C, hipMemcpyDeviceToHost));
        conv_plan *plan = NULL;
        if (conv_batch_plan_create(2, ins, outs, kk, imgs, CONV_1PASS_FUSED, &plan) != CONV_OK)
            return fail("conv_batch_plan_create");
        for (int rep = 0; rep < 2; ++rep) {
            HIPCHECK(hipMemsetAsync(d_out, 0xff, bytes, st));
            HIPCHECK(hipMemsetAsync(d_o2, 0xff, sizeof(float) * R * C, st));
            if (conv_batch_plan_launch(plan, st) != CONV_OK) return fail("conv_batch_plan_launch");
            HIPCHECK(hipStreamSynchronize(st));
            HIPCHECK(hipMemcpy(out, d_out, bytes, hipMemcpyDeviceToHost));
            HIPCHECK(hipMemcpy(got2, d_o2, sizeof(float) * R * C, hipMemcpyDeviceToHost));
            if (memcmp(out, want, bytes) != 0 || memcmp(got2, want2, sizeof(float) * R * C) != 0)
                return fail("plan replay differs from the eager batch");
        }
        if (conv_batch_plan_destroy(plan) != CONV_OK) return fail("conv_batch_plan_destroy");
        HIPCHECK(hipFree(d_o2));

        conv_tile_cfg orig, alt, best;
        if (conv_get_tile_cfg(CONV_F32, 0, &orig) != CONV_OK) return fail("conv_get_tile_cfg");
        if (conv_sep5_1pass(d_in, d_out, k, &img, CONV_1PASS_FUSED, st) != CONV_OK)
            return fail("fused (config reference)");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(want, d_out, bytes, hipMemcpyDeviceToHost));
        alt = orig;
        alt.rows_per_tile = 13;
        alt.waves_per_wg = 2;
        alt.xcd_slabs = 1;
        if (conv_set_tile_cfg(CONV_F32, 0, &alt) != CONV_OK) return fail("conv_set_tile_cfg");
        alt.rows_per_tile = 0;
        if (conv_set_tile_cfg(CONV_F32, 0, &alt) != CONV_EINVAL) return fail("bad tile config accepted");
        float best_ms = 0.0f;
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1) {
                const void *tin[1] = {d_in};
                void *tout[1] = {d_out};
                if (conv_tune(0, 1, tin, tout, k, &img, 2, st, &best, &best_ms) != CONV_OK ||
                    !(best_ms > 0.0f))
                    return fail("conv_tune");
            }
            HIPCHECK(hipMemsetAsync(d_out, 0xff, bytes, st));
            if (conv_sep5_1pass(d_in, d_out, k, &img, CONV_1PASS_FUSED, st) != CONV_OK)
                return fail("fused with another tile config");
            HIPCHECK(hipStreamSynchronize(st));
            HIPCHECK(hipMemcpy(out, d_out, bytes, hipMemcpyDeviceToHost));
            if (memcmp(out, want, bytes) != 0) return fail("tile config changed the result");
        }
        if (conv_set_tile_cfg(CONV_F32, 0, &orig) != CONV_OK) return fail("restoring the tile config");
        printf("plan, tile configs, tuner: OK (tuned: %d rows, %d waves, %.4f ms)\n",
               (int)best.rows_per_tile, (int)best.waves_per_wg, (double)best_ms);
    }

    /* the two-pass form with a 16-bit intermediate: CONV_F32 is the FP32 form
     * bit for bit; with pixels 0..3 and binomial taps every intermediate is
     * exact in FP16 and BF16, so the result equals the oracle's definition
     * (row pass, one rounding per intermediate, column pass) exactly */
    {
        static float out2[N], host3[N];
        static double a3[N], aux[R * C];
        if (conv_sep5_2pass_ex(d_in, d_out, NULL, tap_sets[1], &img, CONV_F32, st) != CONV_OK ||
            conv_sep5_2pass(d_in, d_cb, NULL, tap_sets[1], &img, st) != CONV_OK)
            return fail("2pass_ex F32");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(out, d_out, bytes, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(out2, d_cb, bytes, hipMemcpyDeviceToHost));
        if (memcmp(out, out2, bytes) != 0) return fail("2pass_ex F32 differs from 2pass");
        for (int i = 0; i < N; ++i) {
            s = s * 1664525u + 1013904223u;
            host3[i] = (float)(s >> 30);
            a3[i] = host3[i];
        }
        HIPCHECK(hipMemcpy(d_in, host3, bytes, hipMemcpyHostToDevice));
        const double k64[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
        const int32_t fmts[2] = {CONV_F16, CONV_BF16};
        for (int f = 0; f < 2; ++f) {
            HIPCHECK(hipMemsetAsync(d_out, 0xff, bytes, st));
            if (conv_sep5_2pass_ex(d_in, d_out, NULL, tap_sets[0], &img, fmts[f], st) != CONV_OK)
                return fail("2pass_ex 16-bit");
            HIPCHECK(hipStreamSynchronize(st));
            HIPCHECK(hipMemcpy(out, d_out, bytes, hipMemcpyDeviceToHost));
            oracle_conv5_twopass_q(a3, ref, aux, k64, P, R, C, f + 1);
            if (compare(out, ref, 1) != 0.0) return fail("2pass_ex 16-bit vs its oracle");
        }
        if (conv_sep5_2pass_ex(d_in, d_out, NULL, tap_sets[0], &img, 5, st) != CONV_EINVAL)
            return fail("bad tmp_dtype accepted");
        printf("2pass_ex: OK\n");
    }

    /* the server: 12 requests (the whole image and its first plane, with the
     * inputs written on the caller's stream just before each submit, so that
     * producer_wait orders the launch after the copy), polled to completion;
     * each result equals the lone fused call bit for bit */
    {
        static float want[N], want1[R * C], got1[R * C];
        const float *k = tap_sets[1];
        HIPCHECK(hipMemcpy(d_in, host, bytes, hipMemcpyHostToDevice));
        if (conv_sep5_1pass(d_in, d_out, k, &img, CONV_1PASS_FUSED, st) != CONV_OK)
            return fail("server reference");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(want, d_out, bytes, hipMemcpyDeviceToHost));
        for (int i = 0; i < R * C; ++i) want1[i] = want[i];
        enum { NREQ = 12 };
        void *rin[NREQ], *rout[NREQ];
        uint64_t tickets[NREQ];
        conv_serve_cfg cfg;
        memset(&cfg, 0, sizeof cfg);
        cfg.hbm_budget_bytes = (uint64_t)8 * bytes;
        cfg.max_slots = 8;
        cfg.n_streams = 2;
        cfg.max_batch = 4;
        cfg.device = -1;
        cfg.producer_wait = 1;
        conv_server *srv = NULL;
        if (conv_serve_create(&cfg, &srv) != CONV_OK) return fail("conv_serve_create");
        const conv_image plane0 = {1, R, C, CONV_F32, 0, 0};
        for (int q = 0; q < NREQ; ++q) {
            const size_t nb = q % 2 ? sizeof(float) * R * C : bytes;
            HIPCHECK(hipMalloc(&rin[q], nb));
            HIPCHECK(hipMalloc(&rout[q], nb));
            HIPCHECK(hipMemsetAsync(rout[q], 0xff, nb, st));
            HIPCHECK(hipMemcpyAsync(rin[q], d_in, nb, hipMemcpyDeviceToDevice, st));
            if (conv_serve_submit(srv, rin[q], rout[q], k, q % 2 ? &plane0 : &img, st, &tickets[q]) !=
                CONV_OK)
                return fail("conv_serve_submit");
        }
        int done = 0;
        conv_req_times t;
        for (int spins = 0; done < NREQ && spins < 20000000; ++spins) {
            done = 0;
            for (int q = 0; q < NREQ; ++q) {
                if (!tickets[q]) {
                    ++done;
                    continue;
                }
                const conv_status ps = conv_serve_poll(srv, tickets[q], &t);
                if (ps == CONV_OK) {
                    if (!(t.submit_ns <= t.admit_ns && t.admit_ns <= t.launch_ns &&
                          t.launch_ns <= t.done_ns) || t.batch_size < 1)
                        return fail("request times out of order");
                    tickets[q] = 0;
                    ++done;
                } else if (ps != CONV_EAGAIN) {
                    return fail("conv_serve_poll");
                }
            }
        }
        if (done < NREQ) return fail("server did not finish");
        if (conv_serve_drain(srv) != CONV_OK) return fail("conv_serve_drain");
        conv_serve_stats ss;
        if (conv_serve_get_stats(srv, &ss) != CONV_OK || ss.completed != NREQ || ss.failed != 0)
            return fail("server stats");
        if (conv_serve_poll(srv, 987654321u, &t) != CONV_ENOTFOUND) return fail("unknown ticket");
        if (conv_serve_destroy(srv) != CONV_OK) return fail("conv_serve_destroy");
        for (int q = 0; q < NREQ; ++q) {
            if (q % 2) {
                HIPCHECK(hipMemcpy(got1, rout[q], sizeof(float) * R * C, hipMemcpyDeviceToHost));
                if (memcmp(got1, want1, sizeof(float) * R * C) != 0)
                    return fail("served plane differs from the lone call");
            } else {
                HIPCHECK(hipMemcpy(out, rout[q], bytes, hipMemcpyDeviceToHost));
                if (memcmp(out, want, bytes) != 0) return fail("served image differs from the lone call");
            }
            HIPCHECK(hipFree(rin[q]));
            HIPCHECK(hipFree(rout[q]));
        }
        printf("server: OK (%llu launches, largest %d)\n", (unsigned long long)ss.launches,
               (int)ss.max_batch);
    }

    /* width 7 (the three separable forms and the full-kernel form) and one
     * pyramid level, exact case: pixels m/256 with binomial taps make every
     * FP32 operation exact, so each result equals its oracle bit for bit */
    {
        enum { NW = 7, RO = (R + 1) / 2, CO = (C + 1) / 2 };
        const float k7[NW] = {1 / 64.f, 6 / 64.f, 15 / 64.f, 20 / 64.f, 15 / 64.f, 6 / 64.f, 1 / 64.f};
        float K7[NW * NW];
        double K64[NW * NW];
        for (int a = 0; a < NW; ++a)
            for (int b = 0; b < NW; ++b) {
                K64[a * NW + b] = (double)k7[a] * (double)k7[b];
                K7[a * NW + b] = (float)K64[a * NW + b];
            }
        oracle_conv_direct_n(a64, ref, K64, NW, P, R, C, 1);
        const char *wn[4] = {"sepn fused", "sepn direct", "sepn 2pass", "2d direct"};
        for (int form = 0; form < 4; ++form) {
            HIPCHECK(hipMemsetAsync(d_out, 0xff, bytes, st));
            conv_status rc;
            if (form == 0) rc = conv_sepn_1pass(d_in, d_out, k7, NW, &img, CONV_1PASS_FUSED, st);
            else if (form == 1) rc = conv_sepn_1pass(d_in, d_out, k7, NW, &img, CONV_1PASS_DIRECT25, st);
            else if (form == 2) rc = conv_sepn_2pass(d_in, d_out, NULL, k7, NW, &img, st);
            else rc = conv_2d_direct(d_in, d_out, K7, NW, &img, st);
            if (rc != CONV_OK) return fail(wn[form]);
            HIPCHECK(hipStreamSynchronize(st));
            HIPCHECK(hipMemcpy(out, d_out, bytes, hipMemcpyDeviceToHost));
            if (compare(out, ref, 1) != 0.0) return fail(wn[form]);
        }
        if (conv_sepn_1pass(d_in, d_out, k7, 8, &img, CONV_1PASS_FUSED, st) != CONV_EINVAL)
            return fail("even width accepted");
        printf("width 7: OK\n");

        static float pyr[P * RO * CO];
        const conv_image oimg = {P, RO, CO, CONV_F32, 0, 0};
        void *d_pyr;
        HIPCHECK(hipMalloc(&d_pyr, sizeof pyr));
        HIPCHECK(hipMemsetAsync(d_pyr, 0xff, sizeof pyr, st));
        if (conv_pyr_down(d_in, &img, d_pyr, &oimg, tap_sets[0], st) != CONV_OK)
            return fail("conv_pyr_down");
        HIPCHECK(hipStreamSynchronize(st));
        HIPCHECK(hipMemcpy(pyr, d_pyr, sizeof pyr, hipMemcpyDeviceToHost));
        HIPCHECK(hipFree(d_pyr));
        const double kb[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
        oracle_conv5_direct(a64, ref, kb, P, R, C, 1);
        for (int p = 0; p < P; ++p)
            for (int yo = 0; yo < RO; ++yo)
                for (int xo = 0; xo < CO; ++xo) {
                    const float g = pyr[((size_t)p * RO + yo) * CO + xo];
                    const double r = ref[((size_t)p * R + 2 * yo) * C + 2 * xo];
                    if (g != (float)r || (r == 0.0 && signbit(g))) return fail("pyramid level vs oracle");
                }
        printf("pyramid: OK\n");
    }

    /* errors come back as a status and a message, before any HIP call */
    {
        conv_image bad = img;
        bad.dtype = 7;
        if (conv_sep5_1pass(d_in, d_out, tap_sets[0], &bad, CONV_1PASS_FUSED, st) != CONV_EINVAL ||
            strlen(conv_last_error()) == 0)
            return fail("bad dtype accepted");
        if (conv_sep5_1pass(d_in, (char *)d_in + 4, tap_sets[0], &img, CONV_1PASS_FUSED, st) !=
            CONV_EALIAS)
            return fail("partial overlap accepted");
    }

    HIPCHECK(hipStreamDestroy(st));
    HIPCHECK(hipFree(d_in));
    HIPCHECK(hipFree(d_out));
    HIPCHECK(hipFree(d_cb));
    printf("abi_check OK (%s)\n", conv_version());
    return 0;
}
