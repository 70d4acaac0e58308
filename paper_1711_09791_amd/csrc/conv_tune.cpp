// conv_tune.cpp -- the tile-shape autotuner.  It times every candidate
// configuration on the caller's workload with HIP events and installs the
// fastest.  All candidates compute bitwise identical results; only the
// decomposition into tiles (rows per band, wavefronts per workgroup, the
// persistent grid size, the XCD order and the packing of narrow last strips)
// changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "conv_common.h"

using namespace convsep5;

namespace {

// Configurations whose kernels can pack a narrow last strip are tried with
// packing on and off; for the others the setting has no effect.
void add(std::vector<conv_tile_cfg> &c, int th, int w, int p, int x) {
    if (w == 1 && (th == 4 || th == 8)) {
        c.push_back({th, w, p, x, -1});
        c.push_back({th, w, p, x, 1});
    } else {
        c.push_back({th, w, p, x, 0});
    }
}

std::vector<conv_tile_cfg> candidates(int kind) {
    std::vector<conv_tile_cfg> c;
    const int ths[] = {4, 8, 16, 32, 64};
    const int waves[] = {1, 2, 4};
    if (kind == 0) {
        const int xcd[] = {0, 1, 4, 8, 16};
        for (int x : xcd)
            for (int th : ths)
                for (int w : waves) add(c, th, w, 0, x);
        return c;
    }
    const int persist[] = {0, 4, 8, 16};
    const int xcd[] = {0, 1, 8};
    for (int x : xcd)
        for (int th : ths)
            for (int w : waves)
                for (int p : persist) add(c, th, w, p, x);
    return c;
}

}  // namespace

extern "C" conv_status conv_tune(int32_t kind, int32_t n, const void *const *d_in,
                                 void *const *d_out, const float *k, const conv_image *imgs,
                                 int32_t reps, hipStream_t stream, conv_tile_cfg *best,
                                 float *best_ms) {
    clear_error();
    if (kind != 0 && kind != 1) return set_error(CONV_EINVAL, "kind %d is not 0 or 1", kind);
    if (n < 1 || !d_in || !d_out || !k || !imgs || !best || reps < 1 || reps > 10000)
        return set_error(CONV_EINVAL, "bad tuner arguments");
    const int dtype = imgs[0].dtype;
    if (dtype < 0 || dtype > 2) return set_error(CONV_EINVAL, "bad dtype %d", dtype);
    conv_tile_cfg orig;
    conv_get_tile_cfg(dtype, kind, &orig);

    std::vector<hipEvent_t> ev(2 * reps);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) return set_error(CONV_EHIP, "hipEventCreate failed");
    auto run_once = [&]() -> conv_status {
        if (kind == 0) return conv_sep5_1pass(d_in[0], d_out[0], k, &imgs[0], CONV_1PASS_FUSED, stream);
        return conv_sep5_batch(n, d_in, d_out, k, imgs, CONV_1PASS_FUSED, stream);
    };
    conv_status rc = CONV_OK;
    float best_t = 1e30f;
    conv_tile_cfg best_c = orig;
    std::vector<float> t(reps);
    for (const conv_tile_cfg &c : candidates(kind)) {
        conv_set_tile_cfg(dtype, kind, &c);
        rc = run_once();
        if (rc != CONV_OK) break;
        for (int r = 0; r < reps && rc == CONV_OK; ++r) {
            hipEventRecord(ev[2 * r], stream);
            rc = run_once();
            hipEventRecord(ev[2 * r + 1], stream);
        }
        if (rc != CONV_OK) break;
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            rc = hip_error(e, "hipStreamSynchronize (tuner)");
            break;
        }
        for (int r = 0; r < reps; ++r) hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]);
        std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
        const float med = t[reps / 2];
        if (med < best_t) {
            best_t = med;
            best_c = c;
        }
    }
    for (auto &e : ev) hipEventDestroy(e);
    if (rc != CONV_OK) {
        conv_set_tile_cfg(dtype, kind, &orig);
        return rc;
    }
    conv_set_tile_cfg(dtype, kind, &best_c);
    conv_get_tile_cfg(dtype, kind, best);
    if (best_ms) *best_ms = best_t;
    return CONV_OK;
}
