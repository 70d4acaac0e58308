// conv_api_n.cpp -- C ABI of the width-n kernels: validation, tap tables and
// dispatch for conv_sepn_1pass, conv_sepn_2pass and conv_2d_direct.
#include <hip/hip_runtime.h>

#include <cstring>

#include "conv_common.h"
#include "conv_internal.h"
#include "conv_sep5.h"

using namespace convsep5;

namespace {

constexpr float kNoTaps[5] = {0.f, 0.f, 0.f, 0.f, 0.f};

conv_status check_width(int32_t n) {
    if (n < 1 || n > kMaxWidthN || n % 2 == 0)
        return set_error(CONV_EINVAL, "width %d is not odd in 1..%d", n, kMaxWidthN);
    return CONV_OK;
}

// Descriptor of one width-n launch: the row-band height and workgroup width
// are fixed per dtype and form; the width-5 taps inside stay unused.
int64_t fill_desc_n(ImgDev *d, const void *in, void *out, float *tmp, const conv_image *img,
                    const Layout &L, bool direct, int radius) {
    conv_tile_cfg cfg{};
    cfg.rows_per_tile = direct ? th_direct_n(img->dtype == CONV_F32, radius) : kThSepN;
    cfg.waves_per_wg = waves_n(img->dtype);
    cfg.xcd_slabs = kXcdChunkRowsN / cfg.rows_per_tile;
    return fill_desc(d, in, out, tmp, img, L, kNoTaps, cfg);
}

void fill_taps_sep(TapsN *t, const float *k, int n) {
    std::memset(t, 0, sizeof *t);
    for (int i = 0; i < n; ++i) t->k[i] = k[i];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) t->K[a * n + b] = (float)((double)k[a] * (double)k[b]);
}

// One launch of the width-n kernel in `mode`, or -- with copy-back -- the
// launch into stream-ordered scratch followed by the copy kernel over d_out.
conv_status run_single(const void *d_in, void *d_out, const TapsN &tp, int n,
                       const conv_image *img, const Layout &L, int kmode, hipStream_t stream) {
    const bool direct = kmode == MODE_DIRECT25;
    const int radius = n / 2;
    ImgDev d;
    if (d_in != (const void *)d_out) {
        const int64_t nblocks = fill_desc_n(&d, d_in, d_out, nullptr, img, L, direct, radius);
        const hipError_t e = launch_image_n(d, tp, img->dtype, radius, kmode, nblocks, stream);
        return e == hipSuccess ? CONV_OK : hip_error(e, "width-n kernel launch");
    }
    void *scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, (size_t)L.extent_bytes, stream);
    if (e != hipSuccess)
        return set_error(CONV_ENOMEM, "hipMallocAsync(%lld): %s", (long long)L.extent_bytes,
                         hipGetErrorString(e));
    int64_t nblocks = fill_desc_n(&d, d_in, scratch, nullptr, img, L, direct, radius);
    d.keep_out = 1;  // cached stores: the copy reads the scratch next
    e = launch_image_n(d, tp, img->dtype, radius, kmode, nblocks, stream);
    if (e == hipSuccess) e = launch_copy(scratch, d_out, img, L,
                                                 get_cfg_for(img->dtype, 0, 2 * (uint64_t)L.extent_bytes),
                                                 stream);
    (void)hipFreeAsync(scratch, stream);
    return e == hipSuccess ? CONV_OK : hip_error(e, "width-n (copy-back) kernel launch");
}

// Checks shared by the single-kernel entry points.
conv_status check_common(const void *d_in, void *d_out, const void *taps, int32_t n,
                         const conv_image *img, Layout *L) {
    conv_status st = check_image(img, L);
    if (st != CONV_OK) return st;
    if ((st = reject_hwc(*L, "the width-n entry points")) != CONV_OK) return st;
    if ((st = check_width(n)) != CONV_OK) return st;
    if (!taps) return set_error(CONV_EINVAL, "taps pointer is NULL");
    if (L->empty) return CONV_OK;
    if (!d_in || !d_out) return set_error(CONV_EINVAL, "NULL device pointer");
    if (d_in != (const void *)d_out && overlaps(d_in, L->extent_bytes, d_out, L->extent_bytes))
        return set_error(CONV_EALIAS, "input and output partially overlap");
    return CONV_OK;
}

}  // namespace

extern "C" {

conv_status conv_sepn_1pass(const void *d_in, void *d_out, const float *k, int32_t n,
                            const conv_image *img, int mode, hipStream_t stream) {
    clear_error();
    Layout L;
    conv_status st = check_common(d_in, d_out, k, n, img, &L);
    if (st != CONV_OK) return st;
    if (mode != CONV_1PASS_FUSED && mode != CONV_1PASS_DIRECT25)
        return set_error(CONV_EINVAL, "mode %d is not FUSED or DIRECT25", mode);
    if (L.empty) return CONV_OK;
    TapsN tp;
    fill_taps_sep(&tp, k, n);
    return run_single(d_in, d_out, tp, n, img, L,
                      mode == CONV_1PASS_FUSED ? MODE_FUSED : MODE_DIRECT25, stream);
}

conv_status conv_2d_direct(const void *d_in, void *d_out, const float *K, int32_t n,
                           const conv_image *img, hipStream_t stream) {
    clear_error();
    Layout L;
    conv_status st = check_common(d_in, d_out, K, n, img, &L);
    if (st != CONV_OK) return st;
    if (L.empty) return CONV_OK;
    TapsN tp;
    std::memset(&tp, 0, sizeof tp);
    std::memcpy(tp.K, K, sizeof(float) * (size_t)(n * n));
    return run_single(d_in, d_out, tp, n, img, L, MODE_DIRECT25, stream);
}

conv_status conv_sepn_2pass(const void *d_in, void *d_out, float *d_tmp, const float *k,
                            int32_t n, const conv_image *img, hipStream_t stream) {
    clear_error();
    Layout L;
    conv_status st = check_common(d_in, d_out, k, n, img, &L);
    if (st != CONV_OK) return st;
    if (L.empty) return CONV_OK;
    const int64_t tmp_bytes = (int64_t)img->planes * img->rows * img->cols * 4;
    if (d_tmp && (overlaps(d_tmp, tmp_bytes, d_in, L.extent_bytes) ||
                  overlaps(d_tmp, tmp_bytes, d_out, L.extent_bytes)))
        return set_error(CONV_EALIAS, "workspace overlaps the input or output");
    float *tmp = d_tmp;
    hipError_t e;
    if (!tmp) {
        e = hipMallocAsync((void **)&tmp, (size_t)tmp_bytes, stream);
        if (e != hipSuccess)
            return set_error(CONV_ENOMEM, "hipMallocAsync(%lld): %s", (long long)tmp_bytes,
                             hipGetErrorString(e));
    }
    TapsN tp;
    fill_taps_sep(&tp, k, n);
    ImgDev d;
    const int64_t nblocks = fill_desc_n(&d, d_in, d_out, tmp, img, L, false, n / 2);
    e = launch_image_n(d, tp, img->dtype, n / 2, MODE_ROWPASS, nblocks, stream);
    if (e == hipSuccess) e = launch_image_n(d, tp, img->dtype, n / 2, MODE_COLPASS, nblocks, stream);
    if (!d_tmp) (void)hipFreeAsync(tmp, stream);
    return e == hipSuccess ? CONV_OK : hip_error(e, "width-n 2pass kernel launch");
}

}  // extern "C"
