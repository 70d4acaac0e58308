// conv_api_pyr.cpp -- C ABI of the pyramid level (blur + 2x decimation):
// validation of the two image descriptors, tile geometry and dispatch.
#include <hip/hip_runtime.h>

#include <cstring>

#include "conv_common.h"
#include "conv_internal.h"
#include "conv_sep5.h"

using namespace convsep5;

namespace {

constexpr int kPyrChunkRows = 32;  // output rows per XCD chunk

}  // namespace

extern "C" {

conv_status conv_pyr_down(const void *d_in, const conv_image *in_img, void *d_out,
                          const conv_image *out_img, const float k[5], hipStream_t stream) {
    clear_error();
    Layout Li, Lo;
    conv_status st = check_image(in_img, &Li);
    if (st != CONV_OK) return st;
    if ((st = check_image(out_img, &Lo)) != CONV_OK) return st;
    if ((st = reject_hwc(Li, "conv_pyr_down")) != CONV_OK) return st;
    if ((st = reject_hwc(Lo, "conv_pyr_down")) != CONV_OK) return st;
    if (!k) return set_error(CONV_EINVAL, "taps pointer is NULL");
    if (in_img->dtype != out_img->dtype || in_img->planes != out_img->planes)
        return set_error(CONV_EINVAL, "input and output differ in dtype or planes");
    const int orows = (in_img->rows + 1) / 2, ocols = (in_img->cols + 1) / 2;
    if (out_img->rows != orows || out_img->cols != ocols)
        return set_error(CONV_EINVAL, "output is %d x %d, needs ceil(rows/2) x ceil(cols/2) = %d x %d",
                         out_img->rows, out_img->cols, orows, ocols);
    if (Li.empty) return CONV_OK;
    if (!d_in || !d_out) return set_error(CONV_EINVAL, "NULL device pointer");
    if (overlaps(d_in, Li.extent_bytes, d_out, Lo.extent_bytes))
        return set_error(CONV_EALIAS, "input and output overlap");
    PyrDev pd;
    std::memset(&pd, 0, sizeof pd);
    pd.in = d_in;
    pd.out = d_out;
    pd.in_pitch = Li.pitch;
    pd.in_ps = Li.ps;
    pd.out_pitch = Lo.pitch;
    pd.out_ps = Lo.ps;
    pd.planes = in_img->planes;
    pd.rows = in_img->rows;
    pd.cols = in_img->cols;
    pd.orows = orows;
    pd.ocols = ocols;
    const int v = Li.vec, hv = v / 2;
    pd.aligned = ((uintptr_t)d_in % 16 == 0) && ((uintptr_t)d_out % 8 == 0) &&
                 in_img->cols % v == 0 && Li.pitch % v == 0 && Li.ps % v == 0 &&
                 Lo.pitch % hv == 0 && Lo.ps % hv == 0;
    pd.ns = (in_img->cols + 64 * v - 1) / (64 * v);
    pd.nb = (orows + kThPyr - 1) / kThPyr;
    pd.xcd_chunk = kPyrChunkRows / kThPyr;
    for (int i = 0; i < 5; ++i) pd.k[i] = k[i];
    const int64_t nblocks = (int64_t)pd.planes * pd.nb * pd.ns;
    const hipError_t e = launch_pyr(pd, in_img->dtype, nblocks, stream);
    return e == hipSuccess ? CONV_OK : hip_error(e, "pyramid kernel launch");
}

}  // extern "C"
