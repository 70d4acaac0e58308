// conv_kernels_n_f16.hip -- instantiates the width-n kernels for F16 storage.
#include "conv_kernels_n.h"

namespace convsep5 {

hipError_t launch_image_n_f16(const ImgDev &im, const TapsN &tp, int radius, int mode,
                            int64_t nblocks, hipStream_t s) {
    return launch_image_n_t<F16>(im, tp, radius, mode, nblocks, s);
}

}  // namespace convsep5
