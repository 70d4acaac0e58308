// conv_kernels_n_bf16.hip -- instantiates the width-n kernels for BF16 storage.
#include "conv_kernels_n.h"

namespace convsep5 {

hipError_t launch_image_n_bf16(const ImgDev &im, const TapsN &tp, int radius, int mode,
                            int64_t nblocks, hipStream_t s) {
    return launch_image_n_t<BF16>(im, tp, radius, mode, nblocks, s);
}

}  // namespace convsep5
