// conv_kernels_n_f32.hip -- instantiates the width-n kernels for F32 storage.
#include "conv_kernels_n.h"

namespace convsep5 {

hipError_t launch_image_n_f32(const ImgDev &im, const TapsN &tp, int radius, int mode,
                            int64_t nblocks, hipStream_t s) {
    return launch_image_n_t<F32>(im, tp, radius, mode, nblocks, s);
}

}  // namespace convsep5
