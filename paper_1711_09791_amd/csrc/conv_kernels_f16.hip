// conv_kernels_f16.hip -- instantiates the convolution kernels for F16 storage.
#include "conv_kernels_n.h"

namespace convsep5 {

hipError_t launch_image_f16(const ImgDev &im, int mode, int waves, int64_t nblocks,
                          hipStream_t s) {
    // the direct 25-tap form on its 16-row walking geometry runs the width-n
    // walking band at n = 5 (bitwise the same results, faster)
    if (mode == MODE_DIRECT25 && waves == 1 && im.th == kThWalkN)
        return launch_direct25_walk<F16>(im, nblocks, s);
    return launch_image_t<F16>(im, mode, waves, nblocks, s);
}

hipError_t launch_batch_f16(const ImgDev *d_descs, int n, int64_t total_tiles, int mode,
                          int waves, int th, int grid, int flags, hipStream_t s) {
    return launch_batch_t<F16>(d_descs, n, total_tiles, mode, waves, th, grid, flags, s);
}

hipError_t launch_batch_args_f16(const BatchArgs &a, int mode, int waves, int th, int grid,
                              int flags, hipStream_t s) {
    return launch_batch_args_t<F16>(a, mode, waves, th, grid, flags, s);
}

}  // namespace convsep5
