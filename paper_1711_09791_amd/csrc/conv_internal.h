// conv_internal.h -- types shared by the kernels and the host side of
// libconvsep5 (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace convsep5 {

enum Mode : int {
    MODE_FUSED = 0,     // row filter -> register window -> column filter
    MODE_DIRECT25 = 1,  // 25 multiply-adds per pixel (paper's single pass)
    MODE_ROWPASS = 2,   // two-pass, first kernel: input -> FP32 intermediate
    MODE_COLPASS = 3,   // two-pass, second kernel: FP32 intermediate -> output
    MODE_COPY = 4,      // copy-back of the single-pass result (in -> out, same layout)
    // two-pass with the intermediate stored in 16 bits (FP16 or BF16, RNE)
    MODE_ROWPASS_F16T = 5,
    MODE_COLPASS_F16T = 6,
    MODE_ROWPASS_BF16T = 7,
    MODE_COLPASS_BF16T = 8
};

// Taps as the kernels read them: k for the separable forms, K = fl32(k_a k_b)
// (rounded once on the host from the FP64 product) for the direct form.
struct Taps {
    float k[5];
    float K[25];
};

// One image as the kernels see it (kernel argument for single launches, one
// row of the device descriptor table for batch launches).  Strides are in
// elements of the storage type.
struct ImgDev {
    const void *in;
    void *out;
    float *tmp;           // two-pass intermediate, dense [plane][row][col] (FP32, or
                          // 16-bit values for the *_F16T / *_BF16T modes)
    int64_t pitch;
    int64_t pstride;
    int32_t planes, rows, cols;
    int32_t aligned;      // 1: 16-byte vector path allowed
    int32_t ns;           // column strips of 64*VEC columns
    int32_t nsg;          // strip groups (waves_per_wg strips each)
    int32_t nb;           // row bands
    int32_t th;           // output rows per band
    int32_t xcd_slabs;    // 1: each XCD takes one contiguous slab of tiles;
                          // c >= 2: XCDs take turns on chunks of c band rows
    int32_t keep_out;     // 1: output stores stay cached (copy-back scratch read next)
    int32_t tq;           // fused/direct with one wave per workgroup, aligned images:
                          // > 1 packs the last (narrow) strip, cut into pieces of
                          // 32 and 16 lanes' width: a 32-lane piece serves 2 bands
                          // per wave, a 16-lane piece 4; the bands go in groups of
                          // tq (4 when there is a 16-lane piece, else 2);
                          // 0 or 1: no packing
    int16_t pk32;         // packed pieces, left to right: 32-lane pieces (0 or 1)
    int16_t pk16;         //   then 16-lane pieces (0 .. 2)
    int64_t tile_begin;   // batch: this image's first tile in the launch
    int64_t tile_end;     // batch: one past its last tile
    Taps tp;
};

// Batches of up to kMaxArgImages images travel as one kernel argument (no
// descriptor copy before the launch); larger ones use a device table.
constexpr int kMaxArgImages = 16;
struct BatchArgs {
    ImgDev d[kMaxArgImages];
    int32_t n;
    int32_t reserved;
    int64_t total;
};

// One pyramid level (blur + 2x decimation): input planes x rows x cols,
// output planes x orows x ocols with orows = ceil(rows/2), ocols = ceil(cols/2);
// each image has its own strides (elements of the storage type).
struct PyrDev {
    const void *in;
    void *out;
    int64_t in_pitch, in_ps, out_pitch, out_ps;
    int32_t planes, rows, cols, orows, ocols;
    int32_t aligned;      // 1: vector loads and stores allowed
    int32_t ns;           // column strips of 64*VEC input columns
    int32_t nb;           // bands of kThPyr output rows
    int32_t xcd_chunk;    // >= 2: XCDs take turns on chunks of this many band rows
    int32_t reserved;
    float k[5];
};
constexpr int kThPyr = 4;

// Taps of the width-n kernels (n = 2R+1 <= 9).
struct TapsN {
    float k[9];    // separable taps k[0..n)
    float K[81];   // n x n kernel, row-major: K[a*n + b] weights A[y+a-R][x+b-R]
};
constexpr int kMaxWidthN = 9;
constexpr int kThSepN = 8;     // rows per band: fused, row and column kernels
constexpr int kThDirectN = 4;  // rows per band: direct n x n
constexpr int kThWalkN = 16;   // rows per band: direct n x n, walking bands
// rows per band of the direct n x n form: walking bands from n = 7 on, and at
// n = 5 for 16-bit storage (where the form is bound by the arithmetic)
constexpr int th_direct_n(bool f32, int radius) {
    return radius >= 3 || (radius == 2 && !f32) ? kThWalkN : kThDirectN;
}
constexpr int waves_n(int) { return 1; }
constexpr int kXcdChunkRowsN = 64;  // rows per XCD chunk of the width-n kernels

// Elements per lane per row: 16 bytes of storage.
inline int vec_of(int dtype) { return dtype == 0 ? 4 : 8; }
inline int esize_of(int dtype) { return dtype == 0 ? 4 : 2; }

// Batch launch flags: the kernel variant must carry the element-wise path
// (some image is not aligned) and the packed last strip (some image has tq > 1).
constexpr int kBatchAnyUnaligned = 1;
constexpr int kBatchAnyPacked = 2;

// Kernel launchers, one translation unit per storage type
// (conv_kernels_{f32,f16,bf16}.hip).  `waves` is 1, 2 or 4; bands of 4 or 8
// rows (im.th / th) select the fully unrolled band kernels.
hipError_t launch_image_f32(const ImgDev &im, int mode, int waves, int64_t nblocks, hipStream_t s);
hipError_t launch_image_f16(const ImgDev &im, int mode, int waves, int64_t nblocks, hipStream_t s);
hipError_t launch_image_bf16(const ImgDev &im, int mode, int waves, int64_t nblocks, hipStream_t s);
hipError_t launch_batch_f32(const ImgDev *d, int n, int64_t total, int mode, int waves, int th,
                            int grid, int flags, hipStream_t s);
hipError_t launch_batch_f16(const ImgDev *d, int n, int64_t total, int mode, int waves, int th,
                            int grid, int flags, hipStream_t s);
hipError_t launch_batch_bf16(const ImgDev *d, int n, int64_t total, int mode, int waves, int th,
                            int grid, int flags, hipStream_t s);
hipError_t launch_batch_args_f32(const BatchArgs &a, int mode, int waves, int th, int grid,
                                 int flags, hipStream_t s);
hipError_t launch_batch_args_f16(const BatchArgs &a, int mode, int waves, int th, int grid,
                                 int flags, hipStream_t s);
hipError_t launch_batch_args_bf16(const BatchArgs &a, int mode, int waves, int th, int grid,
                                 int flags, hipStream_t s);

hipError_t launch_image_n_f32(const ImgDev &im, const TapsN &tp, int radius, int mode,
                             int64_t nblocks, hipStream_t s);
hipError_t launch_image_n_f16(const ImgDev &im, const TapsN &tp, int radius, int mode,
                             int64_t nblocks, hipStream_t s);
hipError_t launch_image_n_bf16(const ImgDev &im, const TapsN &tp, int radius, int mode,
                              int64_t nblocks, hipStream_t s);

inline hipError_t launch_image_n(const ImgDev &im, const TapsN &tp, int dtype, int radius, int mode,
                                 int64_t nblocks, hipStream_t s) {
    return dtype == 0 ? launch_image_n_f32(im, tp, radius, mode, nblocks, s)
         : dtype == 1 ? launch_image_n_f16(im, tp, radius, mode, nblocks, s)
                      : launch_image_n_bf16(im, tp, radius, mode, nblocks, s);
}

hipError_t launch_pyr(const PyrDev &pd, int dtype, int64_t nblocks, hipStream_t s);

// Pixel-interleaved (HWC) images: planes = channels per pixel (2..4), pitch in
// elements between rows, cols in pixels; tiles are (band of kThHwc rows,
// strip of 64*8 flat elements), ns strips.
constexpr int kThHwc = 8;
constexpr int kMaxHwcChannels = 4;
// Flat elements a strip produces: the wave's lanes minus the halo lanes
// (ceil(2P / vec) at each end, which only load).
constexpr int hwc_out_per_strip(int vec, int channels) {
    return (64 - 2 * ((2 * channels + vec - 1) / vec)) * vec;
}
hipError_t launch_hwc(const ImgDev &im, int dtype, int mode, int64_t nblocks, hipStream_t s);

inline hipError_t launch_image(const ImgDev &im, int dtype, int mode, int waves, int64_t nblocks,
                               hipStream_t s) {
    return dtype == 0 ? launch_image_f32(im, mode, waves, nblocks, s)
         : dtype == 1 ? launch_image_f16(im, mode, waves, nblocks, s)
                      : launch_image_bf16(im, mode, waves, nblocks, s);
}

inline hipError_t launch_batch(const ImgDev *d, int n, int64_t total, int dtype, int mode,
                               int waves, int th, int grid, int flags, hipStream_t s) {
    return dtype == 0 ? launch_batch_f32(d, n, total, mode, waves, th, grid, flags, s)
         : dtype == 1 ? launch_batch_f16(d, n, total, mode, waves, th, grid, flags, s)
                      : launch_batch_bf16(d, n, total, mode, waves, th, grid, flags, s);
}

inline hipError_t launch_batch_args(const BatchArgs &a, int dtype, int mode, int waves, int th,
                                    int grid, int flags, hipStream_t s) {
    return dtype == 0 ? launch_batch_args_f32(a, mode, waves, th, grid, flags, s)
         : dtype == 1 ? launch_batch_args_f16(a, mode, waves, th, grid, flags, s)
                      : launch_batch_args_bf16(a, mode, waves, th, grid, flags, s);
}

}  // namespace convsep5
