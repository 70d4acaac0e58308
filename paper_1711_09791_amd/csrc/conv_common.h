// conv_common.h -- host-side helpers shared by the C ABI translation units.
#pragma once

#include <stdint.h>

#include <vector>

#include "conv_internal.h"
#include "conv_sep5.h"

namespace convsep5 {

// Limits that keep every 32-bit buffer offset and row index in range.
constexpr int kMaxRows = 1 << 30;
constexpr int64_t kMaxRowBytes = (int64_t)1 << 30;
constexpr int kDescSlots = 32;                 // batch descriptor ring depth
constexpr size_t kDescSlotMinBytes = 256 * sizeof(ImgDev);

struct Layout {
    int64_t pitch = 0, ps = 0;   // elements
    int64_t extent_bytes = 0;    // bytes from the base to one past the last element
    int esz = 4, vec = 4;
    bool empty = true;
    bool hwc = false;            // planes interleaved per pixel (plane_stride == 1)
};

// Tile configuration kinds: 0 the single-image kernels (fused single pass,
// two-pass, copy), 1 the batch kernel, 2 the single-image direct 25-tap
// kernel (VALU-bound where the others are memory-bound, so it takes its own
// tiles).
constexpr int kKinds = 3;
constexpr int kKindImage = 0, kKindBatch = 1, kKindDirect = 2;

conv_status set_error(conv_status st, const char *fmt, ...);
void clear_error();
conv_status hip_error(hipError_t e, const char *what);
conv_status check_image(const conv_image *img, Layout *L);
bool overlaps(const void *a, int64_t na, const void *b, int64_t nb);
conv_tile_cfg get_cfg(int dtype, int kind);  // the default for (dtype, kind)
bool cfg_ok(const conv_tile_cfg *c, int kind);

// Tuned configurations, per storage type, kind and size class of the
// workload's input + output bytes: <= 64 MiB, <= 256 MiB (the GPU's last-level
// cache), <= 1 GiB, larger.
constexpr int kSizeClasses = 4;
struct TunedEntry {
    int valid = 0;
    conv_tile_cfg cfg{};
    float ms = 0.0f;  // the tuner's median time per launch
};
int size_class(uint64_t footprint_bytes);
// The configuration a workload of this footprint runs with: tuned for its
// class if any, else the default.
conv_tile_cfg get_cfg_for(int dtype, int kind, uint64_t footprint_bytes);
TunedEntry get_tuned(int dtype, int kind, int cls);
void put_tuned(int dtype, int kind, int cls, const TunedEntry &e);
void put_default_cfg(int dtype, int kind, const conv_tile_cfg &c);
// Loads the file named by CONV_TUNE_CACHE, once per process (conv_tune.cpp).
void load_tune_cache_once();
uint64_t batch_footprint(int32_t n, const conv_image *imgs);
conv_tile_cfg batch_cfg(int32_t n, const conv_image *imgs);
void fill_taps(Taps *t, const float *k);
bool packs_last_strip(int mode, int dtype);
int batch_flags(const std::vector<ImgDev> &descs);  // kBatchAny*
// pack: the launch's kernel takes packed last strips (packs_last_strip)
int64_t fill_desc(ImgDev *d, const void *in, void *out, float *tmp, const conv_image *img,
                  const Layout &L, const float *k, const conv_tile_cfg &cfg, bool pack = false);
int device_cus();
conv_status build_batch(int32_t n, const void *const *d_in, void *const *d_out, const float *k,
                        const conv_image *imgs, int mode, const conv_tile_cfg &cfg,
                        std::vector<ImgDev> *descs, int64_t *total, int *dtype_out);
int64_t fill_desc_hwc(ImgDev *d, const void *in, void *out, float *tmp, const conv_image *img,
                      const Layout &L, const float *k);
conv_status reject_hwc(const Layout &L, const char *what);
int batch_grid(int64_t total, int cus, const conv_tile_cfg &cfg);
hipError_t launch_copy(const void *d_in, void *d_out, const conv_image *img, const Layout &L,
                       const conv_tile_cfg &cfg, hipStream_t stream);
conv_status enqueue_batch(const std::vector<ImgDev> &descs, int64_t total, int dtype, int mode,
                          const conv_tile_cfg &cfg, hipStream_t s);

}  // namespace convsep5
