// conv_api.cpp -- C ABI of libconvsep5: argument validation, tile geometry,
// dispatch, the batch descriptor ring, captured batch plans and the tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "conv_internal.h"
#include "conv_sep5.h"
#include "conv_common.h"

using namespace convsep5;

namespace convsep5 {

static thread_local std::string g_err;

conv_status set_error(conv_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err.clear(); }

conv_status hip_error(hipError_t e, const char *what) {
    return set_error(CONV_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---- validation ----------------------------------------------------------------
conv_status check_image(const conv_image *img, Layout *L) {
    if (!img) return set_error(CONV_EINVAL, "image descriptor is NULL");
    if (img->dtype < CONV_F32 || img->dtype > CONV_BF16)
        return set_error(CONV_EINVAL, "dtype %d is not CONV_F32/F16/BF16", img->dtype);
    if (img->planes < 0 || img->rows < 0 || img->cols < 0)
        return set_error(CONV_EINVAL, "negative shape %d x %d x %d", img->planes, img->rows,
                         img->cols);
    L->esz = esize_of(img->dtype);
    L->vec = vec_of(img->dtype);
    if (img->rows > kMaxRows)
        return set_error(CONV_EINVAL, "rows %d exceed the limit %d", img->rows, kMaxRows);
    if ((int64_t)img->cols * 4 > kMaxRowBytes)
        return set_error(CONV_EINVAL, "cols %d exceed the limit %lld", img->cols,
                         (long long)(kMaxRowBytes / 4));
    const int64_t rows = img->rows, cols = img->cols, planes = img->planes;
    if (planes > 1 && img->plane_stride == 1) {
        // planes interleaved per pixel (packed HWC): element (p, y, x) at
        // y*pitch + x*planes + p
        if (planes > kMaxHwcChannels)
            return set_error(CONV_EINVAL, "pixel-interleaved images have 2..%d planes, not %d",
                             kMaxHwcChannels, img->planes);
        if (cols * planes * 4 > kMaxRowBytes)
            return set_error(CONV_EINVAL, "cols %d x planes %d exceed the row limit", img->cols,
                             img->planes);
        L->hwc = true;
        L->pitch = img->pitch == 0 ? cols * planes : img->pitch;
        if (L->pitch < cols * planes)
            return set_error(CONV_EINVAL, "pitch %lld < cols * planes = %lld", (long long)img->pitch,
                             (long long)(cols * planes));
        if (L->pitch > ((int64_t)1 << 40))
            return set_error(CONV_EINVAL, "pitch %lld too large", (long long)L->pitch);
        L->ps = 1;
        L->empty = rows == 0 || cols == 0;
        if (L->empty) {
            L->extent_bytes = 0;
            return CONV_OK;
        }
        L->extent_bytes = ((rows - 1) * L->pitch + cols * planes) * L->esz;
        return CONV_OK;
    }
    L->pitch = img->pitch == 0 ? img->cols : img->pitch;
    if (L->pitch < img->cols)
        return set_error(CONV_EINVAL, "pitch %lld < cols %d", (long long)img->pitch, img->cols);
    if (L->pitch > ((int64_t)1 << 40))
        return set_error(CONV_EINVAL, "pitch %lld too large", (long long)L->pitch);
    const int64_t min_ps = rows > 0 ? (rows - 1) * L->pitch + cols : 0;
    L->ps = img->plane_stride == 0 ? rows * L->pitch : img->plane_stride;
    // Planes must not overlap: either one after another (planar), or side by
    // side within each row (row-interleaved, the 3R x C layout).
    const bool planar = L->ps >= min_ps;
    const bool interleaved = L->ps >= cols && (planes - 1) * L->ps + cols <= L->pitch;
    if (img->plane_stride != 0 && planes > 1 && !planar && !interleaved)
        return set_error(CONV_EINVAL,
                         "plane_stride %lld makes planes overlap (needs >= %lld, or planes "
                         "side by side within a row of pitch %lld)",
                         (long long)img->plane_stride, (long long)min_ps, (long long)L->pitch);
    if (L->ps > ((int64_t)1 << 50))
        return set_error(CONV_EINVAL, "plane_stride %lld too large", (long long)L->ps);
    L->empty = planes == 0 || rows == 0 || cols == 0;
    if (L->empty) {
        L->extent_bytes = 0;
        return CONV_OK;
    }
    const __int128 ext = (__int128)(planes - 1) * L->ps + (__int128)(rows - 1) * L->pitch + cols;
    if (ext * L->esz > ((__int128)1 << 60))
        return set_error(CONV_EINVAL, "image spans too many bytes");
    L->extent_bytes = (int64_t)ext * L->esz;
    return CONV_OK;
}

bool overlaps(const void *a, int64_t na, const void *b, int64_t nb) {
    const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
    if (na <= 0 || nb <= 0) return false;
    return pa < pb + (uintptr_t)nb && pb < pa + (uintptr_t)na;
}

// ---- tile configuration ---------------------------------------------------------
static std::mutex g_cfg_mu;
// Defaults from tile sweeps on MI355X (3 x 4096 x 4096 single image; the
// 64-image uneven batch): 8-row bands, one wave per workgroup, XCDs taking
// turns on chunks of 8 band rows (batch: of 64 tiles), and for batches one
// workgroup per tile.  The 16-bit direct 25-tap kernel, bound by its vector
// ALU work, runs 16-row bands (a walking band): 50.0 / 48.2 us against
// 52.1 / 53.1 us with 8-row bands for FP16 / BF16; on that geometry a single
// image now runs the width-n walking band at n = 5 (47 / 43.5 us, bitwise the
// same).  conv_tune re-derives them for a given workload.
static conv_tile_cfg g_cfg[3][kKinds] = {
    {{8, 1, 0, 8, 0}, {8, 1, 0, 8, 0}, {8, 1, 0, 8, 0}},
    {{8, 1, 0, 8, 0}, {8, 1, 0, 8, 0}, {16, 1, 0, 8, 0}},
    {{8, 1, 0, 8, 0}, {8, 1, 0, 8, 0}, {16, 1, 0, 8, 0}},
};

// Configurations the tuner installed, per storage type, kind and workload
// size class (conv_tune, conv_tune_load); they take precedence over the
// defaults above for workloads of their class.
static TunedEntry g_tuned[3][kKinds][kSizeClasses];

conv_tile_cfg get_cfg(int dtype, int kind) {
    std::lock_guard<std::mutex> g(g_cfg_mu);
    return g_cfg[dtype][kind];
}

int size_class(uint64_t footprint) {
    const uint64_t MiB = 1ull << 20;
    return footprint <= 64 * MiB ? 0 : footprint <= 256 * MiB ? 1 : footprint <= 1024 * MiB ? 2 : 3;
}

conv_tile_cfg get_cfg_for(int dtype, int kind, uint64_t footprint) {
    load_tune_cache_once();
    std::lock_guard<std::mutex> g(g_cfg_mu);
    const TunedEntry &t = g_tuned[dtype][kind][size_class(footprint)];
    return t.valid ? t.cfg : g_cfg[dtype][kind];
}

TunedEntry get_tuned(int dtype, int kind, int cls) {
    std::lock_guard<std::mutex> g(g_cfg_mu);
    return g_tuned[dtype][kind][cls];
}

void put_tuned(int dtype, int kind, int cls, const TunedEntry &e) {
    std::lock_guard<std::mutex> g(g_cfg_mu);
    g_tuned[dtype][kind][cls] = e;
    if (kind != kKindBatch) g_tuned[dtype][kind][cls].cfg.persist_wgs_per_cu = 0;
}

void put_default_cfg(int dtype, int kind, const conv_tile_cfg &c) {
    std::lock_guard<std::mutex> g(g_cfg_mu);
    g_cfg[dtype][kind] = c;
    if (kind != kKindBatch) g_cfg[dtype][kind].persist_wgs_per_cu = 0;
}

bool cfg_ok(const conv_tile_cfg *c, int kind) {
    if (c->rows_per_tile < 1 || c->rows_per_tile > 4096) return false;
    if (c->waves_per_wg != 1 && c->waves_per_wg != 2 && c->waves_per_wg != 4) return false;
    if (kind == kKindBatch && (c->persist_wgs_per_cu < 0 || c->persist_wgs_per_cu > 32)) return false;
    if (c->xcd_slabs < 0 || c->xcd_slabs > 4096) return false;
    if (c->pack_tail < -1 || c->pack_tail > 1) return false;
    return true;
}

void fill_taps(Taps *t, const float *k) {
    for (int i = 0; i < 5; ++i) t->k[i] = k[i];
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) t->K[5 * a + b] = (float)((double)k[a] * (double)k[b]);
}

// The fused kernels of every storage type and the FP32 direct25 kernel take
// packed last strips (mode: CONV_1PASS_*).
bool packs_last_strip(int mode, int dtype) {
    return mode == CONV_1PASS_FUSED || (mode == CONV_1PASS_DIRECT25 && dtype == CONV_F32);
}

// Packing only pays when the launch has more waves than the GPU holds at once
// (16 per CU: 4 SIMDs at the kernels' occupancy of 4); below that every wave
// starts at once and fewer of them do not end the launch sooner.
bool pack_pays(int64_t unpacked_tiles, const conv_tile_cfg &cfg) {
    if (cfg.pack_tail != 0) return cfg.pack_tail > 0;
    return unpacked_tiles > (int64_t)device_cus() * 16;
}

int64_t fill_desc(ImgDev *d, const void *in, void *out, float *tmp, const conv_image *img,
                  const Layout &L, const float *k, const conv_tile_cfg &cfg, bool pack) {
    std::memset(d, 0, sizeof *d);
    d->in = in;
    d->out = out;
    d->tmp = tmp;
    d->pitch = L.pitch;
    d->pstride = L.ps;
    d->planes = img->planes;
    d->rows = img->rows;
    d->cols = img->cols;
    const int v = L.vec;
    const bool al = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0) &&
                    (tmp == nullptr || (uintptr_t)tmp % 16 == 0) && img->cols % v == 0 &&
                    L.pitch % v == 0 && L.ps % v == 0;
    d->aligned = al ? 1 : 0;
    const int sw = 64 * v;
    d->ns = (img->cols + sw - 1) / sw;
    d->nsg = (d->ns + cfg.waves_per_wg - 1) / cfg.waves_per_wg;
    d->th = cfg.rows_per_tile;
    d->nb = (img->rows + d->th - 1) / d->th;
    d->xcd_slabs = cfg.xcd_slabs;
    fill_taps(&d->tp, k);
    if (L.empty) return 0;
    // The last strip of an aligned image, when narrower than a wave, is packed:
    // cut into a piece of 32 lanes (one wave for 2 bands) and pieces of 16
    // lanes (one wave for 4 bands), so that at most 15 lanes of the last piece
    // stay idle.  The rows of a packed tile share one buffer resource, whose
    // span must stay below the out-of-range offset.
    if (pack && al && cfg.waves_per_wg == 1 && (d->th == 4 || d->th == 8) && d->nb >= 2) {
        const int lanes = (img->cols - (d->ns - 1) * sw) / v;  // cols % v == 0 here
        const int p32 = lanes > 16 && lanes < 64 ? 1 : 0;
        const int p16 = lanes <= 16 ? 1 : (lanes <= 32 ? 0 : (lanes <= 48 ? 1 : (lanes < 64 ? 2 : 0)));
        const int G = p16 ? 4 : 2;
        if ((p32 || p16) && (int64_t)(G * d->th + 4) * L.pitch * L.esz < ((int64_t)1 << 31) - 64) {
            d->tq = G;
            d->pk32 = (int16_t)p32;
            d->pk16 = (int16_t)p16;
            const int64_t nb = d->nb, m = d->ns - 1;
            return (int64_t)img->planes * (nb * m + p32 * ((nb + 1) / 2) + p16 * ((nb + G - 1) / G));
        }
    }
    return (int64_t)img->planes * d->nsg * d->nb;
}

// Pixel-interleaved image: tiles are (band, strip of flat elements); the XCDs
// take turns on chunks of 64 rows.
int64_t fill_desc_hwc(ImgDev *d, const void *in, void *out, float *tmp, const conv_image *img,
                      const Layout &L, const float *k) {
    std::memset(d, 0, sizeof *d);
    d->in = in;
    d->out = out;
    d->tmp = tmp;
    d->pitch = L.pitch;
    d->pstride = 1;
    d->planes = img->planes;
    d->rows = img->rows;
    d->cols = img->cols;
    const int v = L.vec;
    const int64_t wf = (int64_t)img->cols * img->planes;
    d->aligned = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0) &&
                 (tmp == nullptr || (uintptr_t)tmp % 16 == 0) && wf % v == 0 && L.pitch % v == 0;
    const int out_w = hwc_out_per_strip(v, img->planes);
    d->ns = (int)((wf + out_w - 1) / out_w);
    d->nsg = d->ns;
    d->th = kThHwc;
    d->nb = (img->rows + kThHwc - 1) / kThHwc;
    d->xcd_slabs = 64 / kThHwc;
    fill_taps(&d->tp, k);
    if (L.empty) return 0;
    return (int64_t)d->nb * d->ns;
}

conv_status reject_hwc(const Layout &L, const char *what) {
    if (!L.hwc) return CONV_OK;
    return set_error(CONV_EINVAL,
                     "%s does not take pixel-interleaved (plane_stride 1) images; "
                     "conv_sep5_1pass and conv_sep5_2pass do",
                     what);
}

// ---- per-device state --------------------------------------------------------------
struct DescSlot {
    void *host = nullptr;
    void *dev = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};

struct DeviceState {
    int cus = 0;
    std::mutex mu;
    DescSlot slots[kDescSlots];
    int next = 0;
};

static std::mutex g_dev_mu;
static std::vector<DeviceState *> g_devs;

conv_status device_state(DeviceState **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_dev_mu);
    if ((int)g_devs.size() <= dev) g_devs.resize(dev + 1, nullptr);
    if (!g_devs[dev]) {
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_error(e, "hipDeviceGetAttribute");
        auto *st = new DeviceState;
        st->cus = cus > 0 ? cus : 1;
        g_devs[dev] = st;
    }
    *out = g_devs[dev];
    return CONV_OK;
}

int device_cus() {
    DeviceState *st = nullptr;
    return device_state(&st) == CONV_OK ? st->cus : 256;
}

// Stage `bytes` of descriptors through a pinned slot and copy them to device
// memory on stream s.  Returns the device copy; the caller records the slot's
// event after the kernel that reads it.
static conv_status stage_descs(DeviceState *st, const void *src, size_t bytes, hipStream_t s,
                               DescSlot **slot_out) {
    std::lock_guard<std::mutex> g(st->mu);
    DescSlot &sl = st->slots[st->next];
    st->next = (st->next + 1) % kDescSlots;
    hipError_t e;
    if (sl.pending) {
        e = hipEventSynchronize(sl.ev);
        if (e != hipSuccess) return hip_error(e, "hipEventSynchronize(descriptor slot)");
        sl.pending = false;
    }
    if (!sl.ev) {
        e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_error(e, "hipEventCreate");
    }
    if (sl.cap < bytes) {
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
        sl.host = sl.dev = nullptr;
        sl.cap = 0;
        size_t cap = std::max(bytes, (size_t)kDescSlotMinBytes);
        e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault);
        if (e != hipSuccess) return set_error(CONV_ENOMEM, "hipHostMalloc(%zu) failed", cap);
        e = hipMalloc(&sl.dev, cap);
        if (e != hipSuccess) {
            (void)hipHostFree(sl.host);
            sl.host = nullptr;
            return set_error(CONV_ENOMEM, "hipMalloc(%zu) failed", cap);
        }
        sl.cap = cap;
    }
    std::memcpy(sl.host, src, bytes);
    e = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(descriptors)");
    *slot_out = &sl;
    return CONV_OK;
}

static conv_status finish_slot(DescSlot *sl, hipStream_t s) {
    hipError_t e = hipEventRecord(sl->ev, s);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord");
    sl->pending = true;
    return CONV_OK;
}

// ---- batch validation and descriptor building --------------------------------------
// Input plus output bytes of a batch (images that fail validation count 0;
// build_batch rejects them).
uint64_t batch_footprint(int32_t n, const conv_image *imgs) {
    uint64_t f = 0;
    for (int32_t i = 0; imgs && i < n; ++i) {
        Layout L;
        if (check_image(&imgs[i], &L) == CONV_OK) f += 2 * (uint64_t)L.extent_bytes;
    }
    clear_error();
    return f;
}

// Tile configuration of a batch launch: the tuned one for its storage type and
// size class, else the batch default.
conv_tile_cfg batch_cfg(int32_t n, const conv_image *imgs) {
    const int dt0 = (n > 0 && imgs && imgs[0].dtype >= 0 && imgs[0].dtype <= 2) ? imgs[0].dtype : 0;
    return get_cfg_for(dt0, 1, batch_footprint(n, imgs));
}

conv_status build_batch(int32_t n, const void *const *d_in, void *const *d_out, const float *k,
                        const conv_image *imgs, int mode, const conv_tile_cfg &cfg,
                        std::vector<ImgDev> *descs, int64_t *total, int *dtype_out) {
    if (n < 0) return set_error(CONV_EINVAL, "n = %d < 0", n);
    if (mode != CONV_1PASS_FUSED && mode != CONV_1PASS_DIRECT25)
        return set_error(CONV_EINVAL, "mode %d is not FUSED or DIRECT25", mode);
    descs->clear();
    *total = 0;
    if (n == 0) return CONV_OK;
    if (!d_in || !d_out || !k || !imgs)
        return set_error(CONV_EINVAL, "NULL array argument");
    const int dtype = imgs[0].dtype;
    *dtype_out = dtype;
    struct Span {
        uintptr_t lo, hi;
        int idx;
    };
    std::vector<Span> outs, ins;
    descs->resize(n);
    std::vector<Layout> layouts(n);
    int64_t t = 0;
    for (int i = 0; i < n; ++i) {
        Layout L;
        conv_status st = check_image(&imgs[i], &L);
        if (st != CONV_OK)
            return set_error(st, "image %d: %s", i, conv_last_error());
        if (imgs[i].dtype != dtype)
            return set_error(CONV_EINVAL, "image %d dtype %d differs from image 0 (%d)", i,
                             imgs[i].dtype, dtype);
        if (reject_hwc(L, "the batch kernel") != CONV_OK)
            return set_error(CONV_EINVAL, "image %d: %s", i, conv_last_error());
        if (!L.empty) {
            if (!d_in[i] || !d_out[i])
                return set_error(CONV_EINVAL, "image %d: NULL device pointer", i);
            if (overlaps(d_in[i], L.extent_bytes, d_out[i], L.extent_bytes))
                return set_error(CONV_EALIAS, "image %d: input and output overlap", i);
            outs.push_back({(uintptr_t)d_out[i], (uintptr_t)d_out[i] + L.extent_bytes, i});
            ins.push_back({(uintptr_t)d_in[i], (uintptr_t)d_in[i] + L.extent_bytes, i});
        }
        ImgDev &d = (*descs)[i];
        const int64_t tiles = fill_desc(&d, d_in[i], d_out[i], nullptr, &imgs[i], L, k + 5 * i, cfg);
        d.tile_begin = t;
        t += tiles;
        d.tile_end = t;
        layouts[i] = L;
    }
    if (packs_last_strip(mode, dtype) && pack_pays(t, cfg)) {
        t = 0;
        for (int i = 0; i < n; ++i) {
            ImgDev &d = (*descs)[i];
            const int64_t tiles = fill_desc(&d, d_in[i], d_out[i], nullptr, &imgs[i], layouts[i],
                                            k + 5 * i, cfg, true);
            d.tile_begin = t;
            t += tiles;
            d.tile_end = t;
        }
    }
    std::sort(outs.begin(), outs.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].lo < outs[i - 1].hi)
            return set_error(CONV_EALIAS, "outputs of images %d and %d overlap", outs[i - 1].idx,
                             outs[i].idx);
    for (const Span &in : ins) {
        // first output starting at or after in.hi is past it; check the one before
        auto it = std::lower_bound(outs.begin(), outs.end(), in.hi,
                                   [](const Span &o, uintptr_t v) { return o.lo < v; });
        if (it != outs.begin()) {
            const Span &o = *(it - 1);
            if (o.hi > in.lo && o.idx != in.idx)
                return set_error(CONV_EALIAS, "output of image %d overlaps input of image %d",
                                 o.idx, in.idx);
        }
    }
    *total = t;
    return CONV_OK;
}

int batch_flags(const std::vector<ImgDev> &descs) {
    int f = 0;
    for (const ImgDev &d : descs) {
        if (d.tile_end == d.tile_begin) continue;
        if (!d.aligned) f |= kBatchAnyUnaligned;
        if (d.tq > 1) f |= kBatchAnyPacked;
    }
    return f;
}

// Batch grid: persist_wgs_per_cu workgroups per CU (a persistent grid that
// strides over the tiles), or 0: one workgroup per tile up to 2^20.
int batch_grid(int64_t total, int cus, const conv_tile_cfg &cfg) {
    const int64_t cap = cfg.persist_wgs_per_cu > 0 ? (int64_t)cus * cfg.persist_wgs_per_cu
                                                   : (int64_t)1 << 20;
    return (int)std::max<int64_t>(1, std::min<int64_t>(total, cap));
}

conv_status enqueue_batch(const std::vector<ImgDev> &descs, int64_t total, int dtype, int mode,
                          const conv_tile_cfg &cfg, hipStream_t s) {
    if (total == 0) return CONV_OK;
    DeviceState *st = nullptr;
    conv_status rc = device_state(&st);
    if (rc != CONV_OK) return rc;
    if ((int)descs.size() <= kMaxArgImages) {
        // small batch: descriptors ride in the kernel argument
        BatchArgs a;
        std::memset(&a, 0, sizeof a);
        std::memcpy(a.d, descs.data(), descs.size() * sizeof(ImgDev));
        a.n = (int)descs.size();
        a.total = total;
        const int grid = batch_grid(total, st->cus, cfg);
        hipError_t e = launch_batch_args(a, dtype, mode, cfg.waves_per_wg, cfg.rows_per_tile, grid,
                                         batch_flags(descs), s);
        if (e != hipSuccess) return hip_error(e, "batch kernel launch");
        return CONV_OK;
    }
    DescSlot *slot = nullptr;
    rc = stage_descs(st, descs.data(), descs.size() * sizeof(ImgDev), s, &slot);
    if (rc != CONV_OK) return rc;
    const int grid = batch_grid(total, st->cus, cfg);
    hipError_t e = launch_batch((const ImgDev *)slot->dev, (int)descs.size(), total, dtype, mode,
                                cfg.waves_per_wg, cfg.rows_per_tile, grid, batch_flags(descs), s);
    rc = finish_slot(slot, s);
    if (e != hipSuccess) return hip_error(e, "batch kernel launch");
    return rc;
}

// The copy kernel over an image of either layout (the copy-back step).  The
// copy is elementwise: a pixel-interleaved image copies as one plane of
// cols*planes elements per row.
hipError_t launch_copy(const void *d_in, void *d_out, const conv_image *img, const Layout &L,
                       const conv_tile_cfg &cfg, hipStream_t stream) {
    conv_image flat = *img;
    Layout LF = L;
    if (L.hwc) {
        flat.cols = img->cols * img->planes;
        flat.planes = 1;
        flat.plane_stride = 0;
        LF.ps = (int64_t)img->rows * L.pitch;
    }
    ImgDev d;
    const float k0[5] = {0, 0, 0, 0, 0};
    const int64_t nblocks = fill_desc(&d, d_in, d_out, nullptr, &flat, LF, k0, cfg);
    return launch_image(d, img->dtype, MODE_COPY, cfg.waves_per_wg, nblocks, stream);
}

}  // namespace convsep5

// ==== public entry points ===========================================================
extern "C" {

const char *conv_last_error(void) { return g_err.c_str(); }

const char *conv_version(void) { return "convsep5 1.0 gfx950"; }

conv_status conv_sep5_1pass(const void *d_in, void *d_out, const float k[5],
                            const conv_image *img, int mode, hipStream_t stream) {
    clear_error();
    Layout L;
    conv_status st = check_image(img, &L);
    if (st != CONV_OK) return st;
    if (!k) return set_error(CONV_EINVAL, "taps pointer is NULL");
    if (mode != CONV_1PASS_FUSED && mode != CONV_1PASS_DIRECT25)
        return set_error(CONV_EINVAL, "mode %d is not FUSED or DIRECT25", mode);
    if (L.empty) return CONV_OK;
    if (!d_in || !d_out) return set_error(CONV_EINVAL, "NULL device pointer");
    const bool copy_back = d_in == (const void *)d_out;
    if (!copy_back && overlaps(d_in, L.extent_bytes, d_out, L.extent_bytes))
        return set_error(CONV_EALIAS, "input and output partially overlap");
    const conv_tile_cfg cfg = get_cfg_for(img->dtype, mode == CONV_1PASS_FUSED ? kKindImage : kKindDirect,
                                          2 * (uint64_t)L.extent_bytes);
    const int kmode = mode == CONV_1PASS_FUSED ? MODE_FUSED : MODE_DIRECT25;
    ImgDev d;
    if (!copy_back) {
        hipError_t e;
        if (L.hwc) {
            const int64_t nblocks = fill_desc_hwc(&d, d_in, d_out, nullptr, img, L, k);
            e = launch_hwc(d, img->dtype, kmode, nblocks, stream);
        } else {
            int64_t nblocks = fill_desc(&d, d_in, d_out, nullptr, img, L, k, cfg);
            if (packs_last_strip(mode, img->dtype) && pack_pays(nblocks, cfg))
                nblocks = fill_desc(&d, d_in, d_out, nullptr, img, L, k, cfg, true);
            e = launch_image(d, img->dtype, kmode, cfg.waves_per_wg, nblocks, stream);
        }
        if (e != hipSuccess) return hip_error(e, "1pass kernel launch");
        return CONV_OK;
    }
    // Single-pass with copy-back (the paper's in-place single-pass): convolve
    // into stream-ordered scratch of the image's layout, then copy the result
    // over the input.
    void *scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, (size_t)L.extent_bytes, stream);
    if (e != hipSuccess)
        return set_error(CONV_ENOMEM, "hipMallocAsync(%lld): %s", (long long)L.extent_bytes,
                         hipGetErrorString(e));
    // the scratch is written with cached stores: the copy reads it next
    int64_t nblocks;
    if (L.hwc) {
        nblocks = fill_desc_hwc(&d, d_in, scratch, nullptr, img, L, k);
        d.keep_out = 1;
        e = launch_hwc(d, img->dtype, kmode, nblocks, stream);
    } else {
        nblocks = fill_desc(&d, d_in, scratch, nullptr, img, L, k, cfg);
        if (packs_last_strip(mode, img->dtype) && pack_pays(nblocks, cfg))
            nblocks = fill_desc(&d, d_in, scratch, nullptr, img, L, k, cfg, true);
        d.keep_out = 1;
        e = launch_image(d, img->dtype, kmode, cfg.waves_per_wg, nblocks, stream);
    }
    if (e == hipSuccess) e = launch_copy(scratch, d_out, img, L, cfg, stream);
    (void)hipFreeAsync(scratch, stream);
    if (e != hipSuccess) return hip_error(e, "1pass (copy-back) kernel launch");
    return CONV_OK;
}

conv_status conv_image_copy(const void *d_in, void *d_out, const conv_image *img,
                            hipStream_t stream) {
    clear_error();
    Layout L;
    conv_status st = check_image(img, &L);
    if (st != CONV_OK) return st;
    if (L.empty) return CONV_OK;
    if (!d_in || !d_out) return set_error(CONV_EINVAL, "NULL device pointer");
    if (d_in == (const void *)d_out) return CONV_OK;
    if (overlaps(d_in, L.extent_bytes, d_out, L.extent_bytes))
        return set_error(CONV_EALIAS, "input and output partially overlap");
    hipError_t e = launch_copy(d_in, d_out, img, L,
                               get_cfg_for(img->dtype, 0, 2 * (uint64_t)L.extent_bytes), stream);
    if (e != hipSuccess) return hip_error(e, "copy kernel launch");
    return CONV_OK;
}

// The two-pass form with its intermediate in tmp_dtype (CONV_F32: the FP32
// form; CONV_F16 / CONV_BF16: the 16-bit intermediate, one wave per workgroup).
static conv_status twopass(const void *d_in, void *d_out, void *d_tmp, const float k[5],
                           const conv_image *img, int32_t tmp_dtype, hipStream_t stream) {
    clear_error();
    Layout L;
    conv_status st = check_image(img, &L);
    if (st != CONV_OK) return st;
    if (!k) return set_error(CONV_EINVAL, "taps pointer is NULL");
    if (tmp_dtype != CONV_F32 && tmp_dtype != CONV_F16 && tmp_dtype != CONV_BF16)
        return set_error(CONV_EINVAL, "tmp_dtype %d is not CONV_F32, CONV_F16 or CONV_BF16",
                         tmp_dtype);
    if (L.hwc && tmp_dtype != CONV_F32)
        return set_error(CONV_EINVAL,
                         "pixel-interleaved (plane_stride 1) images take an FP32 intermediate only");
    if (L.empty) return CONV_OK;
    if (!d_in || !d_out) return set_error(CONV_EINVAL, "NULL device pointer");
    if (d_in != (const void *)d_out && overlaps(d_in, L.extent_bytes, d_out, L.extent_bytes))
        return set_error(CONV_EALIAS, "input and output partially overlap");
    const int64_t tmp_bytes =
        (int64_t)img->planes * img->rows * img->cols * (tmp_dtype == CONV_F32 ? 4 : 2);
    if (d_tmp && (overlaps(d_tmp, tmp_bytes, d_in, L.extent_bytes) ||
                  overlaps(d_tmp, tmp_bytes, d_out, L.extent_bytes)))
        return set_error(CONV_EALIAS, "workspace overlaps the input or output");
    void *tmp = d_tmp;
    hipError_t e;
    if (!tmp) {
        e = hipMallocAsync(&tmp, (size_t)tmp_bytes, stream);
        if (e != hipSuccess)
            return set_error(CONV_ENOMEM, "hipMallocAsync(%lld): %s", (long long)tmp_bytes,
                             hipGetErrorString(e));
    }
    conv_tile_cfg cfg = get_cfg_for(img->dtype, 0, 2 * (uint64_t)L.extent_bytes);
    int row_mode = MODE_ROWPASS, col_mode = MODE_COLPASS;
    if (tmp_dtype != CONV_F32) {
        cfg.waves_per_wg = 1;
        row_mode = tmp_dtype == CONV_F16 ? MODE_ROWPASS_F16T : MODE_ROWPASS_BF16T;
        col_mode = tmp_dtype == CONV_F16 ? MODE_COLPASS_F16T : MODE_COLPASS_BF16T;
    }
    ImgDev d;
    if (L.hwc) {
        const int64_t nblocks = fill_desc_hwc(&d, d_in, d_out, (float *)tmp, img, L, k);
        e = launch_hwc(d, img->dtype, MODE_ROWPASS, nblocks, stream);
        if (e == hipSuccess) e = launch_hwc(d, img->dtype, MODE_COLPASS, nblocks, stream);
    } else {
        const int64_t nblocks = fill_desc(&d, d_in, d_out, (float *)tmp, img, L, k, cfg);
        e = launch_image(d, img->dtype, row_mode, cfg.waves_per_wg, nblocks, stream);
        if (e == hipSuccess)
            e = launch_image(d, img->dtype, col_mode, cfg.waves_per_wg, nblocks, stream);
    }
    if (!d_tmp) (void)hipFreeAsync(tmp, stream);
    if (e != hipSuccess) return hip_error(e, "2pass kernel launch");
    return CONV_OK;
}

conv_status conv_sep5_2pass(const void *d_in, void *d_out, float *d_tmp, const float k[5],
                            const conv_image *img, hipStream_t stream) {
    return twopass(d_in, d_out, d_tmp, k, img, CONV_F32, stream);
}

// ---- the two-pass without allocation ----------------------------------------------
// The intermediate of conv_sep5_2pass_noalloc lives in this array: every GPU that
// loads the library's code object holds its own copy, at its own address, until the
// process ends.  In host code the name is only a stand-in for the symbol; its
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[CONV_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices];

// The current device's copy of `scratch` (looked up on its first use on that device).
static conv_status scratch_of_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return set_error(CONV_EINVAL, "device %d: the static workspace serves devices 0..%d", dev,
                         kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return set_error(CONV_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CONV_OK;
}

conv_status conv_sep5_2pass_noalloc(const void *d_in, void *d_out, const float k[5],
                                    const conv_image *img, int32_t tmp_dtype,
                                    hipStream_t stream) {
    clear_error();
    Layout L;
    conv_status st = check_image(img, &L);
    if (st != CONV_OK) return st;
    if (tmp_dtype != CONV_F32 && tmp_dtype != CONV_F16 && tmp_dtype != CONV_BF16)
        return set_error(CONV_EINVAL, "tmp_dtype %d is not CONV_F32, CONV_F16 or CONV_BF16",
                         tmp_dtype);
    const uint64_t tmp_bytes =
        (uint64_t)img->planes * img->rows * img->cols * (tmp_dtype == CONV_F32 ? 4 : 2);
    if (tmp_bytes > CONV_NOALLOC_SCRATCH_BYTES)
        return set_error(CONV_ENOMEM,
                         "the intermediate takes %llu bytes, more than the %llu-byte static "
                         "workspace of conv_sep5_2pass_noalloc",
                         (unsigned long long)tmp_bytes,
                         (unsigned long long)CONV_NOALLOC_SCRATCH_BYTES);
    if (L.empty) return CONV_OK;
    void *tmp = nullptr;
    st = scratch_of_current_device(&tmp);
    if (st != CONV_OK) return st;
    return twopass(d_in, d_out, tmp, k, img, tmp_dtype, stream);
}

conv_status conv_sep5_2pass_ex(const void *d_in, void *d_out, void *d_tmp, const float k[5],
                               const conv_image *img, int32_t tmp_dtype, hipStream_t stream) {
    return twopass(d_in, d_out, d_tmp, k, img, tmp_dtype, stream);
}

conv_status conv_sep5_batch(int32_t n, const void *const *d_in, void *const *d_out,
                            const float *k, const conv_image *imgs, int mode,
                            hipStream_t stream) {
    clear_error();
    std::vector<ImgDev> descs;
    int64_t total = 0;
    int dtype = 0;
    const conv_tile_cfg cfg = batch_cfg(n, imgs);
    conv_status st = build_batch(n, d_in, d_out, k, imgs, mode, cfg, &descs, &total, &dtype);
    if (st != CONV_OK) return st;
    return enqueue_batch(descs, total, dtype, mode == CONV_1PASS_FUSED ? MODE_FUSED : MODE_DIRECT25,
                         cfg, stream);
}

conv_status conv_get_tile_cfg(int32_t dtype, int32_t kind, conv_tile_cfg *cfg) {
    clear_error();
    if (dtype < 0 || dtype > 2 || kind < 0 || kind >= kKinds || !cfg)
        return set_error(CONV_EINVAL, "bad dtype/kind/cfg");
    *cfg = get_cfg(dtype, kind);
    return CONV_OK;
}

conv_status conv_set_tile_cfg(int32_t dtype, int32_t kind, const conv_tile_cfg *cfg) {
    clear_error();
    if (dtype < 0 || dtype > 2 || kind < 0 || kind >= kKinds || !cfg)
        return set_error(CONV_EINVAL, "bad dtype/kind/cfg");
    if (!cfg_ok(cfg, kind)) return set_error(CONV_EINVAL, "tile configuration out of range");
    put_default_cfg(dtype, kind, *cfg);
    // an explicit configuration replaces what the tuner installed for this
    // storage type and kind
    for (int c = 0; c < kSizeClasses; ++c) put_tuned(dtype, kind, c, TunedEntry{});
    return CONV_OK;
}

conv_status conv_get_tile_cfg_for(int32_t dtype, int32_t kind, uint64_t footprint_bytes,
                                  conv_tile_cfg *cfg, int32_t *tuned) {
    clear_error();
    if (dtype < 0 || dtype > 2 || kind < 0 || kind >= kKinds || !cfg)
        return set_error(CONV_EINVAL, "bad dtype/kind/cfg");
    load_tune_cache_once();
    const TunedEntry t = get_tuned(dtype, kind, size_class(footprint_bytes));
    *cfg = t.valid ? t.cfg : get_cfg(dtype, kind);
    if (tuned) *tuned = t.valid ? 1 : 0;
    return CONV_OK;
}

// ---- captured batch plans -------------------------------------------------------------
struct conv_plan {
    int device;
    ImgDev *d_descs;
    hipStream_t cap;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

conv_status conv_batch_plan_create(int32_t n, const void *const *d_in, void *const *d_out,
                                   const float *k, const conv_image *imgs, int mode,
                                   conv_plan **plan) {
    clear_error();
    if (!plan) return set_error(CONV_EINVAL, "plan is NULL");
    *plan = nullptr;
    std::vector<ImgDev> descs;
    int64_t total = 0;
    int dtype = 0;
    const conv_tile_cfg cfg = batch_cfg(n, imgs);
    conv_status st = build_batch(n, d_in, d_out, k, imgs, mode, cfg, &descs, &total, &dtype);
    if (st != CONV_OK) return st;
    DeviceState *ds = nullptr;
    st = device_state(&ds);
    if (st != CONV_OK) return st;
    auto *p = new conv_plan();
    hipGetDevice(&p->device);
    const size_t bytes = std::max<size_t>(descs.size(), 1) * sizeof(ImgDev);
    hipError_t e = hipMalloc((void **)&p->d_descs, bytes);
    if (e != hipSuccess) {
        delete p;
        return set_error(CONV_ENOMEM, "hipMalloc(plan descriptors) failed");
    }
    if (!descs.empty()) {
        e = hipMemcpy(p->d_descs, descs.data(), descs.size() * sizeof(ImgDev),
                      hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            hipFree(p->d_descs);
            delete p;
            return hip_error(e, "hipMemcpy(plan descriptors)");
        }
    }
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        hipFree(p->d_descs);
        delete p;
        return hip_error(e, "hipStreamCreate");
    }
    e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    hipError_t le = hipSuccess;
    if (e == hipSuccess) {
        if (total > 0) {
            const int grid = batch_grid(total, ds->cus, cfg);
            le = launch_batch(p->d_descs, (int)descs.size(), total, dtype,
                              mode == CONV_1PASS_FUSED ? MODE_FUSED : MODE_DIRECT25,
                              cfg.waves_per_wg, cfg.rows_per_tile, grid, batch_flags(descs),
                              p->cap);
        }
        e = hipStreamEndCapture(p->cap, &p->graph);
    }
    if (e == hipSuccess && le == hipSuccess)
        e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess || le != hipSuccess) {
        const hipError_t bad = le != hipSuccess ? le : e;
        if (p->graph) hipGraphDestroy(p->graph);
        hipStreamDestroy(p->cap);
        hipFree(p->d_descs);
        delete p;
        return hip_error(bad, "graph capture of the batch launch");
    }
    *plan = p;
    return CONV_OK;
}

conv_status conv_batch_plan_launch(conv_plan *plan, hipStream_t stream) {
    clear_error();
    if (!plan) return set_error(CONV_EINVAL, "plan is NULL");
    hipError_t e = hipGraphLaunch(plan->exec, stream);
    if (e != hipSuccess) return hip_error(e, "hipGraphLaunch");
    return CONV_OK;
}

conv_status conv_batch_plan_destroy(conv_plan *plan) {
    clear_error();
    if (!plan) return CONV_OK;
    hipGraphExecDestroy(plan->exec);
    hipGraphDestroy(plan->graph);
    hipStreamDestroy(plan->cap);
    hipFree(plan->d_descs);
    delete plan;
    return CONV_OK;
}

}  // extern "C"
