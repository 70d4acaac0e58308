// conv_tune.cpp -- the tile-shape autotuner and its on-disk cache.  The tuner
// times every candidate configuration on the caller's workload with HIP
// events and installs the fastest for the workload's storage type, kind and
// size class.  All candidates compute bitwise identical results; only the
// decomposition into tiles (rows per band, wavefronts per workgroup, the
// persistent grid size, the XCD order and the packing of narrow last strips)
// changes.  The installed choices can be written to and read from a small
// JSON file; the file named by CONV_TUNE_CACHE is read at the library's first
// use and rewritten after every tuning run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
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
    if (kind != kKindBatch) {
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

const char *kFormat = "convsep5-tune-1";

// ---- the cache file -----------------------------------------------------------
// {"format": "convsep5-tune-1", "arch": "gfx950", "entries": [
//   {"dtype": 0, "kind": 1, "size_class": 3, "rows_per_tile": 8, "waves_per_wg": 1,
//    "persist_wgs_per_cu": 0, "xcd_slabs": 8, "pack_tail": 0, "ms": 0.371}, ...]}

struct FileEntry {
    int dtype, kind, cls;
    TunedEntry e;
};

// The number after "key": inside [b, e); false if absent or malformed.
bool number_of(const char *b, const char *e, const char *key, double *v) {
    const std::string k = std::string("\"") + key + "\"";
    const char *p = std::search(b, e, k.begin(), k.end());
    if (p == e) return false;
    p += k.size();
    while (p < e && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
    if (p >= e || *p != ':') return false;
    ++p;
    char *end = nullptr;
    errno = 0;
    const double d = std::strtod(p, &end);
    if (end == p || end > e || errno != 0) return false;
    *v = d;
    return true;
}

bool int_of(const char *b, const char *e, const char *key, int lo, int hi, int *v) {
    double d;
    if (!number_of(b, e, key, &d) || d != (double)(int)d || d < lo || d > hi) return false;
    *v = (int)d;
    return true;
}

conv_status parse(const std::string &text, std::vector<FileEntry> *out) {
    if (text.find(std::string("\"") + kFormat + "\"") == std::string::npos)
        return set_error(CONV_EINVAL, "not a %s file", kFormat);
    const size_t ent = text.find("\"entries\"");
    if (ent == std::string::npos) return set_error(CONV_EINVAL, "no \"entries\" list");
    size_t pos = text.find('[', ent);
    const size_t stop = text.find(']', ent);
    if (pos == std::string::npos || stop == std::string::npos || stop < pos)
        return set_error(CONV_EINVAL, "malformed \"entries\" list");
    for (;;) {
        const size_t ob = text.find('{', pos);
        if (ob == std::string::npos || ob > stop) break;
        const size_t cb = text.find('}', ob);
        if (cb == std::string::npos || cb > stop) return set_error(CONV_EINVAL, "unterminated entry");
        const char *b = text.data() + ob, *e = text.data() + cb;
        FileEntry f{};
        double ms = 0.0;
        conv_tile_cfg &c = f.e.cfg;
        const bool ok = int_of(b, e, "dtype", 0, 2, &f.dtype) && int_of(b, e, "kind", 0, kKinds - 1, &f.kind) &&
                        int_of(b, e, "size_class", 0, kSizeClasses - 1, &f.cls) &&
                        int_of(b, e, "rows_per_tile", 1, 4096, &c.rows_per_tile) &&
                        int_of(b, e, "waves_per_wg", 1, 4, &c.waves_per_wg) &&
                        int_of(b, e, "persist_wgs_per_cu", 0, 32, &c.persist_wgs_per_cu) &&
                        int_of(b, e, "xcd_slabs", 0, 4096, &c.xcd_slabs) &&
                        int_of(b, e, "pack_tail", -1, 1, &c.pack_tail) && number_of(b, e, "ms", &ms);
        if (!ok || !cfg_ok(&c, f.kind))
            return set_error(CONV_EINVAL, "entry %zu: missing or out-of-range field", out->size());
        f.e.valid = 1;
        f.e.ms = (float)ms;
        out->push_back(f);
        pos = cb + 1;
    }
    return CONV_OK;
}

conv_status load_file(const char *path) {
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return set_error(CONV_ENOTFOUND, "cannot open %s: %s", path, std::strerror(errno));
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, fp)) > 0 && text.size() < (1u << 20))
        text.append(buf, got);
    std::fclose(fp);
    std::vector<FileEntry> es;
    const conv_status st = parse(text, &es);
    if (st != CONV_OK) return st;
    for (const FileEntry &f : es) put_tuned(f.dtype, f.kind, f.cls, f.e);  // all or nothing
    return CONV_OK;
}

conv_status save_file(const char *path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) return set_error(CONV_EINVAL, "cannot write %s: %s", tmp.c_str(), std::strerror(errno));
    std::fprintf(fp, "{\"format\": \"%s\", \"arch\": \"gfx950\", \"entries\": [", kFormat);
    bool first = true;
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < kKinds; ++k)
            for (int c = 0; c < kSizeClasses; ++c) {
                const TunedEntry t = get_tuned(d, k, c);
                if (!t.valid) continue;
                std::fprintf(fp,
                             "%s\n  {\"dtype\": %d, \"kind\": %d, \"size_class\": %d, "
                             "\"rows_per_tile\": %d, \"waves_per_wg\": %d, "
                             "\"persist_wgs_per_cu\": %d, \"xcd_slabs\": %d, \"pack_tail\": %d, "
                             "\"ms\": %.6g}",
                             first ? "" : ",", d, k, c, t.cfg.rows_per_tile, t.cfg.waves_per_wg,
                             t.cfg.persist_wgs_per_cu, t.cfg.xcd_slabs, t.cfg.pack_tail,
                             (double)t.ms);
                first = false;
            }
    std::fprintf(fp, "\n]}\n");
    const bool bad = std::ferror(fp) != 0;
    if (std::fclose(fp) != 0 || bad) {
        std::remove(tmp.c_str());
        return set_error(CONV_EINVAL, "writing %s failed", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return set_error(CONV_EINVAL, "cannot replace %s: %s", path, std::strerror(errno));
    }
    return CONV_OK;
}

std::once_flag g_cache_once;

}  // namespace

namespace convsep5 {

// A missing or unreadable cache file leaves the defaults in place.
void load_tune_cache_once() {
    std::call_once(g_cache_once, [] {
        const char *path = std::getenv("CONV_TUNE_CACHE");
        if (path && *path) (void)load_file(path);
        clear_error();
    });
}

}  // namespace convsep5

extern "C" conv_status conv_tune(int32_t kind, int32_t n, const void *const *d_in,
                                 void *const *d_out, const float *k, const conv_image *imgs,
                                 int32_t reps, hipStream_t stream, conv_tile_cfg *best,
                                 float *best_ms) {
    clear_error();
    if (kind < 0 || kind >= kKinds) return set_error(CONV_EINVAL, "kind %d is not 0, 1 or 2", kind);
    if (n < 1 || !d_in || !d_out || !k || !imgs || !best || reps < 1 || reps > 10000)
        return set_error(CONV_EINVAL, "bad tuner arguments");
    const int dtype = imgs[0].dtype;
    if (dtype < 0 || dtype > 2) return set_error(CONV_EINVAL, "bad dtype %d", dtype);
    load_tune_cache_once();
    // the workload's size class: image 0 alone for kinds 0 and 2, the whole
    // batch for kind 1
    const int cls = size_class(batch_footprint(kind == kKindBatch ? n : 1, imgs));
    const conv_tile_cfg orig = get_cfg(dtype, kind);
    const TunedEntry orig_tuned = get_tuned(dtype, kind, cls);
    // candidates run as the default with this class's tuned entry set aside
    put_tuned(dtype, kind, cls, TunedEntry{});

    std::vector<hipEvent_t> ev(2 * reps);
    conv_status rc = CONV_OK;
    for (auto &e : ev)
        if (rc == CONV_OK && hipEventCreate(&e) != hipSuccess)
            rc = set_error(CONV_EHIP, "hipEventCreate failed");
    auto run_once = [&]() -> conv_status {
        if (kind == kKindImage)
            return conv_sep5_1pass(d_in[0], d_out[0], k, &imgs[0], CONV_1PASS_FUSED, stream);
        if (kind == kKindDirect)
            return conv_sep5_1pass(d_in[0], d_out[0], k, &imgs[0], CONV_1PASS_DIRECT25, stream);
        return conv_sep5_batch(n, d_in, d_out, k, imgs, CONV_1PASS_FUSED, stream);
    };
    float best_t = 1e30f;
    conv_tile_cfg best_c = orig;
    std::vector<float> t(reps);
    for (const conv_tile_cfg &c : candidates(kind)) {
        if (rc != CONV_OK) break;
        put_default_cfg(dtype, kind, c);
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
    for (auto &e : ev)
        if (e) hipEventDestroy(e);
    put_default_cfg(dtype, kind, orig);
    if (rc != CONV_OK) {
        put_tuned(dtype, kind, cls, orig_tuned);
        return rc;
    }
    TunedEntry te;
    te.valid = 1;
    te.cfg = best_c;
    te.ms = best_t;
    put_tuned(dtype, kind, cls, te);
    *best = get_tuned(dtype, kind, cls).cfg;
    if (best_ms) *best_ms = best_t;
    const char *path = std::getenv("CONV_TUNE_CACHE");
    if (path && *path) {
        const conv_status st = save_file(path);
        if (st != CONV_OK) return st;
    }
    return CONV_OK;
}

extern "C" conv_status conv_tune_save(const char *path) {
    clear_error();
    if (!path || !*path) return set_error(CONV_EINVAL, "empty path");
    load_tune_cache_once();
    return save_file(path);
}

extern "C" conv_status conv_tune_load(const char *path) {
    clear_error();
    if (!path || !*path) return set_error(CONV_EINVAL, "empty path");
    load_tune_cache_once();
    return load_file(path);
}
