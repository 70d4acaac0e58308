// conv_kernels_n.h -- Eq. 1 of arXiv 1711.09791 for any odd width n = 2R+1,
// R = 0..4: the separable forms (fused single pass, two-pass row and column
// kernels, direct n*n with K = k k^T) and the direct form with a general,
// non-separable n x n kernel K.  The O(n) separable passes against the O(n^2)
// direct sum are the trade-off of Section 5.1.
//
// Same machinery as the width-5 kernels (conv_kernels.h): a wave64 tile of
// 64*VEC columns x a band of TH rows, strip-fastest launch order, one 16-byte
// buffer load per lane per row, R-column halos from neighbouring lanes by DPP,
// per-row buffer resources so that lanes past the edge read 0 and drop their
// stores.  Every band is fully unrolled: all TH+2R input rows are issued
// first; a short last band computes TH rows and stores only its own (the
// direct form at n >= 7 walks 16-row bands instead, loading rows as it goes).
// The output frame of R pixels is written as +0.0.
//
// Arithmetic (fixed for every tile shape):
//   horizontal  h = v[x-R]*k0; h = fma(v[x-R+1], k1, h); ... (n taps)
//   vertical    o = h[y-R]*k0; o = fma(h[y-R+1], k1, o); ...
//   direct      p_a = the same n-term chain over kernel row a with K[a][.],
//               then a pairwise sum of the n row partials: the first half is
//               the largest power of two below n, recursively.
// For n = 5 this is exactly the arithmetic of the width-5 kernels.
#pragma once

#include "conv_kernels.h"

namespace convsep5 {
namespace {

// ---- rows with R-column halos ---------------------------------------------------
template <class D, bool AL, int R> struct RawN;
template <class D, int R> struct RawN<D, true, R> {
    static constexpr int HW = (R * D::ESZ + 3) / 4;  // halo words on each side
    u4 m;
    uint32_t h[HW > 0 ? HW : 1];
};
template <class D, int R> struct RawN<D, false, R> { uint32_t e[D::VEC + 2 * R]; };

template <int HW>
__device__ __forceinline__ void load_words(uint32_t (&h)[HW > 0 ? HW : 1],
                                           __amdgpu_buffer_rsrc_t rs, int off) {
    if constexpr (HW == 1) {
        h[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    } else if constexpr (HW == 2) {
        const u2 q = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        h[0] = q.x;
        h[1] = q.y;
    } else if constexpr (HW == 3) {
        typedef uint32_t u3 __attribute__((ext_vector_type(3)));
        const u3 q = __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0);
        h[0] = q.x;
        h[1] = q.y;
        h[2] = q.z;
    } else if constexpr (HW == 4) {
        const u4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        h[0] = q.x;
        h[1] = q.y;
        h[2] = q.z;
        h[3] = q.w;
    }
}

// Byte offset of the halo load: lane 0 loads the HW words left of the strip,
// lane 63 the HW words right of it; other lanes (and halos outside the row)
// get an out-of-range offset.
template <class D, int R>
__device__ __forceinline__ int halo_offset_n(int xs, int W, int lane) {
    constexpr int HW = (R * D::ESZ + 3) / 4;
    constexpr int HE = HW * 4 / D::ESZ;  // halo elements covered by HW words
    if constexpr (HW == 0) {
        return OOB;
    } else {
        const int hl = xs - HE, hr = xs + WAVE * D::VEC;
        return lane == 0 ? (hl >= 0 ? hl * D::ESZ : OOB)
                         : (lane == WAVE - 1 ? (hr < W ? hr * D::ESZ : OOB) : OOB);
    }
}

template <class D, int R>
__device__ __forceinline__ void issue_n(RawN<D, true, R> &r, const char *row, uint32_t rbytes,
                                        int x, int hoff) {
    const auto rs = row_rsrc(row, rbytes);
    r.m = __builtin_amdgcn_raw_buffer_load_b128(rs, x * D::ESZ, 0, 0);
    load_words<RawN<D, true, R>::HW>(r.h, rs, hoff);
}
template <class D, int R>
__device__ __forceinline__ void issue_n(RawN<D, false, R> &r, const char *row, uint32_t rbytes,
                                        int x, int) {
    const auto rs = row_rsrc(row, rbytes);
#pragma unroll
    for (int e = 0; e < D::VEC + 2 * R; ++e) {
        const int c = x - R + e;
        const int off = c >= 0 ? c * D::ESZ : OOB;
        if constexpr (D::ESZ == 4)
            r.e[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        else
            r.e[e] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
    }
}

// Each decoded FP16 value as a value of its own: an empty asm statement keeps
// the compiler from folding the conversion into mixed-precision FMAs (used by
// the walking band, where those issued slower; no value changes).
template <class D> __device__ __forceinline__ float dec_kept(uint32_t b) {
    float f = dec(D{}, b);
    if constexpr (std::is_same<D, F16>::value) asm volatile("" : "+v"(f));
    return f;
}

// v[i] = A[x - R + i], i = 0 .. VEC+2R-1, as FP32; KEEP: FP16 values through
// dec_kept.
template <class D, int R, bool KEEP = false>
__device__ __forceinline__ void decode_n(const RawN<D, true, R> &r, float (&v)[D::VEC + 2 * R]) {
    constexpr int HW = RawN<D, true, R>::HW;
    const uint32_t m[4] = {r.m.x, r.m.y, r.m.z, r.m.w};
    // words of the lane's extended row: HW from the left lane, its own 4, HW
    // from the right lane (lane 0 / 63 keep their own halo words instead)
    uint32_t ext[4 + 2 * HW];
#pragma unroll
    for (int j = 0; j < HW; ++j) ext[j] = from_left(m[4 - HW + j], r.h[j]);
#pragma unroll
    for (int j = 0; j < 4; ++j) ext[HW + j] = m[j];
#pragma unroll
    for (int j = 0; j < HW; ++j) ext[HW + 4 + j] = from_right(m[j], r.h[j]);
    if constexpr (D::ESZ == 4) {
#pragma unroll
        for (int i = 0; i < D::VEC + 2 * R; ++i) v[i] = __uint_as_float(ext[i]);
    } else {
        constexpr int SH = 2 * HW - R;  // halves of ext before A[x - R]
#pragma unroll
        for (int i = 0; i < D::VEC + 2 * R; ++i) {
            const int j = i + SH;
            const uint32_t b = (j & 1) ? (ext[j >> 1] >> 16) : ext[j >> 1];
            v[i] = KEEP ? dec_kept<D>(b) : dec(D{}, b);
        }
    }
}
template <class D, int R, bool KEEP = false>
__device__ __forceinline__ void decode_n(const RawN<D, false, R> &r, float (&v)[D::VEC + 2 * R]) {
#pragma unroll
    for (int e = 0; e < D::VEC + 2 * R; ++e) v[e] = KEEP ? dec_kept<D>(r.e[e]) : dec(D{}, r.e[e]);
}

// ---- the arithmetic ---------------------------------------------------------------

template <int N, int R>
__device__ __forceinline__ void hfilter_n(const float (&v)[N + 2 * R], const float *k, float (&h)[N]) {
#pragma unroll
    for (int e = 0; e < N; ++e) {
        float t = v[e] * k[0];
#pragma unroll
        for (int b = 1; b <= 2 * R; ++b) t = __builtin_fmaf(v[e + b], k[b], t);
        h[e] = t;
    }
}

// Direct n x n sums for a whole band: out[j][e] = pairwise sum over kernel
// rows a of the chains sum_b w[j+a][e+b] K[a][b].  Subtrees of the pairwise
// split are evaluated left to right and each leaf (one kernel row) for all
// TH x VEC outputs at once, so one weight K[a][b] serves TH*VEC FMAs in a
// row.  Each output's row partials are added pairwise, the first half of
// every split being the largest power of two below its length.
template <int LO, int HI, int NT_, int TH, int VEC, int WN>
__device__ __forceinline__ void direct_tree(const float (&w)[TH + NT_ - 1][WN], const float *K,
                                            float (&s)[TH][VEC]) {
    if constexpr (HI - LO == 1) {
        constexpr int a = LO;
#pragma unroll
        for (int j = 0; j < TH; ++j)
#pragma unroll
            for (int e = 0; e < VEC; ++e) s[j][e] = w[j + a][e] * K[a * NT_];
#pragma unroll
        for (int b = 1; b < NT_; ++b) {
            const float kab = K[a * NT_ + b];
#pragma unroll
            for (int j = 0; j < TH; ++j)
#pragma unroll
                for (int e = 0; e < VEC; ++e) s[j][e] = __builtin_fmaf(w[j + a][e + b], kab, s[j][e]);
        }
    } else {
        constexpr int n = HI - LO;
        constexpr int half = n >= 8 ? (n > 8 ? 8 : 4) : (n > 4 ? 4 : (n > 2 ? 2 : 1));
        float r[TH][VEC];
        direct_tree<LO, LO + half, NT_, TH, VEC, WN>(w, K, s);
        direct_tree<LO + half, HI, NT_, TH, VEC, WN>(w, K, r);
#pragma unroll
        for (int j = 0; j < TH; ++j)
#pragma unroll
            for (int e = 0; e < VEC; ++e) s[j][e] = s[j][e] + r[j][e];
    }
}


// ---- walking band of the direct form (n >= 7) --------------------------------------
// One wave walks down a band of TH output rows, one row per step.  The n input
// rows of the window and kWalkAhead rows in flight live in a ring of
// Q = n + kWalkAhead slots: once output row j is stored, the slot of input row
// j (its last reader) takes the load of row j + Q, which is first read
// kWalkAhead steps later.  Each input row is loaded and its halos moved across
// lanes once per band rather than once per 4-row band, and only the window and
// the rows in flight are live (FP32: n = 7 124 VGPRs, 4 waves per SIMD; n = 9
// 168, 3 waves; 16-bit storage, 8 values per lane: 165 / 217 VGPRs).  The
// 4-row form loaded all its rows up front: FP32 n = 9 needed 213 VGPRs and
// 16-bit n = 9 345 (one wave per SIMD).  The n x n weights do not fit the
// scalar registers next to the addressing (the compiler parked them in vector
// lanes and read them back, one read-back per ~8 multiply-adds), so each
// workgroup copies them to LDS and each leaf of the pairwise sum reads its n
// just before its chains.  Plain LDS reads were hoisted to the top of the band
// (and pinned the weights in registers), and scheduling barriers do not hold
// arithmetic in place, so each leaf's results pass through empty asm
// statements chained on a token that the next leaf's weight address consumes:
// no value changes, but nothing of leaf a+1 can move above leaf a.  Every
// output is the same pairwise sum of n row chains as direct_tree, in the same
// order, so the results are bitwise those of the 4-row band form.
constexpr int kWalkAhead = 2;  // ring slots beyond the window
// the walking form, which also is the one that reads its weights from LDS:
// from n = 7 on, and at n = 5 in 16-bit storage (FP32 at n = 5 is bound by
// memory, where the 4-row form, which issues all its rows at once, is faster)
template <class D, int R, int MODE> constexpr bool walk_n() {
    return MODE == MODE_DIRECT25 && (R >= 3 || (R == 2 && D::ESZ == 2));
}

// The pairwise sum over kernel rows LO..HI-1 of one output row; leaf(a, s)
// writes row a's chain for the lane's VEC outputs.
template <int LO, int HI, int VEC, class Leaf>
__device__ __forceinline__ void walk_tree(const Leaf &leaf, float (&s)[VEC]) {
    if constexpr (HI - LO == 1) {
        leaf(std::integral_constant<int, LO>{}, s);
    } else {
        constexpr int n = HI - LO;
        constexpr int half = n >= 8 ? (n > 8 ? 8 : 4) : (n > 4 ? 4 : (n > 2 ? 2 : 1));
        float r[VEC];
        walk_tree<LO, LO + half, VEC>(leaf, s);
        walk_tree<LO + half, HI, VEC>(leaf, r);
#pragma unroll
        for (int e = 0; e < VEC; ++e) s[e] = s[e] + r[e];
    }
}

// f(integral_constant<J>) for J = LO, LO+1, ... < HI while f returns true.
template <int LO, int HI, class F> __device__ __forceinline__ void each_step(const F &f) {
    if constexpr (LO < HI) {
        if (f(std::integral_constant<int, LO>{})) each_step<LO + 1, HI>(f);
    }
}

template <class D, bool AL, int R, bool EDGE, int TH, int SAUX>
__device__ __forceinline__ void band_walk(const ImgDev &im, const float *Kl, int plane, int xs, int y0,
                                          int y1, int lane) {
    constexpr int VEC = D::VEC;
    constexpr int NT_ = 2 * R + 1;
    constexpr int Q = NT_ + kWalkAhead;
    constexpr int WN = VEC + 2 * R;
    const int H = im.rows, W = im.cols;
    const int x = xs + lane * VEC;
    bool cm[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) cm[e] = (x + e >= R) && (x + e < W - R);
    const char *sbase = (const char *)im.in + (int64_t)plane * im.pstride * D::ESZ;
    const int64_t sstride = im.pitch * D::ESZ;
    const uint32_t sbytes = (uint32_t)W * D::ESZ;
    char *dbase = (char *)im.out + (int64_t)plane * im.pstride * D::ESZ;
    const int hoff = halo_offset_n<D, R>(xs, W, lane);
    const int nrows = y1 - y0;
    const int last = nrows - 1 + 2 * R;  // last window row of the band, counted from y0 - R
    // rows past the band's last window row are issued with an empty buffer
    // range (no memory access) rather than skipped: a load under a branch makes
    // the compiler's wait counts assume the shorter path and wait for the load
    // issued one step earlier, which removes the prefetch
    const auto issue_row = [&](RawN<D, AL, R> &r, int i) {
        const bool need = i <= last;
        issue_n<D, R>(r, sbase + (int64_t)clampi(y0 - R + i, 0, H - 1) * sstride, need ? sbytes : 0u,
                      x, hoff);
    };

    RawN<D, AL, R> raw[Q];
    float win[Q][WN];
#pragma unroll
    for (int i = 0; i < Q; ++i) issue_row(raw[i], i);
#pragma unroll
    for (int i = 0; i < 2 * R; ++i) decode_n<D, R, true>(raw[i], win[i]);

    // the LDS weight reads are ordered leaf by leaf through an opaque address,
    // kept in one register for the whole band
    float dep = 0.0f;
    uint32_t kaddr = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) float *)Kl;
    // one output row; u = j mod Q, known at compile time, names the ring slots
    const auto step = [&](auto U, int j) {
        constexpr int u = decltype(U)::value;
        if (j >= nrows) return false;
        // FP16 rows are kept as converted FP32 values (dec_kept): mixed-precision
        // FMAs ran this kernel 2-4% slower at n = 5, 7 and 9 (same results)
        decode_n<D, R, true>(raw[(u + 2 * R) % Q], win[(u + 2 * R) % Q]);
        float o[VEC];
        const auto leaf = [&](auto A, float (&s)[VEC]) {
            constexpr int a = decltype(A)::value;
            const float(&w)[WN] = win[(u + a) % Q];
            float k[NT_];
            asm volatile("" : "+v"(kaddr) : "v"(dep));
            const __attribute__((address_space(3))) float *Ka =
                (const __attribute__((address_space(3))) float *)(uintptr_t)kaddr;
#pragma unroll
            for (int b = 0; b < NT_; ++b) k[b] = Ka[a * NT_ + b];
#pragma unroll
            for (int e = 0; e < VEC; ++e) s[e] = w[e] * k[0];
#pragma unroll
            for (int b = 1; b < NT_; ++b)
#pragma unroll
                for (int e = 0; e < VEC; ++e) s[e] = __builtin_fmaf(w[e + b], k[b], s[e]);
#pragma unroll
            for (int e = 0; e < VEC; ++e) asm volatile("" : "+v"(s[e]), "+v"(dep));
        };
        walk_tree<0, NT_, VEC>(leaf, o);
        const int y = y0 + j;
        if constexpr (EDGE) {
            const bool vr = (y >= R) && (y < H - R);
#pragma unroll
            for (int e = 0; e < VEC; ++e) o[e] = (vr && cm[e]) ? o[e] : 0.0f;
        }
        store_out<D, AL, SAUX>(dbase + (int64_t)y * sstride, sbytes, x, o);
        issue_row(raw[u], j + Q);
        return true;
    };
    // every step expanded at compile time: a loop this large is not unrolled, and
    // a loop over ring periods kept copies of the ring at its back edge
    each_step<0, TH>([&](auto J) {
        return step(std::integral_constant<int, decltype(J)::value % Q>{}, decltype(J)::value);
    });
}

// ---- one band ---------------------------------------------------------------------
// MODE: MODE_FUSED (separable, register window), MODE_DIRECT25 (direct n x n
// with tp.K), MODE_ROWPASS / MODE_COLPASS (two-pass kernels).
template <class D, bool AL, int R, int MODE, bool EDGE, int TH, int SAUX = NT>
__device__ __forceinline__ void band_n(const ImgDev &im, const TapsN &tp, const float *Kl, int plane,
                                       int xs, int y0, int y1, int lane) {
    constexpr int VEC = D::VEC;
    constexpr int NT_ = 2 * R + 1;
    const int H = im.rows, W = im.cols;
    const int x = xs + lane * VEC;
    bool cm[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) cm[e] = (x + e >= R) && (x + e < W - R);

    if constexpr (MODE == MODE_ROWPASS) {
        const char *sbase = (const char *)im.in + (int64_t)plane * im.pstride * D::ESZ;
        const int64_t sstride = im.pitch * D::ESZ;
        char *tbase = (char *)(im.tmp + (int64_t)plane * H * W);
        const int hoff = halo_offset_n<D, R>(xs, W, lane);
        RawN<D, AL, R> raw[TH];
#pragma unroll
        for (int i = 0; i < TH; ++i)
            issue_n<D, R>(raw[i], sbase + (int64_t)min(y0 + i, y1 - 1) * sstride,
                          (uint32_t)W * D::ESZ, x, hoff);
#pragma unroll
        for (int i = 0; i < TH; ++i) {
            float v[VEC + 2 * R], h[VEC];
            decode_n<D, R>(raw[i], v);
            hfilter_n<VEC, R>(v, tp.k, h);
            if constexpr (EDGE) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) h[e] = cm[e] ? h[e] : 0.0f;
            }
            if (y0 + i < y1)  // T stays cached for the column kernel
                store_t<VEC, AL, 0>(tbase + (int64_t)(y0 + i) * W * 4, (uint32_t)W * 4, x, h);
        }
        return;
    } else {
        constexpr bool COL = MODE == MODE_COLPASS;
        constexpr bool DIRECT = MODE == MODE_DIRECT25;
        constexpr int WN = DIRECT ? VEC + 2 * R : VEC;
        using RawIn = typename std::conditional<COL, RawT<VEC, AL>, RawN<D, AL, R>>::type;
        const char *sbase;
        int64_t sstride;
        uint32_t sbytes;
        if constexpr (COL) {
            sbase = (const char *)(im.tmp + (int64_t)plane * H * W);
            sstride = (int64_t)W * 4;
            sbytes = (uint32_t)W * 4;
        } else {
            sbase = (const char *)im.in + (int64_t)plane * im.pstride * D::ESZ;
            sstride = im.pitch * D::ESZ;
            sbytes = (uint32_t)W * D::ESZ;
        }
        char *dbase = (char *)im.out + (int64_t)plane * im.pstride * D::ESZ;
        const int64_t dstride = im.pitch * D::ESZ;
        const int hoff = halo_offset_n<D, R>(xs, W, lane);
        RawIn raw[TH + 2 * R];
#pragma unroll
        for (int i = 0; i < TH + 2 * R; ++i) {
            const char *p = sbase + (int64_t)clampi(y0 - R + i, 0, H - 1) * sstride;
            if constexpr (COL)
                issue_t<VEC, AL>(raw[i], p, sbytes, x);
            else
                issue_n<D, R>(raw[i], p, sbytes, x, hoff);
        }
        float w[TH + 2 * R][WN];
        float dsum[DIRECT ? TH : 1][VEC];
#pragma unroll
        for (int i = 0; i < TH + 2 * R; ++i) {
            if constexpr (COL) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) w[i][e] = __uint_as_float(raw[i].w[e]);
            } else if constexpr (DIRECT) {
                decode_n<D, R>(raw[i], w[i]);
            } else {
                float v[VEC + 2 * R];
                decode_n<D, R>(raw[i], v);
                hfilter_n<VEC, R>(v, tp.k, w[i]);
            }
        }
        if constexpr (DIRECT) direct_tree<0, NT_, NT_, TH, VEC, WN>(w, tp.K, dsum);
#pragma unroll
        for (int j = 0; j < TH; ++j) {
            const int y = y0 + j;
            if (y >= y1) break;
            float o[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if constexpr (DIRECT) {
                    o[e] = dsum[j][e];
                } else {
                    float t = w[j][e] * tp.k[0];
#pragma unroll
                    for (int a = 1; a < NT_; ++a) t = __builtin_fmaf(w[j + a][e], tp.k[a], t);
                    o[e] = t;
                }
            }
            if constexpr (EDGE) {
                const bool vr = (y >= R) && (y < H - R);
#pragma unroll
                for (int e = 0; e < VEC; ++e) o[e] = (vr && cm[e]) ? o[e] : 0.0f;
            }
            store_out<D, AL, SAUX>(dbase + (int64_t)y * dstride, (uint32_t)W * D::ESZ, x, o);
        }
    }
}

template <class D, bool AL, int R, int MODE, int WAVES, int TH, int SAUX = NT>
__device__ __forceinline__ void run_tile_n(const ImgDev &im, const TapsN &tp, const float *Kl,
                                           int64_t lt, int wave, int lane) {
    const int sg = (int)(lt % im.nsg);
    const int64_t t = lt / im.nsg;
    const int band = (int)(t % im.nb);
    const int plane = (int)(t / im.nb);
    const int strip = sg * WAVES + wave;
    if (strip >= im.ns) return;
    const int xs = strip * (WAVE * D::VEC);
    const int y0 = band * TH;
    const int y1 = min(y0 + TH, im.rows);
    const bool col_edge = xs < R || xs + WAVE * D::VEC > im.cols - R;
    const bool row_edge = MODE != MODE_ROWPASS && (y0 < R || y0 + TH > im.rows - R);
    if constexpr (walk_n<D, R, MODE>()) {
        if (col_edge || row_edge)
            band_walk<D, AL, R, true, TH, SAUX>(im, Kl, plane, xs, y0, y1, lane);
        else
            band_walk<D, AL, R, false, TH, SAUX>(im, Kl, plane, xs, y0, y1, lane);
    } else if (col_edge || row_edge) {
        band_n<D, AL, R, MODE, true, TH, SAUX>(im, tp, Kl, plane, xs, y0, y1, lane);
    } else {
        band_n<D, AL, R, MODE, false, TH, SAUX>(im, tp, Kl, plane, xs, y0, y1, lane);
    }
}

// One workgroup per logical tile (grids above 2^20 workgroups loop); with
// xcd_slabs = c >= 2 the XCDs take turns on chunks of c band rows, as in the
// width-5 kernels.
template <class D, bool AL, int R, int MODE, int WAVES, int TH, int SAUX = NT>
__global__ __launch_bounds__(WAVE *WAVES) void k_image_n(ImgDev im, TapsN tp, int64_t nblocks) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const float *Kl = nullptr;
    if constexpr (walk_n<D, R, MODE>()) {
        constexpr int NK = (2 * R + 1) * (2 * R + 1);
        __shared__ float sK[NK];
        for (int i = threadIdx.x; i < NK; i += WAVE * WAVES) sK[i] = tp.K[i];
        __syncthreads();
        Kl = sK;
    }
    for (int64_t base = 0; base < nblocks; base += gridDim.x) {
        const int64_t left = nblocks - base;
        const int cnt = left < (int64_t)gridDim.x ? (int)left : (int)gridDim.x;
        if ((int)blockIdx.x >= cnt) break;
        const int b = im.xcd_slabs > 1
                          ? xcd_chunk_remap(blockIdx.x, cnt, (int64_t)im.xcd_slabs * im.nsg)
                          : (int)blockIdx.x;
        run_tile_n<D, AL, R, MODE, WAVES, TH, SAUX>(im, tp, Kl, base + b, wave, lane);
    }
}

// Band heights and workgroup widths of the width-n kernels (shared with the
// host, which builds the tile geometry).
template <class D> struct GeomN {
    static constexpr int WAVES = waves_n(D::ESZ == 4 ? 0 : 1);
    static constexpr int TH_SEP = kThSepN;
};

template <class D, bool AL, int R, int MODE>
hipError_t launch_n_m(const ImgDev &im, const TapsN &tp, int64_t nblocks, hipStream_t s) {
    constexpr int W = GeomN<D>::WAVES;
    constexpr int TH = MODE == MODE_DIRECT25 ? th_direct_n(D::ESZ == 4, R)
                                             : GeomN<D>::TH_SEP;
    static_assert(walk_n<D, R, MODE>() == (MODE == MODE_DIRECT25 && TH == kThWalkN),
                  "the host's band height must match the kernel form");
    const int grid = (int)(nblocks < (1 << 20) ? nblocks : (1 << 20));
    // keep_out (the copy-back scratch): cached output stores in kernels of
    // their own
    if constexpr (MODE == MODE_FUSED || MODE == MODE_DIRECT25) {
        if (im.keep_out) {
            hipLaunchKernelGGL((k_image_n<D, AL, R, MODE, W, TH, 0>), dim3(grid), dim3(WAVE * W), 0, s,
                               im, tp, nblocks);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_image_n<D, AL, R, MODE, W, TH>), dim3(grid), dim3(WAVE * W), 0, s, im, tp,
                       nblocks);
    return hipGetLastError();
}

template <class D, bool AL, int R>
hipError_t launch_n_r(const ImgDev &im, const TapsN &tp, int mode, int64_t nblocks, hipStream_t s) {
    switch (mode) {
    case MODE_FUSED: return launch_n_m<D, AL, R, MODE_FUSED>(im, tp, nblocks, s);
    case MODE_DIRECT25: return launch_n_m<D, AL, R, MODE_DIRECT25>(im, tp, nblocks, s);
    case MODE_ROWPASS: return launch_n_m<D, AL, R, MODE_ROWPASS>(im, tp, nblocks, s);
    default: return launch_n_m<D, AL, R, MODE_COLPASS>(im, tp, nblocks, s);
    }
}

template <class D, bool AL>
hipError_t launch_n_a(const ImgDev &im, const TapsN &tp, int radius, int mode, int64_t nblocks,
                      hipStream_t s) {
    switch (radius) {
    case 0: return launch_n_r<D, AL, 0>(im, tp, mode, nblocks, s);
    case 1: return launch_n_r<D, AL, 1>(im, tp, mode, nblocks, s);
    case 2: return launch_n_r<D, AL, 2>(im, tp, mode, nblocks, s);
    case 3: return launch_n_r<D, AL, 3>(im, tp, mode, nblocks, s);
    default: return launch_n_r<D, AL, 4>(im, tp, mode, nblocks, s);
    }
}

template <class D>
hipError_t launch_image_n_t(const ImgDev &im, const TapsN &tp, int radius, int mode,
                            int64_t nblocks, hipStream_t s) {
    return im.aligned ? launch_n_a<D, true>(im, tp, radius, mode, nblocks, s)
                      : launch_n_a<D, false>(im, tp, radius, mode, nblocks, s);
}

// The width-5 direct 25-tap form in 16-bit storage, on its 16-row walking
// geometry, runs the walking band above at n = 5: the same products K = k k^T
// (rounded once on the host) and the same pairwise row sums, so the results are
// bitwise those of the width-5 walking band, which it outruns (3x4096x4096:
// FP16 50 -> 47 us, BF16 48 -> 43.5 us).  The descriptor is the width-5 one.
template <class D>
hipError_t launch_direct25_walk(const ImgDev &im, int64_t nblocks, hipStream_t s) {
    static_assert(D::ESZ == 2 && walk_n<D, 2, MODE_DIRECT25>(), "16-bit storage walks at n = 5");
    TapsN tp;
    std::memset(&tp, 0, sizeof tp);
    for (int i = 0; i < 5; ++i) tp.k[i] = im.tp.k[i];
    for (int i = 0; i < 25; ++i) tp.K[i] = im.tp.K[i];
    return im.aligned ? launch_n_m<D, true, 2, MODE_DIRECT25>(im, tp, nblocks, s)
                      : launch_n_m<D, false, 2, MODE_DIRECT25>(im, tp, nblocks, s);
}

}  // namespace
}  // namespace convsep5
