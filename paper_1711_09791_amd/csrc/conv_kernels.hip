// conv_kernels.hip -- gfx950 kernels of the width-5 separable convolution.
//
// Operation: Eq. 1 of arXiv 1711.09791 (Section 1) with K[i][j] = k_i k_j,
// correlation form, computed on pixels whose 5x5 neighbourhood is inside the
// image (Section 4); the 2-pixel frame is written as +0.0.
//
// Work decomposition (one wavefront = one tile):
//   * a lane owns VEC = 16 bytes of consecutive columns of storage (4 FP32 or
//     8 FP16/BF16), so one wavefront row access is 1 KiB of contiguous,
//     fully coalesced memory;
//   * a tile is a column strip of 64*VEC columns times a band of `th` output
//     rows of one plane; the wavefront walks down the band row by row;
//   * horizontal neighbours come from the adjacent lanes through DPP
//     wave_shr:1 / wave_shl:1 moves; lane 0 and lane 63 fetch the 2-column
//     halo outside the strip themselves;
//   * the vertical 5-row window (row-filtered rows, or raw rows for the
//     direct form) lives in VGPRs and rotates through five register slots
//     with no moves (the loop is unrolled by 5);
//   * input rows are prefetched 5 rows ahead into a ring of raw registers;
//   * all global accesses are raw buffer instructions on a per-row buffer
//     resource whose size is the row's byte length: lanes past the right
//     edge read 0 and their stores are dropped by the hardware range check,
//     so no lane ever diverges and no address is ever clamped per lane.
//
// Arithmetic (identical in every kernel and every tile shape):
//   horizontal  h = A[x-2]*k0; h = fma(A[x-1],k1,h); ...; h = fma(A[x+2],k4,h)
//   vertical    o = h[y-2]*k0; o = fma(h[y-1],k1,o); ...; o = fma(h[y+2],k4,o)
//   direct25    p_a = chain over the 5 taps of kernel row a with K[a][b];
//               o = ((p_0 + p_1) + (p_2 + p_3)) + p_4
// Built with -ffp-contract=off so that nothing else is fused.
#include "conv_internal.h"

#include <type_traits>

namespace convsep5 {
namespace {

typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));

constexpr int WAVE = 64;
constexpr int NT = 2;                      // buffer store cache policy: nt (streaming)
constexpr int OOB = (int)0x80000000;       // an offset beyond any row (rows < 2^30 bytes)
constexpr int RSRC_WORD3 = 0x00020000;     // raw buffer, 32-bit data format

struct F32 { static constexpr int ESZ = 4, VEC = 4; };
struct F16 { static constexpr int ESZ = 2, VEC = 8; };
struct BF16 { static constexpr int ESZ = 2, VEC = 8; };

// ---- storage conversions -------------------------------------------------
__device__ __forceinline__ float dec(F32, uint32_t b) { return __uint_as_float(b); }
__device__ __forceinline__ float dec(F16, uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
}
__device__ __forceinline__ float dec(BF16, uint32_t b) { return __uint_as_float(b << 16); }

__device__ __forceinline__ uint32_t enc(F32, float f) { return __float_as_uint(f); }
__device__ __forceinline__ uint32_t enc(F16, float f) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f);  // v_cvt_f16_f32, RNE
}
__device__ __forceinline__ uint32_t enc(BF16, float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// ---- buffer resources, DPP ----------------------------------------------
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             RSRC_WORD3);
}
// lane i receives lane i-1's value; lane 0 keeps `old`.
__device__ __forceinline__ uint32_t from_left(uint32_t src, uint32_t old) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x138, 0xf, 0xf, false);
}
// lane i receives lane i+1's value; lane 63 keeps `old`.
__device__ __forceinline__ uint32_t from_right(uint32_t src, uint32_t old) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x130, 0xf, 0xf, false);
}

// ---- one raw input row per lane: VEC elements + 2-column halos ------------
template <class D, bool AL> struct Raw;
template <class D> struct Raw<D, true> { u4 m; uint32_t h0, h1; };
template <class D> struct Raw<D, false> { uint32_t e[D::VEC + 4]; };

// Aligned: one 16-byte load per lane; lane 0 / lane 63 also load the two
// elements left / right of the strip (offset `hoff`, OOB for other lanes).
template <class D>
__device__ __forceinline__ void issue(Raw<D, true> &r, const char *row, uint32_t rbytes, int x,
                                      int hoff) {
    const auto rs = row_rsrc(row, rbytes);
    r.m = __builtin_amdgcn_raw_buffer_load_b128(rs, x * D::ESZ, 0, 0);
    if constexpr (D::ESZ == 4) {
        const u2 h = __builtin_amdgcn_raw_buffer_load_b64(rs, hoff, 0, 0);
        r.h0 = h.x;
        r.h1 = h.y;
    } else {
        r.h0 = __builtin_amdgcn_raw_buffer_load_b32(rs, hoff, 0, 0);
        r.h1 = 0;
    }
}
// Unaligned layouts: element loads of columns x-2 .. x+VEC+1; columns left
// of 0 get an explicit out-of-range offset, columns >= W fail the range check.
template <class D>
__device__ __forceinline__ void issue(Raw<D, false> &r, const char *row, uint32_t rbytes, int x,
                                      int) {
    const auto rs = row_rsrc(row, rbytes);
#pragma unroll
    for (int e = 0; e < D::VEC + 4; ++e) {
        const int c = x - 2 + e;
        const int off = c >= 0 ? c * D::ESZ : OOB;
        if constexpr (D::ESZ == 4)
            r.e[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        else
            r.e[e] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
    }
}

// v[i] = A[x - 2 + i], i = 0 .. VEC+3, as FP32.
template <class D>
__device__ __forceinline__ void decode(const Raw<D, true> &r, float (&v)[D::VEC + 4]) {
    if constexpr (D::ESZ == 4) {
        v[0] = __uint_as_float(from_left(r.m.z, r.h0));
        v[1] = __uint_as_float(from_left(r.m.w, r.h1));
        v[2] = __uint_as_float(r.m.x);
        v[3] = __uint_as_float(r.m.y);
        v[4] = __uint_as_float(r.m.z);
        v[5] = __uint_as_float(r.m.w);
        v[6] = __uint_as_float(from_right(r.m.x, r.h0));
        v[7] = __uint_as_float(from_right(r.m.y, r.h1));
    } else {
        const uint32_t l = from_left(r.m.w, r.h0);
        const uint32_t rr = from_right(r.m.x, r.h0);
        const uint32_t w[4] = {r.m.x, r.m.y, r.m.z, r.m.w};
        v[0] = dec(D{}, l);
        v[1] = dec(D{}, l >> 16);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            v[2 + 2 * i] = dec(D{}, w[i]);
            v[3 + 2 * i] = dec(D{}, w[i] >> 16);
        }
        v[10] = dec(D{}, rr);
        v[11] = dec(D{}, rr >> 16);
    }
}
template <class D>
__device__ __forceinline__ void decode(const Raw<D, false> &r, float (&v)[D::VEC + 4]) {
#pragma unroll
    for (int e = 0; e < D::VEC + 4; ++e) v[e] = dec(D{}, r.e[e]);
}

// ---- FP32 intermediate rows (two-pass) -------------------------------------
template <int N, bool AL> struct RawT { uint32_t w[N]; };

template <int N, bool AL>
__device__ __forceinline__ void issue_t(RawT<N, AL> &r, const char *row, uint32_t rbytes, int x) {
    const auto rs = row_rsrc(row, rbytes);
    if constexpr (AL) {
#pragma unroll
        for (int j = 0; j < N / 4; ++j) {
            const u4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, (x + 4 * j) * 4, 0, 0);
            r.w[4 * j + 0] = q.x;
            r.w[4 * j + 1] = q.y;
            r.w[4 * j + 2] = q.z;
            r.w[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < N; ++e)
            r.w[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, (x + e) * 4, 0, 0);
    }
}

template <int N, bool AL>
__device__ __forceinline__ void store_t(char *row, uint32_t rbytes, int x, const float (&o)[N]) {
    const auto rs = row_rsrc(row, rbytes);
    if constexpr (AL) {
#pragma unroll
        for (int j = 0; j < N / 4; ++j) {
            const u4 q = {__float_as_uint(o[4 * j]), __float_as_uint(o[4 * j + 1]),
                          __float_as_uint(o[4 * j + 2]), __float_as_uint(o[4 * j + 3])};
            __builtin_amdgcn_raw_buffer_store_b128(q, rs, (x + 4 * j) * 4, 0, NT);
        }
    } else {
#pragma unroll
        for (int e = 0; e < N; ++e)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o[e]), rs, (x + e) * 4, 0, NT);
    }
}

// ---- output rows in the storage type ------------------------------------
template <class D, bool AL>
__device__ __forceinline__ void store_out(char *row, uint32_t rbytes, int x,
                                          const float (&o)[D::VEC]) {
    const auto rs = row_rsrc(row, rbytes);
    if constexpr (AL) {
        u4 q;
        if constexpr (D::ESZ == 4) {
            q = u4{enc(D{}, o[0]), enc(D{}, o[1]), enc(D{}, o[2]), enc(D{}, o[3])};
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                q[i] = enc(D{}, o[2 * i]) | (enc(D{}, o[2 * i + 1]) << 16);
        }
        __builtin_amdgcn_raw_buffer_store_b128(q, rs, x * D::ESZ, 0, NT);
    } else {
#pragma unroll
        for (int e = 0; e < D::VEC; ++e) {
            if constexpr (D::ESZ == 4)
                __builtin_amdgcn_raw_buffer_store_b32(enc(D{}, o[e]), rs, (x + e) * 4, 0, NT);
            else
                __builtin_amdgcn_raw_buffer_store_b16((uint16_t)enc(D{}, o[e]), rs, (x + e) * 2,
                                                      0, NT);
        }
    }
}

// ---- the arithmetic ----------------------------------------------------------
template <int N>
__device__ __forceinline__ void hfilter(const float (&v)[N + 4], const float *k, float (&h)[N]) {
#pragma unroll
    for (int e = 0; e < N; ++e) {
        float t = v[e] * k[0];
        t = __builtin_fmaf(v[e + 1], k[1], t);
        t = __builtin_fmaf(v[e + 2], k[2], t);
        t = __builtin_fmaf(v[e + 3], k[3], t);
        t = __builtin_fmaf(v[e + 4], k[4], t);
        h[e] = t;
    }
}

template <int N>
__device__ __forceinline__ void vfilter(const float (&a)[N], const float (&b)[N],
                                        const float (&c)[N], const float (&d)[N],
                                        const float (&e)[N], const float *k, float (&o)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        float t = a[i] * k[0];
        t = __builtin_fmaf(b[i], k[1], t);
        t = __builtin_fmaf(c[i], k[2], t);
        t = __builtin_fmaf(d[i], k[3], t);
        t = __builtin_fmaf(e[i], k[4], t);
        o[i] = t;
    }
}

template <int N>
__device__ __forceinline__ float row5(const float (&r)[N + 4], int i, const float *Ka) {
    float p = r[i] * Ka[0];
    p = __builtin_fmaf(r[i + 1], Ka[1], p);
    p = __builtin_fmaf(r[i + 2], Ka[2], p);
    p = __builtin_fmaf(r[i + 3], Ka[3], p);
    p = __builtin_fmaf(r[i + 4], Ka[4], p);
    return p;
}

template <int N>
__device__ __forceinline__ void direct25(const float (&r0)[N + 4], const float (&r1)[N + 4],
                                         const float (&r2)[N + 4], const float (&r3)[N + 4],
                                         const float (&r4)[N + 4], const float *K,
                                         float (&o)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float p0 = row5<N>(r0, i, K + 0);
        const float p1 = row5<N>(r1, i, K + 5);
        const float p2 = row5<N>(r2, i, K + 10);
        const float p3 = row5<N>(r3, i, K + 15);
        const float p4 = row5<N>(r4, i, K + 20);
        o[i] = ((p0 + p1) + (p2 + p3)) + p4;
    }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---- one band of a vertical-filter kernel (fused, direct25, column pass) ----
template <class D, bool AL, int MODE>
__device__ __forceinline__ void band_vertical(const ImgDev &im, int plane, int xs, int y0, int y1,
                                              int lane) {
    constexpr int VEC = D::VEC;
    constexpr bool DIRECT = MODE == MODE_DIRECT25;
    constexpr bool COL = MODE == MODE_COLPASS;
    constexpr int WN = DIRECT ? VEC + 4 : VEC;
    using RawIn = typename std::conditional<COL, RawT<VEC, AL>, Raw<D, AL>>::type;

    const int H = im.rows, W = im.cols;
    const int x = xs + lane * VEC;
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
    const uint32_t dbytes = (uint32_t)W * D::ESZ;
    const int hl = xs - 2, hr = xs + WAVE * VEC;
    const int hoff = lane == 0 ? (hl >= 0 ? hl * D::ESZ : OOB)
                               : (lane == WAVE - 1 ? (hr < W ? hr * D::ESZ : OOB) : OOB);
    bool cm[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) cm[e] = (x + e >= 2) && (x + e < W - 2);
    const int rlim = min(y1 + 1, H - 1);

    auto fetch = [&](RawIn &r, int row) {
        const char *p = sbase + (int64_t)clampi(row, 0, rlim) * sstride;
        if constexpr (COL)
            issue_t<VEC, AL>(r, p, sbytes, x);
        else
            issue<D>(r, p, sbytes, x, hoff);
    };
    auto produce = [&](const RawIn &r, float (&w)[WN]) {
        if constexpr (COL) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) w[e] = __uint_as_float(r.w[e]);
        } else if constexpr (DIRECT) {
            decode<D>(r, w);
        } else {
            float v[VEC + 4];
            decode<D>(r, v);
            hfilter<VEC>(v, im.tp.k, w);
        }
    };
    auto emit = [&](int y, const float (&a)[WN], const float (&b)[WN], const float (&c)[WN],
                    const float (&d)[WN], const float (&e)[WN]) {
        float o[VEC];
        if constexpr (DIRECT)
            direct25<VEC>(a, b, c, d, e, im.tp.K, o);
        else
            vfilter<VEC>(a, b, c, d, e, im.tp.k, o);
        const bool vr = (y >= 2) && (y < H - 2);
#pragma unroll
        for (int i = 0; i < VEC; ++i) o[i] = (vr && cm[i]) ? o[i] : 0.0f;
        store_out<D, AL>(dbase + (int64_t)y * dstride, dbytes, x, o);
    };

    float w[5][WN];
    RawIn ring[5];
    {
        RawIn p0, p1, p2, p3;
        fetch(p0, y0 - 2);
        fetch(p1, y0 - 1);
        fetch(p2, y0);
        fetch(p3, y0 + 1);
        produce(p0, w[0]);
        produce(p1, w[1]);
        produce(p2, w[2]);
        produce(p3, w[3]);
    }
    fetch(ring[4], y0 + 2);
    fetch(ring[0], y0 + 3);
    fetch(ring[1], y0 + 4);
    fetch(ring[2], y0 + 5);
    fetch(ring[3], y0 + 6);

    int y = y0;
    // Output row y: slot S holds row y+2 (just produced), (S+4)%5 row y+1,
    // (S+3)%5 row y, (S+2)%5 row y-1, (S+1)%5 row y-2.  ring[S] holds row
    // y+2 on entry and is refilled with row y+7.
#define CONV_VSTEP(S)                                                                   \
    {                                                                                    \
        produce(ring[S], w[S]);                                                          \
        fetch(ring[S], y + 7);                                                           \
        emit(y, w[((S) + 1) % 5], w[((S) + 2) % 5], w[((S) + 3) % 5], w[((S) + 4) % 5], \
             w[S]);                                                                      \
        ++y;                                                                             \
    }
    while (y + 5 <= y1) {
        CONV_VSTEP(4) CONV_VSTEP(0) CONV_VSTEP(1) CONV_VSTEP(2) CONV_VSTEP(3)
    }
    if (y < y1) {
        CONV_VSTEP(4)
        if (y < y1) {
            CONV_VSTEP(0)
            if (y < y1) {
                CONV_VSTEP(1)
                if (y < y1) CONV_VSTEP(2)
            }
        }
    }
#undef CONV_VSTEP
}

// ---- one band of the two-pass row kernel -------------------------------------
template <class D, bool AL>
__device__ __forceinline__ void band_rowpass(const ImgDev &im, int plane, int xs, int y0, int y1,
                                             int lane) {
    constexpr int VEC = D::VEC;
    const int H = im.rows, W = im.cols;
    const int x = xs + lane * VEC;
    const char *sbase = (const char *)im.in + (int64_t)plane * im.pstride * D::ESZ;
    const int64_t sstride = im.pitch * D::ESZ;
    const uint32_t sbytes = (uint32_t)W * D::ESZ;
    char *tbase = (char *)(im.tmp + (int64_t)plane * H * W);
    const int64_t tstride = (int64_t)W * 4;
    const uint32_t tbytes = (uint32_t)W * 4;
    const int hl = xs - 2, hr = xs + WAVE * VEC;
    const int hoff = lane == 0 ? (hl >= 0 ? hl * D::ESZ : OOB)
                               : (lane == WAVE - 1 ? (hr < W ? hr * D::ESZ : OOB) : OOB);
    bool cm[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) cm[e] = (x + e >= 2) && (x + e < W - 2);
    const int rlim = y1 - 1;

    auto fetch = [&](Raw<D, AL> &r, int row) {
        issue<D>(r, sbase + (int64_t)min(row, rlim) * sstride, sbytes, x, hoff);
    };
    Raw<D, AL> ring[5];
    fetch(ring[0], y0);
    fetch(ring[1], y0 + 1);
    fetch(ring[2], y0 + 2);
    fetch(ring[3], y0 + 3);
    fetch(ring[4], y0 + 4);
    int y = y0;
#define CONV_RSTEP(S)                                                   \
    {                                                                    \
        float v[VEC + 4], h[VEC];                                        \
        decode<D>(ring[S], v);                                           \
        fetch(ring[S], y + 5);                                           \
        hfilter<VEC>(v, im.tp.k, h);                                     \
        _Pragma("unroll") for (int i = 0; i < VEC; ++i) h[i] = cm[i] ? h[i] : 0.0f; \
        store_t<VEC, AL>(tbase + (int64_t)y * tstride, tbytes, x, h);    \
        ++y;                                                             \
    }
    while (y + 5 <= y1) {
        CONV_RSTEP(0) CONV_RSTEP(1) CONV_RSTEP(2) CONV_RSTEP(3) CONV_RSTEP(4)
    }
    if (y < y1) {
        CONV_RSTEP(0)
        if (y < y1) {
            CONV_RSTEP(1)
            if (y < y1) {
                CONV_RSTEP(2)
                if (y < y1) CONV_RSTEP(3)
            }
        }
    }
#undef CONV_RSTEP
}

// ---- tiles -----------------------------------------------------------------
// Logical tile lt = (plane, strip group, band), band fastest.  Wave `wave` of
// the workgroup takes strip sg*WAVES + wave of the group.
template <class D, bool AL, int MODE, int WAVES>
__device__ __forceinline__ void run_tile(const ImgDev &im, int64_t lt, int wave, int lane) {
    const int64_t per_plane = (int64_t)im.nsg * im.nb;
    const int plane = (int)(lt / per_plane);
    const int64_t rem = lt - (int64_t)plane * per_plane;
    const int sg = (int)(rem / im.nb);
    const int band = (int)(rem - (int64_t)sg * im.nb);
    const int strip = sg * WAVES + wave;
    if (strip >= im.ns) return;
    const int xs = strip * (WAVE * D::VEC);
    const int y0 = band * im.th;
    const int y1 = min(y0 + im.th, im.rows);
    if constexpr (MODE == MODE_ROWPASS)
        band_rowpass<D, AL>(im, plane, xs, y0, y1, lane);
    else
        band_vertical<D, AL, MODE>(im, plane, xs, y0, y1, lane);
}

// Workgroups are handed to the 8 XCDs round-robin (block b -> XCD b % 8).
// Renumber them so that each XCD gets one contiguous run of logical blocks:
// vertically adjacent bands, which share halo rows, then meet in one L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    constexpr int X = 8;
    const int q = n / X, r = n % X;
    const int xcd = b % X, i = b / X;
    return xcd * q + min(xcd, r) + i;
}

template <class D, bool AL, int MODE, int WAVES>
__global__ __launch_bounds__(WAVE *WAVES) void k_image(ImgDev im, int64_t nblocks) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    for (int64_t base = 0; base < nblocks; base += gridDim.x) {
        const int64_t left = nblocks - base;
        const int cnt = left < (int64_t)gridDim.x ? (int)left : (int)gridDim.x;
        if ((int)blockIdx.x >= cnt) break;
        run_tile<D, AL, MODE, WAVES>(im, base + xcd_remap(blockIdx.x, cnt), wave, lane);
    }
}

// Persistent batch kernel: the grid is a fixed multiple of the CU count; each
// workgroup takes one contiguous run of the launch's tiles (images in order,
// then plane, strip group, band), finds the image owning each tile from the
// descriptor table's tile ranges, and runs it.
template <class D, int MODE, int WAVES>
__global__ __launch_bounds__(WAVE *WAVES) void k_batch(const ImgDev *__restrict__ descs, int n,
                                                       int64_t total) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int G = gridDim.x;
    const int64_t L = xcd_remap(blockIdx.x, G);
    const int64_t t0 = total * L / G, t1 = total * (L + 1) / G;
    if (t0 >= t1) return;
    int lo = 0, hi = n - 1;  // last image whose first tile is <= t0
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile_begin <= t0) lo = mid;
        else hi = mid - 1;
    }
    int i = lo;
    for (int64_t t = t0; t < t1; ++t) {
        while (t >= descs[i].tile_end) ++i;
        const ImgDev &im = descs[i];
        if (im.aligned)
            run_tile<D, true, MODE, WAVES>(im, t - im.tile_begin, wave, lane);
        else
            run_tile<D, false, MODE, WAVES>(im, t - im.tile_begin, wave, lane);
    }
}

// ---- dispatch ----------------------------------------------------------------
template <class D, bool AL, int MODE>
hipError_t launch_image_w(const ImgDev &im, int waves, int64_t nblocks, hipStream_t s) {
    const int grid = (int)(nblocks < (1 << 20) ? nblocks : (1 << 20));
    switch (waves) {
    case 1: hipLaunchKernelGGL((k_image<D, AL, MODE, 1>), dim3(grid), dim3(WAVE), 0, s, im, nblocks); break;
    case 2: hipLaunchKernelGGL((k_image<D, AL, MODE, 2>), dim3(grid), dim3(2 * WAVE), 0, s, im, nblocks); break;
    default: hipLaunchKernelGGL((k_image<D, AL, MODE, 4>), dim3(grid), dim3(4 * WAVE), 0, s, im, nblocks); break;
    }
    return hipGetLastError();
}

template <class D, bool AL>
hipError_t launch_image_m(const ImgDev &im, int mode, int waves, int64_t nblocks, hipStream_t s) {
    switch (mode) {
    case MODE_FUSED: return launch_image_w<D, AL, MODE_FUSED>(im, waves, nblocks, s);
    case MODE_DIRECT25: return launch_image_w<D, AL, MODE_DIRECT25>(im, waves, nblocks, s);
    case MODE_ROWPASS: return launch_image_w<D, AL, MODE_ROWPASS>(im, waves, nblocks, s);
    default: return launch_image_w<D, AL, MODE_COLPASS>(im, waves, nblocks, s);
    }
}

template <class D>
hipError_t launch_image_a(const ImgDev &im, int mode, int waves, int64_t nblocks, hipStream_t s) {
    return im.aligned ? launch_image_m<D, true>(im, mode, waves, nblocks, s)
                      : launch_image_m<D, false>(im, mode, waves, nblocks, s);
}

template <class D, int MODE>
hipError_t launch_batch_w(const ImgDev *d, int n, int64_t total, int waves, int grid,
                          hipStream_t s) {
    switch (waves) {
    case 1: hipLaunchKernelGGL((k_batch<D, MODE, 1>), dim3(grid), dim3(WAVE), 0, s, d, n, total); break;
    case 2: hipLaunchKernelGGL((k_batch<D, MODE, 2>), dim3(grid), dim3(2 * WAVE), 0, s, d, n, total); break;
    default: hipLaunchKernelGGL((k_batch<D, MODE, 4>), dim3(grid), dim3(4 * WAVE), 0, s, d, n, total); break;
    }
    return hipGetLastError();
}

template <class D>
hipError_t launch_batch_m(const ImgDev *d, int n, int64_t total, int mode, int waves, int grid,
                          hipStream_t s) {
    return mode == MODE_DIRECT25 ? launch_batch_w<D, MODE_DIRECT25>(d, n, total, waves, grid, s)
                                 : launch_batch_w<D, MODE_FUSED>(d, n, total, waves, grid, s);
}

}  // namespace

hipError_t launch_image(const ImgDev &im, int dtype, int mode, int waves, int64_t nblocks,
                        hipStream_t s) {
    switch (dtype) {
    case 0: return launch_image_a<F32>(im, mode, waves, nblocks, s);
    case 1: return launch_image_a<F16>(im, mode, waves, nblocks, s);
    default: return launch_image_a<BF16>(im, mode, waves, nblocks, s);
    }
}

hipError_t launch_batch(const ImgDev *d_descs, int n, int64_t total_tiles, int dtype, int mode,
                        int waves, int grid, hipStream_t s) {
    switch (dtype) {
    case 0: return launch_batch_m<F32>(d_descs, n, total_tiles, mode, waves, grid, s);
    case 1: return launch_batch_m<F16>(d_descs, n, total_tiles, mode, waves, grid, s);
    default: return launch_batch_m<BF16>(d_descs, n, total_tiles, mode, waves, grid, s);
    }
}

}  // namespace convsep5
