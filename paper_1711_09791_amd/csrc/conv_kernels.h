// conv_kernels.h -- gfx950 kernels of the width-5 separable convolution
// (templates; instantiated per storage type by conv_kernels_{f32,f16,bf16}.hip).
//
// Operation: Eq. 1 of arXiv 1711.09791 (Section 1) with K[i][j] = k_i k_j,
// correlation form, computed on pixels whose 5x5 neighbourhood is inside the
// image (Section 5, opening paragraph); the 2-pixel frame is written as +0.0.
//
// Work decomposition (one wavefront = one tile):
//   * a lane owns VEC = 16 bytes of consecutive columns of storage (4 FP32 or
//     8 FP16/BF16), so one wavefront row access is 1 KiB of contiguous,
//     fully coalesced memory;
//   * a tile is a column strip of 64*VEC columns times a band of `th` output
//     rows of one plane.  Tiles are numbered strip-fastest (plane, band,
//     strip group), so the waves resident at any moment cover whole image
//     rows of a compact window that sweeps down the image (DRAM page
//     locality); with the round-robin workgroup-to-XCD dispatch, a column
//     strip then stays on one XCD whenever the strip-group count is a
//     multiple of 8, so the halo rows shared by vertically adjacent bands
//     meet in that XCD's L2;
//   * bands of 4 or 8 rows are fully unrolled: all th+4 input rows are
//     loaded before the first is used; other heights walk down the band
//     with a 5-row prefetch ring;
//   * horizontal neighbours come from the adjacent lanes through DPP
//     wave_shr:1 / wave_shl:1 moves; lane 0 and lane 63 fetch the 2-column
//     halo outside the strip themselves;
//   * the vertical 5-row window (row-filtered rows, or raw rows for the
//     direct form) lives in VGPRs; in the walking form it rotates through
//     five register slots with no moves (the loop is unrolled by 5);
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
#pragma once

#include "conv_internal.h"

#include <cstring>
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

// The two-pass kernels and the storage type of their intermediate.
constexpr bool is_rowpass(int m) {
    return m == MODE_ROWPASS || m == MODE_ROWPASS_F16T || m == MODE_ROWPASS_BF16T;
}
constexpr bool is_colpass(int m) {
    return m == MODE_COLPASS || m == MODE_COLPASS_F16T || m == MODE_COLPASS_BF16T;
}
template <int MODE> struct TmpOf { using T = F32; };
template <> struct TmpOf<MODE_ROWPASS_F16T> { using T = F16; };
template <> struct TmpOf<MODE_COLPASS_F16T> { using T = F16; };
template <> struct TmpOf<MODE_ROWPASS_BF16T> { using T = BF16; };
template <> struct TmpOf<MODE_COLPASS_BF16T> { using T = BF16; };

// ---- storage conversions -------------------------------------------------
__device__ __forceinline__ float dec(F32, uint32_t b) { return __uint_as_float(b); }
__device__ __forceinline__ float dec(F16, uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
}
__device__ __forceinline__ float dec(BF16, uint32_t b) { return __uint_as_float(b << 16); }

__device__ __forceinline__ uint32_t enc(F32, float f) { return __float_as_uint(f); }

typedef float f2v __attribute__((ext_vector_type(2)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
// Two FP32 values -> one packed word of two 16-bit values (low half = a),
// rounded to nearest even by the hardware converters (v_cvt_pk_f16_f32 /
// v_cvt_pk_bf16_f32 on gfx950).  Every 16-bit store goes through this pair
// conversion: a lone float->half conversion lets the compiler fold it with
// the last FMA of the filter into one mixed-precision FMA that rounds once,
// straight to 16 bits, which skips the FP32 result and can differ from it by
// one unit at ties.
__device__ __forceinline__ uint32_t enc2(F16, float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, h2v));
}
__device__ __forceinline__ uint32_t enc2(BF16, float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, b2v));
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
// LAUX: cache policy of the row load (0, or NT for rows read only once).
template <class D, int LAUX = 0>
__device__ __forceinline__ void issue(Raw<D, true> &r, const char *row, uint32_t rbytes, int x,
                                      int hoff) {
    const auto rs = row_rsrc(row, rbytes);
    r.m = __builtin_amdgcn_raw_buffer_load_b128(rs, x * D::ESZ, 0, LAUX);
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
template <class D, int LAUX = 0>
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

// SAUX: cache policy of the stores (NT streams them out; 0 keeps the FP32
// intermediate of the two-pass form cached for the column kernel that reads
// it next).
template <int N, bool AL, int SAUX = NT>
__device__ __forceinline__ void store_t(char *row, uint32_t rbytes, int x, const float (&o)[N]) {
    const auto rs = row_rsrc(row, rbytes);
    if constexpr (AL) {
#pragma unroll
        for (int j = 0; j < N / 4; ++j) {
            const u4 q = {__float_as_uint(o[4 * j]), __float_as_uint(o[4 * j + 1]),
                          __float_as_uint(o[4 * j + 2]), __float_as_uint(o[4 * j + 3])};
            __builtin_amdgcn_raw_buffer_store_b128(q, rs, (x + 4 * j) * 4, 0, SAUX);
        }
    } else {
#pragma unroll
        for (int e = 0; e < N; ++e)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o[e]), rs, (x + e) * 4, 0, SAUX);
    }
}

// ---- intermediate rows in 16 bits (two-pass with a 16-bit intermediate) -----
// N values per lane: packed in pairs (N/2 words) on the vector path, one per
// word on the element-wise path.
template <class TD, int N, bool AL> struct RawTT {
    static constexpr int NW = (TD::ESZ == 2 && AL) ? N / 2 : N;
    uint32_t w[NW];
};

template <class TD, int N, bool AL>
__device__ __forceinline__ void issue_tt(RawTT<TD, N, AL> &r, const char *row, uint32_t rbytes,
                                         int x) {
    static_assert(TD::ESZ == 2, "16-bit intermediates only");
    const auto rs = row_rsrc(row, rbytes);
    if constexpr (AL && N == 4) {
        const u2 q = __builtin_amdgcn_raw_buffer_load_b64(rs, x * 2, 0, 0);
        r.w[0] = q.x;
        r.w[1] = q.y;
    } else if constexpr (AL) {
#pragma unroll
        for (int j = 0; j < N / 8; ++j) {
            const u4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, (x + 8 * j) * 2, 0, 0);
            r.w[4 * j + 0] = q.x;
            r.w[4 * j + 1] = q.y;
            r.w[4 * j + 2] = q.z;
            r.w[4 * j + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < N; ++e)
            r.w[e] = __builtin_amdgcn_raw_buffer_load_b16(rs, (x + e) * 2, 0, 0);
    }
}

template <class TD, int N, bool AL>
__device__ __forceinline__ void decode_tt(const RawTT<TD, N, AL> &r, float (&w)[N]) {
    if constexpr (AL) {
#pragma unroll
        for (int i = 0; i < N / 2; ++i) {
            w[2 * i] = dec(TD{}, r.w[i]);
            w[2 * i + 1] = dec(TD{}, r.w[i] >> 16);
        }
    } else {
#pragma unroll
        for (int e = 0; e < N; ++e) w[e] = dec(TD{}, r.w[e]);
    }
}

// The FP32 row-filter values rounded to TD (RNE, pairwise conversion) and
// stored; SAUX as for store_t.
template <class TD, int N, bool AL, int SAUX>
__device__ __forceinline__ void store_tt(char *row, uint32_t rbytes, int x, const float (&o)[N]) {
    const auto rs = row_rsrc(row, rbytes);
    uint32_t q[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) q[i] = enc2(TD{}, o[2 * i], o[2 * i + 1]);
    if constexpr (AL && N == 4) {
        __builtin_amdgcn_raw_buffer_store_b64(u2{q[0], q[1]}, rs, x * 2, 0, SAUX);
    } else if constexpr (AL) {
#pragma unroll
        for (int j = 0; j < N / 8; ++j)
            __builtin_amdgcn_raw_buffer_store_b128(u4{q[4 * j], q[4 * j + 1], q[4 * j + 2], q[4 * j + 3]},
                                                   rs, (x + 8 * j) * 2, 0, SAUX);
    } else {
#pragma unroll
        for (int i = 0; i < N / 2; ++i) {
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(q[i] & 0xffffu), rs, (x + 2 * i) * 2, 0, SAUX);
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(q[i] >> 16), rs, (x + 2 * i + 1) * 2, 0, SAUX);
        }
    }
}

// ---- output rows in the storage type ------------------------------------
// SAUX: cache policy (NT streams the output out; 0 keeps it cached when the
// next kernel reads it, as the copy of the copy-back single pass does).
template <class D, bool AL, int SAUX = NT>
__device__ __forceinline__ void store_out(char *row, uint32_t rbytes, int x,
                                          const float (&o)[D::VEC]) {
    const auto rs = row_rsrc(row, rbytes);
    if constexpr (AL) {
        u4 q;
        if constexpr (D::ESZ == 4) {
            q = u4{enc(D{}, o[0]), enc(D{}, o[1]), enc(D{}, o[2]), enc(D{}, o[3])};
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = enc2(D{}, o[2 * i], o[2 * i + 1]);
        }
        __builtin_amdgcn_raw_buffer_store_b128(q, rs, x * D::ESZ, 0, SAUX);
    } else if constexpr (D::ESZ == 4) {
#pragma unroll
        for (int e = 0; e < D::VEC; ++e)
            __builtin_amdgcn_raw_buffer_store_b32(enc(D{}, o[e]), rs, (x + e) * 4, 0, SAUX);
    } else {
#pragma unroll
        for (int e = 0; e < D::VEC; e += 2) {
            const uint32_t w = enc2(D{}, o[e], o[e + 1]);
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w & 0xffffu), rs, (x + e) * 2, 0, SAUX);
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w >> 16), rs, (x + e + 1) * 2, 0, SAUX);
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


// ---- per-band context of the vertical-filter kernels -------------------------
// (fused, direct25 and the two-pass column kernel)
// EDGE = false: the tile touches no border row or column, so no output of it
// needs the zero frame and the selects are compiled out.
template <class D, bool AL, int MODE, bool EDGE, int SAUX = NT>
struct VBand {
    static constexpr int VEC = D::VEC;
    static constexpr bool DIRECT = MODE == MODE_DIRECT25;
    static constexpr bool COL = is_colpass(MODE);
    static constexpr int WN = DIRECT ? VEC + 4 : VEC;  // floats per window row
    using TD = typename TmpOf<MODE>::T;                // the intermediate's type
    static constexpr bool T16 = COL && TD::ESZ == 2;
    using RawCol = typename std::conditional<T16, RawTT<TD, VEC, AL>, RawT<VEC, AL>>::type;
    using RawIn = typename std::conditional<COL, RawCol, Raw<D, AL>>::type;

    const ImgDev &im;
    int H, W, x, hoff;
    const char *sbase;
    int64_t sstride;
    uint32_t sbytes;
    char *dbase;
    int64_t dstride;
    uint32_t dbytes;
    bool cm[VEC];

    __device__ __forceinline__ VBand(const ImgDev &im_, int plane, int xs, int lane) : im(im_) {
        H = im.rows;
        W = im.cols;
        x = xs + lane * VEC;
        if constexpr (COL) {
            sbase = (const char *)im.tmp + (int64_t)plane * H * W * TD::ESZ;
            sstride = (int64_t)W * TD::ESZ;
            sbytes = (uint32_t)W * TD::ESZ;
        } else {
            sbase = (const char *)im.in + (int64_t)plane * im.pstride * D::ESZ;
            sstride = im.pitch * D::ESZ;
            sbytes = (uint32_t)W * D::ESZ;
        }
        dbase = (char *)im.out + (int64_t)plane * im.pstride * D::ESZ;
        dstride = im.pitch * D::ESZ;
        dbytes = (uint32_t)W * D::ESZ;
        const int hl = xs - 2, hr = xs + WAVE * VEC;
        hoff = lane == 0 ? (hl >= 0 ? hl * D::ESZ : OOB)
                         : (lane == WAVE - 1 ? (hr < W ? hr * D::ESZ : OOB) : OOB);
#pragma unroll
        for (int e = 0; e < VEC; ++e) cm[e] = (x + e >= 2) && (x + e < W - 2);
    }
    // `row` must already lie in [0, H)
    __device__ __forceinline__ void fetch(RawIn &r, int row) const {
        const char *p = sbase + (int64_t)row * sstride;
        if constexpr (T16)
            issue_tt<TD, VEC, AL>(r, p, sbytes, x);
        else if constexpr (COL)
            issue_t<VEC, AL>(r, p, sbytes, x);
        else
            issue<D>(r, p, sbytes, x, hoff);
    }
    __device__ __forceinline__ void produce(const RawIn &r, float (&w)[WN]) const {
        if constexpr (T16) {
            decode_tt<TD, VEC, AL>(r, w);
        } else if constexpr (COL) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) w[e] = __uint_as_float(r.w[e]);
        } else if constexpr (DIRECT) {
            decode<D>(r, w);
        } else {
            float v[VEC + 4];
            decode<D>(r, v);
            hfilter<VEC>(v, im.tp.k, w);
        }
    }
    // Output row y from window rows y-2 .. y+2.
    __device__ __forceinline__ void emit(int y, const float (&a)[WN], const float (&b)[WN],
                                         const float (&c)[WN], const float (&d)[WN],
                                         const float (&e)[WN]) const {
        float o[VEC];
        if constexpr (DIRECT)
            direct25<VEC>(a, b, c, d, e, im.tp.K, o);
        else
            vfilter<VEC>(a, b, c, d, e, im.tp.k, o);
        if constexpr (EDGE) {
            const bool vr = (y >= 2) && (y < H - 2);
#pragma unroll
            for (int i = 0; i < VEC; ++i) o[i] = (vr && cm[i]) ? o[i] : 0.0f;
        }
        store_out<D, AL, SAUX>(dbase + (int64_t)y * dstride, dbytes, x, o);
    }
};

// Band of compile-time height TH: all TH+4 input rows are issued first.
// Rows outside [0, H) are clamped; they only feed border outputs (y < 2 or
// y >= H-2), which are written as zeros.
template <class D, bool AL, int MODE, bool EDGE, int TH, int SAUX = NT>
__device__ __forceinline__ void band_vertical_fixed(const ImgDev &im, int plane, int xs, int y0,
                                                    int lane) {
    using B = VBand<D, AL, MODE, EDGE, SAUX>;
    const B b(im, plane, xs, lane);
    const int Hm1 = b.H - 1;
    typename B::RawIn raw[TH + 4];
#pragma unroll
    for (int i = 0; i < TH + 4; ++i) b.fetch(raw[i], clampi(y0 - 2 + i, 0, Hm1));
    float w[TH + 4][B::WN];
#pragma unroll
    for (int i = 0; i < TH + 4; ++i) b.produce(raw[i], w[i]);
#pragma unroll
    for (int j = 0; j < TH; ++j) b.emit(y0 + j, w[j], w[j + 1], w[j + 2], w[j + 3], w[j + 4]);
}

// Band of any height: walk down with a 5-row window and a 5-row prefetch ring.
template <class D, bool AL, int MODE, bool EDGE, int SAUX = NT>
__device__ __forceinline__ void band_vertical(const ImgDev &im, int plane, int xs, int y0, int y1,
                                              int lane) {
    using B = VBand<D, AL, MODE, EDGE, SAUX>;
    const B b(im, plane, xs, lane);
    const int rlim = min(y1 + 1, b.H - 1);
    auto fetch = [&](typename B::RawIn &r, int row) { b.fetch(r, clampi(row, 0, rlim)); };

    float w[5][B::WN];
    typename B::RawIn ring[5];
    {
        typename B::RawIn p0, p1, p2, p3;
        fetch(p0, y0 - 2);
        fetch(p1, y0 - 1);
        fetch(p2, y0);
        fetch(p3, y0 + 1);
        b.produce(p0, w[0]);
        b.produce(p1, w[1]);
        b.produce(p2, w[2]);
        b.produce(p3, w[3]);
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
#define CONV_VSTEP(S)                                                                     \
    {                                                                                      \
        b.produce(ring[S], w[S]);                                                          \
        fetch(ring[S], y + 7);                                                             \
        b.emit(y, w[((S) + 1) % 5], w[((S) + 2) % 5], w[((S) + 3) % 5], w[((S) + 4) % 5], \
               w[S]);                                                                      \
        ++y;                                                                               \
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

// ---- the two-pass row kernel -----------------------------------------------------
// TD: storage type of the intermediate (F32, or F16 / BF16 for the 16-bit form)
template <class D, bool AL, bool EDGE, class TD = F32>
struct RBand {
    static constexpr int VEC = D::VEC;
    const ImgDev &im;
    int x, hoff;
    const char *sbase;
    int64_t sstride;
    uint32_t sbytes;
    char *tbase;
    int64_t tstride;
    uint32_t tbytes;
    bool cm[VEC];

    __device__ __forceinline__ RBand(const ImgDev &im_, int plane, int xs, int lane) : im(im_) {
        const int H = im.rows, W = im.cols;
        x = xs + lane * VEC;
        sbase = (const char *)im.in + (int64_t)plane * im.pstride * D::ESZ;
        sstride = im.pitch * D::ESZ;
        sbytes = (uint32_t)W * D::ESZ;
        tbase = (char *)im.tmp + (int64_t)plane * H * W * TD::ESZ;
        tstride = (int64_t)W * TD::ESZ;
        tbytes = (uint32_t)W * TD::ESZ;
        const int hl = xs - 2, hr = xs + WAVE * VEC;
        hoff = lane == 0 ? (hl >= 0 ? hl * D::ESZ : OOB)
                         : (lane == WAVE - 1 ? (hr < W ? hr * D::ESZ : OOB) : OOB);
#pragma unroll
        for (int e = 0; e < VEC; ++e) cm[e] = (x + e >= 2) && (x + e < W - 2);
    }
    // each input row is read once by the row kernel: streamed
    __device__ __forceinline__ void fetch(Raw<D, AL> &r, int row) const {
        issue<D, NT>(r, sbase + (int64_t)row * sstride, sbytes, x, hoff);
    }
    // T[row] = horizontal filter on columns 2..W-3, 0 elsewhere; T stays
    // cached for the column kernel.
    __device__ __forceinline__ void filter_store(const Raw<D, AL> &r, int row) const {
        float v[VEC + 4], h[VEC];
        decode<D>(r, v);
        hfilter<VEC>(v, im.tp.k, h);
        if constexpr (EDGE) {
#pragma unroll
            for (int i = 0; i < VEC; ++i) h[i] = cm[i] ? h[i] : 0.0f;
        }
        if constexpr (TD::ESZ == 4)
            store_t<VEC, AL, 0>(tbase + (int64_t)row * tstride, tbytes, x, h);
        else
            store_tt<TD, VEC, AL, 0>(tbase + (int64_t)row * tstride, tbytes, x, h);
    }
};

template <class D, bool AL, bool EDGE, int TH, class TD>
__device__ __forceinline__ void band_rowpass_fixed(const ImgDev &im, int plane, int xs, int y0,
                                                   int lane) {
    const RBand<D, AL, EDGE, TD> b(im, plane, xs, lane);
    Raw<D, AL> raw[TH];
#pragma unroll
    for (int i = 0; i < TH; ++i) b.fetch(raw[i], y0 + i);
#pragma unroll
    for (int i = 0; i < TH; ++i) b.filter_store(raw[i], y0 + i);
}

template <class D, bool AL, bool EDGE, class TD>
__device__ __forceinline__ void band_rowpass(const ImgDev &im, int plane, int xs, int y0, int y1,
                                             int lane) {
    const RBand<D, AL, EDGE, TD> b(im, plane, xs, lane);
    const int rlim = y1 - 1;
    Raw<D, AL> ring[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) b.fetch(ring[i], min(y0 + i, rlim));
    int y = y0;
#define CONV_RSTEP(S)                                 \
    {                                                  \
        const Raw<D, AL> cur = ring[S];                \
        b.fetch(ring[S], min(y + 5, rlim));            \
        b.filter_store(cur, y);                        \
        ++y;                                           \
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

// ---- copy-back (single-pass result written back over the input) ------------------
template <class D, bool AL>
__device__ __forceinline__ void band_copy(const ImgDev &im, int plane, int xs, int y0, int y1,
                                          int lane) {
    constexpr int VEC = D::VEC, G = 8;  // rows per group: all loads, then all stores
    const int x = xs + lane * VEC;
    const char *sbase = (const char *)im.in + (int64_t)plane * im.pstride * D::ESZ;
    char *dbase = (char *)im.out + (int64_t)plane * im.pstride * D::ESZ;
    const int64_t stride = im.pitch * D::ESZ;
    const uint32_t rbytes = (uint32_t)im.cols * D::ESZ;
    for (int y = y0; y < y1; y += G) {
        // the compiler keeps a load after an earlier store to a buffer that
        // might alias it, so one load per row then its store would leave one
        // load in flight per lane: the group's loads are issued first
        uint32_t v[G][AL ? 4 : VEC];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const auto rs = row_rsrc(sbase + (int64_t)min(y + i, y1 - 1) * stride, rbytes);
            if constexpr (AL) {
                const u4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, x * D::ESZ, 0, 0);
                v[i][0] = q.x;
                v[i][1] = q.y;
                v[i][2] = q.z;
                v[i][3] = q.w;
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int off = (x + e) * D::ESZ;
                    v[i][e] = D::ESZ == 4 ? __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0)
                                          : __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (y + i >= y1) break;
            const auto rd = row_rsrc(dbase + (int64_t)(y + i) * stride, rbytes);
            if constexpr (AL) {
                __builtin_amdgcn_raw_buffer_store_b128(u4{v[i][0], v[i][1], v[i][2], v[i][3]}, rd,
                                                       x * D::ESZ, 0, NT);
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int off = (x + e) * D::ESZ;
                    if constexpr (D::ESZ == 4)
                        __builtin_amdgcn_raw_buffer_store_b32(v[i][e], rd, off, 0, NT);
                    else
                        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)v[i][e], rd, off, 0, NT);
                }
            }
        }
    }
}

// ---- packed last strip (fused and direct25) ------------------------------------------
// A last strip narrower than a wave's 64*VEC columns would leave lanes of its
// wave idle, and a wave costs about the same time whether its lanes are busy
// or not.  The last strip is therefore cut into pieces, left to right: at most
// one of 32 lanes' width and up to two of 16 (the last piece may be partly
// past the right edge).  One wave takes a piece for Q consecutive bands (Q = 2
// for a 32-lane piece, 4 for a 16-lane one): lane group g (64/Q lanes) works
// on band band0 + g.  The groups read different rows, so the buffer resource
// spans the rows of all Q bands and each lane adds its own row offset; the
// range check then no longer stops lanes past the right edge, so their stores
// get an out-of-range offset explicitly (their loads may read the next row,
// which only reaches outputs in the zero frame).  The first and last lane of
// each group fetch the group's halo columns.
//
// Horizontal neighbours inside a group, with no per-lane select (a select on
// the lane's position lets the compiler put the move under a lane mask, and a
// DPP move that reads a masked-off lane gets the fallback value instead):
//   left:  row_shr:1 moves within each row of 16 lanes; a row's lane 0 keeps
//          `old`, its own left halo.  With 4 groups the rows are the groups.
//          With 2 groups, lanes 16 and 48 (row 1 and 3, lane 0) then take
//          lane 15's and 47's value from a wave_shr:1 move written only to
//          rows 1 and 3, bank 0 (lanes 16..19, 48..51; on 17..19 and 49..51
//          it writes the value they already hold);
//   right: the mirror image: row_shl:1 within each row, so a row's lane 15
//          keeps its own right halo; with 2 groups, lanes 15 and 47 (row 0
//          and 2, lane 15) then take lane 16's and 48's value from a
//          wave_shl:1 move written only to rows 0 and 2, bank 3 (lanes
//          12..15, 44..47).  A piece that is not the last one thus gets its
//          right neighbours from its own halo load, not from the next group.
__device__ __forceinline__ uint32_t left_in_row(uint32_t src, uint32_t old) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x111, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t left_rows13_bank0(uint32_t src, uint32_t old) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x138, 0xa, 0x1, false);
}
__device__ __forceinline__ uint32_t right_in_row(uint32_t src, uint32_t old) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x101, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t right_rows02_bank3(uint32_t src, uint32_t old) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x130, 0x5, 0x8, false);
}
// q2: groups of 32 lanes (uniform across the wave)
__device__ __forceinline__ uint32_t left_in_group(uint32_t src, uint32_t halo, bool q2) {
    const uint32_t a = left_in_row(src, halo);
    return q2 ? left_rows13_bank0(src, a) : a;
}
__device__ __forceinline__ uint32_t right_in_group(uint32_t src, uint32_t halo, bool q2) {
    const uint32_t a = right_in_row(src, halo);
    return q2 ? right_rows02_bank3(src, a) : a;
}
template <class D>
__device__ __forceinline__ void decode_group(const Raw<D, true> &r, bool q2,
                                             float (&v)[D::VEC + 4]) {
    if constexpr (D::ESZ == 4) {
        v[0] = __uint_as_float(left_in_group(r.m.z, r.h0, q2));
        v[1] = __uint_as_float(left_in_group(r.m.w, r.h1, q2));
        v[2] = __uint_as_float(r.m.x);
        v[3] = __uint_as_float(r.m.y);
        v[4] = __uint_as_float(r.m.z);
        v[5] = __uint_as_float(r.m.w);
        v[6] = __uint_as_float(right_in_group(r.m.x, r.h0, q2));
        v[7] = __uint_as_float(right_in_group(r.m.y, r.h1, q2));
    } else {
        const uint32_t l = left_in_group(r.m.w, r.h0, q2);
        const uint32_t rr = right_in_group(r.m.x, r.h0, q2);
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
__device__ __forceinline__ void decode_group(const Raw<D, false> &r, bool,
                                             float (&v)[D::VEC + 4]) {
    decode<D>(r, v);
}

// One input row of a lane group: `roff` is the row's byte offset in the
// span resource, `hoff` the halo offset (already OOB for lanes without one).
template <class D>
__device__ __forceinline__ void issue_group(Raw<D, true> &r, __amdgpu_buffer_rsrc_t rs,
                                            uint32_t roff, int x, int hoff) {
    r.m = __builtin_amdgcn_raw_buffer_load_b128(rs, roff + x * D::ESZ, 0, 0);
    const int h = hoff == OOB ? OOB : (int)(roff + hoff);
    if constexpr (D::ESZ == 4) {
        const u2 q = __builtin_amdgcn_raw_buffer_load_b64(rs, h, 0, 0);
        r.h0 = q.x;
        r.h1 = q.y;
    } else {
        r.h0 = __builtin_amdgcn_raw_buffer_load_b32(rs, h, 0, 0);
        r.h1 = 0;
    }
}
template <class D>
__device__ __forceinline__ void issue_group(Raw<D, false> &r, __amdgpu_buffer_rsrc_t rs,
                                            uint32_t roff, int x, int) {
#pragma unroll
    for (int e = 0; e < D::VEC + 4; ++e) {
        const int c = x - 2 + e;
        const int off = c >= 0 ? (int)(roff + c * D::ESZ) : OOB;
        if constexpr (D::ESZ == 4)
            r.e[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        else
            r.e[e] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
    }
}

// Output row of a lane group; `ok` is false for rows past the image and for
// the lanes of a group beyond the last band.
template <class D, bool AL, int SAUX>
__device__ __forceinline__ void store_group(__amdgpu_buffer_rsrc_t rs, uint32_t roff, int x,
                                            int W, bool ok, const float (&o)[D::VEC]) {
    if constexpr (AL) {
        u4 q;
        if constexpr (D::ESZ == 4) {
            q = u4{enc(D{}, o[0]), enc(D{}, o[1]), enc(D{}, o[2]), enc(D{}, o[3])};
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = enc2(D{}, o[2 * i], o[2 * i + 1]);
        }
        // aligned images have W % VEC == 0: a lane's vector is all in or all out
        const int off = (ok && x < W) ? (int)(roff + x * D::ESZ) : OOB;
        __builtin_amdgcn_raw_buffer_store_b128(q, rs, off, 0, SAUX);
    } else if constexpr (D::ESZ == 4) {
#pragma unroll
        for (int e = 0; e < D::VEC; ++e) {
            const int off = (ok && x + e < W) ? (int)(roff + (x + e) * 4) : OOB;
            __builtin_amdgcn_raw_buffer_store_b32(enc(D{}, o[e]), rs, off, 0, SAUX);
        }
    } else {
#pragma unroll
        for (int e = 0; e < D::VEC; e += 2) {
            const uint32_t w = enc2(D{}, o[e], o[e + 1]);
            const int o0 = (ok && x + e < W) ? (int)(roff + (x + e) * 2) : OOB;
            const int o1 = (ok && x + e + 1 < W) ? (int)(roff + (x + e + 1) * 2) : OOB;
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w & 0xffffu), rs, o0, 0, SAUX);
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w >> 16), rs, o1, 0, SAUX);
        }
    }
}

// The packed piece starting at column xs (32 lanes wide if q2, else 16) for
// bands band0 .. band0+qg-1 (qg <= Q); every band has TH rows except possibly
// the image's last.
template <class D, bool AL, int MODE, int TH, int SAUX>
__device__ __forceinline__ void band_packed(const ImgDev &im, int plane, int xs, int band0, int qg,
                                            bool q2, int lane) {
    constexpr int VEC = D::VEC;
    constexpr bool DIRECT = MODE == MODE_DIRECT25;
    constexpr int WN = DIRECT ? VEC + 4 : VEC;
    const int H = im.rows, W = im.cols;
    const int lgs = q2 ? 5 : 4;                    // log2 of the lanes per group
    const int grp = lane >> lgs, ln = lane & ((1 << lgs) - 1);
    const bool first = ln == 0, last = ln == (1 << lgs) - 1;
    const int x = xs + ln * VEC;
    const bool act = grp < qg;
    const int y0 = (band0 + grp) * TH;
    // rows ylo .. yhi feed the qg bands
    const int ylo = max(band0 * TH - 2, 0);
    const int yhi = min((band0 + qg) * TH + 1, H - 1);
    const int64_t pb = im.pitch * D::ESZ;
    const char *ib = (const char *)im.in + (int64_t)plane * im.pstride * D::ESZ + ylo * pb;
    char *ob = (char *)im.out + (int64_t)plane * im.pstride * D::ESZ + ylo * pb;
    const uint32_t span = (uint32_t)((int64_t)(yhi - ylo) * pb + (int64_t)W * D::ESZ);
    const auto rin = row_rsrc(ib, span);
    const auto rout = row_rsrc(ob, span);
    const int hl = xs - 2, hr = xs + (VEC << lgs);
    const int hoff = first ? (hl >= 0 ? hl * D::ESZ : OOB)
                           : (last ? (hr < W ? hr * D::ESZ : OOB) : OOB);

    Raw<D, AL> raw[TH + 4];
#pragma unroll
    for (int i = 0; i < TH + 4; ++i) {
        const int row = clampi(y0 - 2 + i, ylo, yhi);
        issue_group<D>(raw[i], rin, (uint32_t)((int64_t)(row - ylo) * pb), x, hoff);
    }
    bool cm[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) cm[e] = (x + e >= 2) && (x + e < W - 2);
    // each output row as soon as its five window rows exist
    float w[TH + 4][WN];
#pragma unroll
    for (int i = 0; i < TH + 4; ++i) {
        if constexpr (DIRECT) {
            decode_group<D>(raw[i], q2, w[i]);
        } else {
            float v[VEC + 4];
            decode_group<D>(raw[i], q2, v);
            hfilter<VEC>(v, im.tp.k, w[i]);
        }
        if (i < 4) continue;
        const int j = i - 4, y = y0 + j;
        float o[VEC];
        if constexpr (DIRECT)
            direct25<VEC>(w[j], w[j + 1], w[j + 2], w[j + 3], w[j + 4], im.tp.K, o);
        else
            vfilter<VEC>(w[j], w[j + 1], w[j + 2], w[j + 3], w[j + 4], im.tp.k, o);
        const bool vr = (y >= 2) && (y < H - 2);
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = (vr && cm[e]) ? o[e] : 0.0f;
        store_group<D, AL, SAUX>(rout, (uint32_t)((int64_t)(y - ylo) * pb), x, W, act && y < H, o);
    }
}

// ---- tiles -----------------------------------------------------------------------
// Logical tile lt = (plane, band, strip group), strip group fastest.  Wave
// `wave` of the workgroup takes strip sg*WAVES + wave of the group.  TH > 0:
// full bands of TH rows use the unrolled form (the host then sets th = TH).
template <class D, bool AL, int MODE, bool EDGE, int TH, int SAUX = NT>
__device__ __forceinline__ void run_band(const ImgDev &im, int plane, int xs, int y0, int y1,
                                         int lane) {
    if constexpr (MODE == MODE_COPY) {
        band_copy<D, AL>(im, plane, xs, y0, y1, lane);
    } else if constexpr (is_rowpass(MODE)) {
        using TD = typename TmpOf<MODE>::T;
        if constexpr (TH > 0) {
            if (y1 - y0 == TH) {
                band_rowpass_fixed<D, AL, EDGE, TH, TD>(im, plane, xs, y0, lane);
                return;
            }
        }
        band_rowpass<D, AL, EDGE, TD>(im, plane, xs, y0, y1, lane);
    } else {
        if constexpr (TH > 0) {
            if (y1 - y0 == TH) {
                band_vertical_fixed<D, AL, MODE, EDGE, TH, SAUX>(im, plane, xs, y0, lane);
                return;
            }
        }
        band_vertical<D, AL, MODE, EDGE, SAUX>(im, plane, xs, y0, y1, lane);
    }
}

template <class D, bool AL, int MODE, int TH, int SAUX>
__device__ __forceinline__ void run_strip_band(const ImgDev &im, int plane, int strip, int band,
                                               int lane);

// Tiles per group of tq bands of an image whose last strip is packed: the
// m = ns-1 full strips of each band, one tile per 2 bands for the 32-lane
// piece, one per group for each 16-lane piece.
__device__ __forceinline__ int64_t packed_group_tiles(const ImgDev &im) {
    return (int64_t)im.tq * (im.ns - 1) + im.pk32 * (im.tq / 2) + im.pk16;
}

// Tiles of an image whose last strip is packed (im.tq = G > 1): per plane, the
// bands go in groups of G; a group's tiles are the m = ns-1 full strips of
// each of its bands (band-major, strip fastest), then the tiles of the
// pieces of the last strip, left to right (for a 32-lane piece one per 2
// bands of the group, for a 16-lane piece one for the whole group).
template <class D, bool AL, int MODE, int TH, int SAUX>
__device__ __forceinline__ void run_tile_packed(const ImgDev &im, int64_t lt, int lane) {
    const int G = im.tq, m = im.ns - 1;
    const int64_t per = packed_group_tiles(im);
    const int64_t TP = (int64_t)im.nb * m + (int64_t)im.pk32 * ((im.nb + 1) / 2) +
                       (int64_t)im.pk16 * ((im.nb + G - 1) / G);
    const int plane = (int)(lt / TP);
    const int64_t r = lt % TP;
    const int g = (int)(r / per);
    int rr = (int)(r % per);
    const int qg = min(G, im.nb - g * G);
    if (rr < qg * m) {
        run_strip_band<D, AL, MODE, TH, SAUX>(im, plane, rr % m, g * G + rr / m, lane);
        return;
    }
    rr -= qg * m;
    const int xs = m * (WAVE * D::VEC);
    const int t32 = im.pk32 ? (qg + 1) / 2 : 0;
    if (rr < t32) {
        band_packed<D, AL, MODE, TH, SAUX>(im, plane, xs, g * G + 2 * rr, min(2, qg - 2 * rr), true,
                                           lane);
        return;
    }
    rr -= t32;
    band_packed<D, AL, MODE, TH, SAUX>(im, plane, xs + (im.pk32 * 32 + rr * 16) * D::VEC, g * G, qg,
                                       false, lane);
}

// Kernels that take packed last strips: fused, and direct25 for FP32 (the
// 16-bit direct25 kernel would need twice its registers for the packed band),
// aligned images, one wave per workgroup, unrolled bands.
template <class D, bool AL, int MODE, int WAVES, int TH>
constexpr bool packs() {
    return AL && WAVES == 1 && TH > 0 &&
           (MODE == MODE_FUSED || (MODE == MODE_DIRECT25 && D::ESZ == 4));
}

// PK: the launch holds images with a packed last strip (kernels of their
// own, so that the others carry no code for it).
template <class D, bool AL, int MODE, int WAVES, int TH, int SAUX = NT, bool PK = false>
__device__ __forceinline__ void run_tile(const ImgDev &im, int64_t lt, int wave, int lane) {
    if constexpr (PK && packs<D, AL, MODE, WAVES, TH>()) {
        if (im.tq > 1) {
            run_tile_packed<D, AL, MODE, TH, SAUX>(im, lt, lane);
            return;
        }
    }
    const int sg = (int)(lt % im.nsg);
    const int64_t t = lt / im.nsg;
    const int band = (int)(t % im.nb);
    const int plane = (int)(t / im.nb);
    const int strip = sg * WAVES + wave;
    if (strip >= im.ns) return;
    run_strip_band<D, AL, MODE, TH, SAUX>(im, plane, strip, band, lane);
}

template <class D, bool AL, int MODE, int TH, int SAUX>
__device__ __forceinline__ void run_strip_band(const ImgDev &im, int plane, int strip, int band,
                                               int lane) {
    const int xs = strip * (WAVE * D::VEC);
    const int y0 = band * im.th;
    const int y1 = min(y0 + im.th, im.rows);
    // Does any output of this tile lie in the 2-pixel frame?  (The row pass
    // writes every row, so only columns matter there.)
    const bool col_edge = xs < 2 || xs + WAVE * D::VEC > im.cols - 2;
    const bool row_edge = !is_rowpass(MODE) && (y0 < 2 || y1 > im.rows - 2);
    if constexpr (MODE == MODE_COPY)
        run_band<D, AL, MODE, false, TH>(im, plane, xs, y0, y1, lane);
    else if (col_edge || row_edge)
        run_band<D, AL, MODE, true, TH, SAUX>(im, plane, xs, y0, y1, lane);
    else
        run_band<D, AL, MODE, false, TH, SAUX>(im, plane, xs, y0, y1, lane);
}

// Workgroups are handed to the 8 XCDs round-robin (block b -> XCD b % 8).
// This renumbering gives each XCD one contiguous run of logical blocks.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    constexpr int X = 8;
    const int q = n / X, r = n % X;
    const int xcd = b % X, i = b / X;
    return xcd * q + min(xcd, r) + i;
}

// Band chunks dealt to the XCDs in turn: XCD x (blocks x, x+8, x+16, ...)
// takes chunks x, x+8, ... of T consecutive logical tiles (c full band rows),
// each in order, so both horizontal neighbours of a tile and the band above
// it were read through the same L2.  Blocks past the last whole round of 8
// chunks keep their own index.
__device__ __forceinline__ int xcd_chunk_remap(int b, int n, int64_t T) {
    constexpr int X = 8;
    const int64_t full = ((int64_t)n / (X * T)) * (X * T);
    if (b >= full) return b;
    const int x = b % X, i = b / X;
    return (int)((x + X * (i / T)) * T + i % T);
}

// Tiles in a chunk of xcd_slabs band rows (with a packed last strip: of
// xcd_slabs / tq band groups, at least one).
template <bool PK>
__device__ __forceinline__ int64_t chunk_tiles(const ImgDev &im) {
    if (PK && im.tq > 1) return (int64_t)max(1, im.xcd_slabs / im.tq) * packed_group_tiles(im);
    return (int64_t)im.xcd_slabs * im.nsg;
}

// Kernel argument of a single-image launch.  The runtime's host cost per
// launch steps up above 112 argument bytes (MI355X: about 2.9 against
// 3.8-4.1 us per launch), and a kernel that reads gridDim receives 256 more
// bytes of hidden arguments.  So the launch passes its grid size, leaves out
// what the kernel recomputes (strips, strip groups, bands) and the batch's
// tile range, and carries the 25 weights of the direct form only for that
// form: 96 bytes, 200 with the weights.
struct ImgArg {
    const void *in;
    void *out;
    float *tmp;
    int64_t pitch, pstride, nblocks;
    int32_t planes, rows, cols, grid;
    int16_t th, xcd_slabs;
    int8_t keep_out, tq, pk32, pk16;
    float k[5];
};
struct ImgArgK : ImgArg {
    float K[25];
};
static_assert(sizeof(ImgArg) <= 96, "single-image kernel argument above 96 bytes");
template <int MODE>
using ImgArgOf = typename std::conditional<MODE == MODE_DIRECT25, ImgArgK, ImgArg>::type;

template <int MODE>
inline ImgArgOf<MODE> image_arg(const ImgDev &im, int64_t nblocks, int grid) {
    ImgArgOf<MODE> a;
    std::memset(&a, 0, sizeof a);
    a.in = im.in;
    a.out = im.out;
    a.tmp = im.tmp;
    a.pitch = im.pitch;
    a.pstride = im.pstride;
    a.nblocks = nblocks;
    a.planes = im.planes;
    a.rows = im.rows;
    a.cols = im.cols;
    a.grid = grid;
    a.th = (int16_t)im.th;
    a.xcd_slabs = (int16_t)im.xcd_slabs;
    a.keep_out = (int8_t)im.keep_out;
    a.tq = (int8_t)im.tq;
    a.pk32 = (int8_t)im.pk32;
    a.pk16 = (int8_t)im.pk16;
    for (int i = 0; i < 5; ++i) a.k[i] = im.tp.k[i];
    if constexpr (MODE == MODE_DIRECT25)
        for (int i = 0; i < 25; ++i) a.K[i] = im.tp.K[i];
    return a;
}

// The descriptor a tile reads, rebuilt from the kernel argument (uniform
// values, held in scalar registers).
template <class D, bool AL, int MODE, int WAVES>
__device__ __forceinline__ ImgDev image_of_arg(const ImgArgOf<MODE> &a) {
    ImgDev d;
    d.in = a.in;
    d.out = a.out;
    d.tmp = a.tmp;
    d.pitch = a.pitch;
    d.pstride = a.pstride;
    d.planes = a.planes;
    d.rows = a.rows;
    d.cols = a.cols;
    d.aligned = AL ? 1 : 0;
    d.ns = (a.cols + WAVE * D::VEC - 1) / (WAVE * D::VEC);
    d.nsg = (d.ns + WAVES - 1) / WAVES;
    d.th = a.th;
    d.nb = (a.rows + a.th - 1) / a.th;
    d.xcd_slabs = a.xcd_slabs;
    d.keep_out = a.keep_out;
    d.tq = a.tq;
    d.pk32 = a.pk32;
    d.pk16 = a.pk16;
    d.tile_begin = 0;
    d.tile_end = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) d.tp.k[i] = a.k[i];
    if constexpr (MODE == MODE_DIRECT25) {
#pragma unroll
        for (int i = 0; i < 25; ++i) d.tp.K[i] = a.K[i];
    }
    return d;
}

// One workgroup per logical tile; grids above 2^20 workgroups loop.  In
// launch order (xcd_slabs = 0) the resident waves sweep the image row-band by
// row-band; with xcd_slabs = 1 each XCD walks its own slab of full rows; with
// xcd_slabs = c >= 2 the XCDs take turns on chunks of c band rows.  SAUX is
// the cache policy of the output stores.
template <class D, bool AL, int MODE, int WAVES, int TH, int SAUX = NT, bool PK = false>
__global__ __launch_bounds__(WAVE *WAVES) void k_image(ImgArgOf<MODE> arg) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const ImgDev im = image_of_arg<D, AL, MODE, WAVES>(arg);
    const int64_t nblocks = arg.nblocks;
    const int grid = arg.grid;
    for (int64_t base = 0; base < nblocks; base += grid) {
        const int64_t left = nblocks - base;
        const int cnt = left < (int64_t)grid ? (int)left : grid;
        if ((int)blockIdx.x >= cnt) break;
        const int b = im.xcd_slabs == 1   ? xcd_remap(blockIdx.x, cnt)
                      : im.xcd_slabs > 1 ? xcd_chunk_remap(blockIdx.x, cnt, chunk_tiles<PK>(im))
                                         : (int)blockIdx.x;
        run_tile<D, AL, MODE, WAVES, TH, SAUX, PK>(im, base + b, wave, lane);
    }
}

// Persistent batch kernel: a fixed grid (a multiple of the CU count) covers
// the launch's tiles (images in order, then plane, band, strip group).  With
// xcd_slabs = 0 the workgroups stride over the tiles, so the resident ones
// always work on one compact window of the batch; with xcd_slabs = c >= 2
// each such window is cut into chunks of 8c consecutive tiles that the XCDs
// take in turn (as in the single-image kernel); with xcd_slabs = 1 each
// workgroup takes one contiguous run, and the runs of one XCD are adjacent.
// The owning image of a workgroup's first tile is found by binary search over
// the descriptor table's tile ranges, later ones by advancing through them
// (tiles only increase within a workgroup).  A grid of one workgroup per tile
// (persist_wgs_per_cu = 0) runs one iteration per workgroup.
// The image that owns tile t: the last one whose tile range starts at or
// before t (an empty image shares its start with the next one).
__device__ __forceinline__ int find_image(const ImgDev *__restrict__ descs, int n, int64_t t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile_begin <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ANY_UNAL: the batch holds images that are not aligned, so the kernel
// carries the element-wise path too (which needs more registers, and so
// lowers the occupancy of the whole kernel).
template <class D, int MODE, int WAVES, int TH, bool ANY_UNAL, bool PK>
__device__ __forceinline__ void batch_body(const ImgDev *__restrict__ descs, int n, int64_t total) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int G = gridDim.x;
    const int b = blockIdx.x;
    const int x = descs[0].xcd_slabs;
    int64_t first = b, last = total;  // x == 1: this workgroup's contiguous run
    if (x == 1) {
        const int64_t L = xcd_remap(b, G);
        first = total * L / G;
        last = total * (L + 1) / G;
    }
    int i = 0;
    for (int64_t j = 0;; ++j) {
        int64_t t;
        if (x == 1) {
            t = first + j;
            if (t >= last) break;
        } else if (x > 1) {
            const int64_t base = j * G;
            if (base >= total) break;
            const int64_t left = total - base;
            const int cnt = left < (int64_t)G ? (int)left : G;
            if (b >= cnt) break;
            t = base + xcd_chunk_remap(b, cnt, (int64_t)8 * x);
        } else {
            t = b + j * G;
            if (t >= total) break;
        }
        if (j == 0)
            i = find_image(descs, n, t);
        else
            while (i < n - 1 && t >= descs[i].tile_end) ++i;
        const ImgDev &im = descs[i];
        if (!ANY_UNAL || im.aligned)
            run_tile<D, true, MODE, WAVES, TH, NT, PK>(im, t - im.tile_begin, wave, lane);
        else if constexpr (ANY_UNAL)
            run_tile<D, false, MODE, WAVES, TH>(im, t - im.tile_begin, wave, lane);
    }
}

template <class D, int MODE, int WAVES, int TH, bool ANY_UNAL, bool PK>
__global__ __launch_bounds__(WAVE *WAVES) void k_batch(const ImgDev *__restrict__ descs, int n,
                                                       int64_t total) {
    batch_body<D, MODE, WAVES, TH, ANY_UNAL, PK>(descs, n, total);
}

// Same kernel with the descriptors in the kernel argument.  The argument is
// read in place through the kernarg segment pointer (it is the only explicit
// argument, so it starts at offset 0): indexing the by-value parameter itself
// would make the compiler copy it to per-lane scratch memory.
template <class D, int MODE, int WAVES, int TH, bool ANY_UNAL, bool PK>
__global__ __launch_bounds__(WAVE *WAVES) void k_batch_args(BatchArgs) {
    typedef const __attribute__((address_space(4))) BatchArgs ConstArgs;
    ConstArgs *a = (ConstArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    batch_body<D, MODE, WAVES, TH, ANY_UNAL, PK>((const ImgDev *)a->d, a->n, a->total);
}

// ---- launchers -------------------------------------------------------------------
template <class D, bool AL, int MODE, int WAVES, int SAUX>
hipError_t launch_image_th_p(const ImgDev &im_, int64_t nblocks, hipStream_t s) {
    const int grid = (int)(nblocks < (1 << 20) ? nblocks : (1 << 20));
    const dim3 blk(WAVE * WAVES);
    const bool pk = im_.tq > 1;
    const ImgArgOf<MODE> im = image_arg<MODE>(im_, nblocks, grid);
    switch (im.th) {
    case 4:
        if constexpr (packs<D, AL, MODE, WAVES, 4>()) {
            if (pk) {
                hipLaunchKernelGGL((k_image<D, AL, MODE, WAVES, 4, SAUX, true>), dim3(grid), blk, 0, s, im);
                break;
            }
        }
        hipLaunchKernelGGL((k_image<D, AL, MODE, WAVES, 4, SAUX>), dim3(grid), blk, 0, s, im);
        break;
    case 8:
        if constexpr (packs<D, AL, MODE, WAVES, 8>()) {
            if (pk) {
                hipLaunchKernelGGL((k_image<D, AL, MODE, WAVES, 8, SAUX, true>), dim3(grid), blk, 0, s, im);
                break;
            }
        }
        hipLaunchKernelGGL((k_image<D, AL, MODE, WAVES, 8, SAUX>), dim3(grid), blk, 0, s, im);
        break;
    default: hipLaunchKernelGGL((k_image<D, AL, MODE, WAVES, 0, SAUX>), dim3(grid), blk, 0, s, im); break;
    }
    return hipGetLastError();
}

// keep_out (the copy-back scratch, read by the copy next): cached output
// stores, compiled as kernels of their own so the streaming ones are unchanged
template <class D, bool AL, int MODE, int WAVES>
hipError_t launch_image_th(const ImgDev &im, int64_t nblocks, hipStream_t s) {
    if constexpr (MODE == MODE_FUSED || MODE == MODE_DIRECT25) {
        if (im.keep_out) return launch_image_th_p<D, AL, MODE, WAVES, 0>(im, nblocks, s);
    }
    return launch_image_th_p<D, AL, MODE, WAVES, NT>(im, nblocks, s);
}

template <class D, bool AL, int MODE>
hipError_t launch_image_w(const ImgDev &im, int waves, int64_t nblocks, hipStream_t s) {
    switch (waves) {
    case 1: return launch_image_th<D, AL, MODE, 1>(im, nblocks, s);
    case 2: return launch_image_th<D, AL, MODE, 2>(im, nblocks, s);
    default: return launch_image_th<D, AL, MODE, 4>(im, nblocks, s);
    }
}

template <class D, bool AL>
hipError_t launch_image_m(const ImgDev &im, int mode, int waves, int64_t nblocks, hipStream_t s) {
    switch (mode) {
    case MODE_FUSED: return launch_image_w<D, AL, MODE_FUSED>(im, waves, nblocks, s);
    case MODE_DIRECT25: return launch_image_w<D, AL, MODE_DIRECT25>(im, waves, nblocks, s);
    case MODE_ROWPASS: return launch_image_w<D, AL, MODE_ROWPASS>(im, waves, nblocks, s);
    case MODE_COPY: return launch_image_w<D, AL, MODE_COPY>(im, waves, nblocks, s);
    // the 16-bit intermediate forms run with one wave per workgroup
    case MODE_ROWPASS_F16T: return launch_image_th<D, AL, MODE_ROWPASS_F16T, 1>(im, nblocks, s);
    case MODE_COLPASS_F16T: return launch_image_th<D, AL, MODE_COLPASS_F16T, 1>(im, nblocks, s);
    case MODE_ROWPASS_BF16T: return launch_image_th<D, AL, MODE_ROWPASS_BF16T, 1>(im, nblocks, s);
    case MODE_COLPASS_BF16T: return launch_image_th<D, AL, MODE_COLPASS_BF16T, 1>(im, nblocks, s);
    default: return launch_image_w<D, AL, MODE_COLPASS>(im, waves, nblocks, s);
    }
}

template <class D>
hipError_t launch_image_t(const ImgDev &im, int mode, int waves, int64_t nblocks, hipStream_t s) {
    return im.aligned ? launch_image_m<D, true>(im, mode, waves, nblocks, s)
                      : launch_image_m<D, false>(im, mode, waves, nblocks, s);
}

// Batch kernel for the launch's flags (kBatchAnyUnaligned, kBatchAnyPacked);
// packed-strip kernels exist for one-wave workgroups with 4- or 8-row bands.
template <class D, int MODE, int WAVES, int TH, bool U>
hipError_t launch_batch_k(const ImgDev *d, int n, int64_t total, bool pk, int grid, hipStream_t s) {
    const dim3 blk(WAVE * WAVES);
    if constexpr (packs<D, true, MODE, WAVES, TH>()) {
        if (pk) {
            hipLaunchKernelGGL((k_batch<D, MODE, WAVES, TH, U, true>), dim3(grid), blk, 0, s, d, n, total);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_batch<D, MODE, WAVES, TH, U, false>), dim3(grid), blk, 0, s, d, n, total);
    return hipGetLastError();
}

template <class D, int MODE, int WAVES, bool U>
hipError_t launch_batch_th(const ImgDev *d, int n, int64_t total, int th, bool pk, int grid,
                           hipStream_t s) {
    switch (th) {
    case 4: return launch_batch_k<D, MODE, WAVES, 4, U>(d, n, total, pk, grid, s);
    case 8: return launch_batch_k<D, MODE, WAVES, 8, U>(d, n, total, pk, grid, s);
    default: return launch_batch_k<D, MODE, WAVES, 0, U>(d, n, total, pk, grid, s);
    }
}

template <class D, int MODE, bool U>
hipError_t launch_batch_w(const ImgDev *d, int n, int64_t total, int waves, int th, bool pk,
                          int grid, hipStream_t s) {
    switch (waves) {
    case 1: return launch_batch_th<D, MODE, 1, U>(d, n, total, th, pk, grid, s);
    case 2: return launch_batch_th<D, MODE, 2, U>(d, n, total, th, pk, grid, s);
    default: return launch_batch_th<D, MODE, 4, U>(d, n, total, th, pk, grid, s);
    }
}

template <class D, bool U>
hipError_t launch_batch_m(const ImgDev *d, int n, int64_t total, int mode, int waves, int th,
                          bool pk, int grid, hipStream_t s) {
    return mode == MODE_DIRECT25
               ? launch_batch_w<D, MODE_DIRECT25, U>(d, n, total, waves, th, pk, grid, s)
               : launch_batch_w<D, MODE_FUSED, U>(d, n, total, waves, th, pk, grid, s);
}

template <class D>
hipError_t launch_batch_t(const ImgDev *d, int n, int64_t total, int mode, int waves, int th,
                          int grid, int flags, hipStream_t s) {
    const bool pk = (flags & kBatchAnyPacked) != 0;
    return (flags & kBatchAnyUnaligned)
               ? launch_batch_m<D, true>(d, n, total, mode, waves, th, pk, grid, s)
               : launch_batch_m<D, false>(d, n, total, mode, waves, th, pk, grid, s);
}

template <class D, int MODE, int WAVES, int TH, bool U>
hipError_t launch_batch_args_k(const BatchArgs &a, bool pk, int grid, hipStream_t s) {
    const dim3 blk(WAVE * WAVES);
    if constexpr (packs<D, true, MODE, WAVES, TH>()) {
        if (pk) {
            hipLaunchKernelGGL((k_batch_args<D, MODE, WAVES, TH, U, true>), dim3(grid), blk, 0, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_batch_args<D, MODE, WAVES, TH, U, false>), dim3(grid), blk, 0, s, a);
    return hipGetLastError();
}

template <class D, int MODE, int WAVES, bool U>
hipError_t launch_batch_args_th(const BatchArgs &a, int th, bool pk, int grid, hipStream_t s) {
    switch (th) {
    case 4: return launch_batch_args_k<D, MODE, WAVES, 4, U>(a, pk, grid, s);
    case 8: return launch_batch_args_k<D, MODE, WAVES, 8, U>(a, pk, grid, s);
    default: return launch_batch_args_k<D, MODE, WAVES, 0, U>(a, pk, grid, s);
    }
}

template <class D, int MODE, bool U>
hipError_t launch_batch_args_w(const BatchArgs &a, int waves, int th, bool pk, int grid,
                               hipStream_t s) {
    switch (waves) {
    case 1: return launch_batch_args_th<D, MODE, 1, U>(a, th, pk, grid, s);
    case 2: return launch_batch_args_th<D, MODE, 2, U>(a, th, pk, grid, s);
    default: return launch_batch_args_th<D, MODE, 4, U>(a, th, pk, grid, s);
    }
}

template <class D, bool U>
hipError_t launch_batch_args_m(const BatchArgs &a, int mode, int waves, int th, bool pk, int grid,
                               hipStream_t s) {
    return mode == MODE_DIRECT25
               ? launch_batch_args_w<D, MODE_DIRECT25, U>(a, waves, th, pk, grid, s)
               : launch_batch_args_w<D, MODE_FUSED, U>(a, waves, th, pk, grid, s);
}

template <class D>
hipError_t launch_batch_args_t(const BatchArgs &a, int mode, int waves, int th, int grid,
                               int flags, hipStream_t s) {
    const bool pk = (flags & kBatchAnyPacked) != 0;
    return (flags & kBatchAnyUnaligned)
               ? launch_batch_args_m<D, true>(a, mode, waves, th, pk, grid, s)
               : launch_batch_args_m<D, false>(a, mode, waves, th, pk, grid, s);
}

}  // namespace

}  // namespace convsep5
