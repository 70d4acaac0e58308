// conv_kernels_hwc.hip -- the width-5 separable convolution of images whose
// colour planes are interleaved per pixel (packed HWC: element (p, y, x) at
// y*pitch + x*P + p, P = 2..4 channels).  Each channel is convolved on its
// own (Eq. 1 of arXiv 1711.09791 per plane), with its own 2-pixel frame of
// zeros.
//
// In a row of P*cols elements, channel p's horizontal neighbours of element
// e are e -+ P and e -+ 2P, so the row filter is a 5-tap filter with stride P
// along the flat row, with a frame of 2P elements; rows and the vertical
// filter are as in the planar kernels.  Each lane holds VEC consecutive
// elements of the flat row (one 16-byte load), regardless of pixel
// boundaries.  The 2P-element halos come from the HL = ceil(2P/VEC)
// neighbouring lanes on each side by DPP; the HL lanes at each end of the
// wave only load (their strips overlap the neighbouring strips), so no lane
// holds extra halo registers.  The FMA chains are those of the planar
// kernels, so results equal the planar result of the same image bitwise.
// Forms: fused and direct 25-tap single pass, two-pass row and column
// kernels (the FP32 intermediate keeps the HWC row layout, dense rows of
// P*cols floats).
#include "conv_kernels.h"

namespace convsep5 {
namespace {

template <class D, int P> struct HwcGeom {
    static constexpr int VEC = D::VEC;
    static constexpr int HL = (2 * P + VEC - 1) / VEC;   // halo lanes per side
    static constexpr int OUT = hwc_out_per_strip(VEC, P);  // output elements per strip
    static constexpr int E = VEC * (2 * HL + 1);          // window elements per lane
};

// The lane's VEC elements of one row: one 16-byte load (aligned layouts) or
// VEC element loads; elements outside the row read 0.
template <class D, bool AL> struct RawH { uint32_t w[AL ? 4 : D::VEC]; };

template <class D, bool AL>
__device__ __forceinline__ void issue_h(RawH<D, AL> &r, const char *row, uint32_t rbytes, int x) {
    const auto rs = row_rsrc(row, rbytes);
    if constexpr (AL) {
        const u4 q = __builtin_amdgcn_raw_buffer_load_b128(rs, x >= 0 ? x * D::ESZ : OOB, 0, 0);
        r.w[0] = q.x;
        r.w[1] = q.y;
        r.w[2] = q.z;
        r.w[3] = q.w;
    } else {
#pragma unroll
        for (int e = 0; e < D::VEC; ++e) {
            const int off = x + e >= 0 ? (x + e) * D::ESZ : OOB;
            if constexpr (D::ESZ == 4)
                r.w[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
            else
                r.w[e] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
        }
    }
}

// The lane's own VEC elements as FP32.
template <class D, bool AL>
__device__ __forceinline__ void own_h(const RawH<D, AL> &r, float (&u)[D::VEC]) {
    if constexpr (!AL || D::ESZ == 4) {
#pragma unroll
        for (int e = 0; e < D::VEC; ++e) u[e] = dec(D{}, r.w[e]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            u[2 * j] = dec(D{}, r.w[j]);
            u[2 * j + 1] = dec(D{}, r.w[j] >> 16);
        }
    }
}

// v[i] = row[x - HL*VEC + i]: the own elements of lanes l-HL .. l+HL, moved
// across lanes one step at a time (end lanes get 0; they produce nothing).
template <class D, int P>
__device__ __forceinline__ void window_h(const float (&u)[D::VEC], float (&v)[HwcGeom<D, P>::E]) {
    constexpr int VEC = D::VEC, HL = HwcGeom<D, P>::HL;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[HL * VEC + e] = u[e];
#pragma unroll
    for (int d = 1; d <= HL; ++d) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            v[(HL - d) * VEC + e] =
                __uint_as_float(from_left(__float_as_uint(v[(HL - d + 1) * VEC + e]), 0u));
            v[(HL + d) * VEC + e] =
                __uint_as_float(from_right(__float_as_uint(v[(HL + d - 1) * VEC + e]), 0u));
        }
    }
}

// One band of TH rows of one strip: lane l loads flat elements x .. x+VEC-1
// (x = xs - HL*VEC + l*VEC) and, for HL <= l < 64-HL, produces them.
template <class D, bool AL, int P, int MODE, bool EDGE, int TH, int SAUX = NT>
__device__ __forceinline__ void band_h(const ImgDev &im, int xs, int y0, int y1, int lane) {
    using G = HwcGeom<D, P>;
    constexpr int VEC = G::VEC, HL = G::HL, E = G::E;
    constexpr int O = HL * VEC - 2 * P;  // window index of the first tap of element 0
    const int H = im.rows, WF = im.cols * P;  // flat row length
    const int x = xs - HL * VEC + lane * VEC;
    const bool producer = lane >= HL && lane < WAVE - HL;
    bool cm[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) cm[e] = (x + e >= 2 * P) && (x + e < WF - 2 * P);
    const char *sbase = (const char *)im.in;
    const int64_t sstride = im.pitch * D::ESZ;
    const uint32_t sbytes = (uint32_t)WF * D::ESZ;
    const float *k = im.tp.k;

    auto hrow = [&](const float (&v)[E], float (&h)[VEC]) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            float t = v[O + e] * k[0];
            t = __builtin_fmaf(v[O + e + P], k[1], t);
            t = __builtin_fmaf(v[O + e + 2 * P], k[2], t);
            t = __builtin_fmaf(v[O + e + 3 * P], k[3], t);
            t = __builtin_fmaf(v[O + e + 4 * P], k[4], t);
            h[e] = t;
        }
    };

    if constexpr (MODE == MODE_ROWPASS) {
        char *tbase = (char *)im.tmp;
        RawH<D, AL> raw[TH];
#pragma unroll
        for (int i = 0; i < TH; ++i)
            issue_h<D, AL>(raw[i], sbase + (int64_t)min(y0 + i, y1 - 1) * sstride, sbytes, x);
#pragma unroll
        for (int i = 0; i < TH; ++i) {
            float u[VEC], v[E], h[VEC];
            own_h<D, AL>(raw[i], u);
            window_h<D, P>(u, v);
            hrow(v, h);
            if constexpr (EDGE) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) h[e] = cm[e] ? h[e] : 0.0f;
            }
            if (producer && y0 + i < y1)  // T stays cached for the column kernel
                store_t<VEC, AL, 0>(tbase + (int64_t)(y0 + i) * WF * 4, (uint32_t)WF * 4, x, h);
        }
        return;
    } else {
        constexpr bool COL = MODE == MODE_COLPASS;
        constexpr bool DIRECT = MODE == MODE_DIRECT25;
        constexpr int WN = DIRECT ? E : VEC;
        using RawIn = typename std::conditional<COL, RawT<VEC, AL>, RawH<D, AL>>::type;
        RawIn raw[TH + 4];
#pragma unroll
        for (int i = 0; i < TH + 4; ++i) {
            const int row = clampi(y0 - 2 + i, 0, H - 1);
            if constexpr (COL) {
                // the column kernel needs no halo: end lanes skip their loads
                issue_t<VEC, AL>(raw[i], (const char *)im.tmp + (int64_t)row * WF * 4,
                                 producer ? (uint32_t)WF * 4 : 0u, x);
            } else {
                issue_h<D, AL>(raw[i], sbase + (int64_t)row * sstride, sbytes, x);
            }
        }
        char *dbase = (char *)im.out;
        const int64_t dstride = im.pitch * D::ESZ;
        // window rows are produced in order and output row j is emitted as
        // soon as rows j .. j+4 exist, so only five window rows are live
        float w[TH + 4][WN];
#pragma unroll
        for (int i = 0; i < TH + 4; ++i) {
            if constexpr (COL) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) w[i][e] = __uint_as_float(raw[i].w[e]);
            } else {
                float u[VEC];
                own_h<D, AL>(raw[i], u);
                if constexpr (DIRECT) {
                    window_h<D, P>(u, w[i]);
                } else {
                    float v[E];
                    window_h<D, P>(u, v);
                    hrow(v, w[i]);
                }
            }
            if (i < 4) continue;
            const int j = i - 4;
            const int y = y0 + j;
            if (y >= y1) continue;
            float o[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if constexpr (DIRECT) {
                    float p[5];
#pragma unroll
                    for (int a = 0; a < 5; ++a) {
                        float t = w[j + a][O + e] * im.tp.K[5 * a];
#pragma unroll
                        for (int b = 1; b < 5; ++b)
                            t = __builtin_fmaf(w[j + a][O + e + b * P], im.tp.K[5 * a + b], t);
                        p[a] = t;
                    }
                    o[e] = ((p[0] + p[1]) + (p[2] + p[3])) + p[4];
                } else {
                    float t = w[j][e] * k[0];
                    t = __builtin_fmaf(w[j + 1][e], k[1], t);
                    t = __builtin_fmaf(w[j + 2][e], k[2], t);
                    t = __builtin_fmaf(w[j + 3][e], k[3], t);
                    t = __builtin_fmaf(w[j + 4][e], k[4], t);
                    o[e] = t;
                }
            }
            if constexpr (EDGE) {
                const bool vr = (y >= 2) && (y < H - 2);
#pragma unroll
                for (int e = 0; e < VEC; ++e) o[e] = (vr && cm[e]) ? o[e] : 0.0f;
            }
            // end lanes store nothing: an empty range drops their stores
            store_out<D, AL, SAUX>(dbase + (int64_t)y * dstride, producer ? (uint32_t)WF * D::ESZ : 0u,
                             x, o);
        }
    }
}

// Logical tile (band, strip), strip fastest; one wave per workgroup; XCDs
// take turns on chunks of im.xcd_slabs band rows when that is >= 2.
template <class D, bool AL, int P, int MODE, int TH, int SAUX = NT>
__global__ __launch_bounds__(WAVE) void k_hwc(ImgDev im, int64_t nblocks) {
    using G = HwcGeom<D, P>;
    const int lane = threadIdx.x;
    for (int64_t base = 0; base < nblocks; base += gridDim.x) {
        const int64_t left = nblocks - base;
        const int cnt = left < (int64_t)gridDim.x ? (int)left : (int)gridDim.x;
        if ((int)blockIdx.x >= cnt) break;
        const int b = im.xcd_slabs > 1
                          ? xcd_chunk_remap(blockIdx.x, cnt, (int64_t)im.xcd_slabs * im.ns)
                          : (int)blockIdx.x;
        const int64_t lt = base + b;
        const int strip = (int)(lt % im.ns);
        const int band = (int)(lt / im.ns);
        const int xs = strip * G::OUT;
        const int y0 = band * TH;
        const int y1 = min(y0 + TH, im.rows);
        const int WF = im.cols * P;
        const bool col_edge = xs < 2 * P || xs + G::OUT > WF - 2 * P;
        const bool row_edge = MODE != MODE_ROWPASS && (y0 < 2 || y0 + TH > im.rows - 2);
        if (col_edge || row_edge)
            band_h<D, AL, P, MODE, true, TH, SAUX>(im, xs, y0, y1, lane);
        else
            band_h<D, AL, P, MODE, false, TH, SAUX>(im, xs, y0, y1, lane);
    }
}

template <class D, bool AL, int P>
hipError_t launch_hwc_p(const ImgDev &im, int mode, int64_t nblocks, hipStream_t s) {
    const int grid = (int)(nblocks < (1 << 20) ? nblocks : (1 << 20));
    constexpr int TH = kThHwc;
    // keep_out (the copy-back scratch): cached output stores in kernels of
    // their own
    const bool keep = im.keep_out != 0;
    switch (mode) {
    case MODE_FUSED:
        if (keep)
            hipLaunchKernelGGL((k_hwc<D, AL, P, MODE_FUSED, TH, 0>), dim3(grid), dim3(WAVE), 0, s, im,
                               nblocks);
        else
            hipLaunchKernelGGL((k_hwc<D, AL, P, MODE_FUSED, TH>), dim3(grid), dim3(WAVE), 0, s, im,
                               nblocks);
        break;
    case MODE_DIRECT25:
        if (keep)
            hipLaunchKernelGGL((k_hwc<D, AL, P, MODE_DIRECT25, TH, 0>), dim3(grid), dim3(WAVE), 0, s,
                               im, nblocks);
        else
            hipLaunchKernelGGL((k_hwc<D, AL, P, MODE_DIRECT25, TH>), dim3(grid), dim3(WAVE), 0, s, im,
                               nblocks);
        break;
    case MODE_ROWPASS:
        hipLaunchKernelGGL((k_hwc<D, AL, P, MODE_ROWPASS, TH>), dim3(grid), dim3(WAVE), 0, s, im,
                           nblocks);
        break;
    default:
        hipLaunchKernelGGL((k_hwc<D, AL, P, MODE_COLPASS, TH>), dim3(grid), dim3(WAVE), 0, s, im,
                           nblocks);
        break;
    }
    return hipGetLastError();
}

template <class D, bool AL>
hipError_t launch_hwc_a(const ImgDev &im, int mode, int64_t nblocks, hipStream_t s) {
    switch (im.planes) {
    case 2: return launch_hwc_p<D, AL, 2>(im, mode, nblocks, s);
    case 3: return launch_hwc_p<D, AL, 3>(im, mode, nblocks, s);
    default: return launch_hwc_p<D, AL, 4>(im, mode, nblocks, s);
    }
}

template <class D>
hipError_t launch_hwc_t(const ImgDev &im, int mode, int64_t nblocks, hipStream_t s) {
    return im.aligned ? launch_hwc_a<D, true>(im, mode, nblocks, s)
                      : launch_hwc_a<D, false>(im, mode, nblocks, s);
}

}  // namespace

hipError_t launch_hwc(const ImgDev &im, int dtype, int mode, int64_t nblocks, hipStream_t s) {
    return dtype == 0 ? launch_hwc_t<F32>(im, mode, nblocks, s)
         : dtype == 1 ? launch_hwc_t<F16>(im, mode, nblocks, s)
                      : launch_hwc_t<BF16>(im, mode, nblocks, s);
}

}  // namespace convsep5
