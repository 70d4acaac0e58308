// conv_kernels_pyr.hip -- one Gaussian-pyramid level: the width-5 separable
// convolution (Eq. 1 of arXiv 1711.09791 with its zero border) sampled at
// every second row and column, fused into one pass.  The paper names image
// scaling as the step of its application next to the convolution but does
// not define it; this is the blur-then-decimate reading:
//   out[p][yo][xo] = B[p][2 yo][2 xo],  yo < ceil(rows/2), xo < ceil(cols/2)
// where B is the convolution with its 2-pixel frame of zeros.
//
// Only the sampled values are computed: the horizontal filter runs at even
// columns of the 2*TH+3 input rows a band of TH output rows needs, the
// vertical filter at even rows.  Each value is the same FMA chain (taps in
// order k0..k4, horizontal then vertical) as in the fused width-5 kernel,
// so the output equals that kernel's result at the sampled pixels bitwise.
// Traffic: 1 read of the input + 1/4 write per input plane-pixel.
#include "conv_kernels.h"

namespace convsep5 {
namespace {

// Aligned stores of the VEC/2 outputs of a lane: 8 bytes (2 FP32 or 4 16-bit
// values); unaligned layouts store element by element.
template <class D, bool AL>
__device__ __forceinline__ void store_half(char *row, uint32_t rbytes, int xo,
                                           const float (&o)[D::VEC / 2]) {
    const auto rs = row_rsrc(row, rbytes);
    constexpr int H = D::VEC / 2;
    if constexpr (AL) {
        u2 q;
        if constexpr (D::ESZ == 4)
            q = u2{__float_as_uint(o[0]), __float_as_uint(o[1])};
        else
            q = u2{enc2(D{}, o[0], o[1]), enc2(D{}, o[2], o[3])};
        __builtin_amdgcn_raw_buffer_store_b64(q, rs, xo * D::ESZ, 0, NT);
    } else if constexpr (D::ESZ == 4) {
#pragma unroll
        for (int e = 0; e < H; ++e)
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o[e]), rs, (xo + e) * 4, 0, NT);
    } else {
#pragma unroll
        for (int e = 0; e < H; e += 2) {
            const uint32_t w = enc2(D{}, o[e], o[e + 1]);
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w & 0xffffu), rs, (xo + e) * 2, 0, NT);
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(w >> 16), rs, (xo + e + 1) * 2, 0, NT);
        }
    }
}

// One band of TH output rows of one column strip.  The lane holds input
// columns x .. x+VEC-1 (x even) and produces output columns x/2 .. x/2+VEC/2-1.
template <class D, bool AL, bool EDGE, int TH>
__device__ __forceinline__ void band_pyr(const PyrDev &pd, int plane, int xs, int yo0, int lane) {
    constexpr int VEC = D::VEC, HV = VEC / 2, NIN = 2 * TH + 3;
    const int H = pd.rows, W = pd.cols;
    const int x = xs + lane * VEC, xo = x / 2;
    const char *sbase = (const char *)pd.in + (int64_t)plane * pd.in_ps * D::ESZ;
    const int64_t sstride = pd.in_pitch * D::ESZ;
    const uint32_t sbytes = (uint32_t)W * D::ESZ;
    char *dbase = (char *)pd.out + (int64_t)plane * pd.out_ps * D::ESZ;
    const int64_t dstride = pd.out_pitch * D::ESZ;
    const uint32_t dbytes = (uint32_t)pd.ocols * D::ESZ;
    const int hl = xs - 2, hr = xs + WAVE * VEC;
    const int hoff = lane == 0 ? (hl >= 0 ? hl * D::ESZ : OOB)
                               : (lane == WAVE - 1 ? (hr < W ? hr * D::ESZ : OOB) : OOB);
    // input rows 2*yo0-2 .. 2*yo0+2*TH, clamped; clamped rows only feed
    // outputs whose source row lies in the frame, which are written as 0
    Raw<D, AL> raw[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i)
        issue<D>(raw[i], sbase + (int64_t)clampi(2 * yo0 - 2 + i, 0, H - 1) * sstride, sbytes, x,
                 hoff);
    float h[NIN][HV];
#pragma unroll
    for (int i = 0; i < NIN; ++i) {
        float v[VEC + 4];
        decode<D>(raw[i], v);
#pragma unroll
        for (int e = 0; e < HV; ++e) {
            float t = v[2 * e] * pd.k[0];
            t = __builtin_fmaf(v[2 * e + 1], pd.k[1], t);
            t = __builtin_fmaf(v[2 * e + 2], pd.k[2], t);
            t = __builtin_fmaf(v[2 * e + 3], pd.k[3], t);
            t = __builtin_fmaf(v[2 * e + 4], pd.k[4], t);
            h[i][e] = t;
        }
    }
    bool cm[HV];
#pragma unroll
    for (int e = 0; e < HV; ++e) cm[e] = (x + 2 * e >= 2) && (x + 2 * e < W - 2);
#pragma unroll
    for (int j = 0; j < TH; ++j) {
        const int yo = yo0 + j;
        if (yo >= pd.orows) break;
        float o[HV];
#pragma unroll
        for (int e = 0; e < HV; ++e) {
            float t = h[2 * j][e] * pd.k[0];
            t = __builtin_fmaf(h[2 * j + 1][e], pd.k[1], t);
            t = __builtin_fmaf(h[2 * j + 2][e], pd.k[2], t);
            t = __builtin_fmaf(h[2 * j + 3][e], pd.k[3], t);
            t = __builtin_fmaf(h[2 * j + 4][e], pd.k[4], t);
            o[e] = t;
        }
        if constexpr (EDGE) {
            const bool vr = (2 * yo >= 2) && (2 * yo < H - 2);
#pragma unroll
            for (int e = 0; e < HV; ++e) o[e] = (vr && cm[e]) ? o[e] : 0.0f;
        }
        store_half<D, AL>(dbase + (int64_t)yo * dstride, dbytes, xo, o);
    }
}

// Logical tile (plane, band, strip), strip fastest; one wave per workgroup.
template <class D, bool AL, int TH>
__global__ __launch_bounds__(WAVE) void k_pyr(PyrDev pd, int64_t nblocks) {
    const int lane = threadIdx.x;
    for (int64_t base = 0; base < nblocks; base += gridDim.x) {
        const int64_t left = nblocks - base;
        const int cnt = left < (int64_t)gridDim.x ? (int)left : (int)gridDim.x;
        if ((int)blockIdx.x >= cnt) break;
        const int b = pd.xcd_chunk > 1
                          ? xcd_chunk_remap(blockIdx.x, cnt, (int64_t)pd.xcd_chunk * pd.ns)
                          : (int)blockIdx.x;
        const int64_t lt = base + b;
        const int strip = (int)(lt % pd.ns);
        const int64_t t = lt / pd.ns;
        const int band = (int)(t % pd.nb);
        const int plane = (int)(t / pd.nb);
        const int xs = strip * (WAVE * D::VEC);
        const int yo0 = band * TH;
        const int W = pd.cols, H = pd.rows;
        const bool col_edge = xs < 2 || xs + WAVE * D::VEC > W - 2;
        const bool row_edge = 2 * yo0 < 2 || 2 * (yo0 + TH - 1) >= H - 2;
        if (col_edge || row_edge)
            band_pyr<D, AL, true, TH>(pd, plane, xs, yo0, lane);
        else
            band_pyr<D, AL, false, TH>(pd, plane, xs, yo0, lane);
    }
}

template <class D>
hipError_t launch_pyr_t(const PyrDev &pd, int64_t nblocks, hipStream_t s) {
    const int grid = (int)(nblocks < (1 << 20) ? nblocks : (1 << 20));
    if (pd.aligned)
        hipLaunchKernelGGL((k_pyr<D, true, kThPyr>), dim3(grid), dim3(WAVE), 0, s, pd, nblocks);
    else
        hipLaunchKernelGGL((k_pyr<D, false, kThPyr>), dim3(grid), dim3(WAVE), 0, s, pd, nblocks);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pyr(const PyrDev &pd, int dtype, int64_t nblocks, hipStream_t s) {
    return dtype == 0 ? launch_pyr_t<F32>(pd, nblocks, s)
         : dtype == 1 ? launch_pyr_t<F16>(pd, nblocks, s)
                      : launch_pyr_t<BF16>(pd, nblocks, s);
}

}  // namespace convsep5
