// Gridding helpers shared by the FP32 and matrix-core kernels: one group of
// kGroup gather entries (antenna index + weight per pol) applied to the decoded
// samples of one spectrum, and the group weight layout.
#pragma once

#include <hip/hip_runtime.h>

#include "epic_device.hpp"
#include "epic_internal.hpp"

namespace epic {

// Gather weight modes: complex weights (re, im per pol), real weights per pol,
// or one real weight shared by both pols (X and Y taps equal, the default
// Gaussian kernel).
constexpr int kWComplex = 0, kWReal = 1, kWShared = 2;

// Decoded samples of one antenna, held in FP32 (float2 per pol) or FP16
// (h2v per pol; the 4-bit values are exact, and the FMAs below convert them
// on the fly, so both give the same sums while FP16 halves the LDS traffic).
__device__ __forceinline__ float4 smp_both(const float2* __restrict__ s, int a) {
    return reinterpret_cast<const float4*>(s)[a];
}
__device__ __forceinline__ float4 smp_both(const h2v* __restrict__ s, int a) {
    const h4v h = reinterpret_cast<const h4v*>(s)[a];
    return make_float4((float)h[0], (float)h[1], (float)h[2], (float)h[3]);
}
__device__ __forceinline__ float2 smp_one(const float2* __restrict__ s, int a) { return s[a]; }
__device__ __forceinline__ float2 smp_one(const h2v* __restrict__ s, int a) {
    const h2v h = s[a];
    return make_float2((float)h[0], (float)h[1]);
}

// ---- gather gridding of one group of kGroup entries ------------------------
template <int P, int WM, typename SmpT>
__device__ __forceinline__ void gather_group(float2& gx, float2& gy, const float4* __restrict__ w,
                                             const uint2 ia, const SmpT* __restrict__ smp) {
    const int a[4] = {(int)(ia.x & 0xFFFFu), (int)(ia.x >> 16), (int)(ia.y & 0xFFFFu), (int)(ia.y >> 16)};
    if constexpr (P == 2) {
        const float4 s0 = smp_both(smp, a[0]), s1 = smp_both(smp, a[1]), s2 = smp_both(smp, a[2]),
                     s3 = smp_both(smp, a[3]);
        if constexpr (WM == kWShared) {
            const float4 ww = w[0];   // (w0, w1, w2, w3), both pols
            gx.x = fmaf(ww.x, s0.x, gx.x); gx.y = fmaf(ww.x, s0.y, gx.y);
            gy.x = fmaf(ww.x, s0.z, gy.x); gy.y = fmaf(ww.x, s0.w, gy.y);
            gx.x = fmaf(ww.y, s1.x, gx.x); gx.y = fmaf(ww.y, s1.y, gx.y);
            gy.x = fmaf(ww.y, s1.z, gy.x); gy.y = fmaf(ww.y, s1.w, gy.y);
            gx.x = fmaf(ww.z, s2.x, gx.x); gx.y = fmaf(ww.z, s2.y, gx.y);
            gy.x = fmaf(ww.z, s2.z, gy.x); gy.y = fmaf(ww.z, s2.w, gy.y);
            gx.x = fmaf(ww.w, s3.x, gx.x); gx.y = fmaf(ww.w, s3.y, gx.y);
            gy.x = fmaf(ww.w, s3.z, gy.x); gy.y = fmaf(ww.w, s3.w, gy.y);
        } else if constexpr (WM == kWReal) {
            const float4 w01 = w[0], w23 = w[1];   // (w0x, w0y, w1x, w1y), (w2x, w2y, w3x, w3y)
            gx.x = fmaf(w01.x, s0.x, gx.x); gx.y = fmaf(w01.x, s0.y, gx.y);
            gy.x = fmaf(w01.y, s0.z, gy.x); gy.y = fmaf(w01.y, s0.w, gy.y);
            gx.x = fmaf(w01.z, s1.x, gx.x); gx.y = fmaf(w01.z, s1.y, gx.y);
            gy.x = fmaf(w01.w, s1.z, gy.x); gy.y = fmaf(w01.w, s1.w, gy.y);
            gx.x = fmaf(w23.x, s2.x, gx.x); gx.y = fmaf(w23.x, s2.y, gx.y);
            gy.x = fmaf(w23.y, s2.z, gy.x); gy.y = fmaf(w23.y, s2.w, gy.y);
            gx.x = fmaf(w23.z, s3.x, gx.x); gx.y = fmaf(w23.z, s3.y, gx.y);
            gy.x = fmaf(w23.w, s3.z, gy.x); gy.y = fmaf(w23.w, s3.w, gy.y);
        } else {
            const float4 ww[4] = {w[0], w[1], w[2], w[3]};   // (wxr, wxi, wyr, wyi) per entry
            const float4 ss[4] = {s0, s1, s2, s3};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                gx = cfma(gx, make_float2(ww[e].x, ww[e].y), make_float2(ss[e].x, ss[e].y));
                gy = cfma(gy, make_float2(ww[e].z, ww[e].w), make_float2(ss[e].z, ss[e].w));
            }
        }
    } else {
        const float2 s0 = smp_one(smp, a[0]), s1 = smp_one(smp, a[1]), s2 = smp_one(smp, a[2]),
                     s3 = smp_one(smp, a[3]);
        if constexpr (WM != kWComplex) {
            const float4 ww = w[0];
            gx.x = fmaf(ww.x, s0.x, gx.x); gx.y = fmaf(ww.x, s0.y, gx.y);
            gx.x = fmaf(ww.y, s1.x, gx.x); gx.y = fmaf(ww.y, s1.y, gx.y);
            gx.x = fmaf(ww.z, s2.x, gx.x); gx.y = fmaf(ww.z, s2.y, gx.y);
            gx.x = fmaf(ww.w, s3.x, gx.x); gx.y = fmaf(ww.w, s3.y, gx.y);
        } else {
            const float4 w01 = w[0], w23 = w[1];
            gx = cfma(gx, make_float2(w01.x, w01.y), s0);
            gx = cfma(gx, make_float2(w01.z, w01.w), s1);
            gx = cfma(gx, make_float2(w23.x, w23.y), s2);
            gx = cfma(gx, make_float2(w23.z, w23.w), s3);
        }
    }
}

template <int P, int WM>
constexpr int group_f4() {   // float4 words of weights per group
    return WM == kWComplex ? (P == 2 ? 4 : 2) : ((WM == kWReal && P == 2) ? 2 : 1);
}

// the same on the host; floats per entry = 4 * group_f4 / kGroup
inline int group_f4_of(int P, int wm) {
    return wm == kWComplex ? (P == 2 ? 4 : 2) : ((wm == kWReal && P == 2) ? 2 : 1);
}

}  // namespace epic
