// Device helpers shared by the HIP translation units of the library: complex
// arithmetic, the 4+4-bit decoder and a register-resident 8-point DFT.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace epic {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc + a * b
__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
    return acc;
}

// Two and four FP16 values (a decoded sample, a dual-pol antenna).
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));

// One 4+4-bit complex sample (Sec. 2.1): two two's-complement nibbles, the
// real part in the high nibble for order 0, in the low nibble for order 1.
// Every value in [-8, 7] is exact in FP32 (and in FP16 / FP8 e4m3).
__device__ __forceinline__ float2 unpack44(uint32_t byte, int order) {
    const int hi = ((int)(byte << 24)) >> 28;
    const int lo = ((int)(byte << 28)) >> 28;
    return order == 0 ? make_float2((float)hi, (float)lo) : make_float2((float)lo, (float)hi);
}

// The same sample held in FP16 (exact: |value| <= 8).
__device__ __forceinline__ h2v unpack44_h(uint32_t byte, int order) {
    const float2 v = unpack44(byte, order);
    return h2v{(_Float16)v.x, (_Float16)v.y};
}

// Radix-4 butterfly with the positive exponent (exp(+2 pi i nk/4) = i^nk):
// (a, b, c, d) -> (Y0, Y1, Y2, Y3).
__device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d) {
    const float2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = csub(b, d);
    a = cadd(s0, s1);
    c = csub(s0, s1);
    b = make_float2(d0.x - d1.y, d0.y + d1.x);   // d0 + i d1
    d = make_float2(d0.x + d1.y, d0.y - d1.x);   // d0 - i d1
}

// In-place 8-point DFT X[m] = sum_n z[n] exp(+2 pi i n m / 8), as 4 x 2
// (n = 2 n1 + n2, m = m1 + 4 m2).  On return X[m] is held in z[fft8_pos(m)].
__device__ __forceinline__ constexpr int fft8_pos(int m) { return 2 * (m & 3) + (m >> 2); }

__device__ __forceinline__ void fft8(float2 (&z)[8]) {
    constexpr float h = 0.707106781186547524f;   // cos(pi/4)
    dft4(z[0], z[2], z[4], z[6]);   // n2 = 0: z[2 m1] = A0[m1]
    dft4(z[1], z[3], z[5], z[7]);   // n2 = 1: z[2 m1 + 1] = A1[m1]
    // A1[m1] *= exp(+2 pi i m1 / 8)
    z[3] = make_float2(h * (z[3].x - z[3].y), h * (z[3].x + z[3].y));     // W^1
    z[5] = make_float2(-z[5].y, z[5].x);                                  // W^2 = i
    z[7] = make_float2(-h * (z[7].x + z[7].y), h * (z[7].x - z[7].y));    // W^3
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1) {
        const float2 a = z[2 * m1], b = z[2 * m1 + 1];
        z[2 * m1] = cadd(a, b);          // X[m1]
        z[2 * m1 + 1] = csub(a, b);      // X[m1 + 4]
    }
}

// Add a workgroup's sum into its partial-accumulator slot.  On the first
// call after a reset the slots hold zeros, so the sum is stored without
// reading the slot first (0 + v == v bitwise: the sums never hold -0).
__device__ __forceinline__ void slot_put(float* p, float v, bool fresh) {
    if (fresh) *p = v;
    else *p += v;
}

}  // namespace epic
