// Counter-based random numbers of the integrators: Philox4x32-10 (Salmon,
// Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11)
// and the Box-Muller map of its words to Gaussians (Section III.C draws the
// random force from Gaussian numbers; this generator replaces the paper's
// Hybrid Taus).
#pragma once

#include <hip/hip_runtime.h>

namespace sop {

__device__ __forceinline__ uint4 philox10(uint4 c, unsigned k0, unsigned k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const unsigned hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const unsigned hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Uniform in (0,1) from the top 23 bits: exact in single precision.
__device__ __forceinline__ float unit23(unsigned w)
{
    return (static_cast<float>(w >> 9) + 0.5f) * 0x1p-23f;
}

// Box-Muller: axis 0/1 = radius(u0) * (cos, sin)(2 pi u1), axis 2 =
// radius(u2) * cos(2 pi u3). The logarithm, sine and cosine are the
// hardware ones (the sine and cosine take the angle in turns, so they give
// sin(2 pi u) directly): over all 2^23 uniforms the radius is within 5.7e-7
// and the sine and cosine within 1.3e-7 of FP64, against 5.7e-7 and 5e-8 for
// the library's FP32 functions, at a third of the instructions.
__device__ __forceinline__ float gaussian_axis(const uint4 &w, int axis)
{
    const float ur = unit23(axis < 2 ? w.x : w.z);
    const float ua = unit23(axis < 2 ? w.y : w.w);
    const float rad = __fsqrt_rn(-2.0f * __logf(ur));
    return rad * (axis == 1 ? __builtin_amdgcn_sinf(ua) : __builtin_amdgcn_cosf(ua));
}

// Axes 0 and 1 together (one radius, one angle); equal to gaussian_axis.
__device__ __forceinline__ float2 gaussian_pair(const uint4 &w)
{
    const float rad = __fsqrt_rn(-2.0f * __logf(unit23(w.x)));
    const float ua = unit23(w.y);
    return make_float2(rad * __builtin_amdgcn_cosf(ua), rad * __builtin_amdgcn_sinf(ua));
}

}  // namespace sop
