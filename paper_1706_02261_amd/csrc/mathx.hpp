// Small device math for the march.
#pragma once

#include <hip/hip_runtime.h>

namespace bpm {

// (cos r, sin r) for |r| <= pi/4: Taylor series of sin and cos truncated
// after r^9 and r^10 (remainders below 2e-11 and 2e-9 on that interval).
__device__ __forceinline__ float2 cos_sin_quarter(float r) {
    const float r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - r^6/7! + r^8/9!)
    float ps = fmaf(r2, 2.75573192239858906526e-6f, -1.98412698412698412698e-4f);
    ps = fmaf(r2, ps, 8.33333333333333333333e-3f);
    ps = fmaf(r2, ps, -1.66666666666666666667e-1f);
    const float s = fmaf(r * r2, ps, r);
    // cos r = 1 - r^2/2! + r^4/4! - r^6/6! + r^8/8! - r^10/10!
    float pc = fmaf(r2, -2.75573192239858906526e-7f, 2.48015873015873015873e-5f);
    pc = fmaf(r2, pc, -1.38888888888888888889e-3f);
    pc = fmaf(r2, pc, 4.16666666666666666667e-2f);
    pc = fmaf(r2, pc, -0.5f);
    const float c = fmaf(r2, pc, 1.0f);
    return make_float2(c, s);
}

constexpr float kQuarterPi = 0.785398163397448309616f;

// (cos x, sin x) in fp32 for |x| up to ~1e4: Cody-Waite reduction
// x = q (pi/2) + r with a two-term pi/2 (the fp32 nearest value plus its
// residual), cos_sin_quarter(r), then the quadrant rotation by q.
__device__ __forceinline__ float2 expi(float x) {
    constexpr float kTwoOverPi = 0.636619772367581343f;
    constexpr float kPio2Hi = 1.57079637050628662109375f;      // fp32(pi/2)
    constexpr float kPio2Lo = -4.37113900018624283e-8f;        // pi/2 - kPio2Hi
    const float q = rintf(x * kTwoOverPi);
    float r = fmaf(q, -kPio2Hi, x);
    r = fmaf(q, -kPio2Lo, r);
    const float2 cs0 = cos_sin_quarter(r);
    const float c = cs0.x, s = cs0.y;
    const int iq = static_cast<int>(q) & 3;
    const float cs = (iq & 1) ? s : c;   // |cos x| candidate
    const float sn = (iq & 1) ? c : s;   // |sin x| candidate
    const float cx = (iq == 1 || iq == 2) ? -cs : cs;
    const float sx = (iq >= 2) ? -sn : sn;
    return make_float2(cx, sx);
}

}  // namespace bpm
