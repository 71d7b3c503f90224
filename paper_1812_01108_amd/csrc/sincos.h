// Branch-free float32 sine/cosine for the angle ingest.
//
// Reduction by pi/2 in the three-part Cody-Waite manner (Cody & Waite,
// "Software Manual for the Elementary Functions", 1980), each part applied
// with an FMA, then polynomials on [-pi/4, pi/4]:
//   sin r = r + r^3 (s1 + s2 r^2 + s3 r^4),
//   cos r = 1 + r^2 (c1 + c2 r^2 + c3 r^4 + c4 r^6),
// whose coefficients were fitted for this library by a discrete minimax
// (Lawson-weighted least squares) in double and rounded to float32.  For
// |x| <= 1e5 the absolute error is below 8e-8 (about 1.5 ulp on (-pi, pi]).
// Callers take sincos_accurate instead when any lane of the wave holds an
// argument outside that range or a non-finite one.
#pragma once
#include <hip/hip_runtime.h>

namespace a2c {

constexpr float kSinCosFastLimit = 1.0e5f;

// The library's sinf and cosf, taken by value: sincosf returns one result
// through a pointer, which makes the caller's destination array addressable
// and moves it to scratch memory for the whole kernel.
__device__ __forceinline__ void sincos_accurate(float x, float &s, float &c)
{
    s = sinf(x);
    c = cosf(x);
}

__device__ __forceinline__ void sincos_fast(float x, float &s, float &c)
{
    const float k = rintf(x * 0.636619772f);            // x / (pi/2), rounded
    float r = fmaf(-k, 1.57079637e+00f, x);             // pi/2 = p1 + p2 + p3
    r = fmaf(-k, -4.37113883e-08f, r);
    r = fmaf(-k, -1.77635684e-15f, r);
    const float r2 = r * r;
    const float ps = fmaf(fmaf(-1.95172994e-04f, r2, 8.33217800e-03f), r2, -1.66666552e-01f);
    const float sr = fmaf(r2 * r, ps, r);
    const float pc = fmaf(fmaf(fmaf(2.43904506e-05f, r2, -1.38867635e-03f), r2, 4.16666232e-02f),
                          r2, -5.0e-01f);
    const float cr = fmaf(r2, pc, 1.0f);
    const int q = (int)k & 3;                            // quadrant
    const float s0 = (q & 1) ? cr : sr;
    const float c0 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
}

__device__ __forceinline__ bool sincos_fast_ok(float x) { return fabsf(x) <= kSinCosFastLimit; }

}  // namespace a2c
