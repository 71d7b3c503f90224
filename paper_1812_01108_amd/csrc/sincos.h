// Branch-free float32 sine/cosine for the angle ingest.
//
// Reduction by pi in the three-part Cody-Waite manner (Cody & Waite,
// "Software Manual for the Elementary Functions", 1980), each part applied
// with an FMA, then polynomials on [-pi/2, pi/2]:
//   sin r = r + r^3 (s1 + s2 r^2 + s3 r^4 + s4 r^6),
//   cos r = 1 + r^2 (c1 + c2 r^2 + c3 r^4 + c4 r^6 + c5 r^8),
// and sin x = (-1)^k sin r, cos x = (-1)^k cos r for x = k pi + r.  The
// quotient k is rounded by adding 1.5 * 2^23, which leaves k in the low
// mantissa bits of the sum, so the sum's lowest bit is the parity of k and
// the sign flip is one shift and an exclusive or.  The coefficients were
// fitted for this library by a discrete minimax (Lawson-weighted least
// squares) in double on |r| <= 1.6 (a margin for the rounded quotient) and
// rounded to float32.  Evaluated in float32 the absolute error is below
// 1.3e-7 (about one ulp of the results near 1) for |x| <= 1e5.  Callers take
// sincos_accurate instead when any lane of the wave holds an argument outside
// that range or a non-finite one.
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
    const float t = fmaf(x, 3.183098733e-01f, 12582912.0f);  // 1.5 * 2^23 + rint(x / pi)
    const float k = t - 12582912.0f;
    float r = fmaf(-k, 3.141592741e+00f, x);                   // pi = p1 + p2 + p3
    r = fmaf(-k, -8.742277657e-08f, r);
    r = fmaf(-k, -3.552713679e-15f, r);
    const float r2 = r * r;
    const float ps = fmaf(fmaf(fmaf(2.594375474e-06f, r2, -1.980401576e-04f), r2,
                               8.332980797e-03f), r2, -1.666665524e-01f);
    const float sr = fmaf(r2 * r, ps, r);
    const float pc = fmaf(fmaf(fmaf(fmaf(-2.602301663e-07f, r2, 2.475890506e-05f), r2,
                                    -1.388834789e-03f), r2, 4.166663811e-02f), r2, -5.0e-01f);
    const float cr = fmaf(r2, pc, 1.0f);
    const uint32_t sign = __float_as_uint(t) << 31;          // (-1)^k
    s = __uint_as_float(__float_as_uint(sr) ^ sign);
    c = __uint_as_float(__float_as_uint(cr) ^ sign);
}

__device__ __forceinline__ bool sincos_fast_ok(float x) { return fabsf(x) <= kSinCosFastLimit; }

}  // namespace a2c
