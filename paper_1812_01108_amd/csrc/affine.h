// 3x4 affine transforms (rotation + translation, implicit bottom row 0 0 0 1)
// held in registers, and the right-multiplication by the paper's elementary
// transform R(alpha, theta, d) = Ry(theta) Tx(d) Rx(alpha) applied column-wise
// instead of as a full matrix product.
#pragma once
#include <hip/hip_runtime.h>

namespace a2c {

struct Aff {
    // rotation columns c0 (x axis), c1, c2 and translation t
    float r00, r10, r20;  // c0
    float r01, r11, r21;  // c1
    float r02, r12, r22;  // c2
    float t0, t1, t2;
};

__device__ __forceinline__ Aff aff_identity()
{
    Aff m;
    m.r00 = 1.f; m.r10 = 0.f; m.r20 = 0.f;
    m.r01 = 0.f; m.r11 = 1.f; m.r21 = 0.f;
    m.r02 = 0.f; m.r12 = 0.f; m.r22 = 1.f;
    m.t0 = 0.f; m.t1 = 0.f; m.t2 = 0.f;
    return m;
}

// M <- M * Ry(theta) * Tx(d) * Rx(alpha), with (ct, st) = cos/sin theta and
// (ca, sa) = cos/sin alpha.  Column form of the printed matrix:
//   c0' = ct c0 - st c2,  c2' = st c0 + ct c2,  t' = t + d c0',
//   c1'' = ca c1 + sa c2', c2'' = ca c2' - sa c1.
__device__ __forceinline__ void aff_apply_transform(Aff &m, float ct, float st, float d,
                                                    float ca, float sa)
{
    const float a0 = ct * m.r00 - st * m.r02;
    const float a1 = ct * m.r10 - st * m.r12;
    const float a2 = ct * m.r20 - st * m.r22;
    const float b0 = st * m.r00 + ct * m.r02;
    const float b1 = st * m.r10 + ct * m.r12;
    const float b2 = st * m.r20 + ct * m.r22;
    m.t0 = fmaf(d, a0, m.t0);
    m.t1 = fmaf(d, a1, m.t1);
    m.t2 = fmaf(d, a2, m.t2);
    m.r00 = a0; m.r10 = a1; m.r20 = a2;
    const float c0 = ca * m.r01 + sa * b0;
    const float c1 = ca * m.r11 + sa * b1;
    const float c2 = ca * m.r21 + sa * b2;
    const float e0 = ca * b0 - sa * m.r01;
    const float e1 = ca * b1 - sa * m.r11;
    const float e2 = ca * b2 - sa * m.r21;
    m.r01 = c0; m.r11 = c1; m.r21 = c2;
    m.r02 = e0; m.r12 = e1; m.r22 = e2;
}

// The identity followed by R(alpha, theta, d): the first transform of a walk,
// without the products with 0 and 1 (the same values as applying it to the
// identity with aff_apply_transform, up to the sign of zeros).
__device__ __forceinline__ Aff aff_first_transform(float ct, float st, float d, float ca,
                                                   float sa)
{
    Aff m;
    m.r00 = ct; m.r10 = 0.f; m.r20 = -st;
    m.r01 = sa * st; m.r11 = ca; m.r21 = sa * ct;
    m.r02 = ca * st; m.r12 = -sa; m.r22 = ca * ct;
    m.t0 = d * ct; m.t1 = 0.f; m.t2 = -(d * st);
    return m;
}

// a * b (a applied after b): rotation a.R b.R, translation a.R b.t + a.t
__device__ __forceinline__ Aff aff_compose(const Aff &a, const Aff &b)
{
    Aff c;
    c.r00 = fmaf(a.r02, b.r20, fmaf(a.r01, b.r10, a.r00 * b.r00));
    c.r10 = fmaf(a.r12, b.r20, fmaf(a.r11, b.r10, a.r10 * b.r00));
    c.r20 = fmaf(a.r22, b.r20, fmaf(a.r21, b.r10, a.r20 * b.r00));
    c.r01 = fmaf(a.r02, b.r21, fmaf(a.r01, b.r11, a.r00 * b.r01));
    c.r11 = fmaf(a.r12, b.r21, fmaf(a.r11, b.r11, a.r10 * b.r01));
    c.r21 = fmaf(a.r22, b.r21, fmaf(a.r21, b.r11, a.r20 * b.r01));
    c.r02 = fmaf(a.r02, b.r22, fmaf(a.r01, b.r12, a.r00 * b.r02));
    c.r12 = fmaf(a.r12, b.r22, fmaf(a.r11, b.r12, a.r10 * b.r02));
    c.r22 = fmaf(a.r22, b.r22, fmaf(a.r21, b.r12, a.r20 * b.r02));
    c.t0 = fmaf(a.r02, b.t2, fmaf(a.r01, b.t1, fmaf(a.r00, b.t0, a.t0)));
    c.t1 = fmaf(a.r12, b.t2, fmaf(a.r11, b.t1, fmaf(a.r10, b.t0, a.t1)));
    c.t2 = fmaf(a.r22, b.t2, fmaf(a.r21, b.t1, fmaf(a.r20, b.t0, a.t2)));
    return c;
}

// y = a.R p + a.t
__device__ __forceinline__ void aff_point(const Aff &a, float px, float py, float pz,
                                          float &x, float &y, float &z)
{
    x = fmaf(a.r02, pz, fmaf(a.r01, py, fmaf(a.r00, px, a.t0)));
    y = fmaf(a.r12, pz, fmaf(a.r11, py, fmaf(a.r10, px, a.t1)));
    z = fmaf(a.r22, pz, fmaf(a.r21, py, fmaf(a.r20, px, a.t2)));
}

// y = a.R v (direction)
__device__ __forceinline__ void aff_dir(const Aff &a, float px, float py, float pz,
                                        float &x, float &y, float &z)
{
    x = fmaf(a.r02, pz, fmaf(a.r01, py, a.r00 * px));
    y = fmaf(a.r12, pz, fmaf(a.r11, py, a.r10 * px));
    z = fmaf(a.r22, pz, fmaf(a.r21, py, a.r20 * px));
}

// One Newton-Schulz polar step on the rotation part, R <- R (3I - R^T R)/2,
// which pulls a nearly orthonormal R back towards the rotation group; the
// translation is left alone.
__device__ __forceinline__ void aff_orthonormalise(Aff &a)
{
    // S = R^T R (symmetric)
    const float s00 = a.r00 * a.r00 + a.r10 * a.r10 + a.r20 * a.r20;
    const float s11 = a.r01 * a.r01 + a.r11 * a.r11 + a.r21 * a.r21;
    const float s22 = a.r02 * a.r02 + a.r12 * a.r12 + a.r22 * a.r22;
    const float s01 = a.r00 * a.r01 + a.r10 * a.r11 + a.r20 * a.r21;
    const float s02 = a.r00 * a.r02 + a.r10 * a.r12 + a.r20 * a.r22;
    const float s12 = a.r01 * a.r02 + a.r11 * a.r12 + a.r21 * a.r22;
    // E = (I - S)/2 is tiny; R <- R + R E
    const float e00 = 0.5f * (1.f - s00), e11 = 0.5f * (1.f - s11), e22 = 0.5f * (1.f - s22);
    const float e01 = -0.5f * s01, e02 = -0.5f * s02, e12 = -0.5f * s12;
    const float n00 = a.r00 + (a.r00 * e00 + a.r01 * e01 + a.r02 * e02);
    const float n10 = a.r10 + (a.r10 * e00 + a.r11 * e01 + a.r12 * e02);
    const float n20 = a.r20 + (a.r20 * e00 + a.r21 * e01 + a.r22 * e02);
    const float n01 = a.r01 + (a.r00 * e01 + a.r01 * e11 + a.r02 * e12);
    const float n11 = a.r11 + (a.r10 * e01 + a.r11 * e11 + a.r12 * e12);
    const float n21 = a.r21 + (a.r20 * e01 + a.r21 * e11 + a.r22 * e12);
    const float n02 = a.r02 + (a.r00 * e02 + a.r01 * e12 + a.r02 * e22);
    const float n12 = a.r12 + (a.r10 * e02 + a.r11 * e12 + a.r12 * e22);
    const float n22 = a.r22 + (a.r20 * e02 + a.r21 * e12 + a.r22 * e22);
    a.r00 = n00; a.r10 = n10; a.r20 = n20;
    a.r01 = n01; a.r11 = n11; a.r21 = n21;
    a.r02 = n02; a.r12 = n12; a.r22 = n22;
}

// Wave-wide shuffles of a whole transform (64-lane wavefront).
__device__ __forceinline__ Aff aff_shfl_up(const Aff &a, int delta)
{
    Aff o;
    o.r00 = __shfl_up(a.r00, delta, 64); o.r10 = __shfl_up(a.r10, delta, 64);
    o.r20 = __shfl_up(a.r20, delta, 64); o.r01 = __shfl_up(a.r01, delta, 64);
    o.r11 = __shfl_up(a.r11, delta, 64); o.r21 = __shfl_up(a.r21, delta, 64);
    o.r02 = __shfl_up(a.r02, delta, 64); o.r12 = __shfl_up(a.r12, delta, 64);
    o.r22 = __shfl_up(a.r22, delta, 64); o.t0 = __shfl_up(a.t0, delta, 64);
    o.t1 = __shfl_up(a.t1, delta, 64); o.t2 = __shfl_up(a.t2, delta, 64);
    return o;
}

__device__ __forceinline__ Aff aff_select(bool take_a, const Aff &a, const Aff &b)
{
    Aff o;
    o.r00 = take_a ? a.r00 : b.r00; o.r10 = take_a ? a.r10 : b.r10;
    o.r20 = take_a ? a.r20 : b.r20; o.r01 = take_a ? a.r01 : b.r01;
    o.r11 = take_a ? a.r11 : b.r11; o.r21 = take_a ? a.r21 : b.r21;
    o.r02 = take_a ? a.r02 : b.r02; o.r12 = take_a ? a.r12 : b.r12;
    o.r22 = take_a ? a.r22 : b.r22; o.t0 = take_a ? a.t0 : b.t0;
    o.t1 = take_a ? a.t1 : b.t1; o.t2 = take_a ? a.t2 : b.t2;
    return o;
}

}  // namespace a2c
