// Block-level segmented scans shared by the backbone and full-atom kernels.
//
// A workgroup of W waves owns one tile: a residue range [ts, te) holding
// whole chains; lane t of the block owns K consecutive residues starting at
// ts + t*K.  Chain heads come from a bit array (bit r set when residue r
// starts a chain; bit R is set too).
//   - forward: segmented exclusive prefix product of per-lane 3x4 affine
//     aggregates, (fa, A) . (fb, B) = (fa | fb, fb ? B : A B);
//   - adjoint: segmented exclusive suffix sum of per-lane wrenches
//     (force, moment), reset at chain ends.
// Each is a 6-step shuffle scan inside the wave, then one workgroup barrier
// and a short scan of the wave totals that every wave repeats for itself.
#pragma once
#include "a2c_internal.h"
#include "affine.h"

namespace a2c {

// K-bit mask: bit j set when residue rs + j starts a chain.  The bit array is
// padded so that reading one word past rs + K is in bounds.
template <int K>
__device__ __forceinline__ uint32_t head_mask(const uint32_t *__restrict__ bits, int64_t rs)
{
    const int64_t w = rs >> 5;
    const int sh = (int)(rs & 31);
    const uint64_t lo = bits[w];
    const uint64_t hi = (sh + K > 32) ? (uint64_t)bits[w + 1] : 0ull;
    const uint64_t v = (hi << 32) | lo;
    return (uint32_t)(v >> sh) & ((1u << K) - 1u);
}

struct Wrench {
    float g0, g1, g2, m0, m1, m2;  // force and moment about the origin
};

__device__ __forceinline__ Wrench wrench_zero()
{
    Wrench w;
    w.g0 = w.g1 = w.g2 = w.m0 = w.m1 = w.m2 = 0.f;
    return w;
}

__device__ __forceinline__ void wrench_add(Wrench &a, const Wrench &b)
{
    a.g0 += b.g0; a.g1 += b.g1; a.g2 += b.g2;
    a.m0 += b.m0; a.m1 += b.m1; a.m2 += b.m2;
}

// add the wrench of force g applied at point p
__device__ __forceinline__ void wrench_add_point(Wrench &a, float px, float py, float pz, float gx,
                                                 float gy, float gz)
{
    a.g0 += gx; a.g1 += gy; a.g2 += gz;
    a.m0 += py * gz - pz * gy;
    a.m1 += pz * gx - px * gz;
    a.m2 += px * gy - py * gx;
}

// u . (S.m - o x S.g): derivative of sum g.r over the subtree carried by S
// when it rotates about the axis u through o
__device__ __forceinline__ float wrench_torque(const Wrench &S, float ox, float oy, float oz,
                                               float ux, float uy, float uz)
{
    const float tx = S.m0 - (oy * S.g2 - oz * S.g1);
    const float ty = S.m1 - (oz * S.g0 - ox * S.g2);
    const float tz = S.m2 - (ox * S.g1 - oy * S.g0);
    return ux * tx + uy * ty + uz * tz;
}

__device__ __forceinline__ Wrench wrench_shfl_down(const Wrench &a, int delta)
{
    Wrench o;
    o.g0 = __shfl_down(a.g0, delta, 64); o.g1 = __shfl_down(a.g1, delta, 64);
    o.g2 = __shfl_down(a.g2, delta, 64); o.m0 = __shfl_down(a.m0, delta, 64);
    o.m1 = __shfl_down(a.m1, delta, 64); o.m2 = __shfl_down(a.m2, delta, 64);
    return o;
}

struct FwdShared {
    float tot[kMaxWaves][12];
    int tot_flag[kMaxWaves];
};

struct BwdShared {
    float tot[kMaxWaves][6];
    int tot_flag[kMaxWaves];
};

__device__ __forceinline__ void aff_store(float *dst, const Aff &m)
{
    dst[0] = m.r00; dst[1] = m.r10; dst[2] = m.r20;
    dst[3] = m.r01; dst[4] = m.r11; dst[5] = m.r21;
    dst[6] = m.r02; dst[7] = m.r12; dst[8] = m.r22;
    dst[9] = m.t0; dst[10] = m.t1; dst[11] = m.t2;
}

__device__ __forceinline__ Aff aff_load(const float *src)
{
    Aff m;
    m.r00 = src[0]; m.r10 = src[1]; m.r20 = src[2];
    m.r01 = src[3]; m.r11 = src[4]; m.r21 = src[5];
    m.r02 = src[6]; m.r12 = src[7]; m.r22 = src[8];
    m.t0 = src[9]; m.t1 = src[10]; m.t2 = src[11];
    return m;
}

__device__ __forceinline__ float lane_bcast(float v, int src_lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src_lane));
}

__device__ __forceinline__ Aff aff_bcast(const Aff &a, int l)
{
    Aff o;
    o.r00 = lane_bcast(a.r00, l); o.r10 = lane_bcast(a.r10, l); o.r20 = lane_bcast(a.r20, l);
    o.r01 = lane_bcast(a.r01, l); o.r11 = lane_bcast(a.r11, l); o.r21 = lane_bcast(a.r21, l);
    o.r02 = lane_bcast(a.r02, l); o.r12 = lane_bcast(a.r12, l); o.r22 = lane_bcast(a.r22, l);
    o.t0 = lane_bcast(a.t0, l); o.t1 = lane_bcast(a.t1, l); o.t2 = lane_bcast(a.t2, l);
    return o;
}

// Exclusive segmented prefix product over the tile.  In: the lane aggregate
// m (product of the lane's transforms since its last chain head, identity
// when the lane is empty) and f (a chain starts inside the lane).  Out: the
// frame X preceding the lane's first transform; meaningful only for residues
// before the lane's first head.  Every thread of the block calls this (one
// barrier); wave_active must be uniform per wave and true for a prefix of
// the waves.
__device__ __forceinline__ Aff block_exclusive_prefix(Aff m, bool f, bool wave_active,
                                                      FwdShared &sh)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave_active) {
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const Aff o = aff_shfl_up(m, off);
            const int fo = __shfl_up((int)f, off, 64);
            if (lane >= off) {
                const Aff c = aff_compose(o, m);
                m = aff_select(f, m, c);
                f = f || (fo != 0);
            }
        }
        if (lane == kWave - 1) {
            aff_store(sh.tot[wave], m);
            sh.tot_flag[wave] = f ? 1 : 0;
        }
    }
    __syncthreads();
    if (!wave_active) return aff_identity();
    // carry-in of this wave: segmented product of the totals of waves
    // 0 .. wave-1 (the tile starts with a chain head: wave 0 has none)
    Aff cw = aff_identity();
    if (wave > 0) {
        Aff t = aff_identity();
        bool tf = false;
        if (lane < wave) {
            t = aff_load(sh.tot[lane]);
            tf = sh.tot_flag[lane] != 0;
        }
        for (int off = 1; off < wave; off <<= 1) {
            const Aff o = aff_shfl_up(t, off);
            const int fo = __shfl_up((int)tf, off, 64);
            if (lane >= off) {
                const Aff c = aff_compose(o, t);
                t = aff_select(tf, t, c);
                tf = tf || (fo != 0);
            }
        }
        cw = aff_bcast(t, wave - 1);
    }
    Aff e = aff_shfl_up(m, 1);
    int fe = __shfl_up((int)f, 1, 64);
    if (lane == 0) {
        e = aff_identity();
        fe = 0;
    }
    const Aff xc = aff_compose(cw, e);
    return fe ? e : xc;
}

// Exclusive segmented suffix sum over the tile.  In: the lane aggregate agg
// (sum over the lane's atoms up to and including the lane's first chain end)
// and f (a chain ends inside the lane).  Out: the wrench of everything after
// the lane, up to the end of the chain the lane's last residue belongs to
// (callers discard it when that residue ends its chain).  nact = number of
// active waves.  Every thread of the block calls this (one barrier).
__device__ __forceinline__ Wrench block_exclusive_suffix(Wrench agg, bool f, bool wave_active,
                                                         int nact, BwdShared &sh)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave_active) {
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const Wrench o = wrench_shfl_down(agg, off);
            const int fo = __shfl_down((int)f, off, 64);
            if (lane + off < kWave) {
                if (!f) wrench_add(agg, o);
                f = f || (fo != 0);
            }
        }
        if (lane == 0) {
            sh.tot[wave][0] = agg.g0; sh.tot[wave][1] = agg.g1; sh.tot[wave][2] = agg.g2;
            sh.tot[wave][3] = agg.m0; sh.tot[wave][4] = agg.m1; sh.tot[wave][5] = agg.m2;
            sh.tot_flag[wave] = f ? 1 : 0;
        }
    }
    __syncthreads();
    if (!wave_active) return wrench_zero();
    // carry-in from the waves after this one (the tile ends at a chain end,
    // so the last active wave has none)
    Wrench cw = wrench_zero();
    const int nafter = nact - 1 - wave;
    if (nafter > 0) {
        Wrench t = wrench_zero();
        bool tf = false;
        if (lane < nafter) {
            const int w2 = wave + 1 + lane;
            t.g0 = sh.tot[w2][0]; t.g1 = sh.tot[w2][1]; t.g2 = sh.tot[w2][2];
            t.m0 = sh.tot[w2][3]; t.m1 = sh.tot[w2][4]; t.m2 = sh.tot[w2][5];
            tf = sh.tot_flag[w2] != 0;
        }
        for (int off = 1; off < nafter; off <<= 1) {
            const Wrench o = wrench_shfl_down(t, off);
            const int fo = __shfl_down((int)tf, off, 64);
            if (lane + off < kWave) {
                if (!tf) wrench_add(t, o);
                tf = tf || (fo != 0);
            }
        }
        cw.g0 = lane_bcast(t.g0, 0); cw.g1 = lane_bcast(t.g1, 0); cw.g2 = lane_bcast(t.g2, 0);
        cw.m0 = lane_bcast(t.m0, 0); cw.m1 = lane_bcast(t.m1, 0); cw.m2 = lane_bcast(t.m2, 0);
    }
    Wrench S = wrench_shfl_down(agg, 1);
    int fs = __shfl_down((int)f, 1, 64);
    if (lane == kWave - 1) {
        S = wrench_zero();
        fs = 0;
    }
    if (!fs) wrench_add(S, cw);
    return S;
}

// ------------------------------------------------------------ LDS staging
// Global memory is read and written with 64 consecutive floats per wave
// instruction while lanes own N consecutive elements in registers; the
// transpose goes through a per-wave LDS buffer with an odd row stride (no
// bank conflicts on either side).
template <int N>
struct Stride {
    static constexpr int value = (N & 1) ? N : N + 1;
};

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Coalesced global loads of a wave's run base[0 .. 64N): element lane + 64m
// goes to v[m].  `base` is wave-uniform and n (>= 1) is the number of valid
// elements; indices past n are clamped so every load is unconditional
// (straight-line code keeps all loads of all planes in flight together) and
// their values are zeroed in the transpose.
template <int N>
__device__ __forceinline__ void gload(const float *__restrict__ base, int n, float (&v)[N])
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const int e = lane + 64 * m;
        v[m] = base[e < n ? e : n - 1];
    }
}

// Coalesced run (from gload) -> lane-blocked layout: lane l receives
// elements l*N .. l*N+N-1 (0 at or past n).
template <int N>
__device__ __forceinline__ void to_blocked(float *buf, const float (&v)[N], int n, float (&out)[N])
{
    constexpr int S = Stride<N>::value;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const int e = lane + 64 * m;
        buf[e + (e / N) * (S - N)] = e < n ? v[m] : 0.f;
    }
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = buf[lane * S + i];
    wave_lds_sync();
}

// base[l*N + i] = in[i] of lane l for indices below n (base wave-uniform),
// written with 64 consecutive floats per instruction.
template <int N>
__device__ __forceinline__ void stage_store(float *buf, const float (&in)[N], float *__restrict__ base,
                                            int n)
{
    constexpr int S = Stride<N>::value;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < N; ++i) buf[lane * S + i] = in[i];
    wave_lds_sync();
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const int e = lane + 64 * m;
        if (e < n) base[e] = buf[e + (e / N) * (S - N)];
    }
    wave_lds_sync();
}

}  // namespace a2c
