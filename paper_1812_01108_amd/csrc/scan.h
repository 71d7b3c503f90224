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
#include "sincos.h"

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

// ------------------------------------------------------------ DPP moves
// Cross-lane moves within the wave through the DPP path of the VALU (no LDS
// round trip): row_shr/row_shl:n shift inside rows of 16 lanes, row_bcast:15
// and row_bcast:31 carry the last lane of a row (of rows 0-1) to the next
// rows, wave_shr/wave_shl:1 shift the whole wave by one lane.  Lanes without
// a source read 0; callers only use lanes that have one.
constexpr int kDppRowShr = 0x110, kDppRowShl = 0x100, kDppBcast15 = 0x142, kDppBcast31 = 0x143,
              kDppWaveShr1 = 0x138, kDppWaveShl1 = 0x130;

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xf, false);
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ Aff aff_dpp(const Aff &a)
{
    Aff o;
    o.r00 = dpp_f<CTRL, ROW_MASK>(a.r00); o.r10 = dpp_f<CTRL, ROW_MASK>(a.r10);
    o.r20 = dpp_f<CTRL, ROW_MASK>(a.r20); o.r01 = dpp_f<CTRL, ROW_MASK>(a.r01);
    o.r11 = dpp_f<CTRL, ROW_MASK>(a.r11); o.r21 = dpp_f<CTRL, ROW_MASK>(a.r21);
    o.r02 = dpp_f<CTRL, ROW_MASK>(a.r02); o.r12 = dpp_f<CTRL, ROW_MASK>(a.r12);
    o.r22 = dpp_f<CTRL, ROW_MASK>(a.r22); o.t0 = dpp_f<CTRL, ROW_MASK>(a.t0);
    o.t1 = dpp_f<CTRL, ROW_MASK>(a.t1); o.t2 = dpp_f<CTRL, ROW_MASK>(a.t2);
    return o;
}

template <int CTRL>
__device__ __forceinline__ Wrench wrench_dpp(const Wrench &a)
{
    Wrench o;
    o.g0 = dpp_f<CTRL>(a.g0); o.g1 = dpp_f<CTRL>(a.g1); o.g2 = dpp_f<CTRL>(a.g2);
    o.m0 = dpp_f<CTRL>(a.m0); o.m1 = dpp_f<CTRL>(a.m1); o.m2 = dpp_f<CTRL>(a.m2);
    return o;
}

// one step of the segmented affine scan: lanes with `take` combine with the
// value o received from earlier lanes
__device__ __forceinline__ void aff_scan_combine(Aff &m, bool &f, const Aff &o, int fo, bool take)
{
    if (take) {
        const Aff c = aff_compose(o, m);
        m = aff_select(f, m, c);
        f = f || (fo != 0);
    }
}

__device__ __forceinline__ void wrench_scan_combine(Wrench &w, bool &f, const Wrench &o, int fo,
                                                    bool take)
{
    if (take) {
        if (!f) wrench_add(w, o);
        f = f || (fo != 0);
    }
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
        // inclusive scan: four shifts inside rows of 16, then the row totals
        const int rl = lane & 15;
        aff_scan_combine(m, f, aff_dpp<kDppRowShr + 1>(m), dpp_i<kDppRowShr + 1>(f), rl >= 1);
        aff_scan_combine(m, f, aff_dpp<kDppRowShr + 2>(m), dpp_i<kDppRowShr + 2>(f), rl >= 2);
        aff_scan_combine(m, f, aff_dpp<kDppRowShr + 4>(m), dpp_i<kDppRowShr + 4>(f), rl >= 4);
        aff_scan_combine(m, f, aff_dpp<kDppRowShr + 8>(m), dpp_i<kDppRowShr + 8>(f), rl >= 8);
        aff_scan_combine(m, f, aff_dpp<kDppBcast15, 0xa>(m), dpp_i<kDppBcast15, 0xa>(f),
                         (lane & 16) != 0);
        aff_scan_combine(m, f, aff_dpp<kDppBcast31, 0xc>(m), dpp_i<kDppBcast31, 0xc>(f),
                         lane >= 32);
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
    Aff e = aff_dpp<kDppWaveShr1>(m);
    int fe = dpp_i<kDppWaveShr1>(f);
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
        // inclusive reverse scan: four shifts inside rows, then the suffix
        // totals of rows 1 and 3 (lanes 16, 48) and of rows 2-3 (lane 32)
        const int rl = lane & 15;
        wrench_scan_combine(agg, f, wrench_dpp<kDppRowShl + 1>(agg), dpp_i<kDppRowShl + 1>(f), rl < 15);
        wrench_scan_combine(agg, f, wrench_dpp<kDppRowShl + 2>(agg), dpp_i<kDppRowShl + 2>(f), rl < 14);
        wrench_scan_combine(agg, f, wrench_dpp<kDppRowShl + 4>(agg), dpp_i<kDppRowShl + 4>(f), rl < 12);
        wrench_scan_combine(agg, f, wrench_dpp<kDppRowShl + 8>(agg), dpp_i<kDppRowShl + 8>(f), rl < 8);
        {
            const int src = lane < 16 ? 16 : 48;
            Wrench o;
            const float a0 = lane_bcast(agg.g0, 16), b0 = lane_bcast(agg.g0, 48);
            const float a1 = lane_bcast(agg.g1, 16), b1 = lane_bcast(agg.g1, 48);
            const float a2 = lane_bcast(agg.g2, 16), b2 = lane_bcast(agg.g2, 48);
            const float a3 = lane_bcast(agg.m0, 16), b3 = lane_bcast(agg.m0, 48);
            const float a4 = lane_bcast(agg.m1, 16), b4 = lane_bcast(agg.m1, 48);
            const float a5 = lane_bcast(agg.m2, 16), b5 = lane_bcast(agg.m2, 48);
            const int fa = __builtin_amdgcn_readlane((int)f, 16), fb = __builtin_amdgcn_readlane((int)f, 48);
            const bool lo = src == 16;
            o.g0 = lo ? a0 : b0; o.g1 = lo ? a1 : b1; o.g2 = lo ? a2 : b2;
            o.m0 = lo ? a3 : b3; o.m1 = lo ? a4 : b4; o.m2 = lo ? a5 : b5;
            wrench_scan_combine(agg, f, o, lo ? fa : fb, (lane & 16) == 0);
        }
        {
            Wrench o;
            o.g0 = lane_bcast(agg.g0, 32); o.g1 = lane_bcast(agg.g1, 32);
            o.g2 = lane_bcast(agg.g2, 32); o.m0 = lane_bcast(agg.m0, 32);
            o.m1 = lane_bcast(agg.m1, 32); o.m2 = lane_bcast(agg.m2, 32);
            const int fo = __builtin_amdgcn_readlane((int)f, 32);
            wrench_scan_combine(agg, f, o, fo, lane < 32);
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
    Wrench S = wrench_dpp<kDppWaveShl1>(agg);
    int fs = dpp_i<kDppWaveShl1>(f);
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
