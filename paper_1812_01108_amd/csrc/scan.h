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
// A workgroup walks its tile in chunks of 64 W K residues and carries the
// scan state from chunk to chunk.  Inside a chunk each scan is a 6-step DPP
// scan inside the wave, then a scan of the wave totals: for the prefix
// product wave 0 scans them between two workgroup barriers and every wave
// reads its prefix from LDS; the suffix sum's totals are scanned by every
// wave for itself after one barrier.
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
// Explicit FMAs here and in wrench_torque: the compiler may contract
// a * b - c * d either way, and may choose differently in different kernels;
// with the operations spelled out every kernel rounds the same way.
__device__ __forceinline__ void wrench_add_point(Wrench &a, float px, float py, float pz, float gx,
                                                 float gy, float gz)
{
    a.g0 += gx; a.g1 += gy; a.g2 += gz;
    a.m0 += fmaf(py, gz, -(pz * gy));
    a.m1 += fmaf(pz, gx, -(px * gz));
    a.m2 += fmaf(px, gy, -(py * gx));
}

// u . (S.m - o x S.g): derivative of sum g.r over the subtree carried by S
// when it rotates about the axis u through o
__device__ __forceinline__ float wrench_torque(const Wrench &S, float ox, float oy, float oz,
                                               float ux, float uy, float uz)
{
    const float tx = S.m0 - fmaf(oy, S.g2, -(oz * S.g1));
    const float ty = S.m1 - fmaf(oz, S.g0, -(ox * S.g2));
    const float tz = S.m2 - fmaf(ox, S.g1, -(oy * S.g0));
    return fmaf(uz, tz, fmaf(uy, ty, ux * tx));
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
    float tot[kMaxWaves][12];   // wave totals
    int tot_flag[kMaxWaves];    // a chain starts in the wave
    float pre[kMaxWaves][12];   // inclusive prefixes of the wave totals
    int pre_flag[kMaxWaves];    // a chain starts in waves 0..w
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

// Sum of v over the block's lanes in a fixed order (deterministic): quad and
// row exchanges by DPP, the four row sums by lane reads, then the wave sums
// in wave order by thread 0.  Every thread calls it (one barrier); the
// result is meaningful in thread 0.
__device__ __forceinline__ float block_sum(float v, float (&wave_tot)[kMaxWaves])
{
    v += dpp_f<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f<0x141>(v);   // row_half_mirror
    v += dpp_f<0x140>(v);   // row_mirror
    const float w = (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wave_tot[wave] = w;
    __syncthreads();
    float t = 0.f;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += wave_tot[i];
    return t;
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

__device__ __forceinline__ float uni(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ Aff aff_uniform(const Aff &a)
{
    Aff o;
    o.r00 = uni(a.r00); o.r10 = uni(a.r10); o.r20 = uni(a.r20);
    o.r01 = uni(a.r01); o.r11 = uni(a.r11); o.r21 = uni(a.r21);
    o.r02 = uni(a.r02); o.r12 = uni(a.r12); o.r22 = uni(a.r22);
    o.t0 = uni(a.t0); o.t1 = uni(a.t1); o.t2 = uni(a.t2);
    return o;
}

// Segmented combine of a carry with a later segment: the later value wins
// when a chain starts inside it, otherwise the carry is applied first.
__device__ __forceinline__ Aff aff_seg_after(const Aff &carry, const Aff &t, bool t_head)
{
    const Aff c = aff_compose(carry, t);
    return aff_select(t_head, t, c);
}

// Lanes at or below `lane` (bit l set for l <= lane) and strictly below it.
__device__ __forceinline__ uint64_t lanes_upto(int lane) { return ~0ull >> (63 - lane); }
__device__ __forceinline__ uint64_t lanes_below(int lane)
{
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lane of the last set bit of `heads` at or below `lane` (0 when none).
__device__ __forceinline__ int last_head_upto(uint64_t heads, int lane)
{
    const uint64_t b = heads & lanes_upto(lane);
    return b ? 63 - __builtin_clzll(b) : 0;
}

// DPP read with bound_ctrl (a lane without a source reads 0) and full row and
// bank masks: the compiler may then fold the move into the instructions that
// consume it.  Callers only use lanes that have a source.
template <int CTRL>
__device__ __forceinline__ float dpp_z(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

template <int CTRL>
__device__ __forceinline__ Aff aff_dpp_z(const Aff &a)
{
    Aff o;
    o.r00 = dpp_z<CTRL>(a.r00); o.r10 = dpp_z<CTRL>(a.r10); o.r20 = dpp_z<CTRL>(a.r20);
    o.r01 = dpp_z<CTRL>(a.r01); o.r11 = dpp_z<CTRL>(a.r11); o.r21 = dpp_z<CTRL>(a.r21);
    o.r02 = dpp_z<CTRL>(a.r02); o.r12 = dpp_z<CTRL>(a.r12); o.r22 = dpp_z<CTRL>(a.r22);
    o.t0 = dpp_z<CTRL>(a.t0); o.t1 = dpp_z<CTRL>(a.t1); o.t2 = dpp_z<CTRL>(a.t2);
    return o;
}

// One step of a segmented inclusive affine scan, branch-free: lanes with
// `take` prepend the value of their source lane.
template <int CTRL>
__device__ __forceinline__ void aff_scan_step(Aff &m, bool take)
{
    const Aff c = aff_compose(aff_dpp_z<CTRL>(m), m);
    m = aff_select(take, c, m);
}

// Segmented inclusive scan of 3x4 affines over the lanes of a wave (or over
// lanes 0..n-1, n <= 16, when ROW0).  heads: bit l set when lane l starts a
// segment.  Lane l prepends the value of lane l - d when that lane is in the
// same segment, i.e. when l - d >= s_l, the last head at or below l; the row
// steps (d = 1, 2, 4, 8 inside rows of 16 lanes) also need l - d in l's row.
template <bool ROW0>
__device__ __forceinline__ void aff_wave_scan(Aff &m, uint64_t heads, int n)
{
    const int lane = threadIdx.x & 63;
    const int s = last_head_upto(heads, lane);
    const int row = lane & ~15;
    const int dist = lane - max(s, row);   // lanes of l's segment before l, in its row
    if (!ROW0 || n > 1) aff_scan_step<kDppRowShr + 1>(m, dist >= 1);
    if (!ROW0 || n > 2) aff_scan_step<kDppRowShr + 2>(m, dist >= 2);
    if (!ROW0 || n > 4) aff_scan_step<kDppRowShr + 4>(m, dist >= 4);
    if (!ROW0 || n > 8) aff_scan_step<kDppRowShr + 8>(m, dist >= 8);
    if (!ROW0) {
        // rows 1 and 3 prepend the last lane of rows 0 and 2; rows 2-3 lane 31
        aff_scan_step<kDppBcast15>(m, (lane & 16) != 0 && s < row);
        aff_scan_step<kDppBcast31>(m, lane >= 32 && s < 32);
    }
}

// Exclusive segmented prefix product over one chunk of a tile.
//   m, f     lane aggregate (product of the lane's transforms since its last
//            chain head; identity for an empty lane) and "a chain starts in
//            this lane";
//   nact     waves of the block holding residues of this chunk (a prefix);
//   carry    (MULTI only) in: the frame after everything of the tile before
//            this chunk (identity for the first chunk: tiles start at a chain
//            head); out: the frame after this chunk, identical in every wave,
//            also in waves idle in this chunk.
// Returns the frame X preceding the lane's first transform (meaningful for
// the lane's residues before its first chain head).  Every thread of the
// block calls this.  Each wave scans its lanes; wave 0 alone then scans the
// wave totals (two barriers) and every wave reads the prefix it needs.
// MULTI = false: the tile is one chunk and the carry is neither read nor
// written.
template <bool MULTI>
__device__ __forceinline__ Aff block_exclusive_prefix(Aff m, bool f, int nact, FwdShared &sh,
                                                      Aff &carry)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool wave_active = wave < nact;
    const uint64_t heads = __builtin_amdgcn_ballot_w64(f);
    if (wave_active) {
        aff_wave_scan<false>(m, heads, kWave);
        if (lane == kWave - 1) {
            aff_store(sh.tot[wave], m);
            sh.tot_flag[wave] = heads != 0ull ? 1 : 0;
        }
    }
    // the wave totals' inclusive prefixes, by wave 0 (block-uniform branch)
    if (MULTI || nact > 1) {
        __syncthreads();
        if (wave == 0) {
            Aff t = aff_identity();
            bool tf = false;
            if (lane < nact) {
                t = aff_load(sh.tot[lane]);
                tf = sh.tot_flag[lane] != 0;
            }
            const uint64_t th = __builtin_amdgcn_ballot_w64(tf);
            aff_wave_scan<true>(t, th, nact);
            if (lane < nact) {
                aff_store(sh.pre[lane], t);
                sh.pre_flag[lane] = (th & lanes_upto(lane)) != 0ull ? 1 : 0;
            }
        }
        __syncthreads();
    }
    // carry-in of this wave (identity for wave 0 of a one-chunk tile)
    Aff cw = aff_identity();
    if (MULTI) cw = carry;
    if (wave_active && wave > 0) {
        const Aff p = aff_load(sh.pre[wave - 1]);
        const bool pf = sh.pre_flag[wave - 1] != 0;
        cw = MULTI ? aff_seg_after(carry, p, pf) : p;
    }
    if (MULTI) {  // every wave advances the carry, also one idle in this chunk
        const Aff p = aff_load(sh.pre[nact - 1]);
        const bool pf = sh.pre_flag[nact - 1] != 0;
        carry = aff_uniform(aff_seg_after(carry, p, pf));
    }
    if (!wave_active) return aff_identity();
    // lane l's prefix inside the wave: the inclusive value of lane l - 1,
    // complete when a chain starts in lanes before l
    Aff e = aff_dpp_z<kDppWaveShr1>(m);
    if (lane == 0) e = aff_identity();
    const bool fe = (heads & lanes_below(lane)) != 0ull;
    return fe ? e : aff_compose(cw, e);
}

// Exclusive segmented suffix sum over one chunk of a tile, chunks visited
// last to first.
//   agg, f   lane aggregate (sum over the lane's atoms up to and including
//            its first chain end) and "a chain ends in this lane";
//   carry    (MULTI only) in: the wrench of what follows this chunk up to the
//            end of the chain its last residue belongs to (zero for the last
//            chunk: tiles end at a chain end); out: the same for the previous
//            chunk, also in waves idle in this chunk (the last chunk, visited
//            first, may leave waves idle that the earlier chunks use).
// Returns the wrench of everything after the lane up to the end of the
// chain the lane's last residue belongs to (callers discard it when that
// residue ends its chain).  Every thread of the block calls this (one
// barrier); callers alternate two buffers sh.
template <bool MULTI>
__device__ __forceinline__ Wrench block_exclusive_suffix(Wrench agg, bool f, int nact,
                                                         BwdShared &sh, Wrench &carry)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool wave_active = wave < nact;
    if (wave_active) {
        // inclusive reverse scan: four shifts inside rows, then the suffix
        // totals of rows 1 and 3 (lanes 16, 48) and of rows 2-3 (lane 32)
        const int rl = lane & 15;
        wrench_scan_combine(agg, f, wrench_dpp<kDppRowShl + 1>(agg), dpp_i<kDppRowShl + 1>(f), rl < 15);
        wrench_scan_combine(agg, f, wrench_dpp<kDppRowShl + 2>(agg), dpp_i<kDppRowShl + 2>(f), rl < 14);
        wrench_scan_combine(agg, f, wrench_dpp<kDppRowShl + 4>(agg), dpp_i<kDppRowShl + 4>(f), rl < 12);
        wrench_scan_combine(agg, f, wrench_dpp<kDppRowShl + 8>(agg), dpp_i<kDppRowShl + 8>(f), rl < 8);
        {
            const bool lo = lane < 16;
            Wrench o;
            const float a0 = lane_bcast(agg.g0, 16), b0 = lane_bcast(agg.g0, 48);
            const float a1 = lane_bcast(agg.g1, 16), b1 = lane_bcast(agg.g1, 48);
            const float a2 = lane_bcast(agg.g2, 16), b2 = lane_bcast(agg.g2, 48);
            const float a3 = lane_bcast(agg.m0, 16), b3 = lane_bcast(agg.m0, 48);
            const float a4 = lane_bcast(agg.m1, 16), b4 = lane_bcast(agg.m1, 48);
            const float a5 = lane_bcast(agg.m2, 16), b5 = lane_bcast(agg.m2, 48);
            const int fa = __builtin_amdgcn_readlane((int)f, 16);
            const int fb = __builtin_amdgcn_readlane((int)f, 48);
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
    if (!MULTI && !wave_active) return wrench_zero();
    // inclusive reverse scan of the wave totals in lanes 0..nact-1 of row 0,
    // over as many of them as are needed: lanes wave+1..nact-1 for this
    // wave, all nact for the chunk carry
    const int span = MULTI ? nact : nact - 1 - wave;
    Wrench t = wrench_zero();
    bool tf = false;
    if (lane < nact) {
        t.g0 = sh.tot[lane][0]; t.g1 = sh.tot[lane][1]; t.g2 = sh.tot[lane][2];
        t.m0 = sh.tot[lane][3]; t.m1 = sh.tot[lane][4]; t.m2 = sh.tot[lane][5];
        tf = sh.tot_flag[lane] != 0;
    }
    const int rl = lane & 15;
    if (span > 1)
        wrench_scan_combine(t, tf, wrench_dpp<kDppRowShl + 1>(t), dpp_i<kDppRowShl + 1>(tf), rl < 15);
    if (span > 2)
        wrench_scan_combine(t, tf, wrench_dpp<kDppRowShl + 2>(t), dpp_i<kDppRowShl + 2>(tf), rl < 14);
    if (span > 4)
        wrench_scan_combine(t, tf, wrench_dpp<kDppRowShl + 4>(t), dpp_i<kDppRowShl + 4>(tf), rl < 12);
    if (span > 8)
        wrench_scan_combine(t, tf, wrench_dpp<kDppRowShl + 8>(t), dpp_i<kDppRowShl + 8>(tf), rl < 8);
    // carry into this wave from the waves after it (and, MULTI, later chunks)
    Wrench cw = wrench_zero();
    if (MULTI) cw = carry;
    if (wave_active && wave + 1 < nact) {
        Wrench p;
        p.g0 = lane_bcast(t.g0, wave + 1); p.g1 = lane_bcast(t.g1, wave + 1);
        p.g2 = lane_bcast(t.g2, wave + 1); p.m0 = lane_bcast(t.m0, wave + 1);
        p.m1 = lane_bcast(t.m1, wave + 1); p.m2 = lane_bcast(t.m2, wave + 1);
        const bool pf = __builtin_amdgcn_readlane((int)tf, wave + 1) != 0;
        if (MULTI && !pf) wrench_add(p, carry);
        cw = p;
    }
    if (MULTI) {  // every wave advances the carry, also one idle in this chunk
        Wrench p;
        p.g0 = lane_bcast(t.g0, 0); p.g1 = lane_bcast(t.g1, 0); p.g2 = lane_bcast(t.g2, 0);
        p.m0 = lane_bcast(t.m0, 0); p.m1 = lane_bcast(t.m1, 0); p.m2 = lane_bcast(t.m2, 0);
        const bool pf = __builtin_amdgcn_readlane((int)tf, 0) != 0;
        if (!pf) wrench_add(p, carry);
        carry = p;
    }
    if (!wave_active) return wrench_zero();
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

// The lane index made opaque to the optimiser, so address arithmetic
// derived from it is recomputed where it is used instead of being hoisted out
// of the chunk loop and held live in registers across it.
__device__ __forceinline__ int lane_id()
{
    int l = threadIdx.x & 63;
    asm volatile("" : "+v"(l));
    return l;
}

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
    const int lane = lane_id();
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
    const int lane = lane_id();
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
    const int lane = lane_id();
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
