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
// product and the suffix sum alike, wave 0 scans them between two
// workgroup barriers and every wave reads the value it needs from LDS.
#pragma once
#include "a2c_internal.h"
#include "affine.h"
#include "sincos.h"

namespace a2c {

// K-bit mask: bit j set when residue rs + j starts a chain.  The bit array is
// padded so that reading one word past rs + K is in bounds for rs <= R + 1;
// both words are read unconditionally (no branch holds the loads back).
template <int K>
__device__ __forceinline__ uint32_t head_mask(const uint32_t *__restrict__ bits, int64_t rs)
{
    const int64_t w = rs >> 5;
    const int sh = (int)(rs & 31);
    const uint64_t v = ((uint64_t)bits[w + 1] << 32) | bits[w];
    return (uint32_t)(v >> sh) & ((1u << K) - 1u);
}

// head_mask of a lane holding cnt residues from rs in a chunk ending at ce:
// the index is clamped to ce (<= R), so the read needs no branch; 0 for an
// empty lane.
template <int K>
__device__ __forceinline__ uint32_t lane_head_mask(const uint32_t *__restrict__ bits, int64_t rs,
                                                   int64_t ce, int cnt)
{
    const uint32_t m = head_mask<K>(bits, rs < ce ? rs : ce);
    return cnt > 0 ? m : 0u;
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

struct FwdShared {
    float tot[kMaxWaves][12];   // wave totals
    int tot_flag[kMaxWaves];    // a chain starts in the wave
    float pre[kMaxWaves][12];   // inclusive prefixes of the wave totals
    int pre_flag[kMaxWaves];    // a chain starts in waves 0..w
};

struct BwdShared {
    float tot[kMaxWaves][6];    // wave totals
    int tot_flag[kMaxWaves];    // a chain ends in the wave
    float suf[kMaxWaves][6];    // inclusive suffixes of the wave totals
    int suf_flag[kMaxWaves];    // a chain ends in waves w..nact-1
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

// The fused step's loss: every tile stores its share (the block sum of v),
// counts itself done with one atomic, and the tile that counts last sums all
// shares in tile order (each thread a fixed strided subset, then block_sum)
// into *out and sets the count back to 0 for the next launch.  No tile waits
// for another; the total does not depend on which tile finishes last.
// Every thread of the block calls this (block-uniform arguments).
__device__ __forceinline__ void loss_commit(float v, float *__restrict__ parts,
                                            uint32_t *__restrict__ count, float *__restrict__ out,
                                            float (&wave_tot)[kMaxWaves])
{
    __shared__ int last;
    const float t = block_sum(v, wave_tot);
    if (threadIdx.x == 0) {
        parts[blockIdx.x] = t;
        __threadfence();   // the share is visible before the count says so
        last = atomicAdd(count, 1u) == gridDim.x - 1 ? 1 : 0;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    float s = 0.f;
    for (unsigned i = threadIdx.x; i < gridDim.x; i += blockDim.x)
        s += __hip_atomic_load(parts + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();   // wave_tot is reused
    const float total = block_sum(s, wave_tot);
    if (threadIdx.x == 0) {
        *out = total;
        __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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

// The lane index made opaque to the optimiser, so address arithmetic
// derived from it is recomputed where it is used instead of being hoisted out
// of the chunk loop and held live in registers across it.
__device__ __forceinline__ int lane_id()
{
    int l = threadIdx.x & 63;
    asm volatile("" : "+v"(l));
    return l;
}

// The backbone constants made opaque to the optimiser at the top of a loop over
// chunks: products of them (the first transforms of a chain head, say) are
// then formed where they are used instead of being hoisted out of the loop,
// where these uniform values would each hold a vector register across it.
__device__ __forceinline__ BBParams opaque_params(BBParams P)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
        asm volatile("" : "+s"(P.ct[i]), "+s"(P.st[i]), "+s"(P.d[i]), "+s"(P.inv_d[i]));
    return P;
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
__device__ __forceinline__ void aff_wave_scan(Aff &m, uint64_t heads, int n, int lane)
{
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
    // opaque inside chunk loops (MULTI), so lane masks are not hoisted out
    const int lane = MULTI ? lane_id() : (int)(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool wave_active = wave < nact;
    const uint64_t heads = __builtin_amdgcn_ballot_w64(f);
    if (wave_active) {
        aff_wave_scan<false>(m, heads, kWave, lane);
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
            aff_wave_scan<true>(t, th, nact, lane);
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

// Lane of the first set bit of `ends` at or above `lane` (63 when none).
__device__ __forceinline__ int first_end_from(uint64_t ends, int lane)
{
    const uint64_t b = ends & (~0ull << lane);
    return b ? __builtin_ctzll(b) : kWave - 1;
}

template <int CTRL>
__device__ __forceinline__ Wrench wrench_dpp_z(const Wrench &a)
{
    Wrench o;
    o.g0 = dpp_z<CTRL>(a.g0); o.g1 = dpp_z<CTRL>(a.g1); o.g2 = dpp_z<CTRL>(a.g2);
    o.m0 = dpp_z<CTRL>(a.m0); o.m1 = dpp_z<CTRL>(a.m1); o.m2 = dpp_z<CTRL>(a.m2);
    return o;
}

// every lane of each 32-lane half reads lane 16 of its half (ds_swizzle in
// bit mode: and_mask 0, or_mask 16)
__device__ __forceinline__ float swz_lane16(float v)
{
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 16 << 5));
}

__device__ __forceinline__ void wrench_add_if(Wrench &w, const Wrench &o, bool take)
{
    w.g0 = take ? w.g0 + o.g0 : w.g0; w.g1 = take ? w.g1 + o.g1 : w.g1;
    w.g2 = take ? w.g2 + o.g2 : w.g2; w.m0 = take ? w.m0 + o.m0 : w.m0;
    w.m1 = take ? w.m1 + o.m1 : w.m1; w.m2 = take ? w.m2 + o.m2 : w.m2;
}

// Segmented inclusive suffix sum of wrenches over the lanes of a wave (or
// over lanes 0..n-1, n <= 16, when ROW0).  ends: bit l set when lane l's
// value closes a segment.  Lane l adds the value of lane l + d when no
// segment closes in lanes l .. l+d-1, i.e. when l + d <= e_l, the first end
// at or after l; the row steps also need l + d in l's row.
template <bool ROW0>
__device__ __forceinline__ void wrench_wave_rscan(Wrench &w, uint64_t ends, int n, int lane)
{
    const int e = first_end_from(ends, lane);
    const int dist = min(e, lane | 15) - lane;
    if (!ROW0 || n > 1) wrench_add_if(w, wrench_dpp_z<kDppRowShl + 1>(w), dist >= 1);
    if (!ROW0 || n > 2) wrench_add_if(w, wrench_dpp_z<kDppRowShl + 2>(w), dist >= 2);
    if (!ROW0 || n > 4) wrench_add_if(w, wrench_dpp_z<kDppRowShl + 4>(w), dist >= 4);
    if (!ROW0 || n > 8) wrench_add_if(w, wrench_dpp_z<kDppRowShl + 8>(w), dist >= 8);
    if (!ROW0) {
        // rows 0 and 2 add the first lane of rows 1 and 3, then rows 0-1 lane 32
        Wrench o;
        o.g0 = swz_lane16(w.g0); o.g1 = swz_lane16(w.g1); o.g2 = swz_lane16(w.g2);
        o.m0 = swz_lane16(w.m0); o.m1 = swz_lane16(w.m1); o.m2 = swz_lane16(w.m2);
        wrench_add_if(w, o, (lane & 16) == 0 && e > (lane | 15));
        o.g0 = lane_bcast(w.g0, 32); o.g1 = lane_bcast(w.g1, 32); o.g2 = lane_bcast(w.g2, 32);
        o.m0 = lane_bcast(w.m0, 32); o.m1 = lane_bcast(w.m1, 32); o.m2 = lane_bcast(w.m2, 32);
        wrench_add_if(w, o, lane < 32 && e >= 32);
    }
}

__device__ __forceinline__ void wrench_store(float *dst, const Wrench &w)
{
    dst[0] = w.g0; dst[1] = w.g1; dst[2] = w.g2; dst[3] = w.m0; dst[4] = w.m1; dst[5] = w.m2;
}

__device__ __forceinline__ Wrench wrench_load(const float *src)
{
    Wrench w;
    w.g0 = src[0]; w.g1 = src[1]; w.g2 = src[2]; w.m0 = src[3]; w.m1 = src[4]; w.m2 = src[5];
    return w;
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
// residue ends its chain).  Every thread of the block calls this.  Each wave
// scans its lanes; wave 0 alone then scans the wave totals (two barriers)
// and every wave reads the suffix it needs.
template <bool MULTI>
__device__ __forceinline__ Wrench block_exclusive_suffix(Wrench agg, bool f, int nact,
                                                         BwdShared &sh, Wrench &carry)
{
    // opaque inside chunk loops (MULTI), so lane masks are not hoisted out
    const int lane = MULTI ? lane_id() : (int)(threadIdx.x & 63);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool wave_active = wave < nact;
    const uint64_t ends = __builtin_amdgcn_ballot_w64(f);
    if (wave_active) {
        wrench_wave_rscan<false>(agg, ends, kWave, lane);
        if (lane == 0) {
            wrench_store(sh.tot[wave], agg);
            sh.tot_flag[wave] = ends != 0ull ? 1 : 0;
        }
    }
    // the wave totals' inclusive suffixes, by wave 0 (block-uniform branch)
    if (MULTI || nact > 1) {
        __syncthreads();
        if (wave == 0) {
            Wrench t = wrench_zero();
            bool tf = false;
            if (lane < nact) {
                t = wrench_load(sh.tot[lane]);
                tf = sh.tot_flag[lane] != 0;
            }
            const uint64_t th = __builtin_amdgcn_ballot_w64(tf);
            wrench_wave_rscan<true>(t, th, nact, lane);
            if (lane < nact) {
                wrench_store(sh.suf[lane], t);
                sh.suf_flag[lane] = (th & (~0ull << lane)) != 0ull ? 1 : 0;
            }
        }
        __syncthreads();
    }
    // carry into this wave from the waves after it (and, MULTI, later chunks)
    Wrench cw = wrench_zero();
    if (MULTI) cw = carry;
    if (wave_active && wave + 1 < nact) {
        Wrench p = wrench_load(sh.suf[wave + 1]);
        if (MULTI && sh.suf_flag[wave + 1] == 0) wrench_add(p, carry);
        cw = p;
    }
    if (MULTI) {  // every wave advances the carry, also one idle in this chunk
        Wrench p = wrench_load(sh.suf[0]);
        if (sh.suf_flag[0] == 0) wrench_add(p, carry);
        carry = p;
    }
    if (!wave_active) return wrench_zero();
    // everything after lane l inside the wave: the inclusive value of lane
    // l + 1, complete when a chain ends in lanes after l
    Wrench S = wrench_dpp_z<kDppWaveShl1>(agg);
    if (lane == kWave - 1) S = wrench_zero();
    const bool fs = lane < kWave - 1 && (ends >> (lane + 1)) != 0ull;
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
    if constexpr (N == 1) {  // the run is already in lane order
        out[0] = lane < n ? v[0] : 0.f;
        return;
    }
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
    if constexpr (N == 1) {  // lane order is already the run's order
        if (lane < n) base[lane] = in[0];
        return;
    }
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


// ------------------------------------------------------- staging for windows
// Same transposes as above for the wave runs of a window, with every LDS and
// global address formed from a per-lane base and compile-time offsets.
// `full` (wave-uniform): all 64 N elements are valid; otherwise only the
// first n are (a window's last wave).

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

// Coalesced loads of run[0 .. 64N): element lane + 64 m goes to v[m] (0 past n).
template <int N>
__device__ __forceinline__ void run_load(const float *__restrict__ run, int n, bool full,
                                         float (&v)[N])
{
    const int lane = threadIdx.x & 63;
    if (full) {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = run[lane + 64 * m];
    } else {
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const int e = lane + 64 * m;
            v[m] = e < n ? run[e] : 0.f;
        }
    }
}

// Coalesced run (from run_load) -> lane l holds elements l N .. l N + N - 1.
// Rows of S = N + (N even) floats in LDS: element e = lane + 64 m sits at
// index e + (e / N)(S - N), which repeats with period P = N / gcd(N, 64) in m
// up to a constant step, so P per-lane bases serve all N writes; each lane
// then reads its own row.
template <int N>
__device__ __forceinline__ void run_to_lanes(float *buf, const float (&v)[N], float (&out)[N])
{
    if constexpr (N == 1) {
        out[0] = v[0];
    } else {
        const int lane = threadIdx.x & 63;
        constexpr int S = (N & 1) ? N : N + 1;
        constexpr int P = N / cgcd(N, 64);
        constexpr int STEP = 64 * P + (64 * P / N) * (S - N);
        int base[P];
#pragma unroll
        for (int m0 = 0; m0 < P; ++m0) {
            const unsigned e = (unsigned)(lane + 64 * m0);
            base[m0] = (int)(e + (e / N) * (S - N));
        }
#pragma unroll
        for (int m = 0; m < N; ++m) buf[base[m % P] + (m / P) * STEP] = v[m];
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < N; ++i) out[i] = buf[lane * S + i];
        wave_lds_sync();
    }
}

// A store that is non-temporal when NT (an output nothing in the same step
// reads again, so that it does not take cache lines from inputs that are).
template <bool NT>
__device__ __forceinline__ void out_store(float *p, float v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// run[l N + i] = in[i] of lane l for indices below n, written with 64
// consecutive floats per instruction.  Rows of N + (N even) floats in LDS;
// the read address of element e = lane + 64 m repeats with period
// P = N / gcd(N, 64) in m up to a constant step, so P per-lane bases serve
// all N reads.  NT: non-temporal stores.
template <int N, bool NT = false>
__device__ __forceinline__ void lanes_to_run(float *buf, const float (&in)[N],
                                             float *__restrict__ run, int n, bool full)
{
    const int lane = threadIdx.x & 63;
    if constexpr (N == 1) {
        if (full || lane < n) out_store<NT>(&run[lane], in[0]);
    } else {
        constexpr int S = (N & 1) ? N : N + 1;
        constexpr int P = N / cgcd(N, 64);
        constexpr int STEP = 64 * P + (64 * P / N) * (S - N);
#pragma unroll
        for (int i = 0; i < N; ++i) buf[lane * S + i] = in[i];
        wave_lds_sync();
        int base[P];
#pragma unroll
        for (int m0 = 0; m0 < P; ++m0) {
            const unsigned e = (unsigned)(lane + 64 * m0);
            base[m0] = (int)(e + (e / N) * (S - N));
        }
        if (full) {
#pragma unroll
            for (int m = 0; m < N; ++m)
                out_store<NT>(&run[lane + 64 * m], buf[base[m % P] + (m / P) * STEP]);
        } else {
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const int e = lane + 64 * m;
                if (e < n) out_store<NT>(&run[e], buf[base[m % P] + (m / P) * STEP]);
            }
        }
        wave_lds_sync();
    }
}

// Window of workgroup b in a launch that takes its n windows last to first.
// Workgroups are spread over the eight XCDs round robin (b mod 8), so within
// each class b mod 8 the windows go last to first: window t then runs on the
// XCD (t mod 8) that ran window t of a launch over the same windows in
// order, whose L2 may still hold what that launch read or wrote.  A window
// waits only on later windows, whose workgroups are at most 7 places further
// in dispatch order; each publishes before it waits, so the launch makes
// progress whenever the device holds 8 of its workgroups at once.
__device__ __forceinline__ int64_t reverse_window(int64_t b, int64_t n)
{
    const int64_t x = b & 7;
    const int64_t c = (n - x + 7) >> 3;  // windows (and workgroups) of class x
    return ((c - 1 - (b >> 3)) << 3) + x;
}

// ------------------------------------------------------ window look-back
// Windows (tiles) of a packed batch hand the scan state across window
// edges through device memory.  Every tile publishes its aggregate (the
// product of its transforms from its last chain head, or from its start if it
// has none, to its end) as kLbWords tagged 64-bit words: high half the launch
// tag, low half one float.  A tile whose first chain started in an earlier
// tile reads the aggregates of the tiles back to the one holding that head
// (a host table) and composes them in order.  Each tile publishes before it
// reads, so no wait depends on another wait; a tile only waits on tiles of
// lower index, which start no later than it does (the adjoints, which wait on
// later windows, take them in reverse: reverse_window).  Words are written and
// read with relaxed device-scope atomics (each word carries its own tag, so
// no ordering between words is needed).  The tag of a launch is one more than
// the one a tile finds in its own words (all tiles start from 0 and every
// launch runs every tile once, so they agree).  A wait gives up after
// kLbSpinLimit polls and takes NaN for the missing aggregate, so every wave
// ends even if a tile it needs never publishes.
constexpr int kLbSpinLimit = 1 << 18;

__device__ __forceinline__ uint64_t lb_load(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void lb_store(uint64_t *p, uint32_t tag, float v)
{
    __hip_atomic_store(p, ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Wait (one lane) for all kLbWords words of one tile to carry `tag`; returns
// the aggregate (NaN when the spin limit is reached first).
__device__ __forceinline__ Aff lb_wait_aff(const uint64_t *w, uint32_t tag)
{
    float v[kLbWords];
    for (int spins = 0;; ++spins) {
        bool ok = true;
#pragma unroll
        for (int k = 0; k < kLbWords; ++k) {
            const uint64_t x = lb_load(w + k);
            ok = ok && (uint32_t)(x >> 32) == tag;
            v[k] = __uint_as_float((uint32_t)x);
        }
        if (ok) break;
        if (spins >= kLbSpinLimit) {
#pragma unroll
            for (int k = 0; k < kLbWords; ++k) v[k] = __builtin_nanf("");
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return aff_load(v);
}

__device__ __forceinline__ Aff aff_readlane(const Aff &a, int l)
{
    Aff o;
    o.r00 = lane_bcast(a.r00, l); o.r10 = lane_bcast(a.r10, l); o.r20 = lane_bcast(a.r20, l);
    o.r01 = lane_bcast(a.r01, l); o.r11 = lane_bcast(a.r11, l); o.r21 = lane_bcast(a.r21, l);
    o.r02 = lane_bcast(a.r02, l); o.r12 = lane_bcast(a.r12, l); o.r22 = lane_bcast(a.r22, l);
    o.t0 = lane_bcast(a.t0, l); o.t1 = lane_bcast(a.t1, l); o.t2 = lane_bcast(a.t2, l);
    return o;
}

// The frame entering tile t: the ordered product of the aggregates of tiles
// first .. t-1 (identity when first == t).  Called by one whole wave; lanes
// wait on up to 64 tiles at a time, then an inclusive scan across the lanes
// forms their product.  The result is wave-uniform.
__device__ __forceinline__ Aff lb_carry_in(const uint64_t *status, int64_t first, int64_t t,
                                           uint32_t tag)
{
    const int lane = threadIdx.x & 63;
    Aff carry = aff_identity();
    for (int64_t b = first; b < t; b += kWave) {
        const int n = (int)min((int64_t)kWave, t - b);
        Aff a = aff_identity();
        if (lane < n) a = lb_wait_aff(status + (b + lane) * kLbWords, tag);
        if (n > 1) aff_wave_scan<false>(a, 1ull, kWave, lane);
        carry = aff_compose(carry, aff_readlane(a, n - 1));
    }
    return carry;
}


// The frame preceding each lane in window t of a launch over windows:
// segmented scan of the lane aggregates m inside each wave, then of the wave
// totals by wave 0, which publishes the window's aggregate and composes those
// of the earlier windows its first chain spans (lb_carry_in).  heads: the
// wave's lanes holding a chain head; prev, first (read by wave 0 early): the
// window's own first tagged word and the first window of its look-back.
// Every thread of the block calls it; inactive waves get the identity.
__device__ __forceinline__ Aff block_prefix_windows(Aff m, uint64_t heads, int nact, bool active,
                                                    FwdShared &sh, float (&carry_sh)[12],
                                                    uint64_t *__restrict__ status, int64_t t,
                                                    int64_t first, uint64_t prev)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (active) {
        aff_wave_scan<false>(m, heads, kWave, lane);
        if (lane == kWave - 1) {
            aff_store(sh.tot[wave], m);
            sh.tot_flag[wave] = heads != 0ull ? 1 : 0;
        }
    }
    __syncthreads();
    if (wave == 0) {
        Aff tw = aff_identity();
        bool tf = false;
        if (lane < nact) {
            tw = aff_load(sh.tot[lane]);
            tf = sh.tot_flag[lane] != 0;
        }
        const uint64_t th = __builtin_amdgcn_ballot_w64(tf);
        aff_wave_scan<true>(tw, th, nact, lane);
        if (lane < nact) {
            aff_store(sh.pre[lane], tw);
            sh.pre_flag[lane] = (th & lanes_upto(lane)) != 0ull ? 1 : 0;
        }
        wave_lds_sync();
        // publish this window's aggregate, then read the earlier windows' ones
        const uint32_t tag = (uint32_t)(__builtin_amdgcn_readfirstlane((uint32_t)(prev >> 32))) + 1u;
        if (lane < kLbWords) lb_store(status + t * kLbWords + lane, tag, sh.pre[nact - 1][lane]);
        const int64_t f = (int64_t)__builtin_amdgcn_readfirstlane((int)first);
        const Aff carry = lb_carry_in(status, f, t, tag);
        if (lane == 0) aff_store(carry_sh, carry);
    }
    __syncthreads();
    if (!active) return aff_identity();
    // frame entering the wave, then entering each lane
    const Aff carry = aff_load(carry_sh);
    Aff cw = carry;
    if (wave > 0) cw = aff_seg_after(carry, aff_load(sh.pre[wave - 1]), sh.pre_flag[wave - 1] != 0);
    Aff e = aff_dpp_z<kDppWaveShr1>(m);
    if (lane == 0) e = aff_identity();
    const bool fe = (heads & lanes_below(lane)) != 0ull;
    return fe ? e : aff_compose(cw, e);
}

// Sum of v over the 64 lanes of a wave in a fixed order (deterministic);
// wave-uniform result.
__device__ __forceinline__ float wave_sum_fixed(float v)
{
    v += dpp_f<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_f<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_f<0x141>(v);   // row_half_mirror
    v += dpp_f<0x140>(v);   // row_mirror
    return (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
}

// The adjoint's windows publish wrenches (kLbWrenchWords of a tile's
// kLbWords slots): the sum over the window from its start up to and
// including its first chain end (all of it when no chain ends there).
constexpr int kLbWrenchWords = 6;

__device__ __forceinline__ Wrench lb_wait_wrench(const uint64_t *w, uint32_t tag)
{
    float v[kLbWrenchWords];
    for (int spins = 0;; ++spins) {
        bool ok = true;
#pragma unroll
        for (int k = 0; k < kLbWrenchWords; ++k) {
            const uint64_t x = lb_load(w + k);
            ok = ok && (uint32_t)(x >> 32) == tag;
            v[k] = __uint_as_float((uint32_t)x);
        }
        if (ok) break;
        if (spins >= kLbSpinLimit) {
#pragma unroll
            for (int k = 0; k < kLbWrenchWords; ++k) v[k] = __builtin_nanf("");
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return wrench_load(v);
}

// The wrench entering window t from the windows after it: the sum of the
// published wrenches of windows t + 1 .. last (zero when last == t), in a
// fixed order.  Called by one whole wave; wave-uniform result.
__device__ __forceinline__ Wrench lb_carry_after(const uint64_t *status, int64_t t, int64_t last,
                                                 uint32_t tag)
{
    const int lane = threadIdx.x & 63;
    Wrench carry = wrench_zero();
    for (int64_t b = t + 1; b <= last; b += kWave) {
        const int n = (int)min((int64_t)kWave, last + 1 - b);
        Wrench w = wrench_zero();
        if (lane < n) w = lb_wait_wrench(status + (b + lane) * kLbWords, tag);
        carry.g0 += wave_sum_fixed(w.g0); carry.g1 += wave_sum_fixed(w.g1);
        carry.g2 += wave_sum_fixed(w.g2); carry.m0 += wave_sum_fixed(w.m0);
        carry.m1 += wave_sum_fixed(w.m1); carry.m2 += wave_sum_fixed(w.m2);
    }
    return carry;
}


// The wrench of everything after each lane, up to the end of its chain, in
// window t of a launch over windows taken last to first: segmented
// suffix scan of the lane aggregates (agg: the lane's atoms up to and
// including its first chain end; ends: lanes where a chain ends) inside each
// wave, then of the wave totals by wave 0, which publishes the window's
// wrench (from its start to its first chain end) and adds those of the later
// windows its last chain runs into (lb_carry_after).  prev, last (read by
// wave 0 early): the window's own first tagged word and the last window of
// its look-ahead.  Every thread of the block calls it; inactive waves get 0.
__device__ __forceinline__ Wrench block_suffix_windows(Wrench agg, uint64_t ends, int nact,
                                                       bool active, BwdShared &sh,
                                                       float (&carry_sh)[6],
                                                       uint64_t *__restrict__ status, int64_t t,
                                                       int64_t last, uint64_t prev)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (active) {
        wrench_wave_rscan<false>(agg, ends, kWave, lane);
        if (lane == 0) {
            wrench_store(sh.tot[wave], agg);
            sh.tot_flag[wave] = ends != 0ull ? 1 : 0;
        }
    }
    __syncthreads();
    if (wave == 0) {
        Wrench tw = wrench_zero();
        bool tf = false;
        if (lane < nact) {
            tw = wrench_load(sh.tot[lane]);
            tf = sh.tot_flag[lane] != 0;
        }
        const uint64_t th = __builtin_amdgcn_ballot_w64(tf);
        wrench_wave_rscan<true>(tw, th, nact, lane);
        if (lane < nact) {
            wrench_store(sh.suf[lane], tw);
            sh.suf_flag[lane] = (th & (~0ull << lane)) != 0ull ? 1 : 0;
        }
        wave_lds_sync();
        // publish this window's wrench, then read the later windows' ones
        const uint32_t tag = (uint32_t)(__builtin_amdgcn_readfirstlane((uint32_t)(prev >> 32))) + 1u;
        if (lane < kLbWrenchWords) lb_store(status + t * kLbWords + lane, tag, sh.suf[0][lane]);
        const int64_t l = (int64_t)__builtin_amdgcn_readfirstlane((int)last);
        const Wrench carry = lb_carry_after(status, t, l, tag);
        if (lane == 0) wrench_store(carry_sh, carry);
    }
    __syncthreads();
    if (!active) return wrench_zero();
    // everything after the wave up to the end of its last chain
    const Wrench carry = wrench_load(carry_sh);
    Wrench cw = carry;
    if (wave + 1 < nact) {
        cw = wrench_load(sh.suf[wave + 1]);
        if (sh.suf_flag[wave + 1] == 0) wrench_add(cw, carry);
    }
    // everything after lane l inside the wave: the inclusive value of lane
    // l + 1, complete when a chain ends in lanes after l
    Wrench S = wrench_dpp_z<kDppWaveShl1>(agg);
    if (lane == kWave - 1) S = wrench_zero();
    if (!(lane < kWave - 1 && (ends >> (lane + 1)) != 0ull)) wrench_add(S, cw);
    return S;
}


// A launch over windows: the sum of one float per window (each window's
// share of a loss) without a counter or a fence.  Every window publishes its
// share (block sum in a fixed order) as tagged word kLbLossWord of its
// look-back words, with the tag of this launch; the window of the last
// workgroup, started after all others, waits for all shares and adds them in
// window order into *out.  Every thread of the block calls it (one barrier).
constexpr int kLbLossWord = kLbWrenchWords;

__device__ __forceinline__ void lb_loss_commit(float v, uint64_t *__restrict__ status, int64_t t,
                                               int64_t n_win, uint64_t prev,
                                               float *__restrict__ out,
                                               float (&wave_tot)[kMaxWaves])
{
    const float share = block_sum(v, wave_tot);  // meaningful in thread 0
    const uint32_t tag = (uint32_t)(__builtin_amdgcn_readfirstlane((uint32_t)(prev >> 32))) + 1u;
    if (threadIdx.x == 0) lb_store(status + t * kLbWords + kLbLossWord, tag, share);
    if (blockIdx.x != gridDim.x - 1 || threadIdx.x >= kWave) return;
    // wave 0 of the last workgroup: lane l adds windows l, l + 64, ... in
    // order, then the lanes' sums are added in a fixed order; the words are
    // read 16 per lane at a time before any is checked (one memory latency
    // per batch)
    constexpr int kBatch = 16;
    const int lane = threadIdx.x;
    float sum = 0.f;
    for (int64_t b = 0; b < n_win; b += (int64_t)kWave * kBatch) {
        uint64_t x[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int64_t u = b + lane + (int64_t)kWave * i;
            x[i] = u < n_win ? lb_load(status + u * kLbWords + kLbLossWord) : (uint64_t)tag << 32;
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const int64_t u = b + lane + (int64_t)kWave * i;
            for (int spins = 0; (uint32_t)(x[i] >> 32) != tag; ++spins) {
                if (spins >= kLbSpinLimit) {
                    x[i] = (uint64_t)__float_as_uint(__builtin_nanf(""));
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                x[i] = lb_load(status + u * kLbWords + kLbLossWord);
            }
            sum += __uint_as_float((uint32_t)x[i]);
        }
    }
    const float total = wave_sum_fixed(sum);
    if (lane == 0) *out = total;
}


// ------------------------------------------- quaternion scan state (variant)
// The comparison form of the forward scan: a rigid transform held as a unit
// quaternion q = (w, x, y, z) and a translation t (7 floats instead of 12),
// composed as (qa, ta) . (qb, tb) = (qa qb, ta + rot(qa) tb).  Lane
// aggregates (3x4, from the walk, after their polar step) are converted to it
// and normalised, the scans and the window look-back run on it, and the
// lane's prefix is converted back to a 3x4 to place its atoms.
struct Quat {
    float w, x, y, z, t0, t1, t2;
};
constexpr int kQuatWords = 7;

__device__ __forceinline__ Quat quat_identity()
{
    Quat q;
    q.w = 1.f; q.x = q.y = q.z = 0.f;
    q.t0 = q.t1 = q.t2 = 0.f;
    return q;
}

// rot(q) v = v + w c + u x c with c = 2 u x v, u = (x, y, z)
__device__ __forceinline__ void quat_rotate(const Quat &q, float vx, float vy, float vz, float &ox,
                                            float &oy, float &oz)
{
    const float cx = 2.f * fmaf(q.y, vz, -(q.z * vy));
    const float cy = 2.f * fmaf(q.z, vx, -(q.x * vz));
    const float cz = 2.f * fmaf(q.x, vy, -(q.y * vx));
    ox = fmaf(q.w, cx, vx) + fmaf(q.y, cz, -(q.z * cy));
    oy = fmaf(q.w, cy, vy) + fmaf(q.z, cx, -(q.x * cz));
    oz = fmaf(q.w, cz, vz) + fmaf(q.x, cy, -(q.y * cx));
}

// a . b (a applied after b)
__device__ __forceinline__ Quat quat_compose(const Quat &a, const Quat &b)
{
    Quat c;
    c.w = fmaf(a.w, b.w, -fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)));
    c.x = fmaf(a.w, b.x, fmaf(a.x, b.w, fmaf(a.y, b.z, -(a.z * b.y))));
    c.y = fmaf(a.w, b.y, fmaf(-a.x, b.z, fmaf(a.y, b.w, a.z * b.x)));
    c.z = fmaf(a.w, b.z, fmaf(a.x, b.y, fmaf(-a.y, b.x, a.z * b.w)));
    float rx, ry, rz;
    quat_rotate(a, b.t0, b.t1, b.t2, rx, ry, rz);
    c.t0 = a.t0 + rx; c.t1 = a.t1 + ry; c.t2 = a.t2 + rz;
    return c;
}

__device__ __forceinline__ Quat quat_select(bool take_a, const Quat &a, const Quat &b)
{
    Quat o;
    o.w = take_a ? a.w : b.w; o.x = take_a ? a.x : b.x; o.y = take_a ? a.y : b.y;
    o.z = take_a ? a.z : b.z; o.t0 = take_a ? a.t0 : b.t0; o.t1 = take_a ? a.t1 : b.t1;
    o.t2 = take_a ? a.t2 : b.t2;
    return o;
}

template <int CTRL>
__device__ __forceinline__ Quat quat_dpp_z(const Quat &a)
{
    Quat o;
    o.w = dpp_z<CTRL>(a.w); o.x = dpp_z<CTRL>(a.x); o.y = dpp_z<CTRL>(a.y); o.z = dpp_z<CTRL>(a.z);
    o.t0 = dpp_z<CTRL>(a.t0); o.t1 = dpp_z<CTRL>(a.t1); o.t2 = dpp_z<CTRL>(a.t2);
    return o;
}

__device__ __forceinline__ Quat quat_readlane(const Quat &a, int l)
{
    Quat o;
    o.w = lane_bcast(a.w, l); o.x = lane_bcast(a.x, l); o.y = lane_bcast(a.y, l);
    o.z = lane_bcast(a.z, l); o.t0 = lane_bcast(a.t0, l); o.t1 = lane_bcast(a.t1, l);
    o.t2 = lane_bcast(a.t2, l);
    return o;
}

__device__ __forceinline__ void quat_store(float *d, const Quat &q)
{
    d[0] = q.w; d[1] = q.x; d[2] = q.y; d[3] = q.z; d[4] = q.t0; d[5] = q.t1; d[6] = q.t2;
}

__device__ __forceinline__ Quat quat_load(const float *s)
{
    Quat q;
    q.w = s[0]; q.x = s[1]; q.y = s[2]; q.z = s[3]; q.t0 = s[4]; q.t1 = s[5]; q.t2 = s[6];
    return q;
}

// Rotation part of a 3x4 to a unit quaternion by Shepperd's method (the
// largest of 1 + trace and 1 + 2 r_kk - trace chooses the component taken from
// the square root, the others from differences and sums of off-diagonal
// entries), then normalised; the translation is copied.
__device__ __forceinline__ Quat quat_from_aff(const Aff &m)
{
    const float d0 = 1.f + m.r00 + m.r11 + m.r22, d1 = 1.f + m.r00 - m.r11 - m.r22;
    const float d2 = 1.f - m.r00 + m.r11 - m.r22, d3 = 1.f - m.r00 - m.r11 + m.r22;
    const float a = m.r21 - m.r12, b = m.r02 - m.r20, c = m.r10 - m.r01;
    const float p = m.r01 + m.r10, q = m.r02 + m.r20, r = m.r12 + m.r21;
    float w, x, y, z;
    if (d0 >= d1 && d0 >= d2 && d0 >= d3) {
        const float s = 2.f * sqrtf(d0), inv = 1.f / s;
        w = 0.25f * s; x = a * inv; y = b * inv; z = c * inv;
    } else if (d1 >= d2 && d1 >= d3) {
        const float s = 2.f * sqrtf(d1), inv = 1.f / s;
        w = a * inv; x = 0.25f * s; y = p * inv; z = q * inv;
    } else if (d2 >= d3) {
        const float s = 2.f * sqrtf(d2), inv = 1.f / s;
        w = b * inv; x = p * inv; y = 0.25f * s; z = r * inv;
    } else {
        const float s = 2.f * sqrtf(d3), inv = 1.f / s;
        w = c * inv; x = q * inv; y = r * inv; z = 0.25f * s;
    }
    const float n = rsqrtf(fmaf(w, w, fmaf(x, x, fmaf(y, y, z * z))));
    Quat o;
    o.w = w * n; o.x = x * n; o.y = y * n; o.z = z * n;
    o.t0 = m.t0; o.t1 = m.t1; o.t2 = m.t2;
    return o;
}

__device__ __forceinline__ Aff aff_from_quat(const Quat &q)
{
    const float xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
    const float xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
    const float wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
    Aff m;
    m.r00 = 1.f - 2.f * (yy + zz); m.r01 = 2.f * (xy - wz); m.r02 = 2.f * (xz + wy);
    m.r10 = 2.f * (xy + wz); m.r11 = 1.f - 2.f * (xx + zz); m.r12 = 2.f * (yz - wx);
    m.r20 = 2.f * (xz - wy); m.r21 = 2.f * (yz + wx); m.r22 = 1.f - 2.f * (xx + yy);
    m.t0 = q.t0; m.t1 = q.t1; m.t2 = q.t2;
    return m;
}

template <int CTRL>
__device__ __forceinline__ void quat_scan_step(Quat &m, bool take)
{
    const Quat c = quat_compose(quat_dpp_z<CTRL>(m), m);
    m = quat_select(take, c, m);
}

// as aff_wave_scan, on the quaternion state
template <bool ROW0>
__device__ __forceinline__ void quat_wave_scan(Quat &m, uint64_t heads, int n, int lane)
{
    const int s = last_head_upto(heads, lane);
    const int row = lane & ~15;
    const int dist = lane - max(s, row);
    if (!ROW0 || n > 1) quat_scan_step<kDppRowShr + 1>(m, dist >= 1);
    if (!ROW0 || n > 2) quat_scan_step<kDppRowShr + 2>(m, dist >= 2);
    if (!ROW0 || n > 4) quat_scan_step<kDppRowShr + 4>(m, dist >= 4);
    if (!ROW0 || n > 8) quat_scan_step<kDppRowShr + 8>(m, dist >= 8);
    if (!ROW0) {
        quat_scan_step<kDppBcast15>(m, (lane & 16) != 0 && s < row);
        quat_scan_step<kDppBcast31>(m, lane >= 32 && s < 32);
    }
}

__device__ __forceinline__ Quat lb_wait_quat(const uint64_t *w, uint32_t tag)
{
    float v[kQuatWords];
    for (int spins = 0;; ++spins) {
        bool ok = true;
#pragma unroll
        for (int k = 0; k < kQuatWords; ++k) {
            const uint64_t x = lb_load(w + k);
            ok = ok && (uint32_t)(x >> 32) == tag;
            v[k] = __uint_as_float((uint32_t)x);
        }
        if (ok) break;
        if (spins >= kLbSpinLimit) {
#pragma unroll
            for (int k = 0; k < kQuatWords; ++k) v[k] = __builtin_nanf("");
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return quat_load(v);
}

// block_prefix_windows on the quaternion state; the lane's prefix returned
// as a 3x4.
__device__ __forceinline__ Aff block_prefix_windows_quat(Quat m, uint64_t heads, int nact,
                                                         bool active, FwdShared &sh,
                                                         float (&carry_sh)[12],
                                                         uint64_t *__restrict__ status, int64_t t,
                                                         int64_t first, uint64_t prev)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (active) {
        quat_wave_scan<false>(m, heads, kWave, lane);
        if (lane == kWave - 1) {
            quat_store(sh.tot[wave], m);
            sh.tot_flag[wave] = heads != 0ull ? 1 : 0;
        }
    }
    __syncthreads();
    if (wave == 0) {
        Quat tw = quat_identity();
        bool tf = false;
        if (lane < nact) {
            tw = quat_load(sh.tot[lane]);
            tf = sh.tot_flag[lane] != 0;
        }
        const uint64_t th = __builtin_amdgcn_ballot_w64(tf);
        quat_wave_scan<true>(tw, th, nact, lane);
        if (lane < nact) {
            quat_store(sh.pre[lane], tw);
            sh.pre_flag[lane] = (th & lanes_upto(lane)) != 0ull ? 1 : 0;
        }
        wave_lds_sync();
        const uint32_t tag = (uint32_t)(__builtin_amdgcn_readfirstlane((uint32_t)(prev >> 32))) + 1u;
        if (lane < kQuatWords) lb_store(status + t * kLbWords + lane, tag, sh.pre[nact - 1][lane]);
        const int64_t f = (int64_t)__builtin_amdgcn_readfirstlane((int)first);
        Quat carry = quat_identity();
        for (int64_t b = f; b < t; b += kWave) {
            const int n = (int)min((int64_t)kWave, t - b);
            Quat a = quat_identity();
            if (lane < n) a = lb_wait_quat(status + (b + lane) * kLbWords, tag);
            if (n > 1) quat_wave_scan<false>(a, 1ull, kWave, lane);
            carry = quat_compose(carry, quat_readlane(a, n - 1));
        }
        if (lane == 0) quat_store(carry_sh, carry);
    }
    __syncthreads();
    if (!active) return aff_identity();
    const Quat carry = quat_load(carry_sh);
    Quat cw = carry;
    if (wave > 0) {
        const Quat p = quat_load(sh.pre[wave - 1]);
        cw = sh.pre_flag[wave - 1] != 0 ? p : quat_compose(carry, p);
    }
    Quat e = quat_dpp_z<kDppWaveShr1>(m);
    if (lane == 0) e = quat_identity();
    const bool fe = (heads & lanes_below(lane)) != 0ull;
    return aff_from_quat(fe ? e : quat_compose(cw, e));
}

}  // namespace a2c
