// Backbone model ("Backbone model" section of the paper) on gfx950.
//
// Scan form.  Whole chains are packed into tiles; one workgroup of W waves
// owns one tile and each lane owns K consecutive residues (3K transforms).
//   1. lane-serial walk from the identity over its 3K transforms, keeping the
//      local translation of every atom and the lane aggregate (reset at chain
//      heads);
//   2. segmented inclusive scan of the lane aggregates across the wave
//      (log2(64) = 6 shuffle steps of a 3x4 affine), then of the wave totals
//      across the workgroup through LDS;
//   3. each lane maps its local translations through its exclusive prefix
//      frame and stores x, y, z planes.
// The adjoint is a reverse segmented scan of the 6-float "wrench"
// (g_k, r_k x g_k); for transform i with bond axis u_i,
//   dL/dalpha_i = u_i . (S_rg(i) - r_i x S_g(i)),
//   S_g(i) = sum_{k>i} g_k, S_rg(i) = sum_{k>i} r_k x g_k (same chain),
// which equals the sums of Eq. BackboneGradOutput because
// M_{i-1} dR_i/dalpha M_i^-1 = M_i G_x M_i^-1 moves a point p by u_i x (p - r_i).
//
// Plain form: the paper's own GPU design, kept as the comparison -- one
// workgroup per chain, a sequential product that stores M_i for every atom,
// and a backward where each thread owns one angle and sums
// g_k . (M_{i-1} dR_i M_i^-1 r_k) over all downstream atoms.
#include "scan.h"

namespace a2c {

namespace {

// Angle plane of each backbone slot: omega places N, phi places CA, psi places C.
__device__ __forceinline__ int slot_plane(int s) { return s == 0 ? 2 : (s == 1 ? 0 : 1); }

// Absolute atom positions of one lane's residues (x[3j+s], ...), given its
// angles, and the position of the atom just before the lane (the origin when
// the lane starts a chain).  Every thread of the block calls this.
template <int K, bool MULTI>
__device__ __forceinline__ void bb_lane_positions(
    const float (&phi)[K], const float (&psi)[K], const float (&om)[K],
    const BBParams &P, int nact, FwdShared &sh, Aff &carry, float (&x)[3 * K],
    float (&y)[3 * K], float (&z)[3 * K], float &px, float &py, float &pz, int cnt, uint32_t hm)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool wave_active = wave < nact;

    Aff m = aff_identity();
    int first_head = K;    // residues before it need the carry-in frame
    // zero first, write only valid residues below: stores to the same
    // element from two branches get merged through a select of addresses,
    // which forces the arrays out of registers into scratch memory
#pragma unroll
    for (int i = 0; i < 3 * K; ++i) x[i] = y[i] = z[i] = 0.f;
    if (wave_active) {
        // sin/cos of all 3K angles up front, with one wave-uniform choice
        // between the branch-free reduction and the library (huge or non-finite
        // arguments), so the independent evaluations interleave
        float so[K], co[K], sp[K], cp[K], ss[K], cs[K];
        bool ok = true;
#pragma unroll
        for (int j = 0; j < K; ++j)
            ok = ok && sincos_fast_ok(om[j]) && sincos_fast_ok(phi[j]) && sincos_fast_ok(psi[j]);
        if (__all(ok)) {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                sincos_fast(om[j], so[j], co[j]);
                sincos_fast(phi[j], sp[j], cp[j]);
                sincos_fast(psi[j], ss[j], cs[j]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                sincos_accurate(om[j], so[j], co[j]);
                sincos_accurate(phi[j], sp[j], cp[j]);
                sincos_accurate(psi[j], ss[j], cs[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j < cnt) {
                if ((hm >> j) & 1u) {
                    m = aff_identity();
                    if (first_head == K) first_head = j;
                }
                aff_apply_transform(m, P.ct[0], P.st[0], P.d[0], co[j], so[j]);
                x[3 * j] = m.t0; y[3 * j] = m.t1; z[3 * j] = m.t2;
                aff_apply_transform(m, P.ct[1], P.st[1], P.d[1], cp[j], sp[j]);
                x[3 * j + 1] = m.t0; y[3 * j + 1] = m.t1; z[3 * j + 1] = m.t2;
                aff_apply_transform(m, P.ct[2], P.st[2], P.d[2], cs[j], ss[j]);
                x[3 * j + 2] = m.t0; y[3 * j + 2] = m.t1; z[3 * j + 2] = m.t2;
            }
        }
        // the fixed rotations repeat every residue, so their float32 rounding
        // drifts the scale of long products coherently; one polar step per
        // lane aggregate (every 3K transforms) removes that drift
        aff_orthonormalise(m);
    }
    const Aff X = block_exclusive_prefix<MULTI>(m, first_head < K, nact, sh, carry);
    px = py = pz = 0.f;
    if (!wave_active) return;
    // previous atom position (origin when the lane's first residue is a head)
    if (!(hm & 1u)) { px = X.t0; py = X.t1; pz = X.t2; }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < first_head) {
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                float gx, gy, gz;
                aff_point(X, x[3 * j + s], y[3 * j + s], z[3 * j + s], gx, gy, gz);
                x[3 * j + s] = gx; y[3 * j + s] = gy; z[3 * j + s] = gz;
            }
        }
    }
}

// Angle gradients of one lane (gr[s][j]: slot s of residue j; slot 0 is
// omega, 1 phi, 2 psi) from absolute positions, upstream gradients and the
// atom before the lane: a reverse segmented scan of wrenches over the tile.
// Every thread of the block calls this.
template <int K, bool MULTI>
__device__ __forceinline__ void bb_lane_adjoint(
    const BBParams &P, int nact, BwdShared &sh, Wrench &carry,
    const float (&x)[3 * K], const float (&y)[3 * K], const float (&z)[3 * K],
    const float (&gx)[3 * K], const float (&gy)[3 * K], const float (&gz)[3 * K], float px,
    float py, float pz, int cnt, uint32_t hm, uint32_t lm, float (&gr)[3][K])
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool wave_active = wave < nact;

    // lm: residue j is the last of its chain when residue j+1 starts one (the
    // bit array also marks R, and tiles end at chain ends)
    Wrench agg = wrench_zero();
    bool f = false;
    if (wave_active) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j < cnt) {
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    const int i = 3 * j + s;
                    if (!f) wrench_add_point(agg, x[i], y[i], z[i], gx[i], gy[i], gz[i]);
                }
                if ((lm >> j) & 1u) f = true;
            }
        }
    }
    Wrench S = block_exclusive_suffix<MULTI>(agg, f, nact, sh, carry);
    if (!wave_active) return;
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
        if (j < cnt) {
            if ((lm >> j) & 1u) S = wrench_zero();
            const bool head = (hm >> j) & 1u;
#pragma unroll
            for (int s = 2; s >= 0; --s) {
                const int i = 3 * j + s;
                float qx, qy, qz;  // atom before i
                if (s > 0) { qx = x[i - 1]; qy = y[i - 1]; qz = z[i - 1]; }
                else if (head) { qx = 0.f; qy = 0.f; qz = 0.f; }
                else if (j > 0) { qx = x[i - 1]; qy = y[i - 1]; qz = z[i - 1]; }
                else { qx = px; qy = py; qz = pz; }
                const float ux = (x[i] - qx) * P.inv_d[s];
                const float uy = (y[i] - qy) * P.inv_d[s];
                const float uz = (z[i] - qz) * P.inv_d[s];
                gr[s][j] = wrench_torque(S, x[i], y[i], z[i], ux, uy, uz);
                wrench_add_point(S, x[i], y[i], z[i], gx[i], gy[i], gz[i]);
            }
        } else {
            gr[0][j] = gr[1][j] = gr[2][j] = 0.f;
        }
    }
}

template <int K>
__device__ __forceinline__ void store_angle_grads(float *buf, float (&gr)[3][K], float *gang,
                                                  int64_t R, int64_t rbase, int nres)
{
    stage_store<K>(buf, gr[1], gang + rbase, nres);           // phi  (slot CA)
    stage_store<K>(buf, gr[2], gang + R + rbase, nres);       // psi  (slot C)
    stage_store<K>(buf, gr[0], gang + 2 * R + rbase, nres);   // omega (slot N)
}

template <int K>
constexpr size_t stage_bytes(int waves)
{
    return (size_t)waves * kWave * Stride<3 * K>::value * sizeof(float);
}

// Chunk c of a tile: residues [cs, ce) handled by the waves wave < nact.
struct Chunk {
    int64_t cs, ce;
    int nact;
};

template <int K>
__device__ __forceinline__ Chunk chunk_of(int64_t ts, int64_t te, int c)
{
    const int nw = blockDim.x >> 6;
    const int64_t ch = (int64_t)kWave * K * nw;
    Chunk k;
    k.cs = ts + (int64_t)c * ch;
    k.ce = min(k.cs + ch, te);
    k.nact = (int)min((int64_t)nw, (k.ce - k.cs + kWave * K - 1) / (kWave * K));
    return k;
}

template <int K>
__device__ __forceinline__ int chunks_of(int64_t ts, int64_t te)
{
    const int64_t ch = (int64_t)kWave * K * (blockDim.x >> 6);
    return (int)((te - ts + ch - 1) / ch);
}

// Angles of one wave's run -> lane-blocked phi, psi, omega.
template <int K>
__device__ __forceinline__ void load_angles(float *buf, const float *__restrict__ ang, int64_t R,
                                            int64_t rbase, int nres, float (&phi)[K],
                                            float (&psi)[K], float (&om)[K])
{
    float v0[K], v1[K], v2[K];
    gload<K>(ang + rbase, nres, v0);
    gload<K>(ang + R + rbase, nres, v1);
    gload<K>(ang + 2 * R + rbase, nres, v2);
    to_blocked<K>(buf, v0, nres, phi);
    to_blocked<K>(buf, v1, nres, psi);
    to_blocked<K>(buf, v2, nres, om);
}

// Forward over windows of the packed batch: window t covers residues
// [wstart[t], wstart[t + 1]), at most C = 64 W K of them (fixed windows
// [t C, t C + C) whatever the chains, or whole chains where every chain
// fits in one); lane l of wave w owns K consecutive residues.  A chain that
// enters the window from an earlier one gets its frame from those windows'
// published aggregates (window look-back); every lane holds K residues
// except in a window's last wave.
//   1. angles: coalesced loads of the three planes, LDS transpose to lanes;
//   2. per lane: sincos, walk from the identity over its 3K transforms
//      (restarting at chain heads), local positions, one polar step;
//   3. segmented scan of the lane aggregates across each wave, then of the
//      wave totals by wave 0, which publishes the tile's aggregate and then
//      composes the aggregates of the earlier tiles its first chain spans;
//   4. each lane maps the positions before its first chain head through its
//      exclusive prefix frame; LDS transpose, coalesced stores of x, y, z.
// QUAT: the comparison form with a unit quaternion + translation scan state
// (Quat) in place of the 3x4 affine (lane aggregates converted after their
// polar step).
template <int K, int LB, bool QUAT = false>
__global__ __launch_bounds__(LB, 4) void bb_forward_flat_kernel(
    const float *__restrict__ ang, float *__restrict__ xyz, const uint32_t *__restrict__ head_bits,
    const int32_t *__restrict__ wstart, const int32_t *__restrict__ look_first,
    uint64_t *__restrict__ status, int64_t R, BBParams P)
{
    extern __shared__ float stage_mem[];
    __shared__ FwdShared sh;
    __shared__ float carry_sh[12];
    constexpr int RUN = kWave * K;  // residues per wave
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = blockIdx.x;
    const int64_t ts = wstart[t], te = wstart[t + 1];
    const int nact = (int)((te - ts + RUN - 1) / RUN);
    const int64_t rbase = ts + (int64_t)wave * RUN;
    const int nres = (int)max((int64_t)0, min((int64_t)RUN, te - rbase));
    const bool active = nres > 0, full = nres == RUN;
    const int64_t rs = rbase + lane * K;
    float *buf = stage_mem + wave * kWave * Stride<3 * K>::value;
    const int64_t A = 3 * R;
    // own words of the previous launch (the tag) and the look-back range,
    // read ahead of the angles so that their latency overlaps
    uint64_t prev = 0;
    int64_t first = t;
    if (wave == 0) {
        prev = lb_load(status + t * kLbWords);
        first = look_first[t];
    }
    const uint32_t hm = head_mask<K>(head_bits, rs < te ? rs : te);
    float phi[K], psi[K], om[K];
    if (active) {
        float v0[K], v1[K], v2[K];
        run_load<K>(ang + rbase, nres, full, v0);
        run_load<K>(ang + R + rbase, nres, full, v1);
        run_load<K>(ang + 2 * R + rbase, nres, full, v2);
        run_to_lanes<K>(buf, v0, phi);
        run_to_lanes<K>(buf, v1, psi);
        run_to_lanes<K>(buf, v2, om);
    }
    float x[3 * K], y[3 * K], z[3 * K];
    Aff m = aff_identity();
    int first_head = K;  // residues before it need the frame entering the lane
    if (active) {
        // one wave-uniform choice between the branch-free sincos and the
        // library (huge or non-finite arguments anywhere in the wave)
        bool ok = true;
#pragma unroll
        for (int j = 0; j < K; ++j)
            ok = ok && sincos_fast_ok(om[j]) && sincos_fast_ok(phi[j]) && sincos_fast_ok(psi[j]);
        const bool fast = __all(ok);
        // Residues past the batch end (last wave only) are walked too: their
        // positions are never stored and nothing after them reads the frame.
#pragma unroll
        for (int j = 0; j < K; ++j) {
            float so, co, sp, cp, ss, cs;
            if (fast) {
                sincos_fast(om[j], so, co);
                sincos_fast(phi[j], sp, cp);
                sincos_fast(psi[j], ss, cs);
            } else {
                sincos_accurate(om[j], so, co);
                sincos_accurate(phi[j], sp, cp);
                sincos_accurate(psi[j], ss, cs);
            }
            // the lane's walk starts from the identity, and so does a chain
            // that starts here (a wave-uniform test keeps the rare restart
            // out of the common path)
            const bool h = (hm >> j) & 1u;
            if (j == 0) {
                m = aff_first_transform(P.ct[0], P.st[0], P.d[0], co, so);
                first_head = h ? 0 : first_head;
            } else if (__builtin_amdgcn_ballot_w64(h) != 0ull) {
                const Aff f = aff_first_transform(P.ct[0], P.st[0], P.d[0], co, so);
                aff_apply_transform(m, P.ct[0], P.st[0], P.d[0], co, so);
                m = aff_select(h, f, m);
                first_head = (h && first_head == K) ? j : first_head;
            } else {
                aff_apply_transform(m, P.ct[0], P.st[0], P.d[0], co, so);
            }
            x[3 * j] = m.t0; y[3 * j] = m.t1; z[3 * j] = m.t2;
            aff_apply_transform(m, P.ct[1], P.st[1], P.d[1], cp, sp);
            x[3 * j + 1] = m.t0; y[3 * j + 1] = m.t1; z[3 * j + 1] = m.t2;
            aff_apply_transform(m, P.ct[2], P.st[2], P.d[2], cs, ss);
            x[3 * j + 2] = m.t0; y[3 * j + 2] = m.t1; z[3 * j + 2] = m.t2;
        }
        // the fixed rotations repeat every residue, so their float32 rounding
        // drifts the scale of long products coherently; one polar step per
        // lane aggregate removes that drift
        aff_orthonormalise(m);
    }
    const uint64_t heads = __builtin_amdgcn_ballot_w64(first_head < K);
    Aff X;
    if constexpr (QUAT)
        X = block_prefix_windows_quat(quat_from_aff(m), heads, nact, active, sh, carry_sh, status, t,
                                      first, prev);
    else
        X = block_prefix_windows(m, heads, nact, active, sh, carry_sh, status, t, first, prev);
    if (!active) return;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < first_head) {
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                float gx, gy, gz;
                aff_point(X, x[3 * j + s], y[3 * j + s], z[3 * j + s], gx, gy, gz);
                x[3 * j + s] = gx; y[3 * j + s] = gy; z[3 * j + s] = gz;
            }
        }
    }
    float *out = xyz + 3 * rbase;
    lanes_to_run<3 * K>(buf, x, out, 3 * nres, full);
    lanes_to_run<3 * K>(buf, y, out + A, 3 * nres, full);
    lanes_to_run<3 * K>(buf, z, out + 2 * A, 3 * nres, full);
}

// Backward that recomputes the frames from the angles (no stored state).
// Tiles of several chunks first run the forward scan alone to record each
// chunk's carry-in frame, then visit the chunks last to first.
//   GM = kGradLoad: the upstream gradient is read from g;
//   GM = kGradMse:  g points at a target t and the upstream gradient is that
//                   of the squared distance, 2 (r - t), formed in registers
//                   from the recomputed positions (the fused training step);
//                   xyz_out (may be NULL) receives the positions, loss_out
//                   (may be NULL) the batch's sum of |r - t|^2 (from the
//                   tiles' shares in loss_part, counted in loss_count).
template <int K, bool MULTI, int LB, int GM>
__global__ __launch_bounds__(LB) void bb_backward_recompute_kernel(
    const float *__restrict__ ang, const float *__restrict__ g, float *__restrict__ gang,
    float *__restrict__ xyz_out, float *__restrict__ loss_out, float *__restrict__ loss_part,
    uint32_t *__restrict__ loss_count, const int32_t *__restrict__ tile_res,
    const uint32_t *__restrict__ head_bits, int64_t R, BBParams P0)
{
    extern __shared__ float stage_mem[];
    __shared__ FwdShared shf[2];
    __shared__ BwdShared shb[2];
    __shared__ float fwd_carry[kMaxChunks][12];
    __shared__ float loss_tot[GM == kGradMse ? kMaxWaves : 1];
    float loss = 0.f;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *buf = stage_mem + wave * kWave * Stride<3 * K>::value;
    const int64_t ts = tile_res[2 * blockIdx.x], te = tile_res[2 * blockIdx.x + 1];
    const int64_t A = 3 * R;
    // MULTI = false: every tile is one chunk (straight-line code)
    const int nch = MULTI ? chunks_of<K>(ts, te) : 1;
    if (nch > 1) {
        Aff carry = aff_identity();
        for (int c = 0; c < nch; ++c) {
            const BBParams P = MULTI ? opaque_params(P0) : P0;
            if (threadIdx.x == 0) aff_store(fwd_carry[c], carry);
            const Chunk k = chunk_of<K>(ts, te, c);
            const int64_t rbase = k.cs + (int64_t)wave * kWave * K;
            const bool active = wave < k.nact;
            const int nres = active ? (int)min((int64_t)kWave * K, k.ce - rbase) : 0;
            const int64_t rs = k.cs + (int64_t)threadIdx.x * K;
            const int cnt = (int)max((int64_t)0, min((int64_t)K, k.ce - rs));
            const uint32_t hm = lane_head_mask<K>(head_bits, rs, k.ce, cnt);
            float phi[K], psi[K], om[K];
            if (active) load_angles<K>(buf, ang, R, rbase, nres, phi, psi, om);
            float x[3 * K], y[3 * K], z[3 * K];
            float px, py, pz;
            bb_lane_positions<K, MULTI>(phi, psi, om, P, k.nact, shf[c & 1], carry, x, y, z, px, py, pz,
                                 cnt, hm);
        }
    }
    Wrench rcarry = wrench_zero();
    for (int c = nch - 1; c >= 0; --c) {
        const BBParams P = MULTI ? opaque_params(P0) : P0;
        const Chunk k = chunk_of<K>(ts, te, c);
        const int64_t rbase = k.cs + (int64_t)wave * kWave * K;
        const bool active = wave < k.nact;
        const int nres = active ? (int)min((int64_t)kWave * K, k.ce - rbase) : 0;
        const int64_t rs = k.cs + (int64_t)threadIdx.x * K;
        const int cnt = (int)max((int64_t)0, min((int64_t)K, k.ce - rs));
        const uint32_t hm = lane_head_mask<K>(head_bits, rs, k.ce, cnt);
        const uint32_t lm = lane_head_mask<K>(head_bits, rs + 1, k.ce + 1, cnt);
        float phi[K], psi[K], om[K];
        float gx[3 * K], gy[3 * K], gz[3 * K];
        if (active) {
            float v0[K], v1[K], v2[K], w0[3 * K], w1[3 * K], w2[3 * K];
            const float *gb = g + 3 * rbase;
            gload<K>(ang + rbase, nres, v0);
            gload<K>(ang + R + rbase, nres, v1);
            gload<K>(ang + 2 * R + rbase, nres, v2);
            gload<3 * K>(gb, 3 * nres, w0);
            gload<3 * K>(gb + A, 3 * nres, w1);
            gload<3 * K>(gb + 2 * A, 3 * nres, w2);
            to_blocked<K>(buf, v0, nres, phi);
            to_blocked<K>(buf, v1, nres, psi);
            to_blocked<K>(buf, v2, nres, om);
            to_blocked<3 * K>(buf, w0, 3 * nres, gx);
            to_blocked<3 * K>(buf, w1, 3 * nres, gy);
            to_blocked<3 * K>(buf, w2, 3 * nres, gz);
        }
        Aff fcarry = aff_identity();
        if (nch > 1) fcarry = aff_load(fwd_carry[c]);
        float x[3 * K], y[3 * K], z[3 * K];
        float px, py, pz;
        // buffers alternate with the pass above: its last chunk used shf[(nch-1) & 1]
        bb_lane_positions<K, MULTI>(phi, psi, om, P, k.nact, shf[(c + 1) & 1], fcarry, x, y, z, px, py,
                             pz, cnt, hm);
        if (GM == kGradMse) {
            // gx.. hold the target: the loss gradient 2 (r - t) of valid atoms
#pragma unroll
            for (int i = 0; i < 3 * K; ++i) {
                const float dx = x[i] - gx[i], dy = y[i] - gy[i], dz = z[i] - gz[i];
                const bool v = i < 3 * cnt;
                loss += v ? dx * dx + dy * dy + dz * dz : 0.f;
                gx[i] = v ? 2.f * dx : 0.f;
                gy[i] = v ? 2.f * dy : 0.f;
                gz[i] = v ? 2.f * dz : 0.f;
            }
            if (xyz_out && active) {
                float *out = xyz_out + 3 * rbase;
                stage_store<3 * K>(buf, x, out, 3 * nres);
                stage_store<3 * K>(buf, y, out + A, 3 * nres);
                stage_store<3 * K>(buf, z, out + 2 * A, 3 * nres);
            }
        }
        float gr[3][K];
        bb_lane_adjoint<K, MULTI>(P, k.nact, shb[c & 1], rcarry, x, y, z, gx, gy, gz, px, py, pz, cnt,
                           hm, lm, gr);
        if (active) store_angle_grads<K>(buf, gr, gang, R, rbase, nres);
    }
    if constexpr (GM == kGradMse) {
        if (loss_out) loss_commit(loss, loss_part, loss_count, loss_out, loss_tot);
    }
}

// Adjoint from the coordinates the forward produced, over windows of the
// packed batch (as the forward), last window first (rev: reverse_window,
// which keeps window t on the XCD of the forward's window t where the two
// schedules cut the same windows).  A window publishes the wrench sum from
// its start up to its first chain end, then adds those of the later windows
// its last chain runs into (window look-back).  Windows that hold whole
// chains wait on none, and go in order (rev = 0): workgroup t then runs on
// the same XCD as the forward's window t (workgroups are spread over the
// XCDs round robin), whose L2 still holds the coordinates it wrote.
//   1. coordinates and upstream gradients: coalesced loads, LDS transpose;
//   2. per lane: wrench sum of its atoms up to and including its first chain
//      end; segmented suffix scan across the wave, then of the wave totals by
//      wave 0, which publishes and reads the window wrenches;
//   3. per lane, last atom first: dL/dalpha = u . (S_rg - r x S_g) with S the
//      wrench of everything after the atom in its chain, then add the atom;
//   4. LDS transpose, coalesced stores of the phi, psi, omega planes
//      (non-temporal when nt: large plans).
template <int K, int LB>
__global__ __launch_bounds__(LB) void bb_backward_coords_flat_kernel(
    const float *__restrict__ xyz, const float *__restrict__ g, float *__restrict__ gang,
    const uint32_t *__restrict__ head_bits, const int32_t *__restrict__ wstart,
    const int32_t *__restrict__ look_last, uint64_t *__restrict__ status, int64_t R, BBParams P,
    int32_t rev, int32_t nt)
{
    extern __shared__ float stage_mem[];
    __shared__ BwdShared sh;
    __shared__ float carry_sh[6];
    constexpr int RUN = kWave * K;  // residues per wave
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = rev ? reverse_window(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t ts = wstart[t], te = wstart[t + 1];
    const int nact = (int)((te - ts + RUN - 1) / RUN);
    const int64_t rbase = ts + (int64_t)wave * RUN;
    const int nres = (int)max((int64_t)0, min((int64_t)RUN, te - rbase));
    const bool active = nres > 0, full = nres == RUN;
    const int64_t rs = rbase + lane * K;
    float *buf = stage_mem + wave * kWave * Stride<3 * K>::value;
    const int64_t A = 3 * R;
    uint64_t prev = 0;
    int64_t last = t;
    if (wave == 0) {
        prev = lb_load(status + t * kLbWords);
        last = look_last[t];
    }
    // heads (hm) and chain ends (lm: residue j ends a chain when j + 1 starts
    // one; bit R is set) of the lane's residues.  Lanes past the batch end
    // hold zero gradients, so whatever bits they read add nothing.
    const uint32_t hm = head_mask<K>(head_bits, rs < te ? rs : te);
    const uint32_t lm = head_mask<K>(head_bits, rs < te ? rs + 1 : te + 1);
    float x[3 * K], y[3 * K], z[3 * K], gx[3 * K], gy[3 * K], gz[3 * K];
    float px = 0.f, py = 0.f, pz = 0.f;  // the atom before the lane's first
    if (active) {
        // the atom before lane 0 of the wave (read ahead of the fenced transposes)
        float px0 = 0.f, py0 = 0.f, pz0 = 0.f;
        if (lane == 0 && !(hm & 1u)) {
            const float *xb = xyz + 3 * rs;
            px0 = xb[-1]; py0 = xb[A - 1]; pz0 = xb[2 * A - 1];
        }
        float w0[3 * K], w1[3 * K], w2[3 * K], w3[3 * K], w4[3 * K], w5[3 * K];
        const float *xb = xyz + 3 * rbase, *gb = g + 3 * rbase;
        run_load<3 * K>(xb, 3 * nres, full, w0);
        run_load<3 * K>(xb + A, 3 * nres, full, w1);
        run_load<3 * K>(xb + 2 * A, 3 * nres, full, w2);
        run_load<3 * K>(gb, 3 * nres, full, w3);
        run_load<3 * K>(gb + A, 3 * nres, full, w4);
        run_load<3 * K>(gb + 2 * A, 3 * nres, full, w5);
        run_to_lanes<3 * K>(buf, w0, x);
        run_to_lanes<3 * K>(buf, w1, y);
        run_to_lanes<3 * K>(buf, w2, z);
        run_to_lanes<3 * K>(buf, w3, gx);
        run_to_lanes<3 * K>(buf, w4, gy);
        run_to_lanes<3 * K>(buf, w5, gz);
        const float lx = dpp_f<kDppWaveShr1>(x[3 * K - 1]);
        const float ly = dpp_f<kDppWaveShr1>(y[3 * K - 1]);
        const float lz = dpp_f<kDppWaveShr1>(z[3 * K - 1]);
        if (!(hm & 1u)) {
            px = lane > 0 ? lx : px0;
            py = lane > 0 ? ly : py0;
            pz = lane > 0 ? lz : pz0;
        }
    }
    // wrench of the lane's atoms up to and including its first chain end
    Wrench agg = wrench_zero();
    bool f = false;
    if (active) {
        if (__builtin_amdgcn_ballot_w64(lm != 0u) == 0ull) {  // no chain ends in the wave
#pragma unroll
            for (int i = 0; i < 3 * K; ++i) wrench_add_point(agg, x[i], y[i], z[i], gx[i], gy[i], gz[i]);
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j) {
#pragma unroll
                for (int s = 0; s < 3; ++s) {
                    const int i = 3 * j + s;
                    if (!f) wrench_add_point(agg, x[i], y[i], z[i], gx[i], gy[i], gz[i]);
                }
                if ((lm >> j) & 1u) f = true;
            }
        }
    }
    const uint64_t ends = __builtin_amdgcn_ballot_w64(f);
    Wrench S = block_suffix_windows(agg, ends, nact, active, sh, carry_sh, status, t, last, prev);
    if (!active) return;
    float gr[3][K];
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
        if ((lm >> j) & 1u) S = wrench_zero();
        const bool head = (hm >> j) & 1u;
#pragma unroll
        for (int s = 2; s >= 0; --s) {
            const int i = 3 * j + s;
            float qx, qy, qz;  // atom before i
            if (s > 0) { qx = x[i - 1]; qy = y[i - 1]; qz = z[i - 1]; }
            else if (head) { qx = 0.f; qy = 0.f; qz = 0.f; }
            else if (j > 0) { qx = x[i - 1]; qy = y[i - 1]; qz = z[i - 1]; }
            else { qx = px; qy = py; qz = pz; }
            const float ux = (x[i] - qx) * P.inv_d[s];
            const float uy = (y[i] - qy) * P.inv_d[s];
            const float uz = (z[i] - qz) * P.inv_d[s];
            gr[s][j] = wrench_torque(S, x[i], y[i], z[i], ux, uy, uz);
            wrench_add_point(S, x[i], y[i], z[i], gx[i], gy[i], gz[i]);
        }
    }
    if (nt) {
        lanes_to_run<K, true>(buf, gr[1], gang + rbase, nres, full);          // phi  (slot CA)
        lanes_to_run<K, true>(buf, gr[2], gang + R + rbase, nres, full);      // psi  (slot C)
        lanes_to_run<K, true>(buf, gr[0], gang + 2 * R + rbase, nres, full);  // omega (slot N)
    } else {
        lanes_to_run<K>(buf, gr[1], gang + rbase, nres, full);
        lanes_to_run<K>(buf, gr[2], gang + R + rbase, nres, full);
        lanes_to_run<K>(buf, gr[0], gang + 2 * R + rbase, nres, full);
    }
}

// ---------------------------------------------------------------- plain form

__global__ __launch_bounds__(64) void bb_forward_plain_kernel(
    const float *__restrict__ ang, float *__restrict__ xyz, float *__restrict__ ws,
    const int32_t *__restrict__ res_off, int64_t R, BBParams P)
{
    if (threadIdx.x != 0) return;
    const int64_t r0 = res_off[blockIdx.x], r1 = res_off[blockIdx.x + 1];
    const int64_t A = 3 * R;
    Aff m = aff_identity();
    for (int64_t r = r0; r < r1; ++r) {
        if (r > r0 && ((r - r0) & 3) == 0) aff_orthonormalise(m);
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            float sa, ca;
            sincos_accurate(ang[(int64_t)slot_plane(s) * R + r], sa, ca);
            aff_apply_transform(m, P.ct[s], P.st[s], P.d[s], ca, sa);
            const int64_t a = 3 * r + s;
            aff_store(ws + 12 * a, m);
            xyz[a] = m.t0;
            xyz[A + a] = m.t1;
            xyz[2 * A + a] = m.t2;
        }
    }
}

constexpr int kPlainBlock = 256;

__global__ __launch_bounds__(kPlainBlock) void bb_backward_plain_kernel(
    const float *__restrict__ ang, const float *__restrict__ g, float *__restrict__ gang,
    const float *__restrict__ ws, const int32_t *__restrict__ res_off, int64_t R, BBParams P)
{
    __shared__ float s_r[3][kPlainBlock];
    __shared__ float s_g[3][kPlainBlock];
    const int64_t r0 = res_off[blockIdx.x];
    const int64_t n = 3 * (res_off[blockIdx.x + 1] - r0);  // atoms (= angles) in chain
    const int64_t ib = (int64_t)blockIdx.y * kPlainBlock;
    if (ib >= n) return;  // whole block past the chain end (padded launch)
    const int64_t A = 3 * R;
    const int64_t a0 = 3 * r0;
    const int tid = threadIdx.x;
    const int64_t i = ib + tid;
    const bool active = i < n;
    // F_i = M_{i-1} dR_i/dalpha M_i^-1 in 3x4 form: F.R = (R_{i-1} dR) R_i^T,
    // F.t = -F.R t_i  (dR has no translation part)
    float f00 = 0, f01 = 0, f02 = 0, f10 = 0, f11 = 0, f12 = 0, f20 = 0, f21 = 0, f22 = 0;
    float tix = 0, tiy = 0, tiz = 0;
    if (active) {
        const int s = (int)(i % 3);
        float sa, ca;
        sincos_accurate(ang[(int64_t)slot_plane(s) * R + r0 + i / 3], sa, ca);
        const float ct = P.ct[s], st = P.st[s];
        // dR (3x3): [[0, ca st, -sa st], [0, -sa, -ca], [0, ca ct, -sa ct]]
        const float d01 = ca * st, d02 = -sa * st, d11 = -sa, d12 = -ca, d21 = ca * ct,
                    d22 = -sa * ct;
        Aff mp = aff_identity();
        if (i > 0) mp = aff_load(ws + 12 * (a0 + i - 1));
        const Aff mi = aff_load(ws + 12 * (a0 + i));
        // B = R_{i-1} dR (first column is zero)
        const float b01 = mp.r00 * d01 + mp.r01 * d11 + mp.r02 * d21;
        const float b11 = mp.r10 * d01 + mp.r11 * d11 + mp.r12 * d21;
        const float b21 = mp.r20 * d01 + mp.r21 * d11 + mp.r22 * d21;
        const float b02 = mp.r00 * d02 + mp.r01 * d12 + mp.r02 * d22;
        const float b12 = mp.r10 * d02 + mp.r11 * d12 + mp.r12 * d22;
        const float b22 = mp.r20 * d02 + mp.r21 * d12 + mp.r22 * d22;
        // F.R = B R_i^T: (B R^T)_{rc} = sum_k B_{rk} R_{ck}
        f00 = b01 * mi.r01 + b02 * mi.r02;
        f01 = b01 * mi.r11 + b02 * mi.r12;
        f02 = b01 * mi.r21 + b02 * mi.r22;
        f10 = b11 * mi.r01 + b12 * mi.r02;
        f11 = b11 * mi.r11 + b12 * mi.r12;
        f12 = b11 * mi.r21 + b12 * mi.r22;
        f20 = b21 * mi.r01 + b22 * mi.r02;
        f21 = b21 * mi.r11 + b22 * mi.r12;
        f22 = b21 * mi.r21 + b22 * mi.r22;
        tix = mi.t0; tiy = mi.t1; tiz = mi.t2;
    }
    float acc = 0.f;
    for (int64_t kb = ib; kb < n; kb += kPlainBlock) {
        const int64_t k = kb + tid;
        if (k < n) {
            const float *mk = ws + 12 * (a0 + k);
            s_r[0][tid] = mk[9]; s_r[1][tid] = mk[10]; s_r[2][tid] = mk[11];
            s_g[0][tid] = g[a0 + k]; s_g[1][tid] = g[A + a0 + k]; s_g[2][tid] = g[2 * A + a0 + k];
        }
        __syncthreads();
        if (active) {
            const int kmax = (int)min((int64_t)kPlainBlock, n - kb);
            const int kmin = (int)max((int64_t)0, i - kb);
            for (int kk = kmin; kk < kmax; ++kk) {
                const float dx = s_r[0][kk] - tix, dy = s_r[1][kk] - tiy, dz = s_r[2][kk] - tiz;
                const float vx = f00 * dx + f01 * dy + f02 * dz;
                const float vy = f10 * dx + f11 * dy + f12 * dz;
                const float vz = f20 * dx + f21 * dy + f22 * dz;
                acc += s_g[0][kk] * vx + s_g[1][kk] * vy + s_g[2][kk] * vz;
            }
        }
        __syncthreads();
    }
    if (active) gang[(int64_t)slot_plane((int)(i % 3)) * R + r0 + i / 3] = acc;
}

template <int K, int LB, bool QUAT>
hipError_t fwd_kl(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s)
{
    const dim3 grid(p.fs.n_win), block(p.fs.W * kWave);
    hipLaunchKernelGGL((bb_forward_flat_kernel<K, LB, QUAT>), grid, block, stage_bytes<K>(p.fs.W), s,
                       ang, xyz, p.d_head_bits, p.fs.d_wstart, p.fs.d_look, p.fs.d_status, p.R,
                       p.bb);
    return hipGetLastError();
}

template <int K, bool QUAT>
hipError_t fwd_kq(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s)
{
    const int threads = p.fs.W * kWave;
    if (threads <= 256) return fwd_kl<K, 256, QUAT>(p, ang, xyz, s);
    if (threads <= kLbSmall) return fwd_kl<K, kLbSmall, QUAT>(p, ang, xyz, s);
    return fwd_kl<K, kLbLarge, QUAT>(p, ang, xyz, s);
}

template <int K>
hipError_t fwd_k(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s, bool quat)
{
    return quat ? fwd_kq<K, true>(p, ang, xyz, s) : fwd_kq<K, false>(p, ang, xyz, s);
}

template <int K, bool MULTI, int LB>
hipError_t bwd_kml(const a2c_plan &p, const float *ang, const float *xyz, const float *g,
                   float *gang, hipStream_t s)
{
    const dim3 grid(p.bs.n_tiles), block(p.bs.W * kWave);
    const size_t lds = stage_bytes<K>(p.bs.W);
    if (xyz)
        hipLaunchKernelGGL((bb_backward_coords_flat_kernel<K, LB>), dim3(p.bs.n_win), block, lds, s,
                           xyz, g, gang, p.d_head_bits, p.bs.d_wstart, p.bs.d_look, p.bs.d_status,
                           p.R, p.bb, p.bs.whole_chains ? 0 : 1, p.nt_grad ? 1 : 0);
    else
        hipLaunchKernelGGL((bb_backward_recompute_kernel<K, MULTI, LB, kGradLoad>), grid, block,
                           lds, s, ang, g, gang, nullptr, nullptr, nullptr, nullptr,
                           p.bs.d_tile_res, p.d_head_bits, p.R, p.bb);
    return hipGetLastError();
}

template <int K, bool MULTI, int LB>
hipError_t mse_kml(const a2c_plan &p, const float *ang, const float *tgt, float *xyz,
                   float *loss, float *gang, hipStream_t s)
{
    hipLaunchKernelGGL((bb_backward_recompute_kernel<K, MULTI, LB, kGradMse>), dim3(p.bs.n_tiles),
                       dim3(p.bs.W * kWave), stage_bytes<K>(p.bs.W), s, ang, tgt, gang, xyz, loss,
                       p.bs.d_loss_part, p.bs.d_loss_count, p.bs.d_tile_res, p.d_head_bits, p.R,
                       p.bb);
    return hipGetLastError();
}

template <int K>
hipError_t mse_k(const a2c_plan &p, const float *ang, const float *tgt, float *xyz,
                 float *loss, float *gang, hipStream_t s)
{
    const bool small = p.bs.W * kWave <= kLbSmall;
    if (p.bs.multi_chunk)
        return small ? mse_kml<K, true, kLbSmall>(p, ang, tgt, xyz, loss, gang, s)
                     : mse_kml<K, true, kLbLarge>(p, ang, tgt, xyz, loss, gang, s);
    return small ? mse_kml<K, false, kLbSmall>(p, ang, tgt, xyz, loss, gang, s)
                 : mse_kml<K, false, kLbLarge>(p, ang, tgt, xyz, loss, gang, s);
}

template <int K>
hipError_t bwd_k(const a2c_plan &p, const float *ang, const float *xyz, const float *g,
                 float *gang, hipStream_t s)
{
    const bool small = p.bs.W * kWave <= kLbSmall;
    if (p.bs.multi_chunk)
        return small ? bwd_kml<K, true, kLbSmall>(p, ang, xyz, g, gang, s)
                     : bwd_kml<K, true, kLbLarge>(p, ang, xyz, g, gang, s);
    return small ? bwd_kml<K, false, kLbSmall>(p, ang, xyz, g, gang, s)
                 : bwd_kml<K, false, kLbLarge>(p, ang, xyz, g, gang, s);
}

}  // namespace

// The 8-residue forward with more than 10 waves stages more than 64 KiB.
void bb_allow_large_lds()
{
    static bool done = false;
    if (done) return;
    for (const void *k : {(const void *)bb_forward_flat_kernel<8, kLbSmall>,
                          (const void *)bb_forward_flat_kernel<8, kLbLarge>,
                          (const void *)bb_forward_flat_kernel<8, kLbSmall, true>,
                          (const void *)bb_forward_flat_kernel<8, kLbLarge, true>})
        (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)stage_bytes<8>(kMaxWaves));
    done = true;
}

hipError_t launch_bb_forward_scan(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s,
                                  bool quat)
{
    if (p.fs.n_win != p.fs.n_tiles || !p.fs.d_look) return hipErrorInvalidValue;
    switch (p.fs.K) {
    case 1: return fwd_k<1>(p, ang, xyz, s, quat);
    case 2: return fwd_k<2>(p, ang, xyz, s, quat);
    case 4: return fwd_k<4>(p, ang, xyz, s, quat);
    case 8: return fwd_k<8>(p, ang, xyz, s, quat);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bb_backward_scan(const a2c_plan &p, const float *ang, const float *xyz,
                                   const float *g, float *gang, hipStream_t s)
{
    switch (p.bs.K) {
    case 1: return bwd_k<1>(p, ang, xyz, g, gang, s);
    case 2: return bwd_k<2>(p, ang, xyz, g, gang, s);
    case 4: return bwd_k<4>(p, ang, xyz, g, gang, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bb_mse_step(const a2c_plan &p, const float *ang, const float *tgt, float *xyz,
                              float *loss, float *gang, hipStream_t s)
{
    switch (p.bs.K) {
    case 1: return mse_k<1>(p, ang, tgt, xyz, loss, gang, s);
    case 2: return mse_k<2>(p, ang, tgt, xyz, loss, gang, s);
    case 4: return mse_k<4>(p, ang, tgt, xyz, loss, gang, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bb_forward_plain(const a2c_plan &p, const float *ang, float *xyz, float *ws,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(bb_forward_plain_kernel, dim3(p.n_chains), dim3(64), 0, s, ang, xyz, ws,
                       p.d_res_off, p.R, p.bb);
    return hipGetLastError();
}

hipError_t launch_bb_backward_plain(const a2c_plan &p, const float *ang, const float *g,
                                    float *gang, const float *ws, hipStream_t s)
{
    const int64_t max_atoms = 3 * (int64_t)p.max_len;
    const unsigned gy = (unsigned)((max_atoms + kPlainBlock - 1) / kPlainBlock);
    if (gy == 0) return hipSuccess;
    hipLaunchKernelGGL(bb_backward_plain_kernel, dim3(p.n_chains, gy), dim3(kPlainBlock), 0, s,
                       ang, g, gang, ws, p.d_res_off, p.R, p.bb);
    return hipGetLastError();
}

}  // namespace a2c
