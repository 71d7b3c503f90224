// Full-atom model ("Full-atom model" section of the paper) on gfx950.
//
// The spine N -> CA -> C of every residue is the backbone chain (same three
// transforms, same segmented affine scan); each residue then hangs its side
// chain off the CA frame through a fixed rotation R' and a chain of up to
// four side frames M_f = M_parent R(chi_f, theta_f, d_f), and places every
// atom as r = M_frame r°.  One lane owns K consecutive residues:
//   forward : lane aggregate of the 3K spine transforms -> block prefix scan
//             -> the lane re-walks its residues from its prefix frame,
//             building spine and side frames and emitting atoms;
//   adjoint : the same walk yields frame origins and axes; per residue the
//             side-frame subtree wrenches give the chi gradients (side frames
//             form a chain, so a suffix over frames), the residue's N, CA
//             (+ side chain) and C (+ O) group wrenches feed a block reverse
//             scan over residues, and u . (S_m - o x S_g) gives phi, psi,
//             omega -- Eq. FAMBackward summed over subtrees in O(N).
// In the adjoint the atom positions either come from the forward's output
// (axes from bond vectors) or are recomputed from the angles.
#include <cmath>
#include <cstring>
#include <string>

#include "scan.h"

namespace a2c {

// ------------------------------------------------------------------ host

namespace {

struct V3 {
    double x, y, z;
};
V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double norm(V3 a) { return std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }

// Natural extension reference frame placement (Parsons et al., J. Comput.
// Chem. 26, 2005): the point d with |d - c| = bond, angle(b, c, d) = angle
// and torsion(a, b, c, d) = torsion.
V3 nerf(V3 a, V3 b, V3 c, double bond, double angle, double torsion)
{
    V3 bc = sub(c, b);
    bc = scale(bc, 1.0 / norm(bc));
    V3 n = cross(sub(b, a), bc);
    n = scale(n, 1.0 / norm(n));
    const V3 m = cross(n, bc);
    const double dx = -bond * std::cos(angle);
    const double dy = bond * std::sin(angle) * std::cos(torsion);
    const double dz = bond * std::sin(angle) * std::sin(torsion);
    return add(c, add(scale(bc, dx), add(scale(m, dy), scale(n, dz))));
}

a2c_status bad_table(int t, const std::string &msg)
{
    set_error("residue table, type " + std::to_string(t) + ": " + msg);
    return A2C_ERR_INVALID_ARG;
}

}  // namespace

// Validate a residue table and convert it to float32 constants (r° of every
// atom in its frame, side-frame transforms).  spine_d: bond lengths of the
// spine frames N, CA, C (their predecessor distances).  Host only.
a2c_status convert_residue_table(const a2c_residue_table *table, const double spine_d[3],
                                 FATable &T)
{
    const double pi = 3.14159265358979323846, d2r = pi / 180.0;
    std::memset(&T, 0, sizeof(T));
    for (int t = 0; t < A2C_NUM_RESIDUE_TYPES; ++t) {
        const a2c_residue_def &rd = table->residues[t];
        FAType &ft = T.t[t];
        if (rd.n_atoms < 3 || rd.n_atoms > A2C_MAX_RESIDUE_ATOMS)
            return bad_table(t, "n_atoms must be 3..14");
        if (rd.n_side_frames < 0 || rd.n_side_frames > A2C_MAX_SIDE_FRAMES)
            return bad_table(t, "n_side_frames must be 0..4");
        ft.n_atoms = rd.n_atoms;
        ft.n_side = rd.n_side_frames;
        double fd[7] = {spine_d[0], spine_d[1], spine_d[2], 0, 0, 0, 0};
        for (int f = 0; f < rd.n_side_frames; ++f) {
            const a2c_side_frame &sf = rd.frames[f];
            if (sf.parent != (f == 0 ? 1 : 3 + f - 1))
                return bad_table(t, "side frame " + std::to_string(f) +
                                        " must hang off CA (frame 0) or the previous side frame");
            if (sf.chi != 0 && sf.chi != f + 1)
                return bad_table(t, "side frame " + std::to_string(f) + " must use chi" +
                                        std::to_string(f + 1) + " or a fixed torsion");
            if (f > 0 && sf.pre_rotation_deg != 0.0)
                return bad_table(t, "only side frame 0 may have a pre-rotation");
            if (!(std::isfinite(sf.bond) && sf.bond > 0) ||
                !(std::isfinite(sf.bond_angle_deg) && sf.bond_angle_deg > 0 &&
                  sf.bond_angle_deg < 180))
                return bad_table(t, "side frame geometry out of range");
            ft.side_chi[f] = sf.chi ? 1 : 0;
            unit_pair(pi - sf.bond_angle_deg * d2r, ft.ct[f], ft.st[f]);
            ft.d[f] = (float)sf.bond;
            ft.inv_d[f] = (float)(1.0 / sf.bond);
            fd[3 + f] = sf.bond;
            if (f == 0) unit_pair(sf.pre_rotation_deg * d2r, ft.pre_c, ft.pre_s);
        }
        const int nframes = 3 + rd.n_side_frames;
        for (int k = 0; k < 7; ++k) ft.origin_slot[k] = -1;
        V3 local[A2C_MAX_RESIDUE_ATOMS];
        for (int a = 0; a < rd.n_atoms; ++a) {
            const a2c_atom_def &ad = rd.atoms[a];
            if (ad.frame < 0 || ad.frame >= nframes) return bad_table(t, "atom frame out of range");
            if (a < 3 && !(ad.frame == a && ad.kind == A2C_ATOM_ORIGIN))
                return bad_table(t, "atoms 0, 1, 2 must be N, CA, C at the spine frame origins");
            if (ad.kind == A2C_ATOM_ORIGIN) {
                if (ft.origin_slot[ad.frame] >= 0) return bad_table(t, "two atoms at one frame origin");
                ft.origin_slot[ad.frame] = a;
                local[a] = {0, 0, 0};
            } else if (ad.kind == A2C_ATOM_AZIMUTH) {
                const double ang = ad.angle_deg * d2r, z = ad.torsion_deg * d2r;
                local[a] = {-ad.bond * std::cos(ang), ad.bond * std::sin(ang) * std::sin(z),
                            -ad.bond * std::sin(ang) * std::cos(z)};
            } else if (ad.kind == A2C_ATOM_ZMATRIX) {
                V3 r[3];
                for (int q = 0; q < 3; ++q) {
                    const int i = ad.ref[q];
                    if (i == -1) r[q] = {-fd[ad.frame], 0, 0};
                    else if (i >= 0 && i < a && rd.atoms[i].frame == ad.frame) r[q] = local[i];
                    else return bad_table(t, "z-matrix reference must be an earlier atom of the "
                                             "same frame or -1");
                }
                local[a] = nerf(r[0], r[1], r[2], ad.bond, ad.angle_deg * d2r, ad.torsion_deg * d2r);
            } else {
                return bad_table(t, "unknown atom kind");
            }
            if (!std::isfinite(local[a].x) || !std::isfinite(local[a].y) || !std::isfinite(local[a].z))
                return bad_table(t, "atom position not finite");
        }
        for (int k = 0; k < nframes; ++k)
            if (ft.origin_slot[k] < 0) return bad_table(t, "every frame needs an atom at its origin");
        int n = 0;
        for (int k = 0; k < 7; ++k) {
            ft.fbegin[k] = n;
            for (int a = 0; a < rd.n_atoms; ++a)
                if (rd.atoms[a].frame == k) {
                    ft.slot[n] = a;
                    ft.rx[n] = (float)local[a].x;
                    ft.ry[n] = (float)local[a].y;
                    ft.rz[n] = (float)local[a].z;
                    ++n;
                }
            ft.fcount[k] = n - ft.fbegin[k];
            T.max_count[k] = std::max(T.max_count[k], ft.fcount[k]);
        }
        T.max_side = std::max(T.max_side, ft.n_side);
    }
    return A2C_OK;
}

a2c_status build_fullatom_tables(a2c_plan *p, const a2c_residue_table *table)
{
    FATable &T = p->fa_host;
    const double spine_d[3] = {p->bb.d[0], p->bb.d[1], p->bb.d[2]};
    const a2c_status st = convert_residue_table(table, spine_d, T);
    if (st != A2C_OK) return st;
    // atom offsets
    p->res_atom_off.assign((size_t)p->R + 1, 0);
    for (int64_t r = 0; r < p->R; ++r)
        p->res_atom_off[r + 1] = p->res_atom_off[r] + T.t[p->seq[r]].n_atoms;
    p->A = p->res_atom_off[p->R];
    p->chain_atom_off.resize(p->n_chains + 1);
    for (int32_t c = 0; c <= p->n_chains; ++c)
        p->chain_atom_off[c] = p->res_atom_off[p->res_off[c]];
    return A2C_OK;
}

}  // namespace a2c

extern "C" a2c_status a2c_residue_table_info(const a2c_residue_table *table, int32_t *n_atoms,
                                            float *local_xyz)
{
    using namespace a2c;
    if (!table) {
        set_error("table is NULL");
        return A2C_ERR_INVALID_ARG;
    }
    // default backbone bond lengths for the spine predecessors
    const double spine_d[3] = {1.329, 1.458, 1.525};
    FATable T;
    const a2c_status st = convert_residue_table(table, spine_d, T);
    if (st != A2C_OK) return st;
    for (int t = 0; t < A2C_NUM_RESIDUE_TYPES; ++t) {
        const FAType &ft = T.t[t];
        if (n_atoms) n_atoms[t] = ft.n_atoms;
        if (local_xyz)
            for (int q = 0; q < ft.n_atoms; ++q) {
                float *o = local_xyz + 3 * (A2C_MAX_RESIDUE_ATOMS * t + ft.slot[q]);
                o[0] = ft.rx[q]; o[1] = ft.ry[q]; o[2] = ft.rz[q];
            }
    }
    return A2C_OK;
}

namespace a2c {

// ---------------------------------------------------------------- device

namespace {

__device__ __forceinline__ void load_table(FATable &tab, const FATable *__restrict__ g)
{
    const int32_t *src = reinterpret_cast<const int32_t *>(g);
    int32_t *dst = reinterpret_cast<int32_t *>(&tab);
    constexpr int n = sizeof(FATable) / sizeof(int32_t);
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// M <- M Rx(b): the fixed pre-rotation of side frame 0
__device__ __forceinline__ void aff_rot_x(Aff &m, float c, float s)
{
    const float a0 = c * m.r01 + s * m.r02, a1 = c * m.r11 + s * m.r12, a2 = c * m.r21 + s * m.r22;
    const float b0 = c * m.r02 - s * m.r01, b1 = c * m.r12 - s * m.r11, b2 = c * m.r22 - s * m.r21;
    m.r01 = a0; m.r11 = a1; m.r21 = a2;
    m.r02 = b0; m.r12 = b1; m.r22 = b2;
}

// Emit the atoms of frame k of type t placed by F.
__device__ __forceinline__ void emit_frame(const FATable &tab, const FAType &ft, int k,
                                           const Aff &F, float *__restrict__ xyz, int64_t A,
                                           int64_t aoff)
{
    for (int i = 0; i < tab.max_count[k]; ++i) {
        if (i < ft.fcount[k]) {
            const int q = ft.fbegin[k] + i;
            float x, y, z;
            aff_point(F, ft.rx[q], ft.ry[q], ft.rz[q], x, y, z);
            const int64_t a = aoff + ft.slot[q];
            xyz[a] = x;
            xyz[A + a] = y;
            xyz[2 * A + a] = z;
        }
    }
}

// Wrench of the atoms of frame k placed by F, with upstream gradients g.
__device__ __forceinline__ void frame_wrench(const FATable &tab, const FAType &ft, int k,
                                             const Aff &F, const float *__restrict__ g, int64_t A,
                                             int64_t aoff, Wrench &w)
{
    for (int i = 0; i < tab.max_count[k]; ++i) {
        if (i < ft.fcount[k]) {
            const int q = ft.fbegin[k] + i;
            float x, y, z;
            aff_point(F, ft.rx[q], ft.ry[q], ft.rz[q], x, y, z);
            const int64_t a = aoff + ft.slot[q];
            wrench_add_point(w, x, y, z, g[a], g[A + a], g[2 * A + a]);
        }
    }
}

// Wrench of the atoms of frame k read from the forward's coordinates.
__device__ __forceinline__ void frame_wrench_xyz(const FATable &tab, const FAType &ft, int k,
                                                 const float *__restrict__ xyz,
                                                 const float *__restrict__ g, int64_t A,
                                                 int64_t aoff, Wrench &w)
{
    for (int i = 0; i < tab.max_count[k]; ++i) {
        if (i < ft.fcount[k]) {
            const int64_t a = aoff + ft.slot[ft.fbegin[k] + i];
            wrench_add_point(w, xyz[a], xyz[A + a], xyz[2 * A + a], g[a], g[A + a], g[2 * A + a]);
        }
    }
}

struct ResidueIn {
    float co, so, cp, sp, cs, ss;  // cos/sin of omega, phi, psi
};

// Lane-serial spine aggregate of K residues; returns whether a chain starts
// in the lane.  Keeps the spine cos/sin per residue for the re-walk.
template <int K>
__device__ __forceinline__ Aff fa_lane_aggregate(const float *__restrict__ ang, int64_t R,
                                                 int64_t rs, int cnt, uint32_t hm,
                                                 const BBParams &P, ResidueIn (&in)[K],
                                                 int &first_head)
{
    Aff m = aff_identity();
    first_head = K;
    float phi[K], psi[K], om[K];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        phi[j] = j < cnt ? ang[rs + j] : 0.f;
        psi[j] = j < cnt ? ang[R + rs + j] : 0.f;
        om[j] = j < cnt ? ang[2 * R + rs + j] : 0.f;
        ok = ok && sincos_fast_ok(om[j]) && sincos_fast_ok(phi[j]) && sincos_fast_ok(psi[j]);
    }
    if (__all(ok)) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            sincos_fast(phi[j], in[j].sp, in[j].cp);
            sincos_fast(psi[j], in[j].ss, in[j].cs);
            sincos_fast(om[j], in[j].so, in[j].co);
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            sincosf(phi[j], &in[j].sp, &in[j].cp);
            sincosf(psi[j], &in[j].ss, &in[j].cs);
            sincosf(om[j], &in[j].so, &in[j].co);
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < cnt) {
            if ((hm >> j) & 1u) {
                m = aff_identity();
                if (first_head == K) first_head = j;
            }
            aff_apply_transform(m, P.ct[0], P.st[0], P.d[0], in[j].co, in[j].so);
            aff_apply_transform(m, P.ct[1], P.st[1], P.d[1], in[j].cp, in[j].sp);
            aff_apply_transform(m, P.ct[2], P.st[2], P.d[2], in[j].cs, in[j].ss);
        }
    }
    aff_orthonormalise(m);
    return m;
}

__device__ __forceinline__ void side_step(Aff &sf, const FAType &ft, int f, float chi)
{
    float c = 1.f, s = 0.f;
    if (ft.side_chi[f]) {
        if (__all(sincos_fast_ok(chi))) sincos_fast(chi, s, c);
        else sincosf(chi, &s, &c);
    }
    aff_apply_transform(sf, ft.ct[f], ft.st[f], ft.d[f], c, s);
}

template <int K>
__global__ __launch_bounds__(1024) void fa_forward_kernel(
    const float *__restrict__ ang, float *__restrict__ xyz, const int32_t *__restrict__ tile_res,
    const uint32_t *__restrict__ head_bits, const int32_t *__restrict__ res_aoff,
    const uint8_t *__restrict__ seq, const FATable *__restrict__ gtab, int64_t R, int64_t A,
    BBParams P)
{
    __shared__ FATable tab;
    __shared__ FwdShared sh;
    load_table(tab, gtab);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t ts = tile_res[blockIdx.x], te = tile_res[blockIdx.x + 1];
    const int64_t rs = ts + (int64_t)tid * K;
    const int cnt = (int)max((int64_t)0, min((int64_t)K, te - rs));
    const bool wave_active = ts + (int64_t)wave * kWave * K < te;
    uint32_t hm = 0;
    ResidueIn in[K];
    int first_head = K;
    Aff m = aff_identity();
    if (wave_active) {
        if (cnt > 0) hm = head_mask<K>(head_bits, rs);
        m = fa_lane_aggregate<K>(ang, R, rs, cnt, hm, P, in, first_head);
    }
    const Aff X = block_exclusive_prefix(m, first_head < K, wave_active, sh);
    if (!wave_active) return;
    Aff cur = X;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < cnt) {
            const int64_t r = rs + j;
            const FAType &ft = tab.t[seq[r]];
            const int64_t aoff = res_aoff[r];
            if ((hm >> j) & 1u) cur = aff_identity();
            aff_apply_transform(cur, P.ct[0], P.st[0], P.d[0], in[j].co, in[j].so);
            emit_frame(tab, ft, 0, cur, xyz, A, aoff);
            aff_apply_transform(cur, P.ct[1], P.st[1], P.d[1], in[j].cp, in[j].sp);
            emit_frame(tab, ft, 1, cur, xyz, A, aoff);
            if (ft.n_side > 0) {
                Aff sf = cur;
                aff_rot_x(sf, ft.pre_c, ft.pre_s);
#pragma unroll
                for (int f = 0; f < A2C_MAX_SIDE_FRAMES; ++f) {
                    if (f < tab.max_side && f < ft.n_side) {
                        side_step(sf, ft, f, ang[(3 + f) * R + r]);
                        emit_frame(tab, ft, 3 + f, sf, xyz, A, aoff);
                    }
                }
            }
            aff_apply_transform(cur, P.ct[2], P.st[2], P.d[2], in[j].cs, in[j].ss);
            emit_frame(tab, ft, 2, cur, xyz, A, aoff);
        }
    }
}

// Per-residue group wrenches of the spine nodes and the spine frame data the
// gradient needs.
struct SpineNode {
    Wrench wN, wCA, wC;         // own-group wrench (CA includes the side chain)
    float oN[3], uN[3], oCA[3], uCA[3], oC[3], uC[3];
};

__device__ __forceinline__ void set_ou(float (&o)[3], float (&u)[3], const Aff &F)
{
    o[0] = F.t0; o[1] = F.t1; o[2] = F.t2;
    u[0] = F.r00; u[1] = F.r10; u[2] = F.r20;
}

__device__ __forceinline__ void set_ou_pts(float (&o)[3], float (&u)[3], float ox, float oy,
                                           float oz, float px, float py, float pz, float inv_d)
{
    o[0] = ox; o[1] = oy; o[2] = oz;
    u[0] = (ox - px) * inv_d; u[1] = (oy - py) * inv_d; u[2] = (oz - pz) * inv_d;
}

template <int K>
__device__ __forceinline__ void fa_store_grads(float *__restrict__ gang, int64_t R, int64_t r,
                                               const SpineNode &sn, const Wrench &S_after,
                                               const float (&gchi)[4], Wrench &S_out)
{
    Wrench S = S_after;
    wrench_add(S, sn.wC);
    gang[R + r] = wrench_torque(S, sn.oC[0], sn.oC[1], sn.oC[2], sn.uC[0], sn.uC[1], sn.uC[2]);
    wrench_add(S, sn.wCA);
    gang[r] = wrench_torque(S, sn.oCA[0], sn.oCA[1], sn.oCA[2], sn.uCA[0], sn.uCA[1], sn.uCA[2]);
    wrench_add(S, sn.wN);
    gang[2 * R + r] = wrench_torque(S, sn.oN[0], sn.oN[1], sn.oN[2], sn.uN[0], sn.uN[1], sn.uN[2]);
#pragma unroll
    for (int f = 0; f < 4; ++f) gang[(3 + f) * R + r] = gchi[f];
    S_out = S;
}

// Backward: the side chains' subtree sums give the chi gradients, the spine
// groups feed a reverse scan over residues.  RECOMPUTE: frames from the
// angles; otherwise positions and axes from the forward's coordinates.
template <int K, bool RECOMPUTE>
__global__ __launch_bounds__(1024) void fa_backward_kernel(
    const float *__restrict__ ang, const float *__restrict__ xyz, const float *__restrict__ g,
    float *__restrict__ gang, const int32_t *__restrict__ tile_res,
    const uint32_t *__restrict__ head_bits, const int32_t *__restrict__ res_aoff,
    const uint8_t *__restrict__ seq, const FATable *__restrict__ gtab, int64_t R, int64_t A,
    BBParams P)
{
    __shared__ FATable tab;
    __shared__ FwdShared shf;
    __shared__ BwdShared shb;
    load_table(tab, gtab);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nw = blockDim.x >> 6;
    const int64_t ts = tile_res[blockIdx.x], te = tile_res[blockIdx.x + 1];
    const int64_t rs = ts + (int64_t)tid * K;
    const int cnt = (int)max((int64_t)0, min((int64_t)K, te - rs));
    const bool wave_active = ts + (int64_t)wave * kWave * K < te;
    const int nact = (int)min((int64_t)nw, (te - ts + kWave * K - 1) / (kWave * K));
    uint32_t hm = 0, lm = 0;
    if (wave_active && cnt > 0) {
        hm = head_mask<K>(head_bits, rs);
        lm = head_mask<K>(head_bits, rs + 1);
    }
    Aff X = aff_identity();
    ResidueIn in[K];
    if (RECOMPUTE) {
        int first_head = K;
        Aff m = aff_identity();
        if (wave_active) m = fa_lane_aggregate<K>(ang, R, rs, cnt, hm, P, in, first_head);
        X = block_exclusive_prefix(m, first_head < K, wave_active, shf);
    }
    SpineNode sn[K];
    float gchi[K][4];
    Wrench agg = wrench_zero();
    bool f_end = false;
    if (wave_active) {
        Aff cur = X;
        // position of the C atom before the lane (coordinate mode)
        float pcx = 0.f, pcy = 0.f, pcz = 0.f;
        if (!RECOMPUTE && cnt > 0 && !(hm & 1u)) {
            const int64_t ac = res_aoff[rs - 1] + 2;
            pcx = xyz[ac]; pcy = xyz[A + ac]; pcz = xyz[2 * A + ac];
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            gchi[j][0] = gchi[j][1] = gchi[j][2] = gchi[j][3] = 0.f;
            sn[j].wN = sn[j].wCA = sn[j].wC = wrench_zero();
            if (j < cnt) {
                const int64_t r = rs + j;
                const FAType &ft = tab.t[seq[r]];
                const int64_t aoff = res_aoff[r];
                const bool head = (hm >> j) & 1u;
                // side-chain frames: origin/axis per frame and own wrenches
                Wrench ws[A2C_MAX_SIDE_FRAMES];
                float so[A2C_MAX_SIDE_FRAMES][3], su[A2C_MAX_SIDE_FRAMES][3];
                if (RECOMPUTE) {
                    if (head) cur = aff_identity();
                    aff_apply_transform(cur, P.ct[0], P.st[0], P.d[0], in[j].co, in[j].so);
                    set_ou(sn[j].oN, sn[j].uN, cur);
                    frame_wrench(tab, ft, 0, cur, g, A, aoff, sn[j].wN);
                    aff_apply_transform(cur, P.ct[1], P.st[1], P.d[1], in[j].cp, in[j].sp);
                    set_ou(sn[j].oCA, sn[j].uCA, cur);
                    frame_wrench(tab, ft, 1, cur, g, A, aoff, sn[j].wCA);
                    Aff sf = cur;
                    aff_rot_x(sf, ft.pre_c, ft.pre_s);
#pragma unroll
                    for (int f = 0; f < A2C_MAX_SIDE_FRAMES; ++f) {
                        ws[f] = wrench_zero();
                        if (f < tab.max_side && f < ft.n_side) {
                            side_step(sf, ft, f, ang[(3 + f) * R + r]);
                            so[f][0] = sf.t0; so[f][1] = sf.t1; so[f][2] = sf.t2;
                            su[f][0] = sf.r00; su[f][1] = sf.r10; su[f][2] = sf.r20;
                            frame_wrench(tab, ft, 3 + f, sf, g, A, aoff, ws[f]);
                        }
                    }
                    aff_apply_transform(cur, P.ct[2], P.st[2], P.d[2], in[j].cs, in[j].ss);
                    set_ou(sn[j].oC, sn[j].uC, cur);
                    frame_wrench(tab, ft, 2, cur, g, A, aoff, sn[j].wC);
                } else {
                    const float nx = xyz[aoff], ny = xyz[A + aoff], nz = xyz[2 * A + aoff];
                    const float cax = xyz[aoff + 1], cay = xyz[A + aoff + 1], caz = xyz[2 * A + aoff + 1];
                    const float cx = xyz[aoff + 2], cy = xyz[A + aoff + 2], cz = xyz[2 * A + aoff + 2];
                    if (head) { pcx = 0.f; pcy = 0.f; pcz = 0.f; }
                    set_ou_pts(sn[j].oN, sn[j].uN, nx, ny, nz, pcx, pcy, pcz, P.inv_d[0]);
                    set_ou_pts(sn[j].oCA, sn[j].uCA, cax, cay, caz, nx, ny, nz, P.inv_d[1]);
                    set_ou_pts(sn[j].oC, sn[j].uC, cx, cy, cz, cax, cay, caz, P.inv_d[2]);
                    frame_wrench_xyz(tab, ft, 0, xyz, g, A, aoff, sn[j].wN);
                    frame_wrench_xyz(tab, ft, 1, xyz, g, A, aoff, sn[j].wCA);
                    frame_wrench_xyz(tab, ft, 2, xyz, g, A, aoff, sn[j].wC);
                    float ppx = cax, ppy = cay, ppz = caz;
#pragma unroll
                    for (int f = 0; f < A2C_MAX_SIDE_FRAMES; ++f) {
                        ws[f] = wrench_zero();
                        if (f < tab.max_side && f < ft.n_side) {
                            const int64_t ao = aoff + ft.origin_slot[3 + f];
                            const float ox = xyz[ao], oy = xyz[A + ao], oz = xyz[2 * A + ao];
                            so[f][0] = ox; so[f][1] = oy; so[f][2] = oz;
                            su[f][0] = (ox - ppx) * ft.inv_d[f];
                            su[f][1] = (oy - ppy) * ft.inv_d[f];
                            su[f][2] = (oz - ppz) * ft.inv_d[f];
                            ppx = ox; ppy = oy; ppz = oz;
                            frame_wrench_xyz(tab, ft, 3 + f, xyz, g, A, aoff, ws[f]);
                        }
                    }
                    pcx = cx; pcy = cy; pcz = cz;
                }
                // chi gradients: side frames form a chain, subtree = suffix
                Wrench Ss = wrench_zero();
#pragma unroll
                for (int f = A2C_MAX_SIDE_FRAMES - 1; f >= 0; --f) {
                    if (f < tab.max_side && f < ft.n_side) {
                        wrench_add(Ss, ws[f]);
                        if (ft.side_chi[f])
                            gchi[j][f] = wrench_torque(Ss, so[f][0], so[f][1], so[f][2], su[f][0],
                                                       su[f][1], su[f][2]);
                    }
                }
                wrench_add(sn[j].wCA, Ss);
                if (!f_end) {
                    wrench_add(agg, sn[j].wN);
                    wrench_add(agg, sn[j].wCA);
                    wrench_add(agg, sn[j].wC);
                }
                if ((lm >> j) & 1u) f_end = true;
            }
        }
    }
    Wrench S = block_exclusive_suffix(agg, f_end, wave_active, nact, shb);
    if (!wave_active) return;
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
        if (j < cnt) {
            if ((lm >> j) & 1u) S = wrench_zero();
            fa_store_grads<K>(gang, R, rs + j, sn[j], S, gchi[j], S);
        }
    }
}

template <int K>
hipError_t fa_fwd_k(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s)
{
    hipLaunchKernelGGL((fa_forward_kernel<K>), dim3(p.n_tiles), dim3(p.W * kWave), 0, s, ang, xyz,
                       p.d_tile_res, p.d_head_bits, p.d_res_atom_off, p.d_seq, p.d_fa, p.R, p.A,
                       p.bb);
    return hipGetLastError();
}

template <int K>
hipError_t fa_bwd_k(const a2c_plan &p, const float *ang, const float *xyz, const float *g,
                    float *gang, hipStream_t s)
{
    const dim3 grid(p.n_tiles), block(p.W * kWave);
    if (xyz)
        hipLaunchKernelGGL((fa_backward_kernel<K, false>), grid, block, 0, s, ang, xyz, g, gang,
                           p.d_tile_res, p.d_head_bits, p.d_res_atom_off, p.d_seq, p.d_fa, p.R,
                           p.A, p.bb);
    else
        hipLaunchKernelGGL((fa_backward_kernel<K, true>), grid, block, 0, s, ang, xyz, g, gang,
                           p.d_tile_res, p.d_head_bits, p.d_res_atom_off, p.d_seq, p.d_fa, p.R,
                           p.A, p.bb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fa_forward_scan(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s)
{
    switch (p.K) {
    case 1: return fa_fwd_k<1>(p, ang, xyz, s);
    case 2: return fa_fwd_k<2>(p, ang, xyz, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fa_backward_scan(const a2c_plan &p, const float *ang, const float *xyz,
                                   const float *g, float *gang, hipStream_t s)
{
    switch (p.K) {
    case 1: return fa_bwd_k<1>(p, ang, xyz, g, gang, s);
    case 2: return fa_bwd_k<2>(p, ang, xyz, g, gang, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace a2c
