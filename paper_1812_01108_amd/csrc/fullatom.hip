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
        // each frame's list starts with its origin atom (the kernels place it
        // at the frame's translation without a product)
        int n = 0;
        for (int k = 0; k < 7; ++k) {
            ft.fbegin[k] = n;
            for (int pass = 0; pass < 2; ++pass)
                for (int a = 0; a < rd.n_atoms; ++a)
                    if (rd.atoms[a].frame == k && (a == ft.origin_slot[k]) == (pass == 0)) {
                        ft.atom[n].slot = a;
                        ft.atom[n].x = (float)local[a].x;
                        ft.atom[n].y = (float)local[a].y;
                        ft.atom[n].z = (float)local[a].z;
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
                float *o = local_xyz + 3 * (A2C_MAX_RESIDUE_ATOMS * t + ft.atom[q].slot);
                o[0] = ft.atom[q].x; o[1] = ft.atom[q].y; o[2] = ft.atom[q].z;
            }
    }
    return A2C_OK;
}

namespace a2c {

// ---------------------------------------------------------------- device

namespace {

// The constant table into LDS: 16-byte pieces, every load of a thread issued
// before its first store (one memory latency also for a one-wave group).
__device__ __forceinline__ void load_table(FATable &tab, const FATable *__restrict__ g)
{
    static_assert(sizeof(FATable) % 16 == 0, "FATable copies in 16-byte pieces");
    constexpr int n = sizeof(FATable) / 16;
    constexpr int per = (n + kWave - 1) / kWave;
    const int4 *src = reinterpret_cast<const int4 *>(g);
    int4 *dst = reinterpret_cast<int4 *>(&tab);
    int4 v[per];
    // indices past the end are clamped: those threads rewrite the last piece
    // with the value it already gets (no branches, so the loads batch)
#pragma unroll
    for (int u = 0; u < per; ++u) v[u] = src[min((int)(threadIdx.x + u * blockDim.x), n - 1)];
#pragma unroll
    for (int u = 0; u < per; ++u) dst[min((int)(threadIdx.x + u * blockDim.x), n - 1)] = v[u];
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

// A wave's atom run [A0, A0 + n): plane p of atom e (relative to A0) lives
// at st[p * ns + e] -- in the per-wave LDS stage (ns = the stage's floats per
// plane), or, for schedules whose stage does not fit the LDS, in global
// memory itself (st = array + A0, ns = A): the same indexing serves both.
struct Stage {
    float *st;
    int64_t ns;
};

// Coalesced copy between a global run (3 planes, plane stride A) and the
// wave's staging buffer, eight rows of 64 atoms at a time: all loads of a
// batch are issued before the first store (indices past the run are clamped
// to its last atom), so a batch costs one memory latency, not eight.
constexpr int kStageBatch = 8;

__device__ __forceinline__ void run_to_lds(const Stage &sg, int plane0, const float *__restrict__ src,
                                           int64_t A, int64_t A0, int n)
{
    const int lane = lane_id();
    const float *s0 = src + A0, *s1 = src + A + A0, *s2 = src + 2 * A + A0;
    float *d0 = sg.st + plane0 * sg.ns, *d1 = d0 + sg.ns, *d2 = d1 + sg.ns;
    for (int base = 0; base < n; base += kStageBatch * kWave) {
        float v0[kStageBatch], v1[kStageBatch], v2[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int e = min(base + lane + u * kWave, n - 1);
            v0[u] = s0[e];
            v1[u] = s1[e];
            v2[u] = s2[e];
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int e = base + lane + u * kWave;
            if (e < n) {
                d0[e] = v0[u];
                d1[e] = v1[u];
                d2[e] = v2[u];
            }
        }
    }
}

__device__ __forceinline__ void lds_to_run(const Stage &sg, float *__restrict__ dst, int64_t A,
                                           int64_t A0, int n)
{
    const int lane = lane_id();
    float *o0 = dst + A0, *o1 = dst + A + A0, *o2 = dst + 2 * A + A0;
    const float *s0 = sg.st, *s1 = s0 + sg.ns, *s2 = s1 + sg.ns;
    for (int base = 0; base < n; base += kStageBatch * kWave) {
        float v0[kStageBatch], v1[kStageBatch], v2[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int e = min(base + lane + u * kWave, n - 1);
            v0[u] = s0[e];
            v1[u] = s1[e];
            v2[u] = s2[e];
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int e = base + lane + u * kWave;
            if (e < n) {
                o0[e] = v0[u];
                o1[e] = v1[u];
                o2[e] = v2[u];
            }
        }
    }
}

// Emit the atoms of frame k of type t placed by F into the staging buffer.
// The frame's first atom is its origin: F's translation, no product.  Frame
// k exists for the type (every existing frame holds its origin atom).
__device__ __forceinline__ void emit_frame(const FATable &tab, const FAType &ft, int k,
                                           const Aff &F, const Stage &sg, int aloc)
{
    {
        const int e = aloc + ft.atom[ft.fbegin[k]].slot;
        sg.st[e] = F.t0;
        sg.st[sg.ns + e] = F.t1;
        sg.st[2 * sg.ns + e] = F.t2;
    }
    for (int i = 1; i < tab.max_count[k]; ++i) {
        if (i < ft.fcount[k]) {
            const FAAtom at = ft.atom[ft.fbegin[k] + i];
            float x, y, z;
            aff_point(F, at.x, at.y, at.z, x, y, z);
            const int e = aloc + at.slot;
            sg.st[e] = x;
            sg.st[sg.ns + e] = y;
            sg.st[2 * sg.ns + e] = z;
        }
    }
}

// Wrench of the atoms of frame k placed by F, upstream gradients staged in
// planes 0..2 (the origin atom first, at F's translation).
__device__ __forceinline__ void frame_wrench(const FATable &tab, const FAType &ft, int k,
                                             const Aff &F, const Stage &sg, int aloc, Wrench &w)
{
    {
        const int e = aloc + ft.atom[ft.fbegin[k]].slot;
        wrench_add_point(w, F.t0, F.t1, F.t2, sg.st[e], sg.st[sg.ns + e], sg.st[2 * sg.ns + e]);
    }
    for (int i = 1; i < tab.max_count[k]; ++i) {
        if (i < ft.fcount[k]) {
            const FAAtom at = ft.atom[ft.fbegin[k] + i];
            float x, y, z;
            aff_point(F, at.x, at.y, at.z, x, y, z);
            const int e = aloc + at.slot;
            wrench_add_point(w, x, y, z, sg.st[e], sg.st[sg.ns + e], sg.st[2 * sg.ns + e]);
        }
    }
}

// The fused training step: the stage holds the target t of each atom; the
// wrench of frame k's atoms takes the loss gradient 2 (r - t), the loss
// accumulates |r - t|^2, and the staged target is replaced by r (so the
// stage ends up holding the coordinates).
__device__ __forceinline__ void atom_mse(float x, float y, float z, int e, const Stage &sg,
                                         const Stage &so, bool write, Wrench &w, float &loss)
{
    const float dx = x - sg.st[e], dy = y - sg.st[sg.ns + e], dz = z - sg.st[2 * sg.ns + e];
    loss += dx * dx + dy * dy + dz * dz;
    wrench_add_point(w, x, y, z, 2.f * dx, 2.f * dy, 2.f * dz);
    if (write) {
        so.st[e] = x;
        so.st[so.ns + e] = y;
        so.st[2 * so.ns + e] = z;
    }
}

__device__ __forceinline__ void frame_wrench_mse(const FATable &tab, const FAType &ft, int k,
                                                 const Aff &F, const Stage &sg, const Stage &so,
                                                 bool write, int aloc, Wrench &w, float &loss)
{
    atom_mse(F.t0, F.t1, F.t2, aloc + ft.atom[ft.fbegin[k]].slot, sg, so, write, w, loss);
    for (int i = 1; i < tab.max_count[k]; ++i) {
        if (i < ft.fcount[k]) {
            const FAAtom at = ft.atom[ft.fbegin[k] + i];
            float x, y, z;
            aff_point(F, at.x, at.y, at.z, x, y, z);
            atom_mse(x, y, z, aloc + at.slot, sg, so, write, w, loss);
        }
    }
}

// Wrench of the atoms of frame k with positions from sx and upstream
// gradients from sg.
__device__ __forceinline__ void frame_wrench_xyz(const FATable &tab, const FAType &ft, int k,
                                                 const Stage &sg, const Stage &sx, int aloc,
                                                 Wrench &w)
{
    for (int i = 0; i < tab.max_count[k]; ++i) {
        if (i < ft.fcount[k]) {
            const int e = aloc + ft.atom[ft.fbegin[k] + i].slot;
            wrench_add_point(w, sx.st[e], sx.st[sx.ns + e], sx.st[2 * sx.ns + e],
                             sg.st[e], sg.st[sg.ns + e], sg.st[2 * sg.ns + e]);
        }
    }
}

struct ResidueIn {
    float co, so, cp, sp, cs, ss;  // cos/sin of omega, phi, psi
};

// Spine angles (phi, psi, omega) of a lane's K residues, 0 past the chunk.
template <int K>
struct SpineAngles {
    float phi[K], psi[K], om[K];
};

template <int K>
__device__ __forceinline__ SpineAngles<K> load_spine_angles(const float *__restrict__ ang,
                                                            int64_t R, int64_t rs, int cnt)
{
    SpineAngles<K> a;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        a.phi[j] = j < cnt ? ang[rs + j] : 0.f;
        a.psi[j] = j < cnt ? ang[R + rs + j] : 0.f;
        a.om[j] = j < cnt ? ang[2 * R + rs + j] : 0.f;
    }
    return a;
}

// Lane-serial spine aggregate of K residues (reset at chain heads), with one
// polar step; keeps the spine cos/sin per residue for the re-walk.
template <int K>
__device__ __forceinline__ Aff fa_lane_aggregate(const SpineAngles<K> &a, int cnt, uint32_t hm,
                                                 const BBParams &P, ResidueIn (&in)[K],
                                                 int &first_head)
{
    Aff m = aff_identity();
    first_head = K;
    const float(&phi)[K] = a.phi;
    const float(&psi)[K] = a.psi;
    const float(&om)[K] = a.om;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < K; ++j)
        ok = ok && sincos_fast_ok(om[j]) && sincos_fast_ok(phi[j]) && sincos_fast_ok(psi[j]);
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
            sincos_accurate(phi[j], in[j].sp, in[j].cp);
            sincos_accurate(psi[j], in[j].ss, in[j].cs);
            sincos_accurate(om[j], in[j].so, in[j].co);
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

template <int K>
__device__ __forceinline__ Aff fa_lane_aggregate(const float *__restrict__ ang, int64_t R,
                                                 int64_t rs, int cnt, uint32_t hm,
                                                 const BBParams &P, ResidueIn (&in)[K],
                                                 int &first_head)
{
    return fa_lane_aggregate<K>(load_spine_angles<K>(ang, R, rs, cnt), cnt, hm, P, in,
                                first_head);
}

__device__ __forceinline__ void side_step(Aff &sf, const FAType &ft, int f, float chi)
{
    float c = 1.f, s = 0.f;
    if (ft.side_chi[f]) {
        if (__all(sincos_fast_ok(chi))) sincos_fast(chi, s, c);
        else sincos_accurate(chi, s, c);
    }
    aff_apply_transform(sf, ft.ct[f], ft.st[f], ft.d[f], c, s);
}

// Chunk c of a tile: residues [cs, ce) handled by the waves wave < nact.
struct FAChunk {
    int64_t cs, ce;
    int nact;
};

template <int K>
__device__ __forceinline__ FAChunk fa_chunk(int64_t ts, int64_t te, int c)
{
    const int nw = blockDim.x >> 6;
    const int64_t ch = (int64_t)kWave * K * nw;
    FAChunk k;
    k.cs = ts + (int64_t)c * ch;
    k.ce = min(k.cs + ch, te);
    k.nact = (int)min((int64_t)nw, (k.ce - k.cs + kWave * K - 1) / (kWave * K));
    return k;
}

template <int K>
__device__ __forceinline__ int fa_chunks(int64_t ts, int64_t te)
{
    const int64_t ch = (int64_t)kWave * K * (blockDim.x >> 6);
    return (int)((te - ts + ch - 1) / ch);
}

// Per-lane bookkeeping of one chunk.
template <int K>
struct LaneRun {
    int64_t rs, rbase, A0;
    int cnt, nres, natoms;
    bool active;
    uint32_t hm, lm;
};

template <int K>
__device__ __forceinline__ LaneRun<K> lane_run(const FAChunk &k,
                                               const uint32_t *__restrict__ head_bits,
                                               const int32_t *__restrict__ res_aoff)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    LaneRun<K> L;
    L.rbase = k.cs + (int64_t)wave * kWave * K;
    L.active = wave < k.nact;
    L.nres = L.active ? (int)min((int64_t)kWave * K, k.ce - L.rbase) : 0;
    L.rs = k.cs + (int64_t)threadIdx.x * K;
    L.cnt = (int)max((int64_t)0, min((int64_t)K, k.ce - L.rs));
    L.hm = lane_head_mask<K>(head_bits, L.rs, k.ce, L.cnt);
    L.lm = lane_head_mask<K>(head_bits, L.rs + 1, k.ce + 1, L.cnt);
    L.A0 = 0;
    L.natoms = 0;
    if (L.active) {
        L.A0 = __builtin_amdgcn_readfirstlane(res_aoff[L.rbase]);
        L.natoms = __builtin_amdgcn_readfirstlane(res_aoff[L.rbase + L.nres]) - (int)L.A0;
    }
    return L;
}

// Per-residue inputs of a lane, read right after the chunk's bookkeeping so
// that their latency overlaps the block scan instead of stalling the walk:
// residue type, first atom and (CHI) the four chi planes (read for every
// residue; a residue without chi f ignores plane f).
template <int K, bool CHI>
struct LaneRes {
    int type[K];
    int aoff[K];
    float chi[CHI ? K : 1][4];
};

template <int K, bool CHI>
__device__ __forceinline__ LaneRes<K, CHI> load_lane_res(const LaneRun<K> &L,
                                                         const uint8_t *__restrict__ seq,
                                                         const int32_t *__restrict__ res_aoff,
                                                         const float *__restrict__ ang, int64_t R)
{
    LaneRes<K, CHI> lr;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const bool v = j < L.cnt;
        const int64_t r = v ? L.rs + j : 0;
        lr.type[j] = v ? seq[r] : 0;
        lr.aoff[j] = v ? res_aoff[r] : 0;
        if (CHI) {
#pragma unroll
            for (int f = 0; f < 4; ++f) lr.chi[j][f] = v ? ang[(3 + f) * R + r] : 0.f;
        }
    }
    return lr;
}

// All atoms of one residue from the frame before it (cur, advanced to the
// residue's C frame): spine transforms omega, phi, psi, and the side chain
// branching off the CA frame, each frame's atoms written to the stage.
__device__ __forceinline__ void fa_emit_residue(const FATable &tab, const FAType &ft, Aff &cur,
                                                const ResidueIn &in, const float (&chi)[4],
                                                const BBParams &P, const Stage &sg, int aloc)
{
    aff_apply_transform(cur, P.ct[0], P.st[0], P.d[0], in.co, in.so);
    emit_frame(tab, ft, 0, cur, sg, aloc);
    aff_apply_transform(cur, P.ct[1], P.st[1], P.d[1], in.cp, in.sp);
    emit_frame(tab, ft, 1, cur, sg, aloc);
    if (ft.n_side > 0) {
        Aff sf = cur;
        aff_rot_x(sf, ft.pre_c, ft.pre_s);
#pragma unroll
        for (int f = 0; f < A2C_MAX_SIDE_FRAMES; ++f) {
            if (f < tab.max_side && f < ft.n_side) {
                side_step(sf, ft, f, chi[f]);
                emit_frame(tab, ft, 3 + f, sf, sg, aloc);
            }
        }
    }
    aff_apply_transform(cur, P.ct[2], P.st[2], P.d[2], in.cs, in.ss);
    emit_frame(tab, ft, 2, cur, sg, aloc);
}

// Forward over windows of the packed batch (window t: residues
// [wstart[t], wstart[t + 1]), at most C = 64 W K), as the backbone forward:
// the spine scan hands frames across window edges by window look-back; then
// every lane re-walks its residues from its prefix frame, building the spine
// and side frames and writing each atom into the wave's LDS stage, which is
// copied out with coalesced stores (STG; otherwise, for schedules whose
// stage does not fit the LDS, straight to global memory).
template <int K, int LB, bool STG = true>
__global__ __launch_bounds__(LB) void fa_forward_flat_kernel(
    const float *__restrict__ ang, float *__restrict__ xyz, const uint32_t *__restrict__ head_bits,
    const int32_t *__restrict__ wstart, const int32_t *__restrict__ res_aoff,
    const uint8_t *__restrict__ seq, const FATable *__restrict__ gtab,
    const int32_t *__restrict__ look_first,
    uint64_t *__restrict__ status, int64_t R, int64_t A, BBParams P, int stage_atoms)
{
    extern __shared__ float stage_mem[];
    __shared__ __align__(16) FATable tab;
    __shared__ FwdShared sh;
    __shared__ float carry_sh[12];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = blockIdx.x;
    FAChunk k;
    k.cs = wstart[t];
    k.ce = wstart[t + 1];
    k.nact = (int)((k.ce - k.cs + kWave * K - 1) / (kWave * K));
    const LaneRun<K> L = lane_run<K>(k, head_bits, res_aoff);
    uint64_t prev = 0;
    int64_t first = t;
    if (wave == 0) {
        prev = lb_load(status + t * kLbWords);
        first = look_first[t];
    }
    // the window's inputs ahead of the table copy (which ends in a barrier)
    SpineAngles<K> a{};
    if (L.active) a = load_spine_angles<K>(ang, R, L.rs, L.cnt);
    const LaneRes<K, true> lr = load_lane_res<K, true>(L, seq, res_aoff, ang, R);
    load_table(tab, gtab);
    ResidueIn in[K];
    int first_head = K;
    Aff m = aff_identity();
    if (L.active) m = fa_lane_aggregate<K>(a, L.cnt, L.hm, P, in, first_head);
    const uint64_t heads = __builtin_amdgcn_ballot_w64(first_head < K);
    const Aff X = block_prefix_windows(m, heads, k.nact, L.active, sh, carry_sh, status, t, first,
                                       prev);
    if (!L.active) return;
    const Stage sg = STG ? Stage{stage_mem + (size_t)wave * 3 * stage_atoms, stage_atoms}
                         : Stage{xyz + L.A0, A};
    Aff cur = X;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (j < L.cnt) {
            if ((L.hm >> j) & 1u) cur = aff_identity();
            fa_emit_residue(tab, tab.t[lr.type[j]], cur, in[j], lr.chi[j], P, sg,
                            lr.aoff[j] - (int)L.A0);
        }
    }
    if (STG) {
        wave_lds_sync();
        lds_to_run(sg, xyz, A, L.A0, L.natoms);
    }
}

// Torque bookkeeping of one rotation axis (a spine node or a side frame):
// the derivative of sum g.r over the atoms a rotation about the axis u
// through o moves is u . (m - o x g) = u . m - v . g with v = u x o, summed
// over the wrenches (g, m) of the atom groups it moves.  It is linear in the
// wrench, so the wrenches of the residue's groups an axis moves are summed
// and folded into c once the residue is walked, and the wrench S of
// everything after the residue enters later as c + u . S.m - v . S.g.
// 7 floats per axis.
struct NodeGrad {
    float c, u0, u1, u2, v0, v1, v2;
};

// What a residue keeps across the block scan: its three spine nodes and W,
// the residue's whole wrench (for earlier residues of the lane).
struct SpineGrad {
    NodeGrad n, ca, cc;
    Wrench W;
};

__device__ __forceinline__ NodeGrad node_at(float ox, float oy, float oz, float ux, float uy,
                                            float uz)
{
    NodeGrad g;
    g.c = 0.f;
    g.u0 = ux; g.u1 = uy; g.u2 = uz;
    // explicit FMAs: no contraction left to the compiler here
    g.v0 = fmaf(uy, oz, -(uz * oy));
    g.v1 = fmaf(uz, ox, -(ux * oz));
    g.v2 = fmaf(ux, oy, -(uy * ox));
    return g;
}

// the axis of frame F: its x axis through its origin
__device__ __forceinline__ NodeGrad node_of_frame(const Aff &F)
{
    return node_at(F.t0, F.t1, F.t2, F.r00, F.r10, F.r20);
}

__device__ __forceinline__ float node_torque(const NodeGrad &g, const Wrench &S)
{
    float t = fmaf(g.u0, S.m0, g.c);
    t = fmaf(g.u1, S.m1, t);
    t = fmaf(g.u2, S.m2, t);
    t = fmaf(-g.v0, S.g0, t);
    t = fmaf(-g.v1, S.g1, t);
    return fmaf(-g.v2, S.g2, t);
}

__device__ __forceinline__ void node_fold(NodeGrad &g, const Wrench &w) { g.c = node_torque(g, w); }

// An angle gradient: a non-temporal store when nt (large plans).
__device__ __forceinline__ void grad_store(float *p, float v, bool nt)
{
    if (nt) out_store<true>(p, v);
    else out_store<false>(p, v);
}

__device__ __forceinline__ void fa_store_grads(float *__restrict__ gang, int64_t R, int64_t r,
                                               const SpineGrad &sp, const Wrench &S_after,
                                               Wrench &S_out, bool nt)
{
    grad_store(&gang[R + r], node_torque(sp.cc, S_after), nt);
    grad_store(&gang[r], node_torque(sp.ca, S_after), nt);
    grad_store(&gang[2 * R + r], node_torque(sp.n, S_after), nt);
    Wrench S = S_after;
    wrench_add(S, sp.W);
    S_out = S;
}

// Spine aggregates for the recomputing full-atom adjoints.  Those take fixed
// windows last to first (for the wrench look-back), so they cannot wait on
// earlier windows' frames themselves: this spine-only pass over the same
// windows publishes each window's aggregate (the product of its spine
// transforms from its last chain head, or its start, to its end) as tagged
// words and waits on nothing; the adjoint then composes the aggregates of
// the windows its first chain spans, all complete by then (lb_carry_in).
template <int K, int LB>
__global__ __launch_bounds__(LB) void fa_spine_aggregate_kernel(
    const float *__restrict__ ang, const uint32_t *__restrict__ head_bits,
    const int32_t *__restrict__ wstart, uint64_t *__restrict__ status, int64_t R, BBParams P)
{
    __shared__ FwdShared sh;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = blockIdx.x;
    FAChunk k;
    k.cs = wstart[t];
    k.ce = wstart[t + 1];
    k.nact = (int)((k.ce - k.cs + kWave * K - 1) / (kWave * K));
    const bool active = wave < k.nact;
    const int64_t rs = k.cs + (int64_t)threadIdx.x * K;
    const int cnt = (int)max((int64_t)0, min((int64_t)K, k.ce - rs));
    const uint32_t hm = lane_head_mask<K>(head_bits, rs, k.ce, cnt);
    uint64_t prev = 0;
    if (wave == 0) prev = lb_load(status + t * kLbWords);
    ResidueIn in[K];
    int first_head = K;
    Aff m = aff_identity();
    if (active) m = fa_lane_aggregate<K>(load_spine_angles<K>(ang, R, rs, cnt), cnt, hm, P, in,
                                         first_head);
    const uint64_t heads = __builtin_amdgcn_ballot_w64(first_head < K);
    if (active) {
        aff_wave_scan<false>(m, heads, kWave, lane);
        if (lane == kWave - 1) {
            aff_store(sh.tot[wave], m);
            sh.tot_flag[wave] = heads != 0ull ? 1 : 0;
        }
    }
    __syncthreads();
    if (wave != 0) return;
    Aff tw = aff_identity();
    bool tf = false;
    if (lane < k.nact) {
        tw = aff_load(sh.tot[lane]);
        tf = sh.tot_flag[lane] != 0;
    }
    const uint64_t th = __builtin_amdgcn_ballot_w64(tf);
    aff_wave_scan<true>(tw, th, k.nact, lane);
    if (lane == k.nact - 1) aff_store(sh.pre[0], tw);
    wave_lds_sync();
    const uint32_t tag = (uint32_t)(__builtin_amdgcn_readfirstlane((uint32_t)(prev >> 32))) + 1u;
    if (lane < kLbWords) lb_store(status + t * kLbWords + lane, tag, sh.pre[0][lane]);
}

// Backward over windows of the packed batch, last window first (rev:
// reverse_window, so that window t runs on the XCD where the spine pass's
// window t read the same angles; in order where the windows hold whole
// chains, as the backbone adjoint): the
// side chains' subtree sums give the chi gradients, the spine groups feed a
// reverse scan over residues (window look-back for the wrench of later
// windows), and u . (S_m - o x S_g) gives phi, psi, omega.
// RECOMPUTE: frames from the angles, the frame entering the window composed
// from the aggregates fa_spine_aggregate_kernel published (status_fwd,
// windows look_fwd[t] .. t - 1); otherwise positions and axes from the
// forward's coordinates.
// GM = kGradMse (with RECOMPUTE): g points at a target t and the upstream
// gradient is 2 (r - t), formed from the recomputed positions (the fused
// training step); xyz_out (may be NULL) receives the positions, loss_out
// (may be NULL) the batch's sum of |r - t|^2 (lb_loss_commit).
// nt: the angle gradients go out with non-temporal stores (large plans).
// STG: atoms go through the per-wave LDS stage; otherwise global memory is
// addressed directly (schedules whose stage does not fit the LDS).
template <int K, bool RECOMPUTE, int LB, int GM = kGradLoad, bool STG = true>
__global__ __launch_bounds__(LB) void fa_backward_flat_kernel(
    const float *__restrict__ ang, const float *__restrict__ xyz, const float *__restrict__ g,
    float *__restrict__ gang, float *__restrict__ xyz_out, float *__restrict__ loss_out,
    const uint32_t *__restrict__ head_bits, const int32_t *__restrict__ wstart,
    const int32_t *__restrict__ res_aoff, const uint8_t *__restrict__ seq,
    const FATable *__restrict__ gtab, const uint64_t *__restrict__ status_fwd,
    const int32_t *__restrict__ look_fwd,
    const int32_t *__restrict__ look_last, uint64_t *__restrict__ status, int64_t R, int64_t A,
    BBParams P, int stage_atoms, int32_t rev, int32_t nt)
{
    static_assert(GM == kGradLoad || RECOMPUTE, "the fused step recomputes the frames");
    extern __shared__ float stage_mem[];
    __shared__ __align__(16) FATable tab;
    __shared__ FwdShared shf;
    __shared__ BwdShared shb;
    __shared__ float rcarry_sh[6];
    __shared__ float loss_tot[GM == kGradMse ? kMaxWaves : 1];
    float loss = 0.f;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = rev ? reverse_window(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    FAChunk k;
    k.cs = wstart[t];
    k.ce = wstart[t + 1];
    k.nact = (int)((k.ce - k.cs + kWave * K - 1) / (kWave * K));
    const LaneRun<K> L = lane_run<K>(k, head_bits, res_aoff);
    uint64_t prev = 0;
    int64_t last = t;
    if (wave == 0) {
        prev = lb_load(status + t * kLbWords);
        last = look_last[t];
    }
    // the window's inputs, and the upstream gradients (or targets) and
    // coordinates into the stage, ahead of the table copy (which ends in a
    // barrier) so that their latencies overlap
    SpineAngles<K> a{};
    if (RECOMPUTE && L.active) a = load_spine_angles<K>(ang, R, L.rs, L.cnt);
    const LaneRes<K, RECOMPUTE> lr = load_lane_res<K, RECOMPUTE>(L, seq, res_aoff, ang, R);
    const int planes = RECOMPUTE ? 3 : 6;
    const Stage lds{stage_mem + (size_t)wave * planes * stage_atoms, stage_atoms};
    if (STG && L.active) {
        run_to_lds(lds, 0, g, A, L.A0, L.natoms);
        if (!RECOMPUTE) run_to_lds(lds, 3, xyz, A, L.A0, L.natoms);
    }
    // the frame entering the window (wave 0; the aggregates are complete)
    __shared__ float fcarry_sh[12];
    if (RECOMPUTE && wave == 0) {
        const uint32_t tag_f =
            (uint32_t)(__builtin_amdgcn_readfirstlane((uint32_t)(lb_load(status_fwd + t * kLbWords) >> 32)));
        const int64_t f = (int64_t)__builtin_amdgcn_readfirstlane(look_fwd[t]);
        const Aff c = lb_carry_in(status_fwd, f, t, tag_f);
        if (lane == 0) aff_store(fcarry_sh, c);
    }
    load_table(tab, gtab);
    Aff X = aff_identity();
    ResidueIn in[K];
    int first_head = K;
    if (RECOMPUTE) {
        Aff m = aff_identity();
        if (L.active) m = fa_lane_aggregate<K>(a, L.cnt, L.hm, P, in, first_head);
        Aff fcarry = aff_load(fcarry_sh);
        X = block_exclusive_prefix<true>(m, first_head < K, k.nact, shf, fcarry);
    }
    // the C atom before the lane's first residue (coordinate mode): in
    // the staged run for lanes > 0, from global memory for lane 0
    float pcx = 0.f, pcy = 0.f, pcz = 0.f;
    if (!RECOMPUTE && lane == 0 && L.cnt > 0 && !(L.hm & 1u)) {
        const int64_t ac = res_aoff[L.rs - 1] + 2;
        pcx = xyz[ac]; pcy = xyz[A + ac]; pcz = xyz[2 * A + ac];
    }
    SpineGrad sp[K];
    Wrench agg = wrench_zero();
    bool f_end = false;
    // upstream gradient (or target) sg, coordinates sx, positions out sout
    const Stage sg = STG ? lds : Stage{const_cast<float *>(g) + L.A0, A};
    const Stage sx = STG ? Stage{lds.st + 3 * lds.ns, lds.ns}
                         : Stage{const_cast<float *>(xyz) + L.A0, A};
    const Stage sout = STG ? sg : Stage{xyz_out + L.A0, A};
    const bool write_so = STG || (GM == kGradMse && xyz_out != nullptr);
    if (L.active) {
        wave_lds_sync();
        // first atom of the residue before the lane: the previous lane's last
        const int prev_aoff = __builtin_amdgcn_mov_dpp(lr.aoff[K - 1], kDppWaveShr1, 0xf, 0xf, true);
        if (!RECOMPUTE && lane > 0 && L.cnt > 0 && !(L.hm & 1u)) {
            const int e = prev_aoff + 2 - (int)L.A0;
            pcx = sx.st[e]; pcy = sx.st[sx.ns + e]; pcz = sx.st[2 * sx.ns + e];
        }
        Aff cur = X;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (j < L.cnt) {
                const FAType &ft = tab.t[lr.type[j]];
                const int aloc = lr.aoff[j] - (int)L.A0;
                const bool head = (L.hm >> j) & 1u;
                // each group's wrench goes to the axes that move it once the
                // residue is walked (N: every group; CA: its own, the side
                // chain, C's; C: its own; side frame f: frames f and after)
                SpineGrad g;
                NodeGrad sc[A2C_MAX_SIDE_FRAMES];
                Wrench wn = wrench_zero(), wca = wrench_zero(), wc = wrench_zero();
                Wrench ws[A2C_MAX_SIDE_FRAMES];
                if (RECOMPUTE) {
                    if (head) cur = aff_identity();
                    aff_apply_transform(cur, P.ct[0], P.st[0], P.d[0], in[j].co, in[j].so);
                    g.n = node_of_frame(cur);
                    if (GM == kGradMse) frame_wrench_mse(tab, ft, 0, cur, sg, sout, write_so, aloc, wn, loss);
                    else frame_wrench(tab, ft, 0, cur, sg, aloc, wn);
                    aff_apply_transform(cur, P.ct[1], P.st[1], P.d[1], in[j].cp, in[j].sp);
                    g.ca = node_of_frame(cur);
                    if (GM == kGradMse) frame_wrench_mse(tab, ft, 1, cur, sg, sout, write_so, aloc, wca, loss);
                    else frame_wrench(tab, ft, 1, cur, sg, aloc, wca);
                    Aff sf = cur;
                    aff_rot_x(sf, ft.pre_c, ft.pre_s);
#pragma unroll
                    for (int f = 0; f < A2C_MAX_SIDE_FRAMES; ++f) {
                        if (f < tab.max_side && f < ft.n_side) {
                            side_step(sf, ft, f, lr.chi[j][f]);
                            sc[f] = node_of_frame(sf);
                            ws[f] = wrench_zero();
                            if (GM == kGradMse) frame_wrench_mse(tab, ft, 3 + f, sf, sg, sout, write_so, aloc, ws[f], loss);
                            else frame_wrench(tab, ft, 3 + f, sf, sg, aloc, ws[f]);
                        }
                    }
                    aff_apply_transform(cur, P.ct[2], P.st[2], P.d[2], in[j].cs, in[j].ss);
                    g.cc = node_of_frame(cur);
                    if (GM == kGradMse) frame_wrench_mse(tab, ft, 2, cur, sg, sout, write_so, aloc, wc, loss);
                    else frame_wrench(tab, ft, 2, cur, sg, aloc, wc);
                } else {
                    const float *px = sx.st, *py = sx.st + sx.ns, *pz = sx.st + 2 * sx.ns;
                    const float nx = px[aloc], ny = py[aloc], nz = pz[aloc];
                    const float cax = px[aloc + 1], cay = py[aloc + 1], caz = pz[aloc + 1];
                    const float cx = px[aloc + 2], cy = py[aloc + 2], cz = pz[aloc + 2];
                    if (head) { pcx = 0.f; pcy = 0.f; pcz = 0.f; }
                    g.n = node_at(nx, ny, nz, (nx - pcx) * P.inv_d[0], (ny - pcy) * P.inv_d[0],
                                  (nz - pcz) * P.inv_d[0]);
                    g.ca = node_at(cax, cay, caz, (cax - nx) * P.inv_d[1],
                                   (cay - ny) * P.inv_d[1], (caz - nz) * P.inv_d[1]);
                    g.cc = node_at(cx, cy, cz, (cx - cax) * P.inv_d[2], (cy - cay) * P.inv_d[2],
                                   (cz - caz) * P.inv_d[2]);
                    frame_wrench_xyz(tab, ft, 0, sg, sx, aloc, wn);
                    frame_wrench_xyz(tab, ft, 1, sg, sx, aloc, wca);
                    float ppx = cax, ppy = cay, ppz = caz;
#pragma unroll
                    for (int f = 0; f < A2C_MAX_SIDE_FRAMES; ++f) {
                        if (f < tab.max_side && f < ft.n_side) {
                            const int eo = aloc + ft.origin_slot[3 + f];
                            const float ox = px[eo], oy = py[eo], oz = pz[eo];
                            sc[f] = node_at(ox, oy, oz, (ox - ppx) * ft.inv_d[f],
                                            (oy - ppy) * ft.inv_d[f], (oz - ppz) * ft.inv_d[f]);
                            ppx = ox; ppy = oy; ppz = oz;
                            ws[f] = wrench_zero();
                            frame_wrench_xyz(tab, ft, 3 + f, sg, sx, aloc, ws[f]);
                        }
                    }
                    frame_wrench_xyz(tab, ft, 2, sg, sx, aloc, wc);
                    pcx = cx; pcy = cy; pcz = cz;
                }
                // side frame f moves frames f and after: their wrench, summed
                // from the last frame back, folds into each axis once
                Wrench side = wrench_zero();
#pragma unroll
                for (int f = A2C_MAX_SIDE_FRAMES - 1; f >= 0; --f) {
                    if (f < tab.max_side && f < ft.n_side) {
                        wrench_add(side, ws[f]);
                        node_fold(sc[f], side);
                    }
                }
                node_fold(g.cc, wc);      // C: the C group (with O)
                wrench_add(wca, side);
                wrench_add(wca, wc);
                node_fold(g.ca, wca);     // CA: its group, the side chain, the C group
                g.W = wn;
                wrench_add(g.W, wca);
                node_fold(g.n, g.W);      // N: the whole residue
                // chi gradients are complete here (their subtrees end in the residue)
#pragma unroll
                for (int f = 0; f < A2C_MAX_SIDE_FRAMES; ++f)
                    grad_store(&gang[(3 + f) * R + L.rs + j],
                               (f < tab.max_side && f < ft.n_side && ft.side_chi[f]) ? sc[f].c : 0.f,
                               nt != 0);
                sp[j] = g;
                if (!f_end) wrench_add(agg, g.W);
                if ((L.lm >> j) & 1u) f_end = true;
            }
        }
        wave_lds_sync();
        if (STG && GM == kGradMse && xyz_out) {
            lds_to_run(sg, xyz_out, A, L.A0, L.natoms);  // the stage now holds r
            wave_lds_sync();
        }
    }
    Wrench S = block_suffix_windows(agg, __builtin_amdgcn_ballot_w64(f_end), k.nact, L.active, shb,
                                    rcarry_sh, status, t, last, prev);
    if (L.active) {
#pragma unroll
        for (int j = K - 1; j >= 0; --j) {
            if (j < L.cnt) {
                if ((L.lm >> j) & 1u) S = wrench_zero();
                fa_store_grads(gang, R, L.rs + j, sp[j], S, S, nt != 0);
            }
        }
    }
    if constexpr (GM == kGradMse) {
        if (loss_out) lb_loss_commit(loss, status, t, gridDim.x, prev, loss_out, loss_tot);
    }
}

template <int K, int LB, bool STG>
hipError_t fa_fwd_kl(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s)
{
    const size_t lds = STG ? (size_t)p.fs.W * 3 * p.fs.fa_stage_atoms * sizeof(float) : 0;
    hipLaunchKernelGGL((fa_forward_flat_kernel<K, LB, STG>), dim3(p.fs.n_win), dim3(p.fs.W * kWave),
                       lds, s, ang, xyz, p.d_head_bits, p.fs.d_wstart, p.d_res_atom_off, p.d_seq,
                       p.d_fa, p.fs.d_look, p.fs.d_status, p.R, p.A, p.bb, p.fs.fa_stage_atoms);
    return hipGetLastError();
}

template <int K, bool STG>
hipError_t fa_fwd_ks(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s)
{
    const int threads = p.fs.W * kWave;
    if (threads <= 256) return fa_fwd_kl<K, 256, STG>(p, ang, xyz, s);
    if (threads <= kLbSmall) return fa_fwd_kl<K, kLbSmall, STG>(p, ang, xyz, s);
    return fa_fwd_kl<K, kLbLarge, STG>(p, ang, xyz, s);
}

template <int K>
hipError_t fa_fwd_k(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s)
{
    if (!p.fs.d_look) return hipErrorInvalidValue;
    return p.fs.fa_unstaged ? fa_fwd_ks<K, false>(p, ang, xyz, s) : fa_fwd_ks<K, true>(p, ang, xyz, s);
}

// The spine pass covers the adjoint's windows (C = 64 W K residues) with
// more residues per lane where C allows (8 or 4 per lane, fewer waves): it
// only walks the spine, so the per-residue walk is cheap and the scan is
// shared by more residues.
template <int K>
void fa_spine_launch(const a2c_plan &p, const float *ang, hipStream_t s)
{
    const int64_t C = (int64_t)kWave * K * p.bs.W;
    const dim3 grid(p.bs.n_win);
    if (C % (kWave * 8) == 0)
        hipLaunchKernelGGL((fa_spine_aggregate_kernel<8, 1024>), grid, dim3(C / 8), 0, s, ang,
                           p.d_head_bits, p.bs.d_wstart, p.bs.d_status_fwd, p.R, p.bb);
    else if (C % (kWave * 4) == 0)
        hipLaunchKernelGGL((fa_spine_aggregate_kernel<4, 1024>), grid, dim3(C / 4), 0, s, ang,
                           p.d_head_bits, p.bs.d_wstart, p.bs.d_status_fwd, p.R, p.bb);
    else
        hipLaunchKernelGGL((fa_spine_aggregate_kernel<K, 1024>), grid, dim3(C / K), 0, s, ang,
                           p.d_head_bits, p.bs.d_wstart, p.bs.d_status_fwd, p.R, p.bb);
}

template <int K, bool RECOMPUTE, int LB, int GM, bool STG>
void fa_bwd_launch(const a2c_plan &p, const float *ang, const float *xyz, const float *g,
                   float *gang, hipStream_t s, float *xyz_out, float *loss_out)
{
    // whole-chain windows start at a chain head: none needs the spine pass
    if (RECOMPUTE && !p.bs.whole_chains) fa_spine_launch<K>(p, ang, s);
    const size_t lds =
        STG ? (size_t)p.bs.W * (RECOMPUTE ? 3 : 6) * p.bs.fa_stage_atoms * sizeof(float) : 0;
    hipLaunchKernelGGL((fa_backward_flat_kernel<K, RECOMPUTE, LB, GM, STG>), dim3(p.bs.n_win),
                       dim3(p.bs.W * kWave), lds, s, ang, xyz, g, gang, xyz_out, loss_out,
                       p.d_head_bits, p.bs.d_wstart, p.d_res_atom_off,
                       p.d_seq, p.d_fa, p.bs.d_status_fwd, p.bs.d_look_fwd, p.bs.d_look,
                       p.bs.d_status, p.R, p.A, p.bb, p.bs.fa_stage_atoms,
                       p.bs.whole_chains ? 0 : 1, p.nt_grad ? 1 : 0);
}

// mode 0: adjoint from coordinates, 1: recompute, 2: fused squared-distance step
template <int K, int MODE, bool STG>
void fa_bwd_dispatch(const a2c_plan &p, const float *ang, const float *xyz, const float *g,
                     float *gang, hipStream_t s, float *xyz_out, float *loss_out)
{
    constexpr bool RC = MODE != 0;
    constexpr int GM = MODE == 2 ? kGradMse : kGradLoad;
    const int threads = p.bs.W * kWave;
    if (threads <= 256) fa_bwd_launch<K, RC, 256, GM, STG>(p, ang, xyz, g, gang, s, xyz_out, loss_out);
    else if (threads <= kLbSmall)
        fa_bwd_launch<K, RC, kLbSmall, GM, STG>(p, ang, xyz, g, gang, s, xyz_out, loss_out);
    else fa_bwd_launch<K, RC, kLbLarge, GM, STG>(p, ang, xyz, g, gang, s, xyz_out, loss_out);
}

template <int K, int MODE>
hipError_t fa_bwd_mode(const a2c_plan &p, const float *ang, const float *xyz, const float *g,
                       float *gang, hipStream_t s, float *xyz_out = nullptr,
                       float *loss_out = nullptr)
{
    if (p.bs.fa_unstaged) fa_bwd_dispatch<K, MODE, false>(p, ang, xyz, g, gang, s, xyz_out, loss_out);
    else fa_bwd_dispatch<K, MODE, true>(p, ang, xyz, g, gang, s, xyz_out, loss_out);
    return hipGetLastError();
}

template <int K>
hipError_t fa_mse_k(const a2c_plan &p, const float *ang, const float *tgt, float *xyz,
                    float *loss_out, float *gang, hipStream_t s)
{
    return fa_bwd_mode<K, 2>(p, ang, nullptr, tgt, gang, s, xyz, loss_out);
}

template <int K>
hipError_t fa_bwd_k(const a2c_plan &p, const float *ang, const float *xyz, const float *g,
                    float *gang, hipStream_t s)
{
    // the staged coordinate form needs six planes; where they do not fit,
    // the recompute form (three planes) computes the same gradient
    if (xyz && !p.bs.fa_unstaged &&
        (size_t)p.bs.W * 6 * p.bs.fa_stage_atoms * sizeof(float) > (size_t)kMaxDynamicLds)
        xyz = nullptr;
    return xyz ? fa_bwd_mode<K, 0>(p, ang, xyz, g, gang, s)
               : fa_bwd_mode<K, 1>(p, ang, xyz, g, gang, s);
}

}  // namespace

hipError_t launch_fa_forward_scan(const a2c_plan &p, const float *ang, float *xyz, hipStream_t s)
{
    switch (p.fs.K) {
    case 1: return fa_fwd_k<1>(p, ang, xyz, s);
    case 2: return fa_fwd_k<2>(p, ang, xyz, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fa_backward_scan(const a2c_plan &p, const float *ang, const float *xyz,
                                   const float *g, float *gang, hipStream_t s)
{
    switch (p.bs.K) {
    case 1: return fa_bwd_k<1>(p, ang, xyz, g, gang, s);
    case 2: return fa_bwd_k<2>(p, ang, xyz, g, gang, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fa_mse_step(const a2c_plan &p, const float *ang, const float *tgt, float *xyz,
                              float *loss_out, float *gang, hipStream_t s)
{
    switch (p.bs.K) {
    case 1: return fa_mse_k<1>(p, ang, tgt, xyz, loss_out, gang, s);
    case 2: return fa_mse_k<2>(p, ang, tgt, xyz, loss_out, gang, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename F>
static void allow_lds(F kernel)
{
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxDynamicLds);
}

template <int K, int LB>
static void allow_lds_kl()
{
    allow_lds(fa_forward_flat_kernel<K, LB>);
    allow_lds(fa_backward_flat_kernel<K, false, LB>);
    allow_lds(fa_backward_flat_kernel<K, true, LB>);
    allow_lds(fa_backward_flat_kernel<K, true, LB, kGradMse, true>);
}

void fa_allow_large_lds()
{
    static bool done = false;
    if (done) return;
    allow_lds_kl<1, 256>();
    allow_lds_kl<2, 256>();
    allow_lds_kl<1, kLbSmall>();
    allow_lds_kl<2, kLbSmall>();
    allow_lds_kl<1, kLbLarge>();
    allow_lds_kl<2, kLbLarge>();
    done = true;
}

}  // namespace a2c
