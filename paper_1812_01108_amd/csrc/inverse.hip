// Inverse map: Cartesian coordinates -> dihedral angles, the step before the
// forward map in a pipeline (targets, initial angles).  The angle of the
// transform placing atom i is the IUPAC torsion about the bond into atom i,
// (i-2, i-1, i, i+1) ("Backbone model" section), so per residue j
//   omega_j = torsion(CA_{j-1}, C_{j-1}, N_j, CA_j),
//   phi_j   = torsion(C_{j-1}, N_j, CA_j, C_j),
//   psi_j   = torsion(N_j, CA_j, C_j, N_{j+1}),
// with the identity start frame's virtual atoms C_{-1} = origin and
// CA_{-1} = (-1, 0, 0) at a chain start; psi of a chain's last residue moves
// no atom and is written as 0.  Side chains ("Full-atom model" section): the
// transform of side frame f carries chi_{f+1}, so
//   chi_{f+1} = torsion(grandparent origin, parent origin, origin of f, D),
// the grandparent of side frame 0 being N and its parent CA, and D an atom
// that lies at y = 0, z < 0 in frame f's own coordinates (where the
// transform puts the next frame's origin, and where the residue table puts
// the atom that defines the last chi): its torsion is exactly the frame's
// angle.  The quadruples are read off the converted residue table on the
// host; chi planes a residue lacks are written as 0.
#include "a2c_internal.h"

#include <cmath>

namespace a2c {

// Residue slots (a, b, c, d) of every chi of every residue type; -1 where
// the type has no such chi or no defining atom.
void build_chi_slots(const FATable &T, int8_t (&out)[A2C_NUM_RESIDUE_TYPES][4][4])
{
    for (int t = 0; t < A2C_NUM_RESIDUE_TYPES; ++t) {
        const FAType &ft = T.t[t];
        for (int f = 0; f < 4; ++f) {
            int8_t *q = out[t][f];
            q[0] = q[1] = q[2] = q[3] = -1;
            if (f >= ft.n_side || !ft.side_chi[f]) continue;
            const int c = ft.origin_slot[3 + f];
            const int b = f == 0 ? 1 : ft.origin_slot[3 + f - 1];
            const int a = f == 0 ? 0 : (f == 1 ? 1 : ft.origin_slot[3 + f - 2]);
            int d = -1;
            if (f + 1 < ft.n_side) {
                d = ft.origin_slot[3 + f + 1];
            } else {
                const int k = 3 + f;
                for (int i = 0; i < ft.fcount[k] && d < 0; ++i) {
                    const int s = ft.fbegin[k] + i;
                    const float x = ft.atom[s].x, y = ft.atom[s].y, z = ft.atom[s].z;
                    const float r = std::sqrt(x * x + y * y + z * z);
                    if (r > 0.f && std::fabs(y) <= 1e-5f * r && z < -1e-3f * r) d = ft.atom[s].slot;
                }
            }
            if (d < 0) continue;
            q[0] = (int8_t)a;
            q[1] = (int8_t)b;
            q[2] = (int8_t)c;
            q[3] = (int8_t)d;
        }
    }
}

namespace {

struct P3 {
    float x, y, z;
};

// atan2 for the torsions.  Octant reduction: t = min(|x|, |y|) / max(|x|, |y|)
// in [0, 1] (reciprocal by v_rcp_f32), atan t = t (a0 + a1 t^2 + ... + a6 t^12)
// with coefficients fitted for this library by a discrete minimax
// (Lawson-weighted least squares) in double and rounded to float32 (maximum
// error 3.3e-7 rad evaluated in float32), then pi/2 - a where |y| > |x|,
// pi - a where x < 0, and the sign of y.  NaN in gives NaN; (0, 0) gives 0.
__device__ __forceinline__ float atan2_poly(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.f ? mn * __builtin_amdgcn_rcpf(mx) : 0.f;
    const float t2 = t * t;
    float p = 6.81179157e-03f;
    p = fmaf(p, t2, -3.36042158e-02f);
    p = fmaf(p, t2, 7.96236694e-02f);
    p = fmaf(p, t2, -1.32333413e-01f);
    p = fmaf(p, t2, 1.98078156e-01f);
    p = fmaf(p, t2, -3.33173692e-01f);
    p = fmaf(p, t2, 9.99996126e-01f);
    float a = p * t;
    a = ay > ax ? 1.57079637f - a : a;
    a = x < 0.f ? 3.14159274f - a : a;
    a = copysignf(a, y);
    return (x != x || y != y) ? x + y : a;
}

// IUPAC torsion angle of p0-p1-p2-p3:
// atan2(|b2| b1 . (b2 x b3), (b1 x b2) . (b2 x b3)).  |b2| only scales the
// first argument, so the 1-ulp hardware square root is enough.
__device__ __forceinline__ float torsion(P3 p0, P3 p1, P3 p2, P3 p3)
{
    const float b1x = p1.x - p0.x, b1y = p1.y - p0.y, b1z = p1.z - p0.z;
    const float b2x = p2.x - p1.x, b2y = p2.y - p1.y, b2z = p2.z - p1.z;
    const float b3x = p3.x - p2.x, b3y = p3.y - p2.y, b3z = p3.z - p2.z;
    const float n1x = b1y * b2z - b1z * b2y, n1y = b1z * b2x - b1x * b2z, n1z = b1x * b2y - b1y * b2x;
    const float n2x = b2y * b3z - b2z * b3y, n2y = b2z * b3x - b2x * b3z, n2z = b2x * b3y - b2y * b3x;
    const float b2n = __builtin_amdgcn_sqrtf(b2x * b2x + b2y * b2y + b2z * b2z);
    const float y = b2n * (b1x * n2x + b1y * n2y + b1z * n2z);
    const float x = n1x * n2x + n1y * n2y + n1z * n2z;
    return atan2_poly(y, x);
}

__device__ __forceinline__ bool head_bit(const uint32_t *__restrict__ bits, int64_t r)
{
    return (bits[r >> 5] >> (r & 31)) & 1u;
}

constexpr int kInvThreads = 256;  // residues per workgroup

// One lane per residue.  The workgroup's atoms, with one residue on either
// side (the neighbours' backbone atoms), are staged once through LDS with
// coalesced loads, every load issued before the first store; the torsions
// then read LDS.  Staged: residues [max(r0 - 1, 0), min(r0 + 257, R)), at
// most 258 residues of at most kAtoms atoms each.
template <bool FA>
__global__ __launch_bounds__(kInvThreads) void inverse_kernel(
    const float *__restrict__ xyz, float *__restrict__ ang, const uint32_t *__restrict__ head_bits,
    const int32_t *__restrict__ res_aoff, const uint8_t *__restrict__ seq,
    const int8_t *__restrict__ chi_slots, int64_t R, int64_t A, int cap)
{
    constexpr int kAtoms = FA ? A2C_MAX_RESIDUE_ATOMS : 3;
    constexpr int kStage = (kInvThreads + 2) * kAtoms;
    constexpr int kPer = (kStage + kInvThreads - 1) / kInvThreads;
    // cap: the largest staged range of any workgroup of this plan (<= kStage),
    // which sizes the dynamic LDS (3 cap floats)
    extern __shared__ float inv_stage[];
    float *const sx = inv_stage, *const sy = inv_stage + cap, *const sz = inv_stage + 2 * cap;
    const int tid = (int)threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * kInvThreads;
    const int64_t rlo = r0 > 0 ? r0 - 1 : 0;
    const int64_t rhi = r0 + kInvThreads + 1 < R ? r0 + kInvThreads + 1 : R;
    // atom indices fit in int32: a plan holds at most INT32_MAX / 16 residues
    const int lo = FA ? res_aoff[rlo] : (int)(3 * rlo);
    const int hi = FA ? res_aoff[rhi] : (int)(3 * rhi);
    const float *__restrict__ px = xyz + lo;
    const float *__restrict__ py = xyz + A + lo;
    const float *__restrict__ pz = xyz + 2 * A + lo;
    const int n_st = hi - lo;
    {
        float vx[kPer], vy[kPer], vz[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = tid + j * kInvThreads;
            const int kc = k < n_st ? k : 0;
            vx[j] = px[kc]; vy[j] = py[kc]; vz[j] = pz[kc];
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = tid + j * kInvThreads;
            if (k < n_st) {
                sx[k] = vx[j]; sy[k] = vy[j]; sz[k] = vz[j];
            }
        }
    }
    __syncthreads();
    const int64_t r = r0 + tid;
    if (r >= R) return;
    auto pt = [&](int64_t atom) -> P3 {
        const int k = (int)atom - lo;
        return {sx[k], sy[k], sz[k]};
    };
    const bool head = head_bit(head_bits, r), last = head_bit(head_bits, r + 1);
    const int64_t a = FA ? (int64_t)res_aoff[r] : 3 * r;
    // neighbours: the previous residue is staged unless r is a chain head,
    // the next one unless r ends its chain (then r's own atoms stand in and
    // the angle is replaced below)
    const int64_t rp = head ? r : r - 1, rn = last ? r : r + 1;
    const int64_t pa = FA ? (int64_t)res_aoff[rp] : 3 * rp;
    const int64_t na = FA ? (int64_t)res_aoff[rn] : 3 * rn;
    const P3 n = pt(a), ca = pt(a + 1), c = pt(a + 2);
    const P3 pca = head ? P3{-1.f, 0.f, 0.f} : pt(pa + 1);
    const P3 pc = head ? P3{0.f, 0.f, 0.f} : pt(pa + 2);
    const float psi = torsion(n, ca, c, pt(na));
    ang[r] = torsion(pc, n, ca, c);
    ang[R + r] = last ? 0.f : psi;
    ang[2 * R + r] = torsion(pca, pc, n, ca);
    if (FA) {
        // the residue type's four (a, b, c, d) slot quadruples in one load
        const int4 qv = *reinterpret_cast<const int4 *>(chi_slots + 16 * seq[r]);
        const int qw[4] = {qv.x, qv.y, qv.z, qv.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int8_t q0 = (int8_t)(qw[k] & 0xff), q1 = (int8_t)((qw[k] >> 8) & 0xff);
            const int8_t q2 = (int8_t)((qw[k] >> 16) & 0xff), q3 = (int8_t)((qw[k] >> 24) & 0xff);
            const bool has = q0 >= 0;
            const float v = torsion(pt(a + (has ? q0 : 0)), pt(a + (has ? q1 : 1)),
                                    pt(a + (has ? q2 : 2)), pt(a + (has ? q3 : 0)));
            ang[(3 + k) * R + r] = has ? v : 0.f;
        }
    }
}

}  // namespace
}  // namespace a2c

using namespace a2c;

extern "C" a2c_status a2c_coords_to_angles(a2c_plan *p, const float *d_coords, float *d_angles,
                                           void *stream)
{
    if (!p) {
        set_error("plan is NULL");
        return A2C_ERR_INVALID_ARG;
    }
    if (p->R == 0) return A2C_OK;
    if (!d_coords || !d_angles) {
        set_error("NULL coords or angles");
        return A2C_ERR_INVALID_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
        set_error("current device is not the plan's device");
        return A2C_ERR_STATE;
    }
    const dim3 grid((unsigned)((p->R + kInvThreads - 1) / kInvThreads)), block(kInvThreads);
    hipStream_t s = (hipStream_t)stream;
    // the largest staged atom range over the workgroups (host offsets)
    int cap = 0;
    for (int64_t r0 = 0; r0 < p->R; r0 += kInvThreads) {
        const int64_t rlo = r0 > 0 ? r0 - 1 : 0;
        const int64_t rhi = r0 + kInvThreads + 1 < p->R ? r0 + kInvThreads + 1 : p->R;
        const int n = p->model == A2C_BACKBONE ? (int)(3 * (rhi - rlo))
                                               : p->res_atom_off[rhi] - p->res_atom_off[rlo];
        cap = n > cap ? n : cap;
    }
    const size_t lds = 3 * (size_t)cap * sizeof(float);
    if (p->model == A2C_BACKBONE)
        hipLaunchKernelGGL(inverse_kernel<false>, grid, block, lds, s, d_coords, d_angles,
                           p->d_head_bits, nullptr, nullptr, nullptr, p->R, p->A, cap);
    else
        hipLaunchKernelGGL(inverse_kernel<true>, grid, block, lds, s, d_coords, d_angles,
                           p->d_head_bits, p->d_res_atom_off, p->d_seq, p->d_chi_slots, p->R,
                           p->A, cap);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? A2C_OK : hip_fail(e, "inverse map launch");
}
