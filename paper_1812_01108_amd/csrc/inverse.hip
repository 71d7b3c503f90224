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

__device__ __forceinline__ P3 pt(const float *__restrict__ xyz, int64_t A, int64_t a)
{
    return {xyz[a], xyz[A + a], xyz[2 * A + a]};
}

// IUPAC torsion angle of p0-p1-p2-p3:
// atan2(|b2| b1 . (b2 x b3), (b1 x b2) . (b2 x b3)).
__device__ __forceinline__ float torsion(P3 p0, P3 p1, P3 p2, P3 p3)
{
    const float b1x = p1.x - p0.x, b1y = p1.y - p0.y, b1z = p1.z - p0.z;
    const float b2x = p2.x - p1.x, b2y = p2.y - p1.y, b2z = p2.z - p1.z;
    const float b3x = p3.x - p2.x, b3y = p3.y - p2.y, b3z = p3.z - p2.z;
    const float n1x = b1y * b2z - b1z * b2y, n1y = b1z * b2x - b1x * b2z, n1z = b1x * b2y - b1y * b2x;
    const float n2x = b2y * b3z - b2z * b3y, n2y = b2z * b3x - b2x * b3z, n2z = b2x * b3y - b2y * b3x;
    const float b2n = sqrtf(b2x * b2x + b2y * b2y + b2z * b2z);
    const float y = b2n * (b1x * n2x + b1y * n2y + b1z * n2z);
    const float x = n1x * n2x + n1y * n2y + n1z * n2z;
    return atan2f(y, x);
}

__device__ __forceinline__ bool head_bit(const uint32_t *__restrict__ bits, int64_t r)
{
    return (bits[r >> 5] >> (r & 31)) & 1u;
}

template <bool FA>
__global__ __launch_bounds__(256) void inverse_kernel(
    const float *__restrict__ xyz, float *__restrict__ ang, const uint32_t *__restrict__ head_bits,
    const int32_t *__restrict__ res_aoff, const uint8_t *__restrict__ seq,
    const int8_t *__restrict__ chi_slots, int64_t R, int64_t A)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const bool head = head_bit(head_bits, r), last = head_bit(head_bits, r + 1);
    const int64_t a = FA ? (int64_t)res_aoff[r] : 3 * r;
    const P3 n = pt(xyz, A, a), ca = pt(xyz, A, a + 1), c = pt(xyz, A, a + 2);
    P3 pca = {-1.f, 0.f, 0.f}, pc = {0.f, 0.f, 0.f};
    if (!head) {
        const int64_t pa = FA ? (int64_t)res_aoff[r - 1] : 3 * (r - 1);
        pca = pt(xyz, A, pa + 1);
        pc = pt(xyz, A, pa + 2);
    }
    float psi = 0.f;
    if (!last) psi = torsion(n, ca, c, pt(xyz, A, FA ? (int64_t)res_aoff[r + 1] : 3 * (r + 1)));
    ang[r] = torsion(pc, n, ca, c);
    ang[R + r] = psi;
    ang[2 * R + r] = torsion(pca, pc, n, ca);
    if (FA) {
        const int8_t *q = chi_slots + 16 * seq[r];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float v = 0.f;
            if (q[4 * k] >= 0)
                v = torsion(pt(xyz, A, a + q[4 * k]), pt(xyz, A, a + q[4 * k + 1]),
                            pt(xyz, A, a + q[4 * k + 2]), pt(xyz, A, a + q[4 * k + 3]));
            ang[(3 + k) * R + r] = v;
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
    const dim3 grid((unsigned)((p->R + 255) / 256)), block(256);
    hipStream_t s = (hipStream_t)stream;
    if (p->model == A2C_BACKBONE)
        hipLaunchKernelGGL(inverse_kernel<false>, grid, block, 0, s, d_coords, d_angles,
                           p->d_head_bits, nullptr, nullptr, nullptr, p->R, p->A);
    else
        hipLaunchKernelGGL(inverse_kernel<true>, grid, block, 0, s, d_coords, d_angles,
                           p->d_head_bits, p->d_res_atom_off, p->d_seq, p->d_chi_slots, p->R,
                           p->A);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? A2C_OK : hip_fail(e, "inverse map launch");
}
