// LRMSD loss ("Loss function" section of arXiv:1812.01108) on the GPU: for
// every chain c, the least root-mean-square deviation between the input
// coordinates y (the map's output) and a target x after the optimal rigid
// superposition, and its gradient with respect to y.
//
// Per chain (N atoms, centred sets x~, y~, correlation R = sum_i x~_i y~_i^T):
//   T       the symmetric traceless 4x4 matrix the section builds from R;
//   lambda  its largest eigenvalue, q the unit eigenvector;
//   LRMSD   = sqrt((sum |x~|^2 + sum |y~|^2 - 2 lambda) / N);
//   U(q)    the rotation the section builds from q; it maps the target onto
//           the input (U x~_i ~ y~_i);
//   dLRMSD / dy_i = (y~_i - U x~_i) / (N LRMSD)   (0 where LRMSD = 0).
// The printed derivative names the target as the variable and leaves out
// the 1 / (N LRMSD) factor; the form above is the derivative with respect to
// the input, which is what a loss on the map's output needs.
//
// Three kernels:
//   lr_partial  one workgroup per segment (<= kLrSegAtoms atoms of one
//               chain): sums of x, y, |x|^2, |y|^2 and x y^T, both sets
//               shifted by the chain's first atom, accumulated in float64
//               (the shift keeps the centring well conditioned; float64
//               makes the sums exact to far below float32 rounding);
//   lr_solve    one lane per chain: folds the chain's segment sums, centres
//               them, finds lambda by Newton's method on the characteristic
//               polynomial of T from above (monotone: lambda <= the bound
//               (sum |x~|^2 + sum |y~|^2) / 2 it starts from), q from the
//               adjugate of T - lambda I (a cyclic Jacobi sweep takes over
//               when the largest eigenvalue is degenerate), and stores
//               LRMSD, U, the means and 1 / (N LRMSD) per chain;
//   lr_grad     one workgroup per piece (<= kLrPieceAtoms atoms of one
//               chain, four per thread, all loads issued first): the
//               gradient above, scaled by the upstream gradient of each
//               chain's LRMSD.
#include "a2c_internal.h"

#include <cmath>
#include <mutex>

namespace a2c {
namespace {

constexpr int kLrThreads = 256;
constexpr int kLrSolveThreads = 64;  // one lane per chain
constexpr int kLrPart = 18;  // doubles per segment record (17 used)
constexpr int kLrState = 16; // floats per chain: U (9), x mean (3), y mean (3), 1/(N LRMSD)
// The gradient runs on pieces of four atoms per thread, so that a thread's
// loads are all in flight at once and small batches still spread over many
// workgroups.
static_assert(kLrPieceAtoms == 4 * kLrThreads, "four gradient atoms per thread");

// --------------------------------------------------------------- reductions

__device__ __forceinline__ double dpp_f64_xor1(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    // quad_perm [1, 0, 3, 2]
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false),
                            __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false));
}

__device__ __forceinline__ double dpp_f64_xor2(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    // quad_perm [2, 3, 0, 1]
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false),
                            __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false));
}

__device__ __forceinline__ double dpp_f64_half_mirror(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false),
                            __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false));
}

__device__ __forceinline__ double dpp_f64_mirror(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false),
                            __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false));
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the 64 lanes of a wave; every lane receives the total.  Within
// rows of 16 by DPP exchanges, then the four row sums by lane reads (exact
// same order in every wave: the result is deterministic).
__device__ __forceinline__ double wave_sum_f64(double v)
{
    v += dpp_f64_xor1(v);
    v += dpp_f64_xor2(v);
    v += dpp_f64_half_mirror(v);
    v += dpp_f64_mirror(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// ------------------------------------------------------------ partial sums
// Record layout: 0-2 sum x_s, 3-5 sum y_s, 6 sum |x_s|^2, 7 sum |y_s|^2,
// 8-16 sum x_s y_s^T (row-major, [i][j] = sum x_s,i y_s,j); x_s, y_s shifted
// by the chain's first atom.

__global__ __launch_bounds__(kLrThreads) void lr_partial_kernel(
    const float *__restrict__ y, const float *__restrict__ x, const int32_t *__restrict__ seg_atom,
    const int32_t *__restrict__ seg_origin, int64_t A, double *__restrict__ part)
{
    __shared__ double red[17][kLrThreads + 1];
    const int s = blockIdx.x;
    const int a0 = seg_atom[s], a1 = seg_atom[s + 1];
    const int r0 = seg_origin[s];  // the chain's first atom
    const double x0 = x[r0], x1 = x[A + r0], x2 = x[2 * A + r0];
    const double y0 = y[r0], y1 = y[A + r0], y2 = y[2 * A + r0];
    double acc[17];
#pragma unroll
    for (int k = 0; k < 17; ++k) acc[k] = 0.0;
    // at most 16 atoms per thread, four at a time with every load issued first
    for (int base = a0 + (int)threadIdx.x; base < a1; base += 4 * kLrThreads) {
        float fx[4][3], fy[4][3];
        bool ok[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int a = base + j * kLrThreads;
            ok[j] = a < a1;
            const int ac = ok[j] ? a : a0;
            fx[j][0] = x[ac]; fx[j][1] = x[A + ac]; fx[j][2] = x[2 * A + ac];
            fy[j][0] = y[ac]; fy[j][1] = y[A + ac]; fy[j][2] = y[2 * A + ac];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!ok[j]) continue;
            const double px = fx[j][0] - x0, py = fx[j][1] - x1, pz = fx[j][2] - x2;
            const double qx = fy[j][0] - y0, qy = fy[j][1] - y1, qz = fy[j][2] - y2;
            acc[0] += px; acc[1] += py; acc[2] += pz;
            acc[3] += qx; acc[4] += qy; acc[5] += qz;
            acc[6] += px * px + py * py + pz * pz;
            acc[7] += qx * qx + qy * qy + qz * qz;
            acc[8] += px * qx; acc[9] += px * qy; acc[10] += px * qz;
            acc[11] += py * qx; acc[12] += py * qy; acc[13] += py * qz;
            acc[14] += pz * qx; acc[15] += pz * qy; acc[16] += pz * qz;
        }
    }
#pragma unroll
    for (int k = 0; k < 17; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    // wave w folds records w, w + 4, ...: four LDS reads per lane, then a
    // wave sum
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int k = wave; k < 17; k += kLrThreads / 64) {
        const double v = (red[k][lane] + red[k][lane + 64]) + (red[k][lane + 128] + red[k][lane + 192]);
        const double t = wave_sum_f64(v);
        if (lane == 0) part[(size_t)s * kLrPart + k] = t;
    }
}

// ----------------------------------------------------------------- 4x4 solve

__device__ __forceinline__ double det3(double a, double b, double c, double d, double e,
                                       double f, double g, double h, double i)
{
    return a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
}

// Cofactor (r, k) of the 4x4 matrix m (r, k compile-time after unrolling).
__device__ __forceinline__ double cofactor4(const double (&m)[4][4], int r, int k)
{
    const int rows[3] = {r == 0 ? 1 : 0, r <= 1 ? 2 : 1, r <= 2 ? 3 : 2};
    const int cols[3] = {k == 0 ? 1 : 0, k <= 1 ? 2 : 1, k <= 2 ? 3 : 2};
    const double d = det3(m[rows[0]][cols[0]], m[rows[0]][cols[1]], m[rows[0]][cols[2]],
                          m[rows[1]][cols[0]], m[rows[1]][cols[1]], m[rows[1]][cols[2]],
                          m[rows[2]][cols[0]], m[rows[2]][cols[1]], m[rows[2]][cols[2]]);
    return ((r + k) & 1) ? -d : d;
}

__device__ __forceinline__ double det4(const double (&m)[4][4])
{
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) d += m[0][k] * cofactor4(m, 0, k);
    return d;
}

// Eigenvector of the largest eigenvalue of a symmetric 4x4 matrix by cyclic
// Jacobi rotations (the degenerate-case fallback).
__device__ void jacobi_top_vector(const double (&t)[4][4], double (&q)[4])
{
    double a[4][4], v[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            a[i][j] = t[i][j];
            v[i][j] = i == j ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < 4; ++i) {
            diag += a[i][i] * a[i][i];
            for (int j = i + 1; j < 4; ++j) off += a[i][j] * a[i][j];
        }
        if (off <= 1e-30 * diag || off == 0.0) break;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = p + 1; r < 4; ++r) {
                if (a[p][r] == 0.0) continue;
                // rotation zeroing a[p][r]: tan of the angle from the
                // smaller root of t^2 + 2 theta t - 1 = 0
                const double theta = (a[r][r] - a[p][p]) / (2.0 * a[p][r]);
                const double tt = (theta >= 0.0 ? 1.0 : -1.0) /
                                  (fabs(theta) + sqrt(theta * theta + 1.0));
                const double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
                for (int k = 0; k < 4; ++k) {
                    const double akp = a[k][p], akr = a[k][r];
                    a[k][p] = cs * akp - sn * akr;
                    a[k][r] = sn * akp + cs * akr;
                }
                for (int k = 0; k < 4; ++k) {
                    const double apk = a[p][k], ark = a[r][k];
                    a[p][k] = cs * apk - sn * ark;
                    a[r][k] = sn * apk + cs * ark;
                }
                for (int k = 0; k < 4; ++k) {
                    const double vkp = v[k][p], vkr = v[k][r];
                    v[k][p] = cs * vkp - sn * vkr;
                    v[k][r] = sn * vkp + cs * vkr;
                }
            }
    }
    double top = a[0][0];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = v[i][0];
#pragma unroll
    for (int j = 1; j < 4; ++j)
        if (a[j][j] > top) {
            top = a[j][j];
#pragma unroll
            for (int i = 0; i < 4; ++i) q[i] = v[i][j];
        }
}

__global__ __launch_bounds__(kLrSolveThreads) void lr_solve_kernel(
    const float *__restrict__ y, const float *__restrict__ x, const int32_t *__restrict__ seg_atom,
    const int32_t *__restrict__ chain_seg, int32_t n_chains, int64_t A,
    const double *__restrict__ part, float *__restrict__ state, float *__restrict__ out)
{
    const int c = blockIdx.x * kLrSolveThreads + (int)threadIdx.x;
    if (c >= n_chains) return;
    const int s0 = chain_seg[c], s1 = chain_seg[c + 1];
    const int r0 = s1 > s0 ? seg_atom[s0] : 0;
    const int64_t n_atoms = s1 > s0 ? (int64_t)seg_atom[s1] - r0 : 0;
    float *st = state + (size_t)c * kLrState;
    if (n_atoms == 0) {
        for (int k = 0; k < kLrState; ++k) st[k] = 0.f;
        st[0] = st[4] = st[8] = 1.f;
        out[c] = 0.f;
        return;
    }
    // the chain's first atom (the shift of the segment sums), loaded ahead of
    // the sums so that the two latencies overlap
    const float x0[3] = {x[r0], x[A + r0], x[2 * A + r0]};
    const float y0[3] = {y[r0], y[A + r0], y[2 * A + r0]};
    // the chain's segment records, folded in segment order
    double acc[17];
#pragma unroll
    for (int k = 0; k < 17; ++k) acc[k] = part[(size_t)s0 * kLrPart + k];
    for (int s = s0 + 1; s < s1; ++s) {
#pragma unroll
        for (int k = 0; k < 17; ++k) acc[k] += part[(size_t)s * kLrPart + k];
    }
    const double N = (double)n_atoms, inv_N = 1.0 / N;
    const double mx[3] = {acc[0] * inv_N, acc[1] * inv_N, acc[2] * inv_N};
    const double my[3] = {acc[3] * inv_N, acc[4] * inv_N, acc[5] * inv_N};
    const double gx = acc[6] - N * (mx[0] * mx[0] + mx[1] * mx[1] + mx[2] * mx[2]);
    const double gy = acc[7] - N * (my[0] * my[0] + my[1] * my[1] + my[2] * my[2]);
    double R[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[i][j] = acc[8 + 3 * i + j] - N * mx[i] * my[j];
    // the symmetric traceless matrix T of the section
    double T[4][4];
    T[0][0] = R[0][0] + R[1][1] + R[2][2];
    T[1][1] = R[0][0] - R[1][1] - R[2][2];
    T[2][2] = -R[0][0] + R[1][1] - R[2][2];
    T[3][3] = -R[0][0] - R[1][1] + R[2][2];
    T[0][1] = T[1][0] = R[1][2] - R[2][1];
    T[0][2] = T[2][0] = R[2][0] - R[0][2];
    T[0][3] = T[3][0] = R[0][1] - R[1][0];
    T[1][2] = T[2][1] = R[0][1] + R[1][0];
    T[1][3] = T[3][1] = R[0][2] + R[2][0];
    T[2][3] = T[3][2] = R[1][2] + R[2][1];
    // characteristic polynomial lambda^4 + c2 lambda^2 + c1 lambda + c0 of a
    // traceless matrix: c2 = -tr(T^2) / 2, c1 = -tr(T^3) / 3, c0 = det T
    double T2[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double v = 0.0;
            for (int k = 0; k < 4; ++k) v += T[i][k] * T[k][j];
            T2[i][j] = v;
        }
    double tr2 = 0.0, tr3 = 0.0;
    for (int i = 0; i < 4; ++i) {
        tr2 += T2[i][i];
        for (int k = 0; k < 4; ++k) tr3 += T2[i][k] * T[k][i];
    }
    const double c2 = -0.5 * tr2, c1 = tr3 * (-1.0 / 3.0), c0 = det4(T);
    const double G = gx + gy;
    // start above the largest root, where Newton descends monotonically:
    // lambda_max <= G / 2 (LRMSD^2 >= 0), and for a traceless symmetric 4x4
    // lambda_max <= sqrt(3/4 tr(T^2)) (the other three eigenvalues sum to
    // -lambda_max, so their squares sum to at least lambda_max^2 / 3)
    double lam = fmin(0.5 * G, sqrt(0.75 * tr2));
    for (int it = 0; it < 100; ++it) {
        const double l2 = lam * lam;
        const double P = (l2 + c2) * l2 + c1 * lam + c0;
        const double dP = (4.0 * l2 + 2.0 * c2) * lam + c1;
        if (!(dP > 0.0)) break;
        const double step = P / dP;
        // every exact step from above is positive: a step that is not has
        // reached the rounding noise of P (which, with a close second
        // eigenvalue, stays above the relative test below)
        if (!(step > 0.0)) break;
        lam -= step;
        if (!(step > 1e-15 * fabs(lam))) break;
    }
    // eigenvector: the largest column of adj(T - lambda I)
    double M[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) M[i][j] = T[i][j] - (i == j ? lam : 0.0);
    double q[4] = {1.0, 0.0, 0.0, 0.0};
    double best = -1.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double v[4], n2 = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cofactor4(M, r, k);
            n2 += v[k] * v[k];
        }
        if (n2 > best) {
            best = n2;
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = v[k];
        }
    }
    const double scale = fmax(0.5 * G, 1e-300);
    if (!(best > 1e-18 * scale * scale * scale * scale * scale * scale)) {
        jacobi_top_vector(T, q);  // the largest eigenvalue is (nearly) repeated
        best = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    }
    const double inv_n = 1.0 / sqrt(best);
    const double q0 = q[0] * inv_n, q1 = q[1] * inv_n, q2 = q[2] * inv_n, q3 = q[3] * inv_n;
    // rotation from q as the section builds it
    st[0] = (float)(q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3);
    st[1] = (float)(2.0 * (q1 * q2 - q0 * q3));
    st[2] = (float)(2.0 * (q1 * q3 + q0 * q2));
    st[3] = (float)(2.0 * (q1 * q2 + q0 * q3));
    st[4] = (float)(q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3);
    st[5] = (float)(2.0 * (q2 * q3 - q0 * q1));
    st[6] = (float)(2.0 * (q1 * q3 - q0 * q2));
    st[7] = (float)(2.0 * (q2 * q3 + q0 * q1));
    st[8] = (float)(q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3);
    st[9] = (float)(x0[0] + mx[0]);
    st[10] = (float)(x0[1] + mx[1]);
    st[11] = (float)(x0[2] + mx[2]);
    st[12] = (float)(y0[0] + my[0]);
    st[13] = (float)(y0[1] + my[1]);
    st[14] = (float)(y0[2] + my[2]);
    const double l = sqrt(fmax(G - 2.0 * lam, 0.0) / N);
    st[15] = l > 0.0 ? (float)(1.0 / (N * l)) : 0.f;
    out[c] = (float)l;
}

// ------------------------------------------------------------------ gradient

__global__ __launch_bounds__(kLrThreads) void lr_grad_kernel(
    const float *__restrict__ y, const float *__restrict__ x, const int32_t *__restrict__ piece_atom,
    const int32_t *__restrict__ piece_chain, int64_t A, const float *__restrict__ state,
    const float *__restrict__ gout, float *__restrict__ gy)
{
    const int pc = blockIdx.x;
    const int64_t a0 = piece_atom[pc], a1 = piece_atom[pc + 1];
    const int c = piece_chain[pc];
    const float *st = state + (size_t)c * kLrState;
    const float u00 = st[0], u01 = st[1], u02 = st[2];
    const float u10 = st[3], u11 = st[4], u12 = st[5];
    const float u20 = st[6], u21 = st[7], u22 = st[8];
    const float xm0 = st[9], xm1 = st[10], xm2 = st[11];
    const float ym0 = st[12], ym1 = st[13], ym2 = st[14];
    const float w = gout[c] * st[15];
    float fx[4][3], fy[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t a = a0 + threadIdx.x + j * kLrThreads;
        const int64_t ac = a < a1 ? a : a0;  // clamped: every load issued
        fx[j][0] = x[ac]; fx[j][1] = x[A + ac]; fx[j][2] = x[2 * A + ac];
        fy[j][0] = y[ac]; fy[j][1] = y[A + ac]; fy[j][2] = y[2 * A + ac];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t a = a0 + threadIdx.x + j * kLrThreads;
        if (a >= a1) continue;
        const float px = fx[j][0] - xm0, py = fx[j][1] - xm1, pz = fx[j][2] - xm2;
        const float qx = fy[j][0] - ym0, qy = fy[j][1] - ym1, qz = fy[j][2] - ym2;
        const float rx = qx - (u00 * px + u01 * py + u02 * pz);
        const float ry = qy - (u10 * px + u11 * py + u12 * pz);
        const float rz = qz - (u20 * px + u21 * py + u22 * pz);
        gy[a] = w * rx;
        gy[A + a] = w * ry;
        gy[2 * A + a] = w * rz;
    }
}

bool lr_ready(const a2c_plan *p)
{
    return p->n_chains == 0 ||
           (p->d_lr_chain_seg && (p->lr_n_seg == 0 || (p->d_lr_seg_atom && p->d_lr_seg_origin)) &&
            (p->lr_n_piece == 0 || (p->d_lr_piece_atom && p->d_lr_piece_chain)));
}

}  // namespace

size_t lrmsd_workspace_bytes(const a2c_plan &p)
{
    return (size_t)p.lr_n_seg * kLrPart * sizeof(double) +
           (size_t)p.n_chains * kLrState * sizeof(float);
}

// ------------------------------------------------------- static scratch
// The no-allocation forward (a2c_lrmsd_forward_noalloc) keeps the segment
// records and per-chain state that a caller's workspace holds for
// a2c_lrmsd_forward in this fixed array instead; every device holds its own
// copy from module load until the process ends.  In host code the name
// `scratch` is a host-side stand-in, not a device address: the address is
// taken once per device (lrmsd_scratch_setup, at plan creation, with that
// device current) and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[A2C_LRMSD_STATIC_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxScratchDevices];  // device address of `scratch`, per device
}  // namespace

a2c_status lrmsd_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return A2C_OK;  // the entry point reports it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return A2C_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(LRMSD scratch)");
    g_scratch_dev[device] = ptr;
    return A2C_OK;
}

static void *lrmsd_scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

// Segments of at most kLrSegAtoms atoms (the sums) and pieces of at most
// kLrPieceAtoms (the gradient), never across a chain boundary.
void build_lrmsd_segments(a2c_plan &p)
{
    p.lr_seg_atom.clear();
    p.lr_seg_origin.clear();
    p.lr_piece_atom.clear();
    p.lr_piece_chain.clear();
    p.lr_chain_seg.assign(p.n_chains + 1, 0);
    for (int32_t c = 0; c < p.n_chains; ++c) {
        p.lr_chain_seg[c] = (int32_t)p.lr_seg_origin.size();
        for (int64_t a = p.chain_atom_off[c]; a < p.chain_atom_off[c + 1]; a += kLrSegAtoms) {
            p.lr_seg_atom.push_back((int32_t)a);
            p.lr_seg_origin.push_back(p.chain_atom_off[c]);
        }
        for (int64_t a = p.chain_atom_off[c]; a < p.chain_atom_off[c + 1]; a += kLrPieceAtoms) {
            p.lr_piece_atom.push_back((int32_t)a);
            p.lr_piece_chain.push_back(c);
        }
    }
    p.lr_chain_seg[p.n_chains] = (int32_t)p.lr_seg_origin.size();
    p.lr_n_seg = (int32_t)p.lr_seg_origin.size();
    p.lr_seg_atom.push_back((int32_t)p.A);
    p.lr_n_piece = (int32_t)p.lr_piece_chain.size();
    p.lr_piece_atom.push_back((int32_t)p.A);
}

}  // namespace a2c

using namespace a2c;

extern "C" {

a2c_status a2c_lrmsd_workspace_bytes(const a2c_plan *p, size_t *bytes)
{
    if (!p || !bytes) {
        set_error("plan or bytes is NULL");
        return A2C_ERR_INVALID_ARG;
    }
    *bytes = lrmsd_workspace_bytes(*p);
    return A2C_OK;
}

static a2c_status lr_check(const a2c_plan *p, void *ws)
{
    if (!p) {
        set_error("plan is NULL");
        return A2C_ERR_INVALID_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
        set_error("current device is not the plan's device");
        return A2C_ERR_STATE;
    }
    if (!lr_ready(p)) {
        set_error("plan has no LRMSD segment tables");
        return A2C_ERR_STATE;
    }
    // a launch's work-items are counted in 32 bits
    if ((uint64_t)p->lr_n_piece * kLrThreads > 0xFFFFFFFFull) {
        set_error("too many LRMSD pieces for one launch");
        return A2C_ERR_UNSUPPORTED;
    }
    if (!ws && lrmsd_workspace_bytes(*p) > 0) {
        set_error("the LRMSD workspace is NULL");
        return A2C_ERR_WORKSPACE;
    }
    return A2C_OK;
}

// The forward's two kernels with the segment records and per-chain state in
// `ws` (a caller's workspace or the static scratch).
static a2c_status lr_forward_launch(a2c_plan *p, const float *d_coords, const float *d_target,
                                    float *d_lrmsd, void *ws, hipStream_t s)
{
    if (p->n_chains == 0) return A2C_OK;
    if (!d_lrmsd || (p->A > 0 && (!d_coords || !d_target))) {
        set_error("a device pointer is NULL");
        return A2C_ERR_INVALID_ARG;
    }
    double *part = (double *)ws;
    float *state = (float *)((char *)ws + (size_t)p->lr_n_seg * kLrPart * sizeof(double));
    if (p->lr_n_seg > 0)
        hipLaunchKernelGGL(lr_partial_kernel, dim3(p->lr_n_seg), dim3(kLrThreads), 0, s, d_coords,
                           d_target, p->d_lr_seg_atom, p->d_lr_seg_origin, p->A, part);
    hipLaunchKernelGGL(lr_solve_kernel,
                       dim3((p->n_chains + kLrSolveThreads - 1) / kLrSolveThreads),
                       dim3(kLrSolveThreads), 0, s, d_coords, d_target, p->d_lr_seg_atom,
                       p->d_lr_chain_seg, p->n_chains, p->A, part, state, d_lrmsd);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? A2C_OK : hip_fail(e, "lrmsd forward launch");
}

a2c_status a2c_lrmsd_forward(a2c_plan *p, const float *d_coords, const float *d_target,
                             float *d_lrmsd, void *d_workspace, void *stream)
{
    const a2c_status st = lr_check(p, d_workspace);
    if (st != A2C_OK) return st;
    return lr_forward_launch(p, d_coords, d_target, d_lrmsd, d_workspace, (hipStream_t)stream);
}

a2c_status a2c_lrmsd_forward_noalloc(a2c_plan *p, const float *d_coords, const float *d_target,
                                     float *d_lrmsd, void *stream)
{
    if (!p) {
        set_error("plan is NULL");
        return A2C_ERR_INVALID_ARG;
    }
    const size_t need = lrmsd_workspace_bytes(*p);
    if (need > (size_t)A2C_LRMSD_STATIC_BYTES) {
        set_error("the plan's LRMSD state needs " + std::to_string(need) +
                  " bytes; the static scratch holds " +
                  std::to_string((size_t)A2C_LRMSD_STATIC_BYTES));
        return A2C_ERR_WORKSPACE;
    }
    void *ws = lrmsd_scratch_ptr(p->device);
    if (!ws) {
        set_error("no static LRMSD scratch on device " + std::to_string(p->device));
        return A2C_ERR_STATE;
    }
    const a2c_status st = lr_check(p, ws);
    if (st != A2C_OK) return st;
    return lr_forward_launch(p, d_coords, d_target, d_lrmsd, ws, (hipStream_t)stream);
}

a2c_status a2c_lrmsd_backward(a2c_plan *p, const float *d_coords, const float *d_target,
                              const float *d_grad_lrmsd, float *d_grad_coords,
                              const void *d_workspace, void *stream)
{
    a2c_status st = lr_check(p, (void *)d_workspace);
    if (st != A2C_OK) return st;
    if (p->lr_n_piece == 0) return A2C_OK;
    if (!d_coords || !d_target || !d_grad_lrmsd || !d_grad_coords) {
        set_error("a device pointer is NULL");
        return A2C_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const float *state =
        (const float *)((const char *)d_workspace + (size_t)p->lr_n_seg * kLrPart * sizeof(double));
    hipLaunchKernelGGL(lr_grad_kernel, dim3(p->lr_n_piece), dim3(kLrThreads), 0, s, d_coords,
                       d_target, p->d_lr_piece_atom, p->d_lr_piece_chain, p->A, state,
                       d_grad_lrmsd, d_grad_coords);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? A2C_OK : hip_fail(e, "lrmsd backward launch");
}

}  // extern "C"
