/*
 * FP64 CPU oracle for the map from dihedral angles to Cartesian coordinates
 * (Derevyanko & Lamoureux, "TorchProteinLibrary", arXiv:1812.01108).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may link,
 * load or call this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table
 * derivation or helper with the GPU library.
 *
 * Everything is plain double precision with explicit 4x4 homogeneous
 * matrices, written to be checked against the paper by eye:
 *
 *   transform      R(alpha, theta, d), the 4x4 matrix printed in the
 *                  "Backbone model" section (= Ry(theta) Tx(d) Rx(alpha) of
 *                  the "Full-atom model" section).
 *   forward        M_i = R_0 R_1 ... R_i and r_i = M_i 0 ("Backbone model"),
 *                  M_node = M_parent R_node and r = M r° ("Full-atom model").
 *   gradient       two forms: the paper's own expression
 *                    dL/dalpha_i = sum_k g_k . (M_parent dR_i/dalpha M_i^-1 r_k)
 *                  over every atom k downstream of node i (Eq. BackboneGradOutput
 *                  and Eq. FAMBackward, O(N^2)), and the equivalent O(N) closed
 *                  form  u_i . sum_k (r_k - r_i) x g_k  with u_i the x axis of
 *                  M_i, which follows from M_parent dR_i M_i^-1 = M_i G_x M_i^-1
 *                  (G_x the generator of rotations about x).  The closed form is
 *                  pinned by the test suite against the paper's form and
 *                  against central finite differences of the forward.
 *
 * Readings of the paper used here (each is listed with its reason in the
 * design notes):
 *   - backbone constants are vertex-named: the transform placing atom i uses
 *     the bond length (i-1, i) and theta = pi - (bond angle at atom i-1);
 *   - per residue j the three transforms are, in order, omega_j (places N_j),
 *     phi_j (places CA_j), psi_j (places C_j); the chain starts from the
 *     identity frame, so N_0 = (d cos theta, 0, -d sin theta);
 *   - omega is read from the input and receives a gradient;
 *   - "children(i)" in Eq. FAMBackward means every atom in the subtree of node
 *     i, the node's own rigid group included, and the matrix there is
 *     M_parent(i) dR_i M_i^-1.
 *
 * Layouts (all ragged over chains through int32 residue offsets):
 *   angles  [K][R]   planes phi, psi, omega (, chi1..chi4), radians
 *   coords  [3][A]   x plane, y plane, z plane
 *   grads   [K][R]   same planes as angles
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI_D 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* 4x4 homogeneous matrices, row-major                                       */
/* ------------------------------------------------------------------------ */

/* R(alpha, theta, d) exactly as printed in the "Backbone model" section. */
void oracle_transform(double alpha, double theta, double d, double out[16])
{
    const double ca = cos(alpha), sa = sin(alpha);
    const double ct = cos(theta), st = sin(theta);
    out[0] = ct;   out[1] = sa * st; out[2] = ca * st;  out[3] = d * ct;
    out[4] = 0.0;  out[5] = ca;      out[6] = -sa;      out[7] = 0.0;
    out[8] = -st;  out[9] = sa * ct; out[10] = ca * ct; out[11] = -d * st;
    out[12] = 0.0; out[13] = 0.0;    out[14] = 0.0;     out[15] = 1.0;
}

/* d R(alpha, theta, d) / d alpha, entry by entry from the printed matrix. */
static void transform_dalpha(double alpha, double theta, double out[16])
{
    const double ca = cos(alpha), sa = sin(alpha);
    const double ct = cos(theta), st = sin(theta);
    out[0] = 0.0;  out[1] = ca * st;  out[2] = -sa * st;  out[3] = 0.0;
    out[4] = 0.0;  out[5] = -sa;      out[6] = -ca;       out[7] = 0.0;
    out[8] = 0.0;  out[9] = ca * ct;  out[10] = -sa * ct; out[11] = 0.0;
    out[12] = 0.0; out[13] = 0.0;     out[14] = 0.0;      out[15] = 0.0;
}

static void mat_identity(double m[16])
{
    memset(m, 0, 16 * sizeof(double));
    m[0] = m[5] = m[10] = m[15] = 1.0;
}

/* C = A B */
static void mat_mul(const double A[16], const double B[16], double C[16])
{
    double T[16];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += A[4 * r + k] * B[4 * k + c];
            T[4 * r + c] = s;
        }
    memcpy(C, T, sizeof(T));
}

/* Inverse of a rigid transform [Rot t; 0 1]: [Rot^T, -Rot^T t; 0 1]
 * (the "simple form" of M^-1 the backbone section mentions). */
static void mat_rigid_inverse(const double M[16], double out[16])
{
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) out[4 * r + c] = M[4 * c + r];
        out[4 * r + 3] = -(M[0 + r] * M[3] + M[4 + r] * M[7] + M[8 + r] * M[11]);
    }
    out[12] = out[13] = out[14] = 0.0;
    out[15] = 1.0;
}

/* y = M (p, 1), xyz part */
static void mat_apply_point(const double M[16], const double p[3], double y[3])
{
    for (int r = 0; r < 3; ++r)
        y[r] = M[4 * r] * p[0] + M[4 * r + 1] * p[1] + M[4 * r + 2] * p[2] + M[4 * r + 3];
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static int pick_threads(int n_threads)
{
#ifdef _OPENMP
    return n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    (void)n_threads;
    return 1;
#endif
}

int oracle_openmp_enabled(void)
{
#ifdef _OPENMP
    return 1;
#else
    return 0;
#endif
}

/* ------------------------------------------------------------------------ */
/* Backbone model                                                           */
/* ------------------------------------------------------------------------ */

/*
 * geom[6] = { d_N, angle_N, d_CA, angle_CA, d_C, angle_C }: for each slot
 * (the transform placing N, CA, C of a residue) the bond length to the atom
 * before it and the bond angle (degrees) at the atom before it:
 *   N  : bond C-N,   angle CA-C-N
 *   CA : bond N-CA,  angle C-N-CA
 *   C  : bond CA-C,  angle N-CA-C
 * theta of the transform is pi minus that bond angle.
 */
typedef struct { double d[3]; double theta[3]; } bb_geom;

static bb_geom bb_geom_from(const double geom[6])
{
    bb_geom g;
    for (int s = 0; s < 3; ++s) {
        g.d[s] = geom[2 * s];
        g.theta[s] = PI_D - geom[2 * s + 1] * (PI_D / 180.0);
    }
    return g;
}

/* Angle plane read by slot s of a residue: omega (plane 2) places N,
 * phi (plane 0) places CA, psi (plane 1) places C. */
static const int BB_SLOT_PLANE[3] = {2, 0, 1};

/* Frames M_i (16 doubles each) of one chain of L residues starting at
 * residue r0: the plain running product from the identity. */
static void bb_chain_frames(const double *angles, int64_t R, int64_t r0, int64_t L,
                            const bb_geom *g, double *M /* [3L][16] */)
{
    double cur[16], T[16];
    mat_identity(cur);
    for (int64_t j = 0; j < L; ++j)
        for (int s = 0; s < 3; ++s) {
            const double alpha = angles[BB_SLOT_PLANE[s] * R + r0 + j];
            oracle_transform(alpha, g->theta[s], g->d[s], T);
            mat_mul(cur, T, cur);
            memcpy(M + 16 * (3 * j + s), cur, sizeof(cur));
        }
}

int oracle_backbone_forward(int32_t n_chains, const int32_t *res_off,
                            const double *angles, const double geom[6],
                            double *coords, int n_threads)
{
    const int64_t R = res_off[n_chains];
    const int64_t A = 3 * R;
    const bb_geom g = bb_geom_from(geom);
#pragma omp parallel for schedule(dynamic) num_threads(pick_threads(n_threads))
    for (int32_t c = 0; c < n_chains; ++c) {
        double cur[16], T[16];
        mat_identity(cur);
        for (int64_t j = res_off[c]; j < res_off[c + 1]; ++j)
            for (int s = 0; s < 3; ++s) {
                const double alpha = angles[BB_SLOT_PLANE[s] * R + j];
                oracle_transform(alpha, g.theta[s], g.d[s], T);
                mat_mul(cur, T, cur);
                const int64_t a = 3 * j + s;
                coords[a] = cur[3];
                coords[A + a] = cur[7];
                coords[2 * A + a] = cur[11];
            }
    }
    return 0;
}

/* The paper's gradient expression, O(N^2) per chain: for transform i,
 * F_i = M_{i-1} dR_i/dalpha M_i^{-1} (M_{-1} = I) and
 * dL/dalpha_i = sum over atoms k >= i of g_k . (F_i r_k). */
int oracle_backbone_backward_direct(int32_t n_chains, const int32_t *res_off,
                                    const double *angles, const double geom[6],
                                    const double *grad_coords, double *grad_angles)
{
    const int64_t R = res_off[n_chains];
    const int64_t A = 3 * R;
    const bb_geom g = bb_geom_from(geom);
    for (int32_t c = 0; c < n_chains; ++c) {
        const int64_t r0 = res_off[c], L = res_off[c + 1] - r0;
        if (L == 0) continue;
        double *M = (double *)malloc(sizeof(double) * 16 * 3 * L);
        if (!M) return -1;
        bb_chain_frames(angles, R, r0, L, &g, M);
        for (int64_t i = 0; i < 3 * L; ++i) {
            const int s = (int)(i % 3);
            const double alpha = angles[BB_SLOT_PLANE[s] * R + r0 + i / 3];
            double Mprev[16], dR[16], Minv[16], F[16];
            if (i == 0) mat_identity(Mprev);
            else memcpy(Mprev, M + 16 * (i - 1), sizeof(Mprev));
            transform_dalpha(alpha, g.theta[s], dR);
            mat_rigid_inverse(M + 16 * i, Minv);
            mat_mul(Mprev, dR, F);
            mat_mul(F, Minv, F);
            double acc = 0.0;
            for (int64_t k = i; k < 3 * L; ++k) {
                const int64_t a = 3 * r0 + k;
                const double rk[3] = {M[16 * k + 3], M[16 * k + 7], M[16 * k + 11]};
                double v[3];
                mat_apply_point(F, rk, v);
                acc += grad_coords[a] * v[0] + grad_coords[A + a] * v[1] +
                       grad_coords[2 * A + a] * v[2];
            }
            grad_angles[BB_SLOT_PLANE[s] * R + r0 + i / 3] = acc;
        }
        free(M);
    }
    return 0;
}

/* O(N) closed form: dL/dalpha_i = u_i . (S_rg(i) - r_i x S_g(i)) with
 * S_g(i) = sum_{k>i} g_k, S_rg(i) = sum_{k>i} r_k x g_k, u_i = M_i e_x. */
int oracle_backbone_backward(int32_t n_chains, const int32_t *res_off,
                             const double *angles, const double geom[6],
                             const double *grad_coords, double *grad_angles,
                             int n_threads)
{
    const int64_t R = res_off[n_chains];
    const int64_t A = 3 * R;
    const bb_geom g = bb_geom_from(geom);
    int err = 0;
#pragma omp parallel for schedule(dynamic) num_threads(pick_threads(n_threads))
    for (int32_t c = 0; c < n_chains; ++c) {
        const int64_t r0 = res_off[c], L = res_off[c + 1] - r0;
        if (L == 0) continue;
        double *M = (double *)malloc(sizeof(double) * 16 * 3 * L);
        if (!M) {
#pragma omp atomic write
            err = -1;
            continue;
        }
        bb_chain_frames(angles, R, r0, L, &g, M);
        double Sg[3] = {0, 0, 0}, Srg[3] = {0, 0, 0};
        for (int64_t i = 3 * L - 1; i >= 0; --i) {
            const double *Mi = M + 16 * i;
            const double r[3] = {Mi[3], Mi[7], Mi[11]};
            const double u[3] = {Mi[0], Mi[4], Mi[8]};
            double rxS[3], t[3];
            cross3(r, Sg, rxS);
            for (int q = 0; q < 3; ++q) t[q] = Srg[q] - rxS[q];
            const int s = (int)(i % 3);
            grad_angles[BB_SLOT_PLANE[s] * R + r0 + i / 3] = dot3(u, t);
            const int64_t a = 3 * r0 + i;
            const double gk[3] = {grad_coords[a], grad_coords[A + a], grad_coords[2 * A + a]};
            double rxg[3];
            cross3(r, gk, rxg);
            for (int q = 0; q < 3; ++q) {
                Sg[q] += gk[q];
                Srg[q] += rxg[q];
            }
        }
        free(M);
    }
    return err;
}
