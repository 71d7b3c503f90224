/*
 * FP64 CPU oracle, full-atom model ("Full-atom model" section of
 * arXiv:1812.01108).  TEST INFRASTRUCTURE ONLY (see a2c_oracle.c).
 *
 * Per residue the graph of transforms is
 *   M_N  = M_C(previous residue) R(omega)          (identity before the chain)
 *   M_CA = M_N  R(phi)
 *   M_C  = M_CA R(psi)
 *   M_f  = M_parent(f) R_x(pre_f) R(chi_f or 0, theta_f, d_f)   side frames
 * and every atom is r = M_frame(atom) r°.  The spine is exactly the backbone
 * chain of the backbone model, so backbone atoms of the two models agree.
 *
 * Gradient, for L = sum_k g_k . r_k:
 *   direct  : Eq. FAMBackward, F_i = M_parent(i) [R_x(pre)] dR_i M_i^-1 and
 *             dL/dalpha_i = sum over atoms k in the subtree of node i of
 *             g_k . (F_i r_k)  (O(N^2) over the chain);
 *   closed  : dL/dalpha_i = u_i . sum_{k in subtree(i)} (r_k - o_i) x g_k with
 *             o_i, u_i the origin and x axis of M_i (O(N)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NT 20
#define MS 4
#define MA 14
#define PI_D 3.14159265358979323846

typedef struct {
    int32_t n_atoms[NT];
    int32_t n_side[NT];
    int32_t side_parent[NT][MS];   /* 1 = CA frame, 3 + f = side frame f */
    int32_t side_chi[NT][MS];      /* 1..4, or 0 for a fixed torsion of 0 */
    double side_pre[NT][MS];       /* radians */
    double side_theta[NT][MS];     /* radians */
    double side_d[NT][MS];
    int32_t atom_frame[NT][MA];    /* 0 N, 1 CA, 2 C, 3 + f */
    double atom_r[NT][MA][3];      /* r° in that frame */
} oracle_table;

void oracle_transform(double alpha, double theta, double d, double out[16]);

static void fa_identity(double m[16])
{
    memset(m, 0, 16 * sizeof(double));
    m[0] = m[5] = m[10] = m[15] = 1.0;
}

static void fa_mul(const double A[16], const double B[16], double C[16])
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

static void fa_rx(double a, double m[16])
{
    fa_identity(m);
    m[5] = cos(a); m[6] = -sin(a);
    m[9] = sin(a); m[10] = cos(a);
}

static void fa_dtransform(double alpha, double theta, double out[16])
{
    const double ca = cos(alpha), sa = sin(alpha), ct = cos(theta), st = sin(theta);
    memset(out, 0, 16 * sizeof(double));
    out[1] = ca * st;  out[2] = -sa * st;
    out[5] = -sa;      out[6] = -ca;
    out[9] = ca * ct;  out[10] = -sa * ct;
}

static void fa_rigid_inverse(const double M[16], double out[16])
{
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) out[4 * r + c] = M[4 * c + r];
        out[4 * r + 3] = -(M[0 + r] * M[3] + M[4 + r] * M[7] + M[8 + r] * M[11]);
    }
    out[12] = out[13] = out[14] = 0.0;
    out[15] = 1.0;
}

static void fa_point(const double M[16], const double p[3], double y[3])
{
    for (int r = 0; r < 3; ++r)
        y[r] = M[4 * r] * p[0] + M[4 * r + 1] * p[1] + M[4 * r + 2] * p[2] + M[4 * r + 3];
}

static int fa_threads(int n)
{
#ifdef _OPENMP
    return n > 0 ? n : omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Frames of one residue: fr[0..2] spine (N, CA, C), fr[3 + f] side frames.
 * `prevC` is the C frame of the previous residue (identity at chain start);
 * `pre_alpha[k]` receives, for node k, the matrix M_parent [R_x(pre)] that
 * multiplies R(alpha_k) (needed by the direct gradient). */
static void residue_frames(const oracle_table *tab, int t, const double *prevC,
                           double phi, double psi, double omega, const double chi[4],
                           const double theta[3], const double dlen[3],
                           double fr[7][16], double pre_alpha[7][16], double alpha[7],
                           double th[7], double dd[7])
{
    double T[16];
    /* N */
    memcpy(pre_alpha[0], prevC, sizeof(double) * 16);
    alpha[0] = omega; th[0] = theta[0]; dd[0] = dlen[0];
    oracle_transform(omega, theta[0], dlen[0], T);
    fa_mul(prevC, T, fr[0]);
    /* CA */
    memcpy(pre_alpha[1], fr[0], sizeof(double) * 16);
    alpha[1] = phi; th[1] = theta[1]; dd[1] = dlen[1];
    oracle_transform(phi, theta[1], dlen[1], T);
    fa_mul(fr[0], T, fr[1]);
    /* C */
    memcpy(pre_alpha[2], fr[1], sizeof(double) * 16);
    alpha[2] = psi; th[2] = theta[2]; dd[2] = dlen[2];
    oracle_transform(psi, theta[2], dlen[2], T);
    fa_mul(fr[1], T, fr[2]);
    for (int f = 0; f < tab->n_side[t]; ++f) {
        const int k = 3 + f;
        double P[16], Rx[16];
        fa_rx(tab->side_pre[t][f], Rx);
        fa_mul(fr[tab->side_parent[t][f]], Rx, P);
        memcpy(pre_alpha[k], P, sizeof(P));
        const int c = tab->side_chi[t][f];
        alpha[k] = c > 0 ? chi[c - 1] : 0.0;
        th[k] = tab->side_theta[t][f];
        dd[k] = tab->side_d[t][f];
        oracle_transform(alpha[k], th[k], dd[k], T);
        fa_mul(P, T, fr[k]);
    }
}

static void bb_theta(const double geom[6], double theta[3], double d[3])
{
    for (int s = 0; s < 3; ++s) {
        d[s] = geom[2 * s];
        theta[s] = PI_D - geom[2 * s + 1] * (PI_D / 180.0);
    }
}

int oracle_fullatom_forward(int32_t n_chains, const int32_t *res_off, const uint8_t *seq,
                            const double *angles, const double geom[6], const oracle_table *tab,
                            const int32_t *res_atom_off, double *coords, int n_threads)
{
    const int64_t R = res_off[n_chains];
    const int64_t A = res_atom_off[R];
    double theta[3], dlen[3];
    bb_theta(geom, theta, dlen);
#pragma omp parallel for schedule(dynamic) num_threads(fa_threads(n_threads))
    for (int32_t c = 0; c < n_chains; ++c) {
        double prevC[16];
        fa_identity(prevC);
        for (int64_t j = res_off[c]; j < res_off[c + 1]; ++j) {
            const int t = seq[j];
            double fr[7][16], pa[7][16], al[7], th[7], dd[7];
            const double chi[4] = {angles[3 * R + j], angles[4 * R + j], angles[5 * R + j],
                                   angles[6 * R + j]};
            residue_frames(tab, t, prevC, angles[j], angles[R + j], angles[2 * R + j], chi, theta,
                           dlen, fr, pa, al, th, dd);
            for (int a = 0; a < tab->n_atoms[t]; ++a) {
                double y[3];
                fa_point(fr[tab->atom_frame[t][a]], tab->atom_r[t][a], y);
                const int64_t k = res_atom_off[j] + a;
                coords[k] = y[0];
                coords[A + k] = y[1];
                coords[2 * A + k] = y[2];
            }
            memcpy(prevC, fr[2], sizeof(prevC));
        }
    }
    return 0;
}

/* angle plane of node k of a residue of type t (-1: no gradient) */
static int node_plane(const oracle_table *tab, int t, int k)
{
    if (k == 0) return 2;  /* omega */
    if (k == 1) return 0;  /* phi */
    if (k == 2) return 1;  /* psi */
    const int c = tab->side_chi[t][k - 3];
    return c > 0 ? 2 + c : -1;
}

/* is frame `f` (frame id) in the subtree of node `k` within one residue */
static int in_subtree(const oracle_table *tab, int t, int k, int f)
{
    while (1) {
        if (f == k) return 1;
        if (f <= 1) return k == 0 && f == 1;   /* N's subtree holds CA's */
        if (f == 2) f = 1;                     /* C hangs off CA */
        else f = tab->side_parent[t][f - 3];
    }
}

int oracle_fullatom_backward(int32_t n_chains, const int32_t *res_off, const uint8_t *seq,
                             const double *angles, const double geom[6], const oracle_table *tab,
                             const int32_t *res_atom_off, const double *grad_coords,
                             double *grad_angles, int direct, int n_threads)
{
    const int64_t R = res_off[n_chains];
    const int64_t A = res_atom_off[R];
    double theta[3], dlen[3];
    bb_theta(geom, theta, dlen);
    for (int p = 0; p < 7; ++p)
        for (int64_t j = 0; j < R; ++j) grad_angles[p * R + j] = 0.0;
    int err = 0;
#pragma omp parallel for schedule(dynamic) num_threads(fa_threads(n_threads))
    for (int32_t c = 0; c < n_chains; ++c) {
        const int64_t r0 = res_off[c], L = res_off[c + 1] - r0;
        if (L == 0) continue;
        /* frames and atoms of the whole chain */
        double(*fr)[7][16] = malloc(sizeof(double) * 7 * 16 * L);
        double(*pa)[7][16] = malloc(sizeof(double) * 7 * 16 * L);
        double(*al)[7] = malloc(sizeof(double) * 7 * L);
        double(*th)[7] = malloc(sizeof(double) * 7 * L);
        double(*dd)[7] = malloc(sizeof(double) * 7 * L);
        const int64_t a0 = res_atom_off[r0], na = res_atom_off[r0 + L] - a0;
        double *r = malloc(sizeof(double) * 3 * (na > 0 ? na : 1));
        if (!fr || !pa || !al || !th || !dd || !r) {
#pragma omp atomic write
            err = -1;
            free(fr); free(pa); free(al); free(th); free(dd); free(r);
            continue;
        }
        double prevC[16];
        fa_identity(prevC);
        for (int64_t j = 0; j < L; ++j) {
            const int64_t rj = r0 + j;
            const int t = seq[rj];
            const double chi[4] = {angles[3 * R + rj], angles[4 * R + rj], angles[5 * R + rj],
                                   angles[6 * R + rj]};
            residue_frames(tab, t, prevC, angles[rj], angles[R + rj], angles[2 * R + rj], chi,
                           theta, dlen, fr[j], pa[j], al[j], th[j], dd[j]);
            for (int a = 0; a < tab->n_atoms[t]; ++a)
                fa_point(fr[j][tab->atom_frame[t][a]], tab->atom_r[t][a],
                         r + 3 * (res_atom_off[rj] + a - a0));
            memcpy(prevC, fr[j][2], sizeof(prevC));
        }
        if (direct) {
            for (int64_t j = 0; j < L; ++j) {
                const int64_t rj = r0 + j;
                const int t = seq[rj];
                for (int k = 0; k < 3 + tab->n_side[t]; ++k) {
                    const int plane = node_plane(tab, t, k);
                    if (plane < 0) continue;
                    double dR[16], inv[16], F[16];
                    fa_dtransform(al[j][k], th[j][k], dR);
                    fa_rigid_inverse(fr[j][k], inv);
                    fa_mul(pa[j][k], dR, F);
                    fa_mul(F, inv, F);
                    double acc = 0.0;
                    /* atoms of this residue in the subtree of node k */
                    for (int a = 0; a < tab->n_atoms[t]; ++a) {
                        if (!in_subtree(tab, t, k, tab->atom_frame[t][a])) continue;
                        const int64_t ka = res_atom_off[rj] + a;
                        double v[3];
                        fa_point(F, r + 3 * (ka - a0), v);
                        acc += grad_coords[ka] * v[0] + grad_coords[A + ka] * v[1] +
                               grad_coords[2 * A + ka] * v[2];
                    }
                    /* spine nodes carry every later residue */
                    if (k <= 2) {
                        for (int64_t ka = res_atom_off[rj + 1]; ka < a0 + na; ++ka) {
                            double v[3];
                            fa_point(F, r + 3 * (ka - a0), v);
                            acc += grad_coords[ka] * v[0] + grad_coords[A + ka] * v[1] +
                                   grad_coords[2 * A + ka] * v[2];
                        }
                    }
                    grad_angles[plane * R + rj] = acc;
                }
            }
        } else {
            /* closed form with subtree sums; S = wrench of everything after
             * the current residue's C group */
            double Sg[3] = {0, 0, 0}, Sm[3] = {0, 0, 0};
            for (int64_t j = L - 1; j >= 0; --j) {
                const int64_t rj = r0 + j;
                const int t = seq[rj];
                double Wg[7][3], Wm[7][3];   /* per-node own-group wrench */
                memset(Wg, 0, sizeof(Wg));
                memset(Wm, 0, sizeof(Wm));
                for (int a = 0; a < tab->n_atoms[t]; ++a) {
                    const int64_t ka = res_atom_off[rj] + a;
                    const double *p = r + 3 * (ka - a0);
                    const double g[3] = {grad_coords[ka], grad_coords[A + ka], grad_coords[2 * A + ka]};
                    const int f = tab->atom_frame[t][a];
                    Wg[f][0] += g[0]; Wg[f][1] += g[1]; Wg[f][2] += g[2];
                    Wm[f][0] += p[1] * g[2] - p[2] * g[1];
                    Wm[f][1] += p[2] * g[0] - p[0] * g[2];
                    Wm[f][2] += p[0] * g[1] - p[1] * g[0];
                }
                /* fold side frames into their parents, deepest first */
                for (int f = tab->n_side[t] - 1; f >= 0; --f) {
                    const int k = 3 + f;
                    const int plane = node_plane(tab, t, k);
                    if (plane >= 0) {
                        const double *M = fr[j][k];
                        const double o[3] = {M[3], M[7], M[11]}, u[3] = {M[0], M[4], M[8]};
                        const double tq[3] = {Wm[k][0] - (o[1] * Wg[k][2] - o[2] * Wg[k][1]),
                                              Wm[k][1] - (o[2] * Wg[k][0] - o[0] * Wg[k][2]),
                                              Wm[k][2] - (o[0] * Wg[k][1] - o[1] * Wg[k][0])};
                        grad_angles[plane * R + rj] = u[0] * tq[0] + u[1] * tq[1] + u[2] * tq[2];
                    }
                    const int par = tab->side_parent[t][f];
                    for (int q = 0; q < 3; ++q) {
                        Wg[par][q] += Wg[k][q];
                        Wm[par][q] += Wm[k][q];
                    }
                }
                /* spine: C group, then CA (with side chain), then N */
                const int order[3] = {2, 1, 0};
                for (int s = 0; s < 3; ++s) {
                    const int k = order[s];
                    for (int q = 0; q < 3; ++q) {
                        Sg[q] += Wg[k][q];
                        Sm[q] += Wm[k][q];
                    }
                    const double *M = fr[j][k];
                    const double o[3] = {M[3], M[7], M[11]}, u[3] = {M[0], M[4], M[8]};
                    const double tq[3] = {Sm[0] - (o[1] * Sg[2] - o[2] * Sg[1]),
                                          Sm[1] - (o[2] * Sg[0] - o[0] * Sg[2]),
                                          Sm[2] - (o[0] * Sg[1] - o[1] * Sg[0])};
                    grad_angles[node_plane(tab, t, k) * R + rj] =
                        u[0] * tq[0] + u[1] * tq[1] + u[2] * tq[2];
                }
            }
        }
        free(fr); free(pa); free(al); free(th); free(dd); free(r);
    }
    return err;
}
