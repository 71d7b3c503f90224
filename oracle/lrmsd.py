"""FP64 oracle of the LRMSD loss ("Loss function" section of arXiv:1812.01108).
TEST INFRASTRUCTURE ONLY.

LRMSD(x, y) = min over rigid motions M of sqrt(sum_i |x_i - M y_i|^2 / N),
x the target and y the input structure of one chain.  Two independent
evaluations:
  - kabsch():    centre both, H = sum_i y~_i x~_i^T, SVD, proper rotation
                 (Kabsch 1976 with the determinant correction);
  - quaternion(): the paper's route -- correlation R = sum_i x~_i y~_i^T, the
                 4x4 matrix T built from R as printed, its largest eigenvalue
                 lambda, LRMSD = sqrt((sum |x~|^2 + |y~|^2 - 2 lambda) / N), and
                 the rotation U from the eigenvector q as printed.
With q the eigenvector of the largest eigenvalue and U built from q as
printed, U maps the target onto the input (U x~ ~ y~): it is the transpose
of the Kabsch rotation.  The printed derivative x_i - U^T y_i is therefore
the one with respect to the target x, without the factor 1 / (N LRMSD).
Here the gradient is taken with respect to the input y:
  d LRMSD / d y_i = (y~_i - U x~_i) / (N LRMSD)      (U from q, as printed)
                  = (y~_i - K^T x~_i) / (N LRMSD)    (K the Kabsch rotation).
"""
from __future__ import annotations

import numpy as np


def _center(p):
    return p - p.mean(axis=0, keepdims=True)


def kabsch(x, y):
    """(lrmsd, U) for one chain; x, y: [N, 3] float64; U y~ ~ x~."""
    xc, yc = _center(np.asarray(x, float)), _center(np.asarray(y, float))
    H = yc.T @ xc
    V, S, Wt = np.linalg.svd(H)
    d = np.sign(np.linalg.det(Wt.T @ V.T))
    D = np.diag([1.0, 1.0, d])
    U = Wt.T @ D @ V.T
    diff = xc - yc @ U.T
    return float(np.sqrt(np.sum(diff * diff) / len(x))), U


def paper_T(R):
    """The 4x4 matrix T printed in the Loss function section."""
    return np.array([
        [R[0, 0] + R[1, 1] + R[2, 2], R[1, 2] - R[2, 1], R[2, 0] - R[0, 2], R[0, 1] - R[1, 0]],
        [R[1, 2] - R[2, 1], R[0, 0] - R[1, 1] - R[2, 2], R[0, 1] + R[1, 0], R[0, 2] + R[2, 0]],
        [R[2, 0] - R[0, 2], R[0, 1] + R[1, 0], -R[0, 0] + R[1, 1] - R[2, 2], R[1, 2] + R[2, 1]],
        [R[0, 1] - R[1, 0], R[0, 2] + R[2, 0], R[1, 2] + R[2, 1], -R[0, 0] - R[1, 1] + R[2, 2]]])


def paper_U(q):
    """Rotation matrix from the quaternion q, as printed."""
    q0, q1, q2, q3 = q
    return np.array([
        [q0 * q0 + q1 * q1 - q2 * q2 - q3 * q3, 2 * (q1 * q2 - q0 * q3), 2 * (q1 * q3 + q0 * q2)],
        [2 * (q1 * q2 + q0 * q3), q0 * q0 - q1 * q1 + q2 * q2 - q3 * q3, 2 * (q2 * q3 - q0 * q1)],
        [2 * (q1 * q3 - q0 * q2), 2 * (q2 * q3 + q0 * q1), q0 * q0 - q1 * q1 - q2 * q2 + q3 * q3]])


def quaternion(x, y):
    """(lrmsd, U_paper, lambda) for one chain by the paper's steps."""
    xc, yc = _center(np.asarray(x, float)), _center(np.asarray(y, float))
    R = xc.T @ yc                      # R = sum_i x_i y_i^T
    T = paper_T(R)
    w, v = np.linalg.eigh(T)
    lam, q = w[-1], v[:, -1]
    e0 = np.sum(xc * xc) + np.sum(yc * yc)
    val = max(e0 - 2.0 * lam, 0.0) / len(x)
    return float(np.sqrt(val)), paper_U(q), float(lam)


def lrmsd_batch(x, y, chain_atom_offsets):
    """Per-chain LRMSD for [3][A] planes x (target) and y (input)."""
    off = np.asarray(chain_atom_offsets)
    out = np.zeros(len(off) - 1)
    for c in range(len(off) - 1):
        a0, a1 = off[c], off[c + 1]
        if a1 > a0:
            out[c] = kabsch(x[:, a0:a1].T, y[:, a0:a1].T)[0]
    return out


def lrmsd_grad_batch(x, y, chain_atom_offsets, grad_out):
    """d(sum_c grad_out[c] * LRMSD_c) / dy, planes [3][A]."""
    off = np.asarray(chain_atom_offsets)
    g = np.zeros_like(np.asarray(y, float))
    for c in range(len(off) - 1):
        a0, a1 = off[c], off[c + 1]
        n = a1 - a0
        if n == 0:
            continue
        xs, ys = x[:, a0:a1].T.astype(float), y[:, a0:a1].T.astype(float)
        val, U = kabsch(xs, ys)
        if val == 0.0:
            continue
        xc, yc = _center(xs), _center(ys)
        g[:, a0:a1] = (grad_out[c] * (yc - xc @ U) / (n * val)).T
    return g
