"""Independent geometry used by the pins: dihedrals, bond angles, screw
parameters of a helix and textbook rotation matrices.  Written from the
definitions, not from the oracle or the library."""
from __future__ import annotations

import numpy as np


def dihedral(p0, p1, p2, p3):
    """IUPAC torsion angle p0-p1-p2-p3 in radians, (-pi, pi]; vectorised over
    leading axes.  atan2(|b2| b1.(b2 x b3), (b1 x b2).(b2 x b3))."""
    b1 = np.asarray(p1) - np.asarray(p0)
    b2 = np.asarray(p2) - np.asarray(p1)
    b3 = np.asarray(p3) - np.asarray(p2)
    n1 = np.cross(b1, b2)
    n2 = np.cross(b2, b3)
    y = np.linalg.norm(b2, axis=-1) * np.sum(b1 * n2, axis=-1)
    x = np.sum(n1 * n2, axis=-1)
    return np.arctan2(y, x)


def bond_angle(a, b, c):
    """Angle a-b-c at vertex b, radians."""
    u = np.asarray(a) - np.asarray(b)
    v = np.asarray(c) - np.asarray(b)
    cosv = np.sum(u * v, axis=-1) / (np.linalg.norm(u, axis=-1) * np.linalg.norm(v, axis=-1))
    return np.arccos(np.clip(cosv, -1.0, 1.0))


def wrapped_diff(a, b):
    """a - b wrapped to (-pi, pi]."""
    d = np.asarray(a) - np.asarray(b)
    return np.pi - np.mod(np.pi - d, 2.0 * np.pi)


def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0, 0], [0, c, -s, 0], [0, s, c, 0], [0, 0, 0, 1.0]])


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s, 0], [0, 1, 0, 0], [-s, 0, c, 0], [0, 0, 0, 1.0]])


def trans_x(d):
    m = np.eye(4)
    m[0, 3] = d
    return m


def residue_frame(n, ca, c):
    """Orthonormal frame (columns) from N, CA, C of one residue."""
    e1 = ca - n
    e1 = e1 / np.linalg.norm(e1)
    v = (c - ca) - np.dot(c - ca, e1) * e1
    e2 = v / np.linalg.norm(v)
    e3 = np.cross(e1, e2)
    return np.stack([e1, e2, e3], axis=1)


def screw_parameters(xyz_res):
    """Residues per turn, rise per residue (A) and handedness sign of the
    rigid motion taking residue j to residue j+1.  xyz_res: [L][3 atoms][3].
    Uses residues in the middle of the chain."""
    j = len(xyz_res) // 2
    F0 = residue_frame(*xyz_res[j])
    F1 = residue_frame(*xyz_res[j + 1])
    Q = F1 @ F0.T
    kappa = np.arccos(np.clip((np.trace(Q) - 1.0) / 2.0, -1.0, 1.0))
    axis = np.array([Q[2, 1] - Q[1, 2], Q[0, 2] - Q[2, 0], Q[1, 0] - Q[0, 1]]) / (2.0 * np.sin(kappa))
    t = xyz_res[j + 1][1] - Q @ xyz_res[j][1]
    rise = float(np.dot(t, axis))
    return 2.0 * np.pi / kappa, rise, Q, t


def coords_by_residue(coords, r0, L):
    """[3][A] planes -> [L][3 atoms][xyz] for backbone chain residues r0..r0+L."""
    a = coords[:, 3 * r0: 3 * (r0 + L)].T
    return a.reshape(L, 3, 3)
