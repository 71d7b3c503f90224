"""FP64 oracle of the inverse map, Cartesian coordinates -> dihedral angles.
TEST INFRASTRUCTURE ONLY (tests, smoke check and the bench's CPU baseline).

The torsion angle of four points (a, b, c, d) is the IUPAC one (IUPAC-IUB
Commission on Biochemical Nomenclature, 1970): the angle between the planes
(a, b, c) and (b, c, d), positive for a clockwise rotation of a-b onto c-d
seen along b -> c; with b1 = b - a, b2 = c - b, b3 = d - c,
  torsion = atan2(|b2| b1 . (b2 x b3), (b1 x b2) . (b2 x b3)).

Backbone ("Backbone model" section): the angle of the transform placing
atom i is the torsion about the bond into atom i, (i-2, i-1, i, i+1), so per
residue j
  omega_j = torsion(CA_{j-1}, C_{j-1}, N_j, CA_j)
  phi_j   = torsion(C_{j-1}, N_j, CA_j, C_j)
  psi_j   = torsion(N_j, CA_j, C_j, N_{j+1}).
At a chain start the identity start frame supplies the virtual atoms
C_{-1} = origin and CA_{-1} = (-1, 0, 0).  psi of a chain's last residue moves
no atom (there is no N_{j+1}) and is returned as 0.

Full-atom: chi_k by the IUPAC atom quadruples of each residue type, looked up
by atom name; planes of chi angles a residue lacks are 0.  Angle planes:
0 phi, 1 psi, 2 omega, 3..6 chi1..chi4.
"""
from __future__ import annotations

import numpy as np

# IUPAC side-chain torsions: four atom names per chi.
IUPAC_CHI = {
    "ARG": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD"), ("CB", "CG", "CD", "NE"),
            ("CG", "CD", "NE", "CZ")],
    "ASN": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "OD1")],
    "ASP": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "OD1")],
    "CYS": [("N", "CA", "CB", "SG")],
    "GLN": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD"), ("CB", "CG", "CD", "OE1")],
    "GLU": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD"), ("CB", "CG", "CD", "OE1")],
    "HIS": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "ND1")],
    "ILE": [("N", "CA", "CB", "CG1"), ("CA", "CB", "CG1", "CD1")],
    "LEU": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD1")],
    "LYS": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD"), ("CB", "CG", "CD", "CE"),
            ("CG", "CD", "CE", "NZ")],
    "MET": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "SD"), ("CB", "CG", "SD", "CE")],
    "PHE": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD1")],
    "PRO": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD")],
    "SER": [("N", "CA", "CB", "OG")],
    "THR": [("N", "CA", "CB", "OG1")],
    "TRP": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD1")],
    "TYR": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD1")],
    "VAL": [("N", "CA", "CB", "CG1")],
    "ALA": [], "GLY": [],
}

_VIRTUAL_C = np.zeros(3)
_VIRTUAL_CA = np.array([-1.0, 0.0, 0.0])


def torsion(a, b, c, d) -> float:
    """IUPAC torsion angle of four points, radians in (-pi, pi]."""
    a, b, c, d = (np.asarray(p, dtype=np.float64) for p in (a, b, c, d))
    b1, b2, b3 = b - a, c - b, d - c
    n1, n2 = np.cross(b1, b2), np.cross(b2, b3)
    return float(np.arctan2(np.linalg.norm(b2) * np.dot(b1, n2), np.dot(n1, n2)))


def _backbone_of_residue(xyz, res_atom_off, r):
    a = res_atom_off[r]
    return xyz[:, a], xyz[:, a + 1], xyz[:, a + 2]


def _spine_angles(xyz, res_off, res_atom_off, out):
    for c in range(len(res_off) - 1):
        r0, r1 = res_off[c], res_off[c + 1]
        for r in range(r0, r1):
            n, ca, cc = _backbone_of_residue(xyz, res_atom_off, r)
            if r == r0:
                pca, pc = _VIRTUAL_CA, _VIRTUAL_C
            else:
                _, pca, pc = _backbone_of_residue(xyz, res_atom_off, r - 1)
            out[2, r] = torsion(pca, pc, n, ca)
            out[0, r] = torsion(pc, n, ca, cc)
            out[1, r] = 0.0 if r == r1 - 1 else torsion(
                n, ca, cc, _backbone_of_residue(xyz, res_atom_off, r + 1)[0])


def backbone_angles(res_offsets, xyz):
    """[3][R] (phi, psi, omega) of a backbone batch, xyz [3][3R]."""
    off = np.asarray(res_offsets, dtype=np.int64)
    R = int(off[-1])
    out = np.zeros((3, R))
    _spine_angles(np.asarray(xyz, dtype=np.float64), off, 3 * np.arange(R + 1), out)
    return out


def fullatom_angles(res_offsets, seq, xyz, res_atom_offsets, type_names, atom_names):
    """[7][R] angles of a full-atom batch.  type_names[t] is the residue's
    three-letter name, atom_names[t] its atom names in output order."""
    off = np.asarray(res_offsets, dtype=np.int64)
    aoff = np.asarray(res_atom_offsets, dtype=np.int64)
    R = int(off[-1])
    xyz = np.asarray(xyz, dtype=np.float64)
    out = np.zeros((7, R))
    _spine_angles(xyz, off, aoff, out)
    for r in range(R):
        t = int(seq[r])
        names = atom_names[t]
        for k, quad in enumerate(IUPAC_CHI[type_names[t]]):
            pts = [xyz[:, aoff[r] + names.index(nm)] for nm in quad]
            out[3 + k, r] = torsion(*pts)
    return out
