"""Pins of the FP64 full-atom oracle ("Full-atom model" section) against what
the paper, chemistry and mathematics fix:
  - backbone atoms equal the backbone model's for the same phi, psi, omega
    (the paper compares the two models this way in its error study);
  - every bond length, bond angle and fixed torsion recomputed from the output
    equals the residue table; IUPAC chi torsions equal the input chi angles;
  - L-chirality at CA and the known configurations of the other stereo
    centres (Thr 2S,3R; Ile 2S,3S; Val CG1 and Leu CD1 pro-R);
  - the gradient agrees three ways: Eq. FAMBackward term by term, the O(N)
    subtree form, and central finite differences.
The table values themselves are the library's authored stereochemistry: the
paper prints none, so agreement with the paper's own table is unpinned."""
import json

import numpy as np
import pytest

import oracle
from oracle.residue_table import default_path
from tests import geom as G
from workloads import ALPHABET, offsets_from_lengths

SPEC = json.load(open(default_path()))

# IUPAC side-chain torsion definitions (four atoms per chi)
CHI_ATOMS = {
    "ARG": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD"), ("CB", "CG", "CD", "NE"), ("CG", "CD", "NE", "CZ")],
    "ASN": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "OD1")],
    "ASP": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "OD1")],
    "CYS": [("N", "CA", "CB", "SG")],
    "GLN": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD"), ("CB", "CG", "CD", "OE1")],
    "GLU": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD"), ("CB", "CG", "CD", "OE1")],
    "HIS": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "ND1")],
    "ILE": [("N", "CA", "CB", "CG1"), ("CA", "CB", "CG1", "CD1")],
    "LEU": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD1")],
    "LYS": [("N", "CA", "CB", "CG"), ("CA", "CB", "CG", "CD"), ("CB", "CG", "CD", "CE"), ("CG", "CD", "CE", "NZ")],
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
CODE_TO_NAME = {v["code"]: k for k, v in SPEC["residues"].items()}


def build_all(seed, length_per_type=3, geom=None):
    """Chains covering every residue type a few times, random angles."""
    rng = np.random.Generator(np.random.PCG64(seed))
    seq = np.repeat(np.arange(20, dtype=np.uint8), length_per_type)
    rng.shuffle(seq)
    off = offsets_from_lengths([len(seq) // 2, len(seq) - len(seq) // 2])
    ang = rng.uniform(-np.pi, np.pi, (7, len(seq)))
    return off, seq, ang


def atoms_of(x, aoff, seq, info):
    out = []
    for j, t in enumerate(seq):
        out.append({n: x[:, aoff[j] + i] for i, n in enumerate(info[t]["atoms"])})
    return out


def test_backbone_atoms_equal_backbone_model(geom):
    off, seq, ang = build_all(1)
    x, aoff = oracle.fullatom_forward(off, seq, ang, geom)
    xb = oracle.backbone_forward(off, ang[:3], geom)
    tab, info = oracle.load_residue_table()
    res = atoms_of(x, aoff, seq, info)
    for j in range(len(seq)):
        for s, nm in enumerate(("N", "CA", "C")):
            assert np.max(np.abs(res[j][nm] - xb[:, 3 * j + s])) < 1e-12


def test_chi_torsions_equal_inputs(geom):
    off, seq, ang = build_all(2)
    x, aoff = oracle.fullatom_forward(off, seq, ang, geom)
    tab, info = oracle.load_residue_table()
    res = atoms_of(x, aoff, seq, info)
    seen = 0
    for j, t in enumerate(seq):
        name = CODE_TO_NAME[ALPHABET[t]]
        for k, quad in enumerate(CHI_ATOMS[name]):
            got = G.dihedral(*(res[j][a] for a in quad))
            assert abs(G.wrapped_diff(got, ang[3 + k, j])) < 1e-10, (name, k)
            seen += 1
    assert seen > 0


def test_table_geometry_recomputed(geom):
    """Every bond, angle and torsion in the residue table, measured on output."""
    off, seq, ang = build_all(3)
    x, aoff = oracle.fullatom_forward(off, seq, ang, geom)
    tab, info = oracle.load_residue_table()
    res = atoms_of(x, aoff, seq, info)
    n_checked = 0
    for j, t in enumerate(seq):
        name = CODE_TO_NAME[ALPHABET[t]]
        spec = SPEC["residues"][name]
        r = res[j]
        pred = {"C": "CA", "CA": "N"}
        for fr in spec["frames"]:
            pred[fr["origin"]] = fr["parent"]
            o, p = fr["origin"], fr["parent"]
            assert abs(np.linalg.norm(r[o] - r[p]) - fr["bond"]) < 1e-10
            assert abs(np.degrees(G.bond_angle(r[pred[p]], r[p], r[o])) - fr["angle"]) < 1e-8
        for at in SPEC["backbone_atoms"] + spec["atoms"]:
            nm, f = at["name"], at["frame"]
            if at["kind"] == "azimuth":
                assert abs(np.linalg.norm(r[nm] - r[f]) - at["bond"]) < 1e-10
                assert abs(np.degrees(G.bond_angle(r[pred[f]], r[f], r[nm])) - at["angle"]) < 1e-8
            elif at["kind"] == "zmatrix":
                a, b, c = at["refs"]
                assert abs(np.linalg.norm(r[nm] - r[c]) - at["bond"]) < 1e-10
                assert abs(np.degrees(G.bond_angle(r[b], r[c], r[nm])) - at["angle"]) < 1e-8
                tor = np.degrees(G.dihedral(r[a], r[b], r[c], r[nm]))
                assert abs(G.wrapped_diff(np.radians(tor), np.radians(at["torsion"]))) < 1e-9
            n_checked += 1
        # carbonyl O is anti to the next N about CA-C: torsion N-CA-C-O = psi + pi
        assert abs(G.wrapped_diff(G.dihedral(r["N"], r["CA"], r["C"], r["O"]), ang[1, j] + np.pi)) < 1e-10
    assert n_checked > 100


def test_stereochemistry(geom):
    off, seq, ang = build_all(4)
    x, aoff = oracle.fullatom_forward(off, seq, ang, geom)
    tab, info = oracle.load_residue_table()
    res = atoms_of(x, aoff, seq, info)

    def tp(c, a, b, d):  # (a-c) . ((b-c) x (d-c))
        return np.dot(a - c, np.cross(b - c, d - c))

    for j, t in enumerate(seq):
        r = res[j]
        name = CODE_TO_NAME[ALPHABET[t]]
        if name != "GLY":
            # CA: N > C > CB; L (S) configuration
            assert tp(r["CA"], r["N"], r["C"], r["CB"]) > 1.0
        if name == "THR":      # CB: OG1 > CA > CG2, R
            assert tp(r["CB"], r["OG1"], r["CA"], r["CG2"]) < -1.0
        if name == "ILE":      # CB: CA > CG1 > CG2, S
            assert tp(r["CB"], r["CA"], r["CG1"], r["CG2"]) > 1.0
        if name == "VAL":      # CG1 pro-R
            assert tp(r["CB"], r["CA"], r["CG1"], r["CG2"]) < -1.0
        if name == "LEU":      # CD1 pro-R
            assert tp(r["CG"], r["CB"], r["CD1"], r["CD2"]) < -1.0


def test_rigid_groups_are_rigid(geom):
    """Distances inside one rigid group do not depend on the angles."""
    off, seq, ang1 = build_all(5)
    ang2 = np.random.Generator(np.random.PCG64(6)).uniform(-np.pi, np.pi, ang1.shape)
    tab, info = oracle.load_residue_table()
    x1, aoff = oracle.fullatom_forward(off, seq, ang1, geom)
    x2, _ = oracle.fullatom_forward(off, seq, ang2, geom)
    for j, t in enumerate(seq):
        frames = np.array([tab.atom_frame[t][a] for a in range(tab.n_atoms[t])])
        for f in set(frames.tolist()):
            idx = aoff[j] + np.nonzero(frames == f)[0]
            p1, p2 = x1[:, idx].T, x2[:, idx].T
            d1 = np.linalg.norm(p1[:, None] - p1[None], axis=-1)
            d2 = np.linalg.norm(p2[:, None] - p2[None], axis=-1)
            assert np.max(np.abs(d1 - d2)) < 1e-10


def test_aromatic_rings_planar(geom):
    off, seq, ang = build_all(7)
    x, aoff = oracle.fullatom_forward(off, seq, ang, geom)
    tab, info = oracle.load_residue_table()
    res = atoms_of(x, aoff, seq, info)
    rings = {"PHE": ["CG", "CD1", "CD2", "CE1", "CE2", "CZ"],
             "TYR": ["CG", "CD1", "CD2", "CE1", "CE2", "CZ", "OH"],
             "HIS": ["CG", "ND1", "CD2", "CE1", "NE2"],
             "TRP": ["CG", "CD1", "CD2", "NE1", "CE2", "CE3", "CZ2", "CZ3", "CH2"]}
    for j, t in enumerate(seq):
        name = CODE_TO_NAME[ALPHABET[t]]
        if name in rings:
            P = np.array([res[j][a] for a in rings[name]])
            P = P - P.mean(axis=0)
            assert np.linalg.svd(P, compute_uv=False)[-1] < 1e-8


def _fd(off, seq, ang, geom, g, h=1e-6):
    out = np.zeros_like(ang)
    for p in range(7):
        for r in range(ang.shape[1]):
            a1 = ang.copy(); a1[p, r] += h
            a2 = ang.copy(); a2[p, r] -= h
            out[p, r] = (np.sum(g * oracle.fullatom_forward(off, seq, a1, geom)[0]) -
                         np.sum(g * oracle.fullatom_forward(off, seq, a2, geom)[0])) / (2 * h)
    return out


def test_gradient_three_ways(geom):
    rng = np.random.Generator(np.random.PCG64(8))
    seq = rng.permutation(20).astype(np.uint8)[:14]
    off = offsets_from_lengths([9, 5])
    ang = rng.uniform(-np.pi, np.pi, (7, 14))
    x, aoff = oracle.fullatom_forward(off, seq, ang, geom)
    g = rng.standard_normal(x.shape)
    closed = oracle.fullatom_backward(off, seq, ang, geom, g)
    direct = oracle.fullatom_backward(off, seq, ang, geom, g, direct=True)
    fd = _fd(off, seq, ang, geom, g)
    scale = np.max(np.abs(closed))
    assert np.max(np.abs(closed - direct)) < 1e-12 * scale
    assert np.max(np.abs(closed - fd)) < 1e-7 * scale
    # chi slots a residue lacks carry no gradient
    tab, info = oracle.load_residue_table()
    for j, t in enumerate(seq):
        for k in range(info[t]["chi"], 4):
            assert closed[3 + k, j] == 0.0


def test_rigid_invariant_loss(geom):
    off, seq, ang = build_all(9, length_per_type=1)
    x, aoff = oracle.fullatom_forward(off, seq, ang, geom)
    for c in range(2):
        r0, r1 = off[c], off[c + 1]
        a0, a1 = aoff[r0], aoff[r1]
        X = x[:, a0:a1]
        g = np.zeros_like(x)
        g[:, a0:a1] = 4.0 * (X.shape[1] * X - X.sum(axis=1, keepdims=True))
        gr = oracle.fullatom_backward(off, seq, ang, geom, g)
        scale = np.max(np.abs(gr[:, r0:r1]))
        assert abs(gr[2, r0]) < 1e-11 * scale    # omega_0
        assert abs(gr[0, r0]) < 1e-11 * scale    # phi_0 (rotates the chain about N-CA)
