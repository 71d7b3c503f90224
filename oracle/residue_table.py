"""Oracle-side reading of the residue table (TEST INFRASTRUCTURE ONLY).

Turns the internal coordinates of the residue data file into the rigid-group
standard coordinates r° of the full-atom model ("Full-atom model" section:
the first atom of a group sits at the frame origin, the others where the
stereochemistry puts them) using the paper's 4x4 transform matrices.  This is
written independently of the library's own conversion.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np

N_TYPES = 20
MAX_SIDE = 4
MAX_ATOMS = 14
SPINE = {"N": 0, "CA": 1, "C": 2}


class OracleTable(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32 * N_TYPES),
        ("n_side", ctypes.c_int32 * N_TYPES),
        ("side_parent", (ctypes.c_int32 * MAX_SIDE) * N_TYPES),
        ("side_chi", (ctypes.c_int32 * MAX_SIDE) * N_TYPES),
        ("side_pre", (ctypes.c_double * MAX_SIDE) * N_TYPES),
        ("side_theta", (ctypes.c_double * MAX_SIDE) * N_TYPES),
        ("side_d", (ctypes.c_double * MAX_SIDE) * N_TYPES),
        ("atom_frame", (ctypes.c_int32 * MAX_ATOMS) * N_TYPES),
        ("atom_r", ((ctypes.c_double * 3) * MAX_ATOMS) * N_TYPES),
    ]


def default_path() -> str:
    here = os.path.dirname(os.path.abspath(__file__))
    return os.path.join(os.path.dirname(here), "paper_1812_01108_amd", "data", "residues.json")


def _rx(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0, 0], [0, c, -s, 0], [0, s, c, 0], [0, 0, 0, 1.0]])


def _paper_transform(alpha, theta, d):
    """R(alpha, theta, d) as printed in the backbone section."""
    ca, sa, ct, st = np.cos(alpha), np.sin(alpha), np.cos(theta), np.sin(theta)
    return np.array([[ct, sa * st, ca * st, d * ct],
                     [0.0, ca, -sa, 0.0],
                     [-st, sa * ct, ca * ct, -d * st],
                     [0.0, 0.0, 0.0, 1.0]])


def _azimuth_point(bond, angle_deg, azimuth_deg):
    """Point bonded to the frame origin: R_x(azimuth) R(0, pi - angle, bond) 0."""
    m = _rx(np.radians(azimuth_deg)) @ _paper_transform(0.0, np.pi - np.radians(angle_deg), bond)
    return m[:3, 3]


def _zmatrix_point(a, b, c, bond, angle_deg, torsion_deg):
    """Atom from three reference points: a frame at c with x along b->c and a
    on its -z side, then the paper's transform with alpha = torsion."""
    ex = (c - b) / np.linalg.norm(c - b)
    v = (a - b) - np.dot(a - b, ex) * ex
    ez = -v / np.linalg.norm(v)
    ey = np.cross(ez, ex)
    F = np.eye(4)
    F[:3, 0], F[:3, 1], F[:3, 2], F[:3, 3] = ex, ey, ez, c
    m = F @ _rx(np.radians(torsion_deg)) @ _paper_transform(0.0, np.pi - np.radians(angle_deg), bond)
    return m[:3, 3]


def load(path: str | None = None):
    """Returns (OracleTable, info) where info maps residue codes to names and
    atom names, in output order (N, CA, C, O, side chain)."""
    with open(path or default_path()) as f:
        spec = json.load(f)
    alphabet = spec["alphabet"]
    by_code = {v["code"]: (k, v) for k, v in spec["residues"].items()}
    tab = OracleTable()
    info = []
    for t, code in enumerate(alphabet):
        name, res = by_code[code]
        frames = res["frames"]
        fid = dict(SPINE)
        frame_bond = {}
        frame_pred = {"C": "CA"}
        for f, fr in enumerate(frames):
            fid[fr["origin"]] = 3 + f
            tab.side_parent[t][f] = fid[fr["parent"]]
            tab.side_chi[t][f] = fr["chi"]
            tab.side_pre[t][f] = np.radians(fr["pre_rotation"])
            tab.side_theta[t][f] = np.pi - np.radians(fr["angle"])
            tab.side_d[t][f] = fr["bond"]
            frame_bond[fr["origin"]] = fr["bond"]
            frame_pred[fr["origin"]] = fr["parent"]
        tab.n_side[t] = len(frames)
        atoms = spec["backbone_atoms"] + res["atoms"]
        tab.n_atoms[t] = len(atoms)
        local = {}
        for a, at in enumerate(atoms):
            fr = at["frame"]
            tab.atom_frame[t][a] = fid[fr]
            if at["kind"] == "origin":
                p = np.zeros(3)
            elif at["kind"] == "azimuth":
                p = _azimuth_point(at["bond"], at["angle"], at["azimuth"])
            else:
                def ref(nm):
                    if nm == frame_pred.get(fr):
                        return np.array([-frame_bond[fr], 0.0, 0.0])
                    return local[(fr, nm)]
                ra, rb, rc = (ref(nm) for nm in at["refs"])
                p = _zmatrix_point(ra, rb, rc, at["bond"], at["angle"], at["torsion"])
            local[(fr, at["name"])] = p
            for q in range(3):
                tab.atom_r[t][a][q] = p[q]
        info.append({"code": code, "name": name, "atoms": [at["name"] for at in atoms],
                     "chi": sum(1 for fr in frames if fr["chi"] > 0)})
    return tab, info


def atom_offsets(seq, tab: OracleTable):
    """Residue atom offsets [R+1] from the sequence."""
    counts = np.array([tab.n_atoms[t] for t in range(N_TYPES)], dtype=np.int64)
    off = np.zeros(len(seq) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts[np.asarray(seq, dtype=np.int64)])
    return off.astype(np.int32)
