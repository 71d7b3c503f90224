"""Residue table for the full-atom model: reads the internal-coordinate data
file (data/residues.json) into the a2c_residue_table struct of the C ABI.
Marshalling only (names to indices); the library converts the internal
coordinates into rigid-group coordinates itself."""
from __future__ import annotations

import json
import os

from . import _lib

DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "residues.json")
SPINE = {"N": 0, "CA": 1, "C": 2}
KINDS = {"origin": _lib.ATOM_ORIGIN, "azimuth": _lib.ATOM_AZIMUTH, "zmatrix": _lib.ATOM_ZMATRIX}


class ResidueTable:
    def __init__(self, path: str = DATA):
        with open(path) as f:
            self.spec = json.load(f)
        self.alphabet = self.spec["alphabet"]
        by_code = {v["code"]: (k, v) for k, v in self.spec["residues"].items()}
        self.names = []
        self.atom_names = []
        self.n_chi = []
        for code in self.alphabet:
            name, res = by_code[code]
            self.names.append(name)
            atoms = self.spec["backbone_atoms"] + res["atoms"]
            self.atom_names.append([a["name"] for a in atoms])
            self.n_chi.append(sum(1 for fr in res["frames"] if fr["chi"] > 0))

    def n_atoms(self, code: int) -> int:
        return len(self.atom_names[code])

    def to_struct(self) -> _lib.ResidueTable:
        tab = _lib.ResidueTable()
        by_code = {v["code"]: v for v in self.spec["residues"].values()}
        for t, code in enumerate(self.alphabet):
            res = by_code[code]
            rd = tab.residues[t]
            frame_id = dict(SPINE)
            pred = {"C": "CA", "CA": "N"}
            for f, fr in enumerate(res["frames"]):
                frame_id[fr["origin"]] = 3 + f
                pred[fr["origin"]] = fr["parent"]
                sf = rd.frames[f]
                sf.parent = frame_id[fr["parent"]]
                sf.chi = fr["chi"]
                sf.pre_rotation_deg = fr["pre_rotation"]
                sf.bond = fr["bond"]
                sf.bond_angle_deg = fr["angle"]
            rd.n_side_frames = len(res["frames"])
            atoms = self.spec["backbone_atoms"] + res["atoms"]
            if len(atoms) > _lib.MAX_RESIDUE_ATOMS:
                raise ValueError(f"{code}: too many atoms")
            rd.n_atoms = len(atoms)
            index = {}
            for a, at in enumerate(atoms):
                ad = rd.atoms[a]
                ad.frame = frame_id[at["frame"]]
                ad.kind = KINDS[at["kind"]]
                if at["kind"] == "azimuth":
                    ad.bond, ad.angle_deg, ad.torsion_deg = at["bond"], at["angle"], at["azimuth"]
                elif at["kind"] == "zmatrix":
                    ad.bond, ad.angle_deg, ad.torsion_deg = at["bond"], at["angle"], at["torsion"]
                    for q, nm in enumerate(at["refs"]):
                        ad.ref[q] = -1 if nm == pred.get(at["frame"]) else index[nm]
                index[at["name"]] = a
        return tab


_DEFAULT = None


def default_table() -> ResidueTable:
    global _DEFAULT
    if _DEFAULT is None:
        _DEFAULT = ResidueTable()
    return _DEFAULT
