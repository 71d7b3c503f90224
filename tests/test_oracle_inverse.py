"""Pins of the inverse-map oracle (coordinates -> dihedral angles): the
torsion of hand-built points, round trips through the forward oracle for the
backbone and every residue type, and invariance of the internal angles under
rigid motions."""
import numpy as np
import pytest

import oracle
from oracle import inverse as inv
from workloads import (ALPHABET, BACKBONE_GEOMETRY, make_angles, offsets_from_lengths,
                       random_sequence)

GEOM = BACKBONE_GEOMETRY


def wrapped(a):
    return (np.asarray(a) + np.pi) % (2 * np.pi) - np.pi


def test_torsion_of_hand_built_points():
    # a-b along +x, b-c along +z; d rotated by tau about z from the +x side
    for tau in (0.0, 0.4, 1.9, -2.5, np.pi):
        d = [np.cos(tau), np.sin(tau), 1.0]
        assert abs(wrapped(inv.torsion([1, 0, 0], [0, 0, 0], [0, 0, 1], d) - tau)) < 1e-14
    # cis / trans of a planar zig-zag
    assert abs(inv.torsion([1, 1, 0], [0, 0, 0], [1, 0, 0], [0, 1, 0])) < 1e-14
    assert abs(abs(inv.torsion([0, 1, 0], [0, 0, 0], [1, 0, 0], [1, -1, 0])) - np.pi) < 1e-14


def test_backbone_round_trip():
    rng = np.random.Generator(np.random.PCG64(71))
    off = offsets_from_lengths([1, 2, 37, 200, 5])
    ang = make_angles(rng, int(off[-1]), "uniform", 3).astype(np.float64)
    xyz = oracle.backbone_forward(off, ang, GEOM)
    back = inv.backbone_angles(off, xyz)
    last = off[1:] - 1
    keep = np.ones(int(off[-1]), bool)
    keep[last] = False
    assert np.max(np.abs(wrapped(back - ang)[:, keep])) < 1e-9
    assert np.max(np.abs(wrapped(back - ang)[[0, 2]][:, last])) < 1e-9
    assert np.all(back[1, last] == 0.0)


def test_fullatom_round_trip_every_type():
    tab, info = oracle.load_residue_table()
    rng = np.random.Generator(np.random.PCG64(73))
    seq = np.repeat(np.arange(20, dtype=np.uint8), 4)
    rng.shuffle(seq)
    off = offsets_from_lengths([30, 1, 49])
    ang = make_angles(rng, len(seq), "uniform", 7).astype(np.float64)
    xyz, aoff = oracle.fullatom_forward(off, seq, ang, GEOM)
    back = inv.fullatom_angles(off, seq, xyz, aoff, [i["name"] for i in info],
                               [i["atoms"] for i in info])
    nchi = np.array([info[t]["chi"] for t in range(20)])[seq]
    last = set((off[1:] - 1).tolist())
    for r in range(len(seq)):
        planes = [0, 2] + ([] if r in last else [1]) + [3 + k for k in range(nchi[r])]
        assert np.max(np.abs(wrapped(back[planes, r] - ang[planes, r]))) < 1e-9, r
        assert np.all(back[3 + nchi[r]:, r] == 0.0)


def test_internal_angles_invariant_under_rigid_motion():
    """Only omega_0 and phi_0 refer to the fixed start frame; every other
    angle is a torsion of the chain's own atoms."""
    rng = np.random.Generator(np.random.PCG64(79))
    off = offsets_from_lengths([60])
    ang = make_angles(rng, 60, "mixture", 3).astype(np.float64)
    xyz = oracle.backbone_forward(off, ang, GEOM)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    moved = q @ xyz + np.array([[3.0], [-7.0], [11.0]])
    a0, a1 = inv.backbone_angles(off, xyz), inv.backbone_angles(off, moved)
    d = np.abs(wrapped(a0 - a1))
    d[[0, 2], 0] = 0.0
    assert np.max(d) < 1e-9
    assert np.max(np.abs(wrapped(a0[[0, 2], 0] - a1[[0, 2], 0]))) > 1e-3
