"""Pins of the FP64 backbone oracle against what the paper and the mathematics
fix: the printed transform equals the product of elementary rotations and a
translation (Full-atom model section vs Backbone model section), bond lengths
and angles are the geometry, recomputed dihedrals equal the input angles, an
ideal alpha-helix is right-handed with ~3.6 residues per turn and ~1.5 A rise,
and the gradient agrees three ways (the paper's O(N^2) expression, the O(N)
closed form and central finite differences)."""
import numpy as np
import pytest

import oracle
from tests import geom as G
from workloads import offsets_from_lengths, uniform_angles, mixture_phi_psi

D2R = np.pi / 180.0


def slot_geometry(geom):
    """(bond length, bond angle at previous atom) for slots N, CA, C."""
    return [(geom["bond_C_N"], geom["angle_CA_C_N"] * D2R),
            (geom["bond_N_CA"], geom["angle_C_N_CA"] * D2R),
            (geom["bond_CA_C"], geom["angle_N_CA_C"] * D2R)]


def random_backbone(seed, lengths, kind="uniform"):
    rng = np.random.Generator(np.random.PCG64(seed))
    off = offsets_from_lengths(lengths)
    R = int(off[-1])
    ang = np.empty((3, R))
    if kind == "uniform":
        ang[0], ang[1], ang[2] = uniform_angles(rng, R), uniform_angles(rng, R), uniform_angles(rng, R)
    else:
        ang[0], ang[1] = mixture_phi_psi(rng, R)
        ang[2] = np.pi
    return off, ang


def with_virtual_atoms(coords, r0, L):
    """Atoms of one chain preceded by the two virtual atoms of the identity
    start frame: CA_{-1} on the -x axis and C_{-1} at the origin."""
    xyz = coords[:, 3 * r0: 3 * (r0 + L)].T
    virt = np.array([[-1.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    return np.concatenate([virt, xyz], axis=0)


def test_dihedral_helper_sign():
    # Looking along b->c (+z), a-b along +x rotated clockwise onto d-c (towards
    # +y when seen from behind) is a positive IUPAC torsion.
    for tau in (0.3, 1.2, -2.0, 3.0):
        d = G.dihedral([1, 0, 0], [0, 0, 0], [0, 0, 1], [np.cos(tau), np.sin(tau), 1])
        assert abs(d - tau) < 1e-14


@pytest.mark.parametrize("alpha,theta,d", [(0.3, 1.1, 1.5), (-2.9, 0.4, 0.7), (np.pi, np.pi - 2.0, 1.33)])
def test_transform_is_ry_tx_rx(alpha, theta, d):
    want = G.rot_y(theta) @ G.trans_x(d) @ G.rot_x(alpha)
    got = oracle.transform(alpha, theta, d)
    assert np.max(np.abs(got - want)) < 1e-15


def test_first_atom_closed_form(geom):
    off, ang = random_backbone(1, [5])
    xyz = oracle.backbone_forward(off, ang, geom)
    d, a = slot_geometry(geom)[0]
    theta = np.pi - a
    assert np.allclose(xyz[:, 0], [d * np.cos(theta), 0.0, -d * np.sin(theta)], atol=1e-15)


@pytest.mark.parametrize("kind", ["uniform", "mixture"])
def test_bond_lengths_angles_dihedrals(geom, kind):
    lengths = [1, 2, 7, 40]
    off, ang = random_backbone(11, lengths, kind)
    xyz = oracle.backbone_forward(off, ang, geom)
    sg = slot_geometry(geom)
    plane_of_slot = [2, 0, 1]
    for c, L in enumerate(lengths):
        r0 = off[c]
        P = with_virtual_atoms(xyz, r0, L)        # P[i + 2] is atom i
        n = 3 * L
        for i in range(n):
            d, a = sg[i % 3]
            assert abs(np.linalg.norm(P[i + 2] - P[i + 1]) - d) < 1e-12
            if i >= 1 or True:
                assert abs(G.bond_angle(P[i], P[i + 1], P[i + 2]) - a) < 1e-10
            # angle of transform i is the torsion (i-2, i-1, i, i+1)
            if i + 1 < n:
                want = ang[plane_of_slot[i % 3], r0 + i // 3]
                got = G.dihedral(P[i], P[i + 1], P[i + 2], P[i + 3])
                assert abs(G.wrapped_diff(got, want)) < 1e-10


def test_alpha_helix_right_handed(geom):
    L = 40
    off = offsets_from_lengths([L])
    for phi, psi, n_want, rise_want in [(-57.0, -47.0, 3.6, 1.5), (-63.0, -43.0, 3.6, 1.5)]:
        ang = np.empty((3, L))
        ang[0], ang[1], ang[2] = phi * D2R, psi * D2R, np.pi
        xyz = oracle.backbone_forward(off, ang, geom)
        n, rise, _, _ = G.screw_parameters(G.coords_by_residue(xyz, 0, L))
        assert abs(n - n_want) < 0.1, n
        assert abs(rise - rise_want) < 0.1, rise     # positive rise: right-handed
    # mirror image angles give the left-handed helix
    ang = np.empty((3, L))
    ang[0], ang[1], ang[2] = 57.0 * D2R, 47.0 * D2R, np.pi
    xyz = oracle.backbone_forward(off, ang, geom)
    n, rise, _, _ = G.screw_parameters(G.coords_by_residue(xyz, 0, L))
    assert rise < -1.4


def test_constant_angles_are_a_screw(geom):
    """For constant angles, r_{i+3} = P r_i with P the per-residue product of
    the three elementary transforms (the start frame is the identity)."""
    L = 25
    off = offsets_from_lengths([L])
    phi, psi, om = -1.1, 2.3, 3.0
    ang = np.empty((3, L))
    ang[0], ang[1], ang[2] = phi, psi, om
    xyz = oracle.backbone_forward(off, ang, geom)
    sg = slot_geometry(geom)
    P = np.eye(4)
    for (d, a), alpha in zip(sg, (om, phi, psi)):
        P = P @ G.rot_y(np.pi - a) @ G.trans_x(d) @ G.rot_x(alpha)
    pts = np.vstack([xyz, np.ones((1, 3 * L))])
    pred = (P @ pts)[:3, : 3 * (L - 1)]
    assert np.max(np.abs(pred - xyz[:, 3:])) < 1e-11


@pytest.mark.parametrize("value", [np.pi, 0.0])
def test_planar_chain(geom, value):
    off = offsets_from_lengths([30])
    ang = np.full((3, 30), value)
    xyz = oracle.backbone_forward(off, ang, geom)
    assert np.max(np.abs(xyz[1])) < 1e-12


def test_chains_are_independent(geom):
    off, ang = random_backbone(5, [9, 0, 13, 4])
    xyz = oracle.backbone_forward(off, ang, geom)
    for c in range(4):
        r0, r1 = off[c], off[c + 1]
        o1 = offsets_from_lengths([r1 - r0])
        alone = oracle.backbone_forward(o1, ang[:, r0:r1], geom)
        assert np.array_equal(alone, xyz[:, 3 * r0: 3 * r1])


def test_subchain_is_rigid_motion(geom):
    """Residues k.. of a chain are the chain started at residue k moved by the
    rigid frame M_{3k-1}: pairwise distances of the tail are preserved."""
    off, ang = random_backbone(8, [30])
    xyz = oracle.backbone_forward(off, ang, geom)
    k = 11
    tail = oracle.backbone_forward(offsets_from_lengths([30 - k]), ang[:, k:], geom)
    a = xyz[:, 3 * k:].T
    b = tail.T
    da = np.linalg.norm(a[:, None] - a[None], axis=-1)
    db = np.linalg.norm(b[:, None] - b[None], axis=-1)
    assert np.max(np.abs(da - db)) < 1e-10


def _loss_grad_fd(off, ang, geom, g, h=1e-6):
    fd = np.zeros_like(ang)
    for p in range(3):
        for r in range(ang.shape[1]):
            a1 = ang.copy(); a1[p, r] += h
            a2 = ang.copy(); a2[p, r] -= h
            fd[p, r] = (np.sum(g * oracle.backbone_forward(off, a1, geom)) -
                        np.sum(g * oracle.backbone_forward(off, a2, geom))) / (2 * h)
    return fd


def test_gradient_three_ways(geom):
    off, ang = random_backbone(21, [6, 1, 3])
    rng = np.random.Generator(np.random.PCG64(3))
    g = rng.standard_normal((3, 3 * ang.shape[1]))
    closed = oracle.backbone_backward(off, ang, geom, g)
    direct = oracle.backbone_backward(off, ang, geom, g, direct=True)
    fd = _loss_grad_fd(off, ang, geom, g)
    scale = np.max(np.abs(closed))
    assert np.max(np.abs(closed - direct)) < 1e-12 * scale
    assert np.max(np.abs(closed - fd)) < 1e-7 * scale


def test_gradient_special_cases(geom):
    off, ang = random_backbone(31, [12, 7])
    rng = np.random.Generator(np.random.PCG64(4))
    g = rng.standard_normal((3, 3 * ang.shape[1]))
    gr = oracle.backbone_backward(off, ang, geom, g)
    # nothing is placed after the last C: psi of the last residue has no effect
    for c in range(2):
        assert gr[1, off[c + 1] - 1] == 0.0
    # a rigid-motion invariant loss: sum of squared pairwise distances in a chain
    xyz = oracle.backbone_forward(off, ang, geom)
    for c in range(2):
        gg = np.zeros_like(xyz)
        a0, a1 = 3 * off[c], 3 * off[c + 1]
        X = xyz[:, a0:a1]
        n = X.shape[1]
        gg[:, a0:a1] = 4.0 * (n * X - X.sum(axis=1, keepdims=True))
        gi = oracle.backbone_backward(off, ang, geom, gg)
        scale = np.max(np.abs(gi[:, off[c]:off[c + 1]]))
        # omega_0 and phi_0 only rotate the whole chain rigidly
        assert abs(gi[2, off[c]]) < 1e-11 * scale
        assert abs(gi[0, off[c]]) < 1e-11 * scale


def test_zero_length_and_threads(geom):
    off, ang = random_backbone(41, [0, 5, 0, 0, 17, 0])
    g = np.random.Generator(np.random.PCG64(5)).standard_normal((3, 3 * ang.shape[1]))
    a = oracle.backbone_forward(off, ang, geom, n_threads=1)
    b = oracle.backbone_forward(off, ang, geom, n_threads=4)
    assert np.array_equal(a, b)
    ga = oracle.backbone_backward(off, ang, geom, g, n_threads=1)
    gb = oracle.backbone_backward(off, ang, geom, g, n_threads=4)
    assert np.array_equal(ga, gb)
