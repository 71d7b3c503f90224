"""GPU parity of the inverse map (a2c_coords_to_angles) against the FP64
oracle on the same float32 coordinates, and the round trip through the
forward map.

Tolerance: each torsion is formed in float32 from coordinate differences
(bond vectors of ~1.5 A, rounded relative ~1e-7) and the library's
polynomial arctangent (<= 5.3e-7 rad): ~1e-6 rad on protein geometry (bond
angles near 110-120 degrees); 2e-5 rad is used.  The
round trip also carries the forward map's coordinate error (<= 1e-3 A at
L <= 1000, i.e. ~1e-3 rad on a 1.5 A bond), checked at 2e-3 rad."""
import numpy as np
import pytest

import oracle
from oracle import inverse as inv
from tests.gpu_util import to_dev
from workloads import (BACKBONE_GEOMETRY, make_angles, make_inputs, offsets_from_lengths,
                       random_sequence)

pytestmark = pytest.mark.gpu
GEOM = BACKBONE_GEOMETRY
TORSION_TOL = 2e-5
ROUND_TRIP_TOL = 2e-3


def _a2c():
    import paper_1812_01108_amd as a2c
    return a2c


def wrapped(a):
    return (np.asarray(a, dtype=np.float64) + np.pi) % (2 * np.pi) - np.pi


def _gpu(plan, xyz):
    import torch
    out = plan.coords_to_angles(to_dev(xyz))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_backbone_against_oracle():
    a2c = _a2c()
    off = offsets_from_lengths([1, 2, 0, 64, 700, 3, 1000])
    rng = np.random.Generator(np.random.PCG64(401))
    ang = make_angles(rng, int(off[-1]), "mixture", 3)
    xyz = oracle.backbone_forward(off, ang, GEOM).astype(np.float32)
    plan = a2c.Plan("backbone", offsets=off)
    got = _gpu(plan, xyz)
    ref = inv.backbone_angles(off, xyz.astype(np.float64))
    err = float(np.max(np.abs(wrapped(got - ref))))
    print(f"backbone inverse: max|dangle|={err:.3e} rad", flush=True)
    assert err <= TORSION_TOL
    assert np.all(got[1, off[1:][np.diff(off) > 0] - 1] == 0.0)


def test_fullatom_against_oracle_every_type():
    a2c = _a2c()
    tab, info = oracle.load_residue_table()
    rng = np.random.Generator(np.random.PCG64(409))
    seq = np.concatenate([np.repeat(np.arange(20, dtype=np.uint8), 5),
                          random_sequence(rng, 400)])
    off = offsets_from_lengths([100, 1, 399])
    ang = make_angles(rng, len(seq), "mixture", 7)
    xyz, aoff = oracle.fullatom_forward(off, seq, ang, GEOM)
    xyz = xyz.astype(np.float32)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    got = _gpu(plan, xyz)
    ref = inv.fullatom_angles(off, seq, xyz.astype(np.float64), aoff,
                              [i["name"] for i in info], [i["atoms"] for i in info])
    err = float(np.max(np.abs(wrapped(got - ref))))
    print(f"full-atom inverse: max|dangle|={err:.3e} rad", flush=True)
    assert err <= TORSION_TOL
    nchi = np.array([info[t]["chi"] for t in range(20)])[seq]
    for k in range(4):
        assert np.all(got[3 + k][nchi <= k] == 0.0)


@pytest.mark.parametrize("name", ["backbone_256x700", "fullatom_64x300"])
def test_round_trip_through_the_forward_map(name):
    """angles -> GPU forward -> GPU inverse returns the angles (psi of chain
    ends is 0; chi a residue lacks is 0; the rest within the tolerance)."""
    import torch
    a2c = _a2c()
    inp = make_inputs(name)
    off, ang = inp["offsets"], inp["angles"]
    if inp["config"].model == "backbone":
        plan = a2c.Plan("backbone", offsets=off)
        nchi = None
    else:
        plan = a2c.Plan("fullatom", offsets=off, seq=inp["seq"])
        info = oracle.load_residue_table()[1]
        nchi = np.array([info[t]["chi"] for t in range(20)])[inp["seq"]]
    coords = plan.forward(to_dev(ang))
    back = plan.coords_to_angles(coords)
    torch.cuda.synchronize()
    back = back.cpu().numpy()
    keep = np.ones_like(back, dtype=bool)
    keep[1, off[1:] - 1] = False
    if nchi is not None:
        for k in range(4):
            keep[3 + k] = nchi > k
    err = float(np.max(np.abs(wrapped(back - ang))[keep]))
    print(f"{name}: round trip max|dangle|={err:.3e} rad", flush=True)
    assert err <= ROUND_TRIP_TOL
    assert np.all(back[~keep] == 0.0)


def test_empty_plan():
    import torch
    a2c = _a2c()
    plan = a2c.Plan("backbone", offsets=np.array([0, 0], np.int32))
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda:0")
    out = plan.coords_to_angles(e)
    torch.cuda.synchronize()
    assert out.shape == (3, 0)


@pytest.mark.parametrize("model", ["backbone", "fullatom"])
def test_chain_ends_on_workgroup_edges(model):
    """Each workgroup of 256 residues stages its atoms with one residue on
    either side; chains here start and end exactly on those edges (and one
    residue either side of them), against the oracle."""
    a2c = _a2c()
    off = offsets_from_lengths([256, 1, 255, 256, 257, 0, 511, 2, 254])
    R = int(off[-1])
    rng = np.random.Generator(np.random.PCG64(419))
    if model == "backbone":
        ang = make_angles(rng, R, "mixture", 3)
        xyz = oracle.backbone_forward(off, ang, GEOM).astype(np.float32)
        plan = a2c.Plan("backbone", offsets=off)
        ref = inv.backbone_angles(off, xyz.astype(np.float64))
    else:
        tab, info = oracle.load_residue_table()
        seq = random_sequence(rng, R)
        ang = make_angles(rng, R, "mixture", 7)
        xyz, aoff = oracle.fullatom_forward(off, seq, ang, GEOM)
        xyz = xyz.astype(np.float32)
        plan = a2c.Plan("fullatom", offsets=off, seq=seq)
        ref = inv.fullatom_angles(off, seq, xyz.astype(np.float64), aoff,
                                  [i["name"] for i in info], [i["atoms"] for i in info])
    got = _gpu(plan, xyz)
    err = float(np.max(np.abs(wrapped(got - ref))))
    print(f"{model} inverse at workgroup edges: max|dangle|={err:.3e} rad", flush=True)
    assert err <= TORSION_TOL


def test_nan_coordinates_stay_local():
    """A NaN coordinate gives NaN only in torsions that use that atom: the
    residue's own angles and its neighbours'; every other angle equals the
    clean result bit for bit."""
    a2c = _a2c()
    off = offsets_from_lengths([300, 400])
    rng = np.random.Generator(np.random.PCG64(421))
    ang = make_angles(rng, int(off[-1]), "mixture", 3)
    xyz = oracle.backbone_forward(off, ang, GEOM).astype(np.float32)
    plan = a2c.Plan("backbone", offsets=off)
    clean = _gpu(plan, xyz)
    j = 450
    bad = xyz.copy()
    bad[1, 3 * j + 1] = np.nan  # y of CA_j
    got = _gpu(plan, bad)
    assert np.isnan(got[0, j]) and np.isnan(got[1, j]) and np.isnan(got[2, j])
    far = np.ones(got.shape[1], dtype=bool)
    far[j - 1:j + 2] = False
    assert np.array_equal(got[:, far], clean[:, far])


def test_training_batch_sampled_chains():
    """The 512-chain full-atom training batch (283 k residues, 2.36 M atoms)
    through the inverse map in one launch, checked against the oracle on 24
    chains: the first, the last, the longest, the shortest and 20 drawn at
    random (the oracle takes about a minute for the whole batch)."""
    a2c = _a2c()
    inp = make_inputs("ragged_fullatom_512")
    off, seq, ang = inp["offsets"], inp["seq"], inp["angles"]
    xyz, aoff = oracle.fullatom_forward(off, seq, ang, GEOM)
    xyz = xyz.astype(np.float32)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    got = _gpu(plan, xyz)
    info = oracle.load_residue_table()[1]
    names, atoms = [i["name"] for i in info], [i["atoms"] for i in info]
    lengths = np.diff(off)
    rng = np.random.Generator(np.random.PCG64(431))
    pick = {0, len(lengths) - 1, int(np.argmax(lengths)),
            int(np.argmin(np.where(lengths > 0, lengths, 1 << 30)))}
    pick |= set(int(c) for c in rng.choice(len(lengths), 20, replace=False))
    aoff = np.asarray(aoff)
    worst, n_res = 0.0, 0
    for c in sorted(pick):
        r0, r1 = int(off[c]), int(off[c + 1])
        if r1 == r0:
            continue
        a0, a1 = int(aoff[r0]), int(aoff[r1])
        ref = inv.fullatom_angles(np.array([0, r1 - r0], np.int32), seq[r0:r1],
                                  xyz[:, a0:a1].astype(np.float64), aoff[r0:r1 + 1] - a0,
                                  names, atoms)
        worst = max(worst, float(np.max(np.abs(wrapped(got[:, r0:r1] - ref)))))
        n_res += r1 - r0
    print(f"training batch inverse: {len(pick)} chains, {n_res} residues, "
          f"max|dangle|={worst:.3e} rad", flush=True)
    assert worst <= TORSION_TOL
