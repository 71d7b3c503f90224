"""GPU parity against the FP64 oracle on the input domains the boundary
promises beyond the workloads' own: angles far outside (-pi, pi] (the
branch-free sine/cosine reduces them by pi/2 up to |angle| = 1e5, beyond
that or for a non-finite lane the whole wave takes the library's sinf/cosf),
and backbone geometries other than the default (the paper's own constant
list, and an arbitrary one), through every call that uses the geometry:
scan forward, both adjoints, the plain form and the fused training step.
The oracle always receives the same float32 angle bits and the same
geometry.  Tolerances: 1e-3 A and 1e-3 relative (normwise per chain), the
accuracy stated for chains up to L = 1000."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import COORD_TOL_A, GRAD_TOL_REL, grad_rel_err, to_dev
from workloads import (BACKBONE_GEOMETRY, PAPER_LITERAL_GEOMETRY, make_angles,
                       offsets_from_lengths, random_sequence, upstream_grad)

pytestmark = pytest.mark.gpu

# a geometry unlike the default and the paper's: every slot constant differs
ODD_GEOMETRY = {"bond_N_CA": 1.40, "bond_CA_C": 1.61, "bond_C_N": 1.27,
                "angle_N_CA_C": 104.5, "angle_CA_C_N": 125.3, "angle_C_N_CA": 117.9}

LENGTHS = [1000, 1, 64, 65, 300, 999, 2, 513]


def _a2c():
    import paper_1812_01108_amd as a2c
    return a2c


def _oracle(model, off, seq, ang, geom, g):
    if model == "backbone":
        return (oracle.backbone_forward(off, ang, geom),
                oracle.backbone_backward(off, ang, geom, g))
    ref, _ = oracle.fullatom_forward(off, seq, ang, geom)
    return ref, oracle.fullatom_backward(off, seq, ang, geom, g)


def _plan(model, off, seq, geom=None):
    a2c = _a2c()
    if model == "backbone":
        return a2c.Plan("backbone", offsets=off, geometry=geom)
    return a2c.Plan("fullatom", offsets=off, seq=seq, geometry=geom)


def _err(label, xyz, ref, gr, gref, off, coord_tol=COORD_TOL_A):
    cerr = float(np.max(np.abs(xyz - ref))) if ref.size else 0.0
    gerr = grad_rel_err(gr, gref, off)
    print(f"{label}: max|dr|={cerr:.3e} A grad_rel={gerr:.3e}", flush=True)
    assert np.all(np.isfinite(xyz)) and np.all(np.isfinite(gr))
    assert cerr <= coord_tol, (label, cerr)
    assert gerr <= GRAD_TOL_REL, (label, gerr)


def _check_all(model, plan, off, seq, ang, geom, label, plain=True, mse=True):
    """Forward, both adjoints, the plain form (backbone) and the fused step,
    each against the oracle on the same float32 inputs and geometry."""
    import torch
    g = upstream_grad(len(off), plan.n_atoms)
    ref, gref = _oracle(model, off, seq, ang, geom, g)
    a, gd = to_dev(ang), to_dev(g)
    xyz = plan.forward(a)
    g_coords = plan.backward(a, gd, coords=xyz)
    g_recomp = plan.backward(a, gd)
    torch.cuda.synchronize()
    x_np = xyz.cpu().numpy()
    _err(f"{label} coords-adjoint", x_np, ref, g_coords.cpu().numpy(), gref, off)
    _err(f"{label} recompute-adjoint", x_np, ref, g_recomp.cpu().numpy(), gref, off)
    if plain and model == "backbone":
        ws = plan.new_workspace("plain")
        xp = plan.forward(a, variant="plain", workspace=ws)
        gp = plan.backward(a, gd, variant="plain", workspace=ws)
        torch.cuda.synchronize()
        _err(f"{label} plain", xp.cpu().numpy(), ref, gp.cpu().numpy(), gref, off)
    if mse:
        # target: the reference structure moved by a fixed offset per axis
        t = (ref + np.array([[0.7], [-1.3], [2.1]])).astype(np.float32)
        coords = torch.empty_like(xyz)
        loss, gm = plan.mse_step(a, to_dev(t), coords=coords)
        torch.cuda.synchronize()
        gl = 2.0 * (ref - t.astype(np.float64))
        _, gmref = _oracle(model, off, seq, ang, geom, gl)
        _err(f"{label} fused step", coords.cpu().numpy(), ref, gm.cpu().numpy(), gmref, off)
        L = float(np.sum((ref - t.astype(np.float64)) ** 2))
        assert abs(float(loss) - L) <= 1e-4 * L


def _shifted(ang, seed, kmax):
    """The angles plus 2 pi k, k uniform in [-kmax, kmax] per angle, rounded
    to float32 (both sides see the rounded value)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(-kmax, kmax + 1, size=ang.shape)
    return (ang.astype(np.float64) + 2.0 * np.pi * k).astype(np.float32)


@pytest.mark.parametrize("model", ["backbone", "fullatom"])
@pytest.mark.parametrize("sched", [None, (1, 16)])
def test_angles_far_outside_pi(model, sched):
    """|angle| up to ~9.4e4 rad (up to 15000 full turns, quadrant counts up
    to ~6e4): the fast path's Cody-Waite reduction far from (-pi, pi]."""
    off = offsets_from_lengths(LENGTHS)
    R = int(off[-1])
    rng = np.random.Generator(np.random.PCG64(601))
    ang = make_angles(rng, R, "mixture", 3 if model == "backbone" else 7)
    seq = random_sequence(rng, R) if model == "fullatom" else None
    ang = _shifted(ang, 603, 15000)
    assert np.max(np.abs(ang)) > 9e4 and np.max(np.abs(ang)) <= 1e5
    plan = _plan(model, off, seq)
    if sched:
        plan.set_schedule(*sched)
    _check_all(model, plan, off, seq, ang, BACKBONE_GEOMETRY, f"{model} |a|<=1e5 {sched}")


@pytest.mark.parametrize("model", ["backbone", "fullatom"])
@pytest.mark.parametrize("K", [1, 2, 4])
def test_library_sincos_in_mixed_waves(model, K):
    """A few lanes hold |angle| in (1e5, 1e8] (the whole wave then takes the
    library's sinf/cosf) among ordinary lanes of the same wave; short chains
    so that several chains share each wave."""
    if model == "fullatom" and K == 4:
        pytest.skip("the full-atom kernels take 1 or 2 residues per lane")
    lengths = [20, 31, 40, 1, 57, 64, 300, 5]
    off = offsets_from_lengths(lengths)
    R = int(off[-1])
    rng = np.random.Generator(np.random.PCG64(607 + K))
    P = 3 if model == "backbone" else 7
    ang = make_angles(rng, R, "mixture", P)
    seq = random_sequence(rng, R) if model == "fullatom" else None
    idx = rng.choice(R, size=12, replace=False)
    planes = rng.integers(0, P, size=12)
    mags = 10.0 ** rng.uniform(5.0, 8.0, size=12) * rng.choice([-1.0, 1.0], size=12)
    ang[planes, idx] = mags.astype(np.float32)
    assert np.sum(np.abs(ang) > 1e5) == 12
    plan = _plan(model, off, seq)
    plan.set_schedule(K, 4)
    _check_all(model, plan, off, seq, ang, BACKBONE_GEOMETRY, f"{model} K={K} mixed")


@pytest.mark.parametrize("model", ["backbone", "fullatom"])
def test_non_finite_lane_leaves_its_wave_exact(model):
    """A NaN and an Inf angle in one chain send their waves to the library
    path; every other chain of those waves still matches the oracle."""
    import torch
    lengths = [30, 45, 20, 60, 33]
    off = offsets_from_lengths(lengths)
    R = int(off[-1])
    rng = np.random.Generator(np.random.PCG64(611))
    P = 3 if model == "backbone" else 7
    ang = make_angles(rng, R, "mixture", P)
    seq = random_sequence(rng, R) if model == "fullatom" else None
    ang[0, 30 + 7] = np.nan
    ang[1, 30 + 20] = np.inf
    plan = _plan(model, off, seq)
    plan.set_schedule(2, 2)
    g = upstream_grad(len(off), plan.n_atoms)
    a, gd = to_dev(ang), to_dev(g)
    xyz = plan.forward(a)
    grs = [plan.backward(a, gd, coords=xyz), plan.backward(a, gd)]
    torch.cuda.synchronize()
    ca, _ = plan.atom_offsets()
    keep = [c for c in range(len(lengths)) if c != 1]
    sub_off = offsets_from_lengths([lengths[c] for c in keep])
    rsel = np.concatenate([np.arange(off[c], off[c + 1]) for c in keep])
    asel = np.concatenate([np.arange(ca[c], ca[c + 1]) for c in keep])
    sub_seq = None if seq is None else seq[rsel]
    ref, gref = _oracle(model, sub_off, sub_seq, np.ascontiguousarray(ang[:, rsel]),
                        BACKBONE_GEOMETRY, np.ascontiguousarray(g[:, asel]))
    x = xyz.cpu().numpy()[:, asel]
    for gr, tag in zip(grs, ("coords", "recompute")):
        _err(f"{model} finite chains {tag}", x, ref, gr.cpu().numpy()[:, rsel], gref, sub_off)


@pytest.mark.parametrize("model", ["backbone", "fullatom"])
@pytest.mark.parametrize("name", ["paper_literal", "odd"])
def test_non_default_geometry(model, name):
    a2c = _a2c()
    geom = PAPER_LITERAL_GEOMETRY if name == "paper_literal" else ODD_GEOMETRY
    if name == "paper_literal":
        # the package's preset is the same data the inputs module states
        assert a2c.PAPER_LITERAL_GEOMETRY == pytest.approx(PAPER_LITERAL_GEOMETRY, abs=1e-12)
        geom_plan = a2c.PAPER_LITERAL_GEOMETRY
    else:
        geom_plan = ODD_GEOMETRY
    off = offsets_from_lengths(LENGTHS)
    R = int(off[-1])
    rng = np.random.Generator(np.random.PCG64(613))
    ang = make_angles(rng, R, "mixture", 3 if model == "backbone" else 7)
    seq = random_sequence(rng, R) if model == "fullatom" else None
    plan = _plan(model, off, seq, geom_plan)
    _check_all(model, plan, off, seq, ang, geom, f"{model} {name} geometry")
    plan.set_schedule(1, 16)
    if model == "backbone":
        plan.set_adjoint_schedule(4, 2)
    _check_all(model, plan, off, seq, ang, geom, f"{model} {name} geometry (1,16)", plain=False)
