"""GPU parity of the full-atom path against the FP64 oracle: every atom and
all seven angle-gradient planes, element by element on the same float32
inputs, for both adjoint modes, the schedules, edge cases and the full-size
workloads."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import (COORD_TOL_A, GRAD_TOL_REL, grad_rel_err, run_fullatom, to_dev,
                            window_counts)
from workloads import (BACKBONE_GEOMETRY, make_angles, make_inputs, offsets_from_lengths,
                       random_sequence, upstream_grad)

pytestmark = pytest.mark.gpu
GEOM = BACKBONE_GEOMETRY


def _a2c():
    import paper_1812_01108_amd as a2c
    return a2c


def _batch(lengths, seed, seq=None):
    off = offsets_from_lengths(lengths)
    R = int(off[-1])
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = make_angles(rng, R, "mixture", 7)
    if seq is None:
        seq = random_sequence(rng, R)
    return off, np.asarray(seq, dtype=np.uint8), ang


def _check(plan, off, seq, ang, mode, label="", coord_tol=COORD_TOL_A, grad_tol=GRAD_TOL_REL):
    ca, ra = plan.atom_offsets()
    ref, aoff = oracle.fullatom_forward(off, seq, ang, GEOM)
    assert np.array_equal(ra, aoff)
    g = upstream_grad(len(seq), int(aoff[-1]))
    xyz, gr = run_fullatom(plan, ang, g, mode)
    gref = oracle.fullatom_backward(off, seq, ang, GEOM, g)
    cerr = float(np.max(np.abs(xyz - ref))) if ref.size else 0.0
    gerr = grad_rel_err(gr, gref, off)
    print(f"{label} mode={mode} atoms={ref.shape[1]} max|dr|={cerr:.3e} A grad_rel={gerr:.3e}",
          flush=True)
    assert np.all(np.isfinite(xyz)) and np.all(np.isfinite(gr))
    assert cerr <= coord_tol, cerr
    assert gerr <= grad_tol, gerr
    # chi planes a residue lacks are exactly zero
    info = oracle.load_residue_table()[1]
    nchi = np.array([info[t]["chi"] for t in range(20)])[seq]
    for k in range(4):
        assert np.all(gr[3 + k][nchi <= k] == 0.0)


@pytest.mark.parametrize("K,W", [(1, 1), (1, 4), (2, 2), (2, 4), (1, 8), (1, 12)])
@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_schedules_all_types(K, W, mode):
    """Chains longer than one chunk (64 K W residues) are walked chunk by chunk."""
    a2c = _a2c()
    off, seq, ang = _batch([1, 2, 20, 63, 64, 65, 0, 130, 7, 200, 1000], 101)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(K, W)
    _check(plan, off, seq, ang, mode, label=f"K={K} W={W}")


@pytest.mark.parametrize("K,W", [(2, 3), (1, 4)])
@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_whole_chain_windows(K, W, mode):
    """Short chains that all fit in one window and pack well: the windows
    hold whole chains (no window composes another's aggregate)."""
    a2c = _a2c()
    rng = np.random.Generator(np.random.PCG64(29))
    lengths = [int(v) for v in rng.integers(0, 26, 200)]
    n_whole, n_fixed = window_counts(lengths, 64 * K * W)
    assert n_whole <= n_fixed + n_fixed // 8
    off, seq, ang = _batch(lengths, 29)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(K, W)
    assert plan.schedule["n_tiles"] == n_whole
    _check(plan, off, seq, ang, mode, label=f"whole chains K={K} W={W}")


@pytest.mark.parametrize("n_win", [2, 7, 8, 9, 17])
@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_adjoint_window_order(n_win, mode):
    """The full-atom adjoints take fixed windows last to first within each
    class of window index mod 8: window counts around multiples of 8, with a
    chain crossing several windows."""
    from tests.test_parity_backbone import window_order_lengths
    a2c = _a2c()
    K, W = 2, 1
    lengths = window_order_lengths(n_win, 64 * K * W)
    off, seq, ang = _batch(lengths, 41 + n_win)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(K, W)
    assert plan.schedule["n_tiles"] == n_win
    _check(plan, off, seq, ang, mode, label=f"{n_win} windows")


@pytest.mark.parametrize("fwd,adj", [((1, 16), (2, 16)), ((2, 4), (1, 1))])
@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_separate_forward_and_adjoint_schedules(fwd, adj, mode):
    """Forward and adjoint on their own schedules (staged and unstaged,
    one- and multi-chunk tiles mixed)."""
    a2c = _a2c()
    off, seq, ang = _batch([1, 2, 20, 63, 64, 65, 0, 130, 7, 200, 1000], 103)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(*fwd)
    plan.set_adjoint_schedule(*adj)
    _check(plan, off, seq, ang, mode, label=f"fwd={fwd} adj={adj}")


@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_max_chunks_per_tile(mode):
    """K = 1, W = 1: a 4096-residue chain is exactly 64 chunks of 64 residues."""
    a2c = _a2c()
    off, seq, ang = _batch([3, 4096, 64, 65, 128, 129, 0, 1], 107)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(1, 1)
    _check(plan, off, seq, ang, mode, coord_tol=4e-3, label="64 chunks")


@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_unstaged_schedule(mode):
    """K = 2, W = 16: sixteen waves of 128 residues would stage ~1000 atoms
    per wave, beyond the LDS a workgroup may use; the kernels then read and
    write the atoms in global memory directly.  Chains up to 3000 residues
    (two 2048-residue chunks) and short ones."""
    a2c = _a2c()
    off, seq, ang = _batch([3000, 5, 2048, 1, 700, 2049], 109)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(2, 16)
    _check(plan, off, seq, ang, mode, coord_tol=4e-3, label=f"unstaged {mode}")


@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_sixteen_waves_coords_falls_back_to_recompute(mode):
    """K = 1, W = 16: three planes fit, six do not; the coordinate-mode
    adjoint recomputes the frames instead and gives the same gradient."""
    a2c = _a2c()
    off, seq, ang = _batch([1500, 1024, 3, 700, 64], 113)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(1, 16)
    _check(plan, off, seq, ang, mode, coord_tol=2e-3, label=f"K=1 W=16 {mode}")


@pytest.mark.parametrize("code", ["G", "W", "R", "P", "A"])
def test_homopolymers(code):
    a2c = _a2c()
    from workloads import ALPHABET
    off, seq, ang = _batch([50, 1, 33], 103, seq=[ALPHABET.index(code)] * 84)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    for mode in ("coords", "recompute"):
        _check(plan, off, seq, ang, mode, label=f"poly-{code}")


@pytest.mark.parametrize("name", ["fullatom_64x300", "ragged_fullatom_512"])
def test_full_size_workloads(name):
    a2c = _a2c()
    inp = make_inputs(name)
    off, seq, ang = inp["offsets"], inp["seq"], inp["angles"]
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    # chains of the ragged batch reach 2000 residues; the stated 1e-3 A bound
    # is at L = 1000, and 9.5e-4 A is what the kernels reach on this batch
    tol = COORD_TOL_A if name == "fullatom_64x300" else 1.2e-3
    for mode in ("coords", "recompute"):
        _check(plan, off, seq, ang, mode, label=name, coord_tol=tol)
    # the launch configuration bench.py times: the autotuner's schedules for
    # this batch, and for the training batch the schedules of its profiles
    # (forward K = 1, W = 16 staged; adjoint K = 2, W = 16 unstaged)
    a = to_dev(ang)
    g = to_dev(upstream_grad(len(seq), plan.n_atoms))
    mode = "coords" if name == "fullatom_64x300" else "recompute"
    fs, bs = plan.autotune(a, g, from_coords=mode == "coords", reps=3)
    tag = (f"{name} autotuned ({fs['res_per_lane']},{fs['waves_per_group']})/"
           f"({bs['res_per_lane']},{bs['waves_per_group']})")
    _check(plan, off, seq, ang, mode, label=tag, coord_tol=tol)
    if name == "ragged_fullatom_512":
        plan.set_schedule(1, 16)
        plan.set_adjoint_schedule(2, 16)
        _check(plan, off, seq, ang, "recompute", label=f"{name} (1,16)/(2,16)", coord_tol=tol)


def test_fullatom_backbone_matches_backbone_model():
    """Backbone atoms of the full-atom path agree with the backbone path's
    output (the paper's own comparison of the two models); the two kernels
    round in different orders, so they agree to the float32 parity bound."""
    a2c = _a2c()
    off, seq, ang = _batch([300, 77, 500], 107)
    fa = a2c.Plan("fullatom", offsets=off, seq=seq)
    bb = a2c.Plan("backbone", offsets=off)
    fa.set_schedule(2, 4)
    bb.set_schedule(2, 4)
    a7 = to_dev(ang)
    a3 = to_dev(np.ascontiguousarray(ang[:3]))
    xf = fa.forward(a7).cpu().numpy()
    xb = bb.forward(a3).cpu().numpy()
    _, ra = fa.atom_offsets()
    for s in range(3):
        assert np.max(np.abs(xf[:, ra[:-1] + s] - xb[:, s::3])) < COORD_TOL_A


@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_nan_stays_in_its_chain(mode):
    """A NaN chi1 poisons only its own residue's side chain; a NaN phi poisons
    its chain from that residue's CA frame on (the CA atom, at the origin of
    the frame phi rotates, is not checked); other chains (packed in the same
    tile) stay finite, forward and adjoint."""
    a2c = _a2c()
    off, seq, ang = _batch([50, 60, 70, 40], 113)
    info = oracle.load_residue_table()[1]
    nchi = np.array([info[t]["chi"] for t in range(20)])[seq]
    j = 50 + int(np.flatnonzero(nchi[50:110] >= 2)[0])        # a residue of chain 1 with chi2
    ang = ang.copy()
    ang[3, j] = np.nan
    ang[0, 110 + 30] = np.nan                                # phi of residue 30 of chain 2
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    ra = plan.atom_offsets()[1]
    xyz, gr = run_fullatom(plan, ang, upstream_grad(len(seq), int(ra[-1])), mode)
    fin = np.all(np.isfinite(xyz), axis=0)
    assert np.all(fin[: ra[50]]) and np.all(fin[ra[180]:])
    assert np.all(np.isfinite(gr[:, :50])) and np.all(np.isfinite(gr[:, 180:]))
    assert np.all(fin[ra[50]: ra[j]]) and np.all(fin[ra[j + 1]: ra[110]])
    assert np.all(fin[ra[j]: ra[j] + 3]) and not np.all(fin[ra[j]: ra[j + 1]])
    assert np.all(fin[ra[110]: ra[140] + 1]) and not np.any(fin[ra[141]: ra[180]])


@pytest.mark.parametrize("mode", ["coords", "recompute"])
def test_autograd_fullatom(mode):
    import torch
    a2c = _a2c()
    off, seq, ang = _batch([40, 0, 90, 5], 109)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    ref, aoff = oracle.fullatom_forward(off, seq, ang, GEOM)
    g = upstream_grad(3, int(aoff[-1]))
    x = to_dev(ang).requires_grad_(True)
    out = a2c.angles_to_coords(x, plan, mode=mode)
    out.backward(to_dev(g))
    torch.cuda.synchronize()
    gref = oracle.fullatom_backward(off, seq, ang, GEOM, g)
    assert np.max(np.abs(out.detach().cpu().numpy() - ref)) < COORD_TOL_A
    assert grad_rel_err(x.grad.cpu().numpy(), gref, off) < GRAD_TOL_REL
