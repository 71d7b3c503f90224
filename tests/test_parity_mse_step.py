"""GPU parity of the fused training step (a2c_mse_step): forward, loss
L = sum |r - t|^2 and its angle gradient in one kernel, against

* the FP64 oracle: forward, g = 2 (r - t) in float64, O(N) adjoint;
* the unfused GPU path: a2c_forward, g = 2 (r - t) in float32 by torch,
  a2c_backward recomputing the frames.  The forward runs on windows of the
  packed batch and the backbone fused step on tiles of whole chains (the
  full-atom one on windows, with a spine pass first), so their scans
  associate differently: both are held to the oracle bounds.

Loss tolerance: the coordinates carry float32 rounding of up to ~1e-3 A
against residuals |r - t| of order 1-10 A, and the sum runs in float32 over
up to ~1e6 terms: 1e-4 relative."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import COORD_TOL_A, GRAD_TOL_REL, grad_rel_err, to_dev
from workloads import (BACKBONE_GEOMETRY, make_angles, make_inputs, offsets_from_lengths,
                       random_sequence, target_perturbation)

pytestmark = pytest.mark.gpu
GEOM = BACKBONE_GEOMETRY
LOSS_RTOL = 1e-4


def _a2c():
    import paper_1812_01108_amd as a2c
    return a2c


def _case(model, lengths, seed):
    off = offsets_from_lengths(lengths)
    R = int(off[-1])
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = make_angles(rng, R, "mixture", 3 if model == "backbone" else 7)
    seq = random_sequence(rng, R) if model == "fullatom" else None
    pert, _, _ = target_perturbation(seed, ang, len(lengths))
    if model == "backbone":
        t = oracle.backbone_forward(off, pert, GEOM)
    else:
        t, _ = oracle.fullatom_forward(off, seq, pert, GEOM)
    return off, seq, ang, t.astype(np.float32)


def _oracle(model, off, seq, ang, t):
    if model == "backbone":
        r = oracle.backbone_forward(off, ang, GEOM)
        g = 2.0 * (r - t.astype(np.float64))
        ga = oracle.backbone_backward(off, ang, GEOM, g)
    else:
        r, _ = oracle.fullatom_forward(off, seq, ang, GEOM)
        g = 2.0 * (r - t.astype(np.float64))
        ga = oracle.fullatom_backward(off, seq, ang, GEOM, g)
    return r, float(np.sum((r - t.astype(np.float64)) ** 2)), ga


def _run(plan, model, off, seq, ang, t, label, coord_tol=COORD_TOL_A):
    import torch
    a, td = to_dev(ang), to_dev(t)
    coords = torch.empty((3, plan.n_atoms), dtype=torch.float32, device=a.device)
    loss, grad = plan.mse_step(a, td, coords=coords)
    # unfused reference on the GPU, same schedule
    c2 = plan.forward(a)
    g2 = plan.backward(a, 2.0 * (c2 - td))
    torch.cuda.synchronize()
    r, L, ga = _oracle(model, off, seq, ang, t)
    xyz, gr = coords.cpu().numpy(), grad.cpu().numpy()
    cerr = float(np.max(np.abs(xyz - r))) if r.size else 0.0
    gerr = grad_rel_err(gr, ga, off)
    lerr = abs(float(loss) - L) / max(L, 1e-30)
    print(f"{label}: max|dr|={cerr:.3e} A grad_rel={gerr:.3e} loss_rel={lerr:.3e}", flush=True)
    assert cerr <= coord_tol and gerr <= GRAD_TOL_REL and lerr <= LOSS_RTOL
    # The forward and the fused step associate their scans differently even at
    # one schedule (windows against whole-chain tiles, or a spine pass): the
    # unfused path is held to the same oracle bounds.
    c2n, g2n = c2.cpu().numpy(), g2.cpu().numpy()
    assert float(np.max(np.abs(c2n - r))) <= coord_tol
    assert grad_rel_err(g2n, ga, off) <= GRAD_TOL_REL


@pytest.mark.parametrize("K,W", [(1, 16), (2, 8), (4, 4), (1, 1), (2, 3), (4, 16)])
def test_backbone_schedules(K, W):
    """Ragged chains, including ones longer than a chunk at the small
    schedules (several chunks per tile)."""
    a2c = _a2c()
    off, seq, ang, t = _case("backbone", [1, 2, 0, 63, 64, 65, 255, 700, 1000, 5], 301)
    plan = a2c.Plan("backbone", offsets=off)
    plan.set_schedule(K, W)
    _run(plan, "backbone", off, seq, ang, t, f"backbone K={K} W={W}")


@pytest.mark.parametrize("K,W", [(1, 16), (1, 8), (2, 4), (1, 1), (2, 8), (2, 16)])
def test_fullatom_schedules(K, W):
    a2c = _a2c()
    off, seq, ang, t = _case("fullatom", [1, 20, 0, 64, 65, 300, 700, 3], 307)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(K, W)
    _run(plan, "fullatom", off, seq, ang, t, f"full-atom K={K} W={W}")


def test_fullatom_whole_chain_windows():
    """Short chains packed whole into the windows of the fused step."""
    a2c = _a2c()
    rng = np.random.Generator(np.random.PCG64(311))
    lengths = [int(v) for v in rng.integers(0, 26, 200)]
    off, seq, ang, t = _case("fullatom", lengths, 311)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(2, 3)
    _run(plan, "fullatom", off, seq, ang, t, "full-atom whole chains K=2 W=3")


@pytest.mark.parametrize("model", ["backbone", "fullatom"])
def test_separate_adjoint_schedule(model):
    """The fused step runs on the adjoint schedule (its loss shares are one
    per adjoint tile) while the forward keeps another."""
    a2c = _a2c()
    lengths = [1, 20, 0, 64, 65, 300, 700, 3]
    off, seq, ang, t = _case(model, lengths, 313)
    plan = (a2c.Plan("backbone", offsets=off) if model == "backbone"
            else a2c.Plan("fullatom", offsets=off, seq=seq))
    plan.set_schedule(1, 4)
    plan.set_adjoint_schedule(2, 8)
    assert plan.adjoint_schedule["n_tiles"] != plan.schedule["n_tiles"]
    _run(plan, model, off, seq, ang, t, f"{model} fwd (1,4) adj (2,8)")


def test_training_workload_full_size():
    """The ragged 512-chain full-atom workload (chains to 2000 residues)."""
    a2c = _a2c()
    inp = make_inputs("ragged_fullatom_512")
    off, seq, ang = inp["offsets"], inp["seq"], inp["angles"]
    pert, _, _ = target_perturbation(inp["config"].seed, ang, inp["n_chains"])
    t, _ = oracle.fullatom_forward(off, seq, pert, GEOM)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    # chains reach 2000 residues; the stated 1e-3 A bound is at L = 1000, and
    # 9.5e-4 A is what the kernels reach on this batch
    _run(plan, "fullatom", off, seq, ang, t.astype(np.float32), "ragged_fullatom_512",
         coord_tol=1.2e-3)


def test_optional_outputs_and_empty_plan():
    import torch
    a2c = _a2c()
    off, seq, ang, t = _case("backbone", [40, 9], 311)
    plan = a2c.Plan("backbone", offsets=off)
    a, td = to_dev(ang), to_dev(t)
    loss_none, g1 = plan.mse_step(a, td, loss=False)
    loss, g2 = plan.mse_step(a, td)
    torch.cuda.synchronize()
    assert loss_none is None and torch.equal(g1, g2) and float(loss) > 0
    empty = a2c.Plan("backbone", offsets=np.array([0, 0], np.int32))
    e = torch.empty((3, 0), dtype=torch.float32, device="cuda:0")
    l0, g0 = empty.mse_step(e, e)
    torch.cuda.synchronize()
    assert float(l0) == 0.0 and g0.numel() == 0
