"""Plan-level behaviour on the GPU: the store-vs-recompute memory budget and
the autograd Function's "auto" mode, the autotuner's schedule cache (hit,
miss, malformed and unreadable files, schedules the plan would reject), and
graphs captured before a schedule change."""
import os

import numpy as np
import pytest

import oracle
from tests.gpu_util import COORD_TOL_A, GRAD_TOL_REL, grad_rel_err, to_dev
from workloads import BACKBONE_GEOMETRY, make_angles, offsets_from_lengths, upstream_grad

pytestmark = pytest.mark.gpu


def _a2c():
    import paper_1812_01108_amd as a2c
    return a2c


def _batch(lengths, seed):
    off = offsets_from_lengths(lengths)
    rng = np.random.Generator(np.random.PCG64(seed))
    return off, make_angles(rng, int(off[-1]), "mixture", 3)


def test_budget_decides_keep_or_recompute():
    a2c = _a2c()
    off, _ = _batch([40, 90, 7], 701)
    A = 3 * int(off[-1])
    assert a2c.Plan("backbone", offsets=off).keep_coords                   # no limit
    assert not a2c.Plan("backbone", offsets=off, mem_budget_bytes=0).keep_coords
    assert a2c.Plan("backbone", offsets=off, mem_budget_bytes=12 * A).keep_coords
    assert not a2c.Plan("backbone", offsets=off, mem_budget_bytes=12 * A - 1).keep_coords


@pytest.mark.parametrize("budget", [0, None])
def test_auto_mode_matches_oracle(budget):
    """Budget 0 (recompute in the adjoint, only the angles kept) and no
    limit (the coordinates kept) both give oracle-parity results through the
    autograd Function's default mode."""
    import torch
    a2c = _a2c()
    off, ang = _batch([1000, 33, 0, 257, 600], 703)
    plan = a2c.Plan("backbone", offsets=off, mem_budget_bytes=budget)
    assert plan.keep_coords == (budget is None)
    g = upstream_grad(5, plan.n_atoms)
    x = to_dev(ang).requires_grad_(True)
    out = a2c.angles_to_coords(x, plan)
    # what the Function kept between the passes
    saved = out.grad_fn.saved_tensors
    assert len(saved) == (2 if budget is None else 1)
    out.backward(to_dev(g))
    torch.cuda.synchronize()
    ref = oracle.backbone_forward(off, ang, BACKBONE_GEOMETRY)
    gref = oracle.backbone_backward(off, ang, BACKBONE_GEOMETRY, g)
    assert np.max(np.abs(out.detach().cpu().numpy() - ref)) <= COORD_TOL_A
    assert grad_rel_err(x.grad.cpu().numpy(), gref, off) <= GRAD_TOL_REL


def _tune(plan, ang, path, mode=True):
    a = to_dev(ang)
    g = to_dev(upstream_grad(3, plan.n_atoms))
    return plan.autotune(a, g, from_coords=mode, reps=1, cache_path=path)


def _key_lines(path):
    with open(path) as f:
        return [ln.split() for ln in f if ln.strip()]


def test_autotune_cache_miss_then_hit(tmp_path):
    a2c = _a2c()
    off, ang = _batch([300, 700, 5], 707)
    path = str(tmp_path / "tune.txt")
    plan = a2c.Plan("backbone", offsets=off)
    fs, bs = _tune(plan, ang, path)
    lines = _key_lines(path)
    assert len(lines) == 1 and lines[0][-5] == "coords"
    assert [int(v) for v in lines[0][-4:]] == [fs["res_per_lane"], fs["waves_per_group"],
                                                bs["res_per_lane"], bs["waves_per_group"]]
    # a different adjoint form is a different key: a miss that appends
    _tune(plan, ang, path, mode=False)
    lines = _key_lines(path)
    assert len(lines) == 2 and lines[1][-5] == "recompute"
    # a hit: a plan of the same shape takes the cached pair without timing
    # and without appending; edit the cached pair to a valid non-default one
    # so that taking it is visible
    with open(path, "w") as f:
        f.write(" ".join(lines[0][:-4] + ["1", "3", "2", "5"]) + "\n")
    plan2 = a2c.Plan("backbone", offsets=off)
    fs2, bs2 = _tune(plan2, ang, path)
    assert (fs2["res_per_lane"], fs2["waves_per_group"]) == (1, 3)
    assert (bs2["res_per_lane"], bs2["waves_per_group"]) == (2, 5)
    assert len(_key_lines(path)) == 1


@pytest.mark.parametrize("bad", ["4 17 1 1", "3 4", "1 0 1 1", "2 4 2", "x y", "1 4 1 4 junk", ""])
def test_autotune_cache_bad_lines_are_ignored(tmp_path, bad):
    """A matching line with schedules the plan would reject (W = 17, K = 3,
    W = 0, K = 4 on a full-atom plan), or malformed, is skipped: the
    schedules are tuned and the new choice appended."""
    a2c = _a2c()
    off, ang = _batch([300, 700, 5], 709)
    path = str(tmp_path / "tune.txt")
    plan = a2c.Plan("backbone", offsets=off)
    _tune(plan, ang, path)
    key = _key_lines(path)[0][:-4]
    with open(path, "w") as f:
        f.write(" ".join(key) + " " + bad + "\n")
    fs, bs = _tune(a2c.Plan("backbone", offsets=off), ang, path)
    lines = _key_lines(path)
    assert len(lines) == 2
    assert [int(v) for v in lines[1][-4:]] == [fs["res_per_lane"], fs["waves_per_group"],
                                                bs["res_per_lane"], bs["waves_per_group"]]


def test_autotune_cache_full_atom_rejects_k4(tmp_path):
    import torch
    a2c = _a2c()
    from workloads import random_sequence
    off = offsets_from_lengths([120, 33])
    rng = np.random.Generator(np.random.PCG64(711))
    ang = make_angles(rng, int(off[-1]), "mixture", 7)
    seq = random_sequence(rng, int(off[-1]))
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    path = str(tmp_path / "tune.txt")
    a = to_dev(ang)
    g = torch.ones((3, plan.n_atoms), device="cuda")
    plan.autotune(a, g, reps=1, cache_path=path)
    key = _key_lines(path)[0][:-4]
    with open(path, "w") as f:
        f.write(" ".join(key) + " 4 4 4 4\n")
    fs, _ = a2c.Plan("fullatom", offsets=off, seq=seq).autotune(a, g, reps=1, cache_path=path)
    assert fs["res_per_lane"] in (1, 2) and len(_key_lines(path)) == 2


def test_autotune_unreadable_cache(tmp_path):
    """A cache path that cannot be read or written (a directory) is ignored."""
    a2c = _a2c()
    off, ang = _batch([300, 70], 713)
    d = tmp_path / "a_directory"
    os.mkdir(d)
    fs, bs = _tune(a2c.Plan("backbone", offsets=off), ang, str(d))
    assert fs["res_per_lane"] in (1, 2, 4)


def test_graph_captured_before_a_schedule_change():
    """A graph captured on one schedule keeps replaying it after the plan
    moves to another (its tile tables stay allocated until the plan is
    destroyed): replays reproduce the eager results of the captured
    schedule, and eager calls after the change run the new one."""
    import torch
    a2c = _a2c()
    off, ang = _batch([700] * 20 + [4100, 13], 717)
    plan = a2c.Plan("backbone", offsets=off)
    plan.set_schedule(2, 8)
    a = to_dev(ang)
    gd = to_dev(upstream_grad(7, plan.n_atoms))
    coords = torch.empty((3, plan.n_atoms), device="cuda")
    grad = torch.empty_like(a)
    loss = torch.empty(1, device="cuda")

    def run():
        plan.forward(a, coords)
        plan.backward(a, gd, grad_angles=grad)
        plan.mse_step(a, gd, loss_out=loss)

    run()
    torch.cuda.synchronize()
    ref = [coords.clone(), grad.clone(), loss.clone()]
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            run()
    torch.cuda.current_stream().wait_stream(s)
    for sched in [(1, 2), (4, 16)]:
        plan.set_schedule(*sched)
        for o in (coords, grad, loss):
            o.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for o, r in zip((coords, grad, loss), ref):
            assert torch.equal(o, r)
    # eager calls use the new schedule and still agree with the oracle
    xyz = plan.forward(a)
    torch.cuda.synchronize()
    assert np.max(np.abs(xyz.cpu().numpy()
                         - oracle.backbone_forward(off, ang, BACKBONE_GEOMETRY))) < 4e-3
