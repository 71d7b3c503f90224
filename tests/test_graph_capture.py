"""HIP-graph capture of the calls the header states are capturable (no
allocation, no synchronisation): the full-atom forward and adjoints, the
fused training step, the LRMSD forward and backward, and the inverse map.
Each graph is replayed several times with eager work (zeroing the outputs,
synchronisations) between replays, and every replay must reproduce the eager
result bit for bit (the same kernels run on the same inputs).  Multi-chunk
tiles are included (their carries live in LDS, not in device scratch)."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import to_dev
from workloads import (BACKBONE_GEOMETRY, make_angles, offsets_from_lengths, random_sequence,
                       target_perturbation)

pytestmark = pytest.mark.gpu


def _a2c():
    import paper_1812_01108_amd as a2c
    return a2c


def _fullatom_case(seed=501):
    lengths = [300, 17, 700, 1, 90]
    off = offsets_from_lengths(lengths)
    R = int(off[-1])
    rng = np.random.Generator(np.random.PCG64(seed))
    ang = make_angles(rng, R, "mixture", 7)
    seq = random_sequence(rng, R)
    pert, _, _ = target_perturbation(seed, ang, len(lengths))
    t, _ = oracle.fullatom_forward(off, seq, pert, BACKBONE_GEOMETRY)
    return off, seq, ang, t.astype(np.float32)


def _capture_and_check(run, outs, replays=3):
    """run() enqueues the work writing into the tensors `outs`; compare the
    eager result with every replay of a captured graph."""
    import torch
    run()
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            run()
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(replays):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r)


@pytest.mark.parametrize("K,W", [(1, 4), (1, 1)])
def test_fullatom_forward_and_adjoints(K, W):
    import torch
    a2c = _a2c()
    off, seq, ang, _ = _fullatom_case()
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    plan.set_schedule(K, W)
    a = to_dev(ang)
    g = torch.randn((3, plan.n_atoms), device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    coords = torch.empty((3, plan.n_atoms), device="cuda")
    ga, gb = torch.empty_like(a), torch.empty_like(a)

    def run():
        plan.forward(a, coords)
        plan.backward(a, g, coords=coords, grad_angles=ga)
        plan.backward(a, g, grad_angles=gb)

    _capture_and_check(run, [coords, ga, gb])


@pytest.mark.parametrize("model", ["backbone", "fullatom"])
def test_fused_step(model):
    import torch
    a2c = _a2c()
    if model == "fullatom":
        off, seq, ang, t = _fullatom_case(503)
        plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    else:
        off = offsets_from_lengths([700, 5, 4096 + 3])
        rng = np.random.Generator(np.random.PCG64(505))
        ang = make_angles(rng, int(off[-1]), "mixture", 3)
        t = rng.normal(0, 20, (3, 3 * int(off[-1]))).astype(np.float32)
        plan = a2c.Plan("backbone", offsets=off)
    a, td = to_dev(ang), to_dev(t)
    coords = torch.empty((3, plan.n_atoms), device="cuda")
    grad = torch.empty_like(a)
    loss_out = torch.empty(1, device="cuda")

    def run():
        plan.mse_step(a, td, coords=coords, grad_angles=grad, loss_out=loss_out)

    # every replay sums the tiles' shares again: the count of finished tiles
    # the last tile re-arms must start each replay at zero
    _capture_and_check(run, [coords, grad, loss_out])
    loss, _ = plan.mse_step(a, td)
    torch.cuda.synchronize()
    assert torch.equal(loss_out[0], loss)


def test_lrmsd_and_inverse_map():
    import torch
    a2c = _a2c()
    off, seq, ang, t = _fullatom_case(507)
    plan = a2c.Plan("fullatom", offsets=off, seq=seq)
    a, td = to_dev(ang), to_dev(t)
    coords = plan.forward(a)
    torch.cuda.synchronize()
    ws = plan.lrmsd_workspace()
    val = torch.empty(plan.n_chains, device="cuda")
    gout = torch.linspace(0.5, 2.0, plan.n_chains, device="cuda")
    gc = torch.empty_like(coords)
    back = torch.empty_like(a)

    def run():
        plan.lrmsd_forward(coords, td, ws, out=val)
        plan.lrmsd_backward(coords, td, gout, ws, grad_coords=gc)
        plan.coords_to_angles(coords, out=back)

    _capture_and_check(run, [val, gc, back])
