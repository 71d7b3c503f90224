"""The no-allocation LRMSD forward (a2c_lrmsd_forward_noalloc) against the
workspace form it varies (a2c_lrmsd_forward): same kernels, so the per-chain
values must agree bit for bit, on two calls in a row (the second with a
smaller input, over the array the first one left behind) and again on the
first input afterwards; both are also held to the FP64 oracle (Kabsch) at
the LRMSD parity tolerance.  A plan whose state exceeds the fixed array is
refused before anything is enqueued."""
import numpy as np
import pytest

from oracle import lrmsd as olr
from tests.gpu_util import to_dev
from workloads import offsets_from_lengths, random_sequence

pytestmark = pytest.mark.gpu
LR_RTOL, LR_ATOL = 1e-5, 1e-6


def _case(model, lengths, seed):
    import paper_1812_01108_amd as a2c
    off = offsets_from_lengths(lengths)
    rng = np.random.Generator(np.random.PCG64(seed))
    if model == "backbone":
        plan = a2c.Plan("backbone", offsets=off)
    else:
        plan = a2c.Plan("fullatom", offsets=off, seq=random_sequence(rng, int(off[-1])))
    A = plan.n_atoms
    y = (rng.standard_normal((3, A)) * 12.0).astype(np.float32)
    x = (y + rng.standard_normal((3, A)) * 2.0).astype(np.float32)
    ca, _ = plan.atom_offsets()
    return plan, y, x, np.asarray(ca, dtype=np.int64)


def _both(plan, y, x):
    import torch
    yd, xd = to_dev(y), to_dev(x)
    ref = plan.lrmsd_forward(yd, xd, plan.lrmsd_workspace())
    out = torch.full((plan.n_chains,), float("nan"), device=yd.device)
    plan.lrmsd_forward_noalloc(yd, xd, out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


def _check(plan, y, x, ca, label):
    got, ref = _both(plan, y, x)
    exact = olr.lrmsd_batch(x.astype(np.float64), y.astype(np.float64), ca)
    print(f"{label}: chains={plan.n_chains} atoms={plan.n_atoms} "
          f"max|noalloc-ws|={np.max(np.abs(got - ref)):.3e} "
          f"max|noalloc-oracle|={np.max(np.abs(got - exact)):.3e}", flush=True)
    assert np.array_equal(got, ref)
    assert np.all(np.abs(got - exact) <= LR_RTOL * exact + LR_ATOL)


def test_noalloc_matches_workspace_form_on_consecutive_calls():
    # full-atom: empty chains, one-residue chains and chains of several
    # 4096-atom segments; then a smaller backbone batch on the same array
    big = [0, 1, 700, 35, 0, 1200, 3, 480, 90]
    small = [5, 0, 17, 2]
    plan1, y1, x1, ca1 = _case("fullatom", big, 77)
    _check(plan1, y1, x1, ca1, "first call (full-atom, 9 chains)")
    plan2, y2, x2, ca2 = _case("backbone", small, 78)
    _check(plan2, y2, x2, ca2, "second call (backbone, 4 chains)")
    _check(plan1, y1, x1, ca1, "first input again")


def test_noalloc_refuses_state_beyond_the_array():
    import torch

    import paper_1812_01108_amd as a2c
    from paper_1812_01108_amd import _lib
    n = 21000   # 21000 one-residue chains: 208 bytes each, beyond 4 MiB
    plan = a2c.Plan("backbone", offsets=np.arange(n + 1, dtype=np.int32))
    assert _lib.load().a2c_lrmsd_forward_noalloc is not None
    y = torch.zeros((3, plan.n_atoms), device="cuda")
    out = torch.full((n,), -1.0, device="cuda")
    with pytest.raises(_lib.A2CError) as ei:
        plan.lrmsd_forward_noalloc(y, y, out)
    assert ei.value.status == -3   # A2C_ERR_WORKSPACE
    assert "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.all(out == -1.0)
