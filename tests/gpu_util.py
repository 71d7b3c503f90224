"""Helpers for the GPU parity tests: run the HIP path through the Python
binding and measure errors against the oracle the way the tolerances are
stated (max-abs Angstrom for coordinates; normwise per chain, max over
chains, for gradients)."""
from __future__ import annotations

import numpy as np
import torch

COORD_TOL_A = 1e-3      # max-abs coordinate error, Angstrom
GRAD_TOL_REL = 1e-3     # ||g_gpu - g_ref||_inf / ||g_ref||_inf per chain


def window_counts(lengths, cap):
    """(windows when whole chains are packed greedily in order into windows
    of at most cap residues, fixed windows of cap residues): the plan uses
    the first layout when every chain fits and it takes at most 1/8 more
    windows than the second, or no more windows than the device has CUs
    (see uses_whole_chains)."""
    n, cur = 0, 0
    for L in lengths:
        if L == 0:
            continue
        if n == 0 or cur + L > cap:
            n += 1
            cur = 0
        cur += L
    R = int(sum(lengths))
    return n, -(-R // cap)


def uses_whole_chains(lengths, cap):
    """The plan's layout rule for windows of at most cap residues."""
    n_whole, n_fixed = window_counts(lengths, cap)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    return max(lengths) <= cap and (n_whole <= n_fixed + n_fixed // 8 or n_whole <= n_cu)


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def grad_rel_err(gpu, ref, res_off):
    """max over chains of ||gpu - ref||_inf / ||ref||_inf over all planes of
    the chain's residues (chains whose reference gradient is 0 use abs)."""
    worst = 0.0
    for c in range(len(res_off) - 1):
        r0, r1 = res_off[c], res_off[c + 1]
        if r1 == r0:
            continue
        d = np.max(np.abs(gpu[:, r0:r1] - ref[:, r0:r1]))
        s = np.max(np.abs(ref[:, r0:r1]))
        worst = max(worst, d / s if s > 0 else d)
    return float(worst)


def run_backbone(plan, angles, g, mode="coords", variant="scan"):
    """Forward + backward through the raw binding; returns numpy (coords, grad)."""
    a = to_dev(angles)
    gg = to_dev(g)
    ws = plan.new_workspace(variant)
    coords = plan.forward(a, variant=variant, workspace=ws)
    grad = plan.backward(a, gg, coords=coords if mode == "coords" else None, variant=variant,
                         workspace=ws)
    torch.cuda.synchronize()
    return coords.cpu().numpy(), grad.cpu().numpy()


def run_fullatom(plan, angles, g, mode="coords"):
    """Full-atom forward + backward; returns numpy (coords, grad [7][R])."""
    a = to_dev(angles)
    gg = to_dev(g)
    coords = plan.forward(a)
    grad = plan.backward(a, gg, coords=coords if mode == "coords" else None)
    torch.cuda.synchronize()
    return coords.cpu().numpy(), grad.cpu().numpy()
