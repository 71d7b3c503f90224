"""Benchmark: forward+backward residues/s of the dihedral -> Cartesian map.

One step = the whole path over one batch: forward coordinates and the adjoint
angle gradient for a fixed upstream gradient, through the torch.autograd
Function.  Steps are captured in HIP graphs, --steps-per-graph complete
steps per graph (one graph launch costs the host more than one step takes
on the GPU); every timed step runs the whole path.  Inputs are resident in
HBM before timing starts.  Prints one JSON line; besides the (warm) timed
steps it carries "cold": the step time when a 512 MiB device write precedes
every step (captured in the same graph as the steps), so that no input or
output is left in the caches, and the plain device-copy bandwidth the HBM
fractions can be read against.

Default workload: the largest single-GPU batch, 4096 backbone chains with
lengths uniform in [20, 1000] (about 2.09 M residues) packed back to back,
Ramachandran-like mixture angles, omega = pi, upstream gradient iid N(0,1).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per launch (float32): what each kernel must move.
# Backbone, per residue: angles 12 B, coordinates 36 B, upstream gradient
# 36 B, angle gradient 12 B.  Full-atom, per residue: angles 4 (3 + n_chi) B,
# residue code 1 B, residue atom offset 4 B, 12 B per atom for coordinates
# and for their gradient, 28 B of angle gradient (seven planes).  The inverse
# map reads the three backbone atoms of every residue (neighbours' are the
# same bytes) and, full-atom, the side atoms its chi torsions use (n_chi + 1
# for a residue with any chi: the first side frame's origin and one atom per
# chi), plus the residue code and atom offset; it writes every angle plane.
def algorithmic_bytes(model, kernel, R, A=None, n_chi_total=None, n_side_used=None):
    if model == "backbone":
        per = {"forward": 12 + 36, "backward_coords": 36 + 36 + 12,
               "backward_recompute": 12 + 36 + 12, "inverse": 36 + 12}[kernel]
        return per * R
    if kernel == "inverse":
        return 36 * R + 12 * n_side_used + 5 * R + 28 * R
    ang = 4 * (3 * R + n_chi_total)
    meta = 5 * R
    return {"forward": ang + meta + 12 * A,
            "backward_recompute": ang + meta + 12 * A + 28 * R,
            "backward_coords": meta + 24 * A + 28 * R}[kernel]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--steps-per-graph", type=int, default=10,
                   help="complete steps captured back to back in one graph")
    p.add_argument("--workload", default="ragged_backbone_4096")
    p.add_argument("--mode", default=None, choices=["coords", "recompute"],
                   help="adjoint reads the forward's coordinates, or recomputes the frames "
                        "(default: coords; recompute for the training-step workload)")
    p.add_argument("--schedule", default=None, help="K,W (residues per lane, waves per group) "
                   "for both the forward and the adjoint, or K,W,aK,aW (forward, adjoint; the "
                   "backbone forward also takes K = 8); default: autotuned")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 256 MiB device copy (HBM counter calibration)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--kernel-reps", type=int, default=50)
    p.add_argument("--fused", action="store_true",
                   help="training-step workload, squared-distance loss: one fused kernel "
                        "(forward, loss gradient and adjoint; a2c_mse_step) per step")
    p.add_argument("--loss", default="mse", choices=["mse", "lrmsd"],
                   help="training-step workload: sum |r - t|^2 (default) or the per-chain "
                        "LRMSD of the Loss function section, summed over chains")
    return p.parse_args()


def make_step(a2c, plan, angles, grad_up, mode, target=None, loss="mse"):
    """One step: forward through the autograd Function, then the adjoint for
    the fixed upstream gradient, or (with a target) for a loss formed inside
    the step: sum |r - t|^2 (gradient 2 (r - t)), or sum over chains of the
    LRMSD (its forward and backward kernels run inside the step)."""
    import torch

    x = angles.clone().requires_grad_(True)

    def step():
        out = a2c.angles_to_coords(x, plan, mode=mode)
        if target is not None and loss == "lrmsd":
            lval = a2c.lrmsd(out, target, plan).sum()
            (gx,) = torch.autograd.grad(lval, x)
            return out, gx
        g = grad_up if target is None else 2.0 * (out - target)
        (gx,) = torch.autograd.grad(out, x, g)
        return out, gx

    return step


def capture(step, warm=3, per_graph=1):
    """Graphs of `per_graph` back-to-back steps and of one step; returns
    ((graph_n, n), graph_1, outputs of the last captured step)."""
    import torch

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(warm):
            step()
    torch.cuda.current_stream().wait_stream(s)
    g1 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g1):
        outs = step()
    n = max(1, per_graph)
    gn = g1
    if n > 1:
        gn = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gn):
            for _ in range(n):
                outs = step()
    return (gn, n), g1, outs


def _run_steps(graphs, k):
    (gn, n), g1 = graphs
    for _ in range(k // n):
        gn.replay()
    for _ in range(k % n):
        g1.replay()


def time_graph(graphs, steps, warmup):
    """Exactly `warmup` untimed steps, then wall time of exactly `steps`."""
    import torch

    _run_steps(graphs, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _run_steps(graphs, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def time_cold(step, R, n=10, reps=5, flush_bytes=512 << 20):
    """Cold-cache step time.  One graph holds n x (512 MiB device write,
    step) and a second graph the n writes alone; the write (twice the
    256 MiB Infinity Cache) evicts the step's data before every step.  The
    cold step time is the difference of the two graphs' durations over n,
    so neither the graph launch nor the writes are counted.  Both graphs are
    timed with HIP events on the stream they run on; best of `reps`."""
    import torch

    buf = torch.empty(flush_bytes // 4, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
        buf.fill_(1.0)
    torch.cuda.current_stream().wait_stream(s)
    g_both, g_flush = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_both):
        for i in range(n):
            buf.fill_(float(i + 1))   # a fill kernel, not a memset node
            step()
    with torch.cuda.graph(g_flush):
        for i in range(n):
            buf.fill_(float(i + 1))
    st = torch.cuda.current_stream()

    def best(g):
        g.replay()
        torch.cuda.synchronize()
        out = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            g.replay()
            e1.record(st)
            e1.synchronize()
            out = min(out, e0.elapsed_time(e1) / 1000.0)
        return out

    t_both, t_flush = best(g_both), best(g_flush)
    del g_both, g_flush, buf
    t = max(t_both - t_flush, 1e-9) / n
    return {"value": R / t, "ms_per_step": t * 1000.0, "steps_per_graph": n,
            "flush": "512 MiB device write before every step, captured with the steps; "
                     "cold step = (graph of writes and steps - graph of writes alone) / n",
            "flush_only_ms_per_step": t_flush * 1000.0 / n}


def copy_bandwidth_gbs(nbytes=1 << 30, reps=5):
    """Plain device-to-device copy of `nbytes` (torch copy_, one kernel):
    (bytes read + bytes written) / duration, best of `reps`, HIP events on
    the current stream.  The HBM fractions are quoted against the 8 TB/s
    peak; this is what a streaming kernel reaches on the same board."""
    import torch

    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        y.copy_(x)
        e1.record(st)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1000.0)
    del x, y
    return 2 * nbytes / best / 1e9


def kernel_avg_us(launch, reps):
    """Average duration of one kernel launch: `reps` back-to-back launches
    captured in a graph, timed with HIP events on the stream they run on."""
    import torch

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        launch()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            launch()
    g.replay()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(5):
        e0.record(st)
        g.replay()
        e1.record(st)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1000.0 / reps)
    return best


# Sources a model's kernels are compiled from: profiles/traffic.json records
# their joint hash, so a counter figure is reported only for the kernels it
# was measured on.
KERNEL_SOURCES = {
    "backbone": ["backbone.hip", "scan.h", "affine.h", "sincos.h", "a2c_internal.h"],
    "fullatom": ["fullatom.hip", "scan.h", "affine.h", "sincos.h", "a2c_internal.h"],
}


def kernel_source_sha(model):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[model]:
        with open(os.path.join(ROOT, "paper_1812_01108_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_key(kernel_key, schedule):
    """Key of a committed counter record: workload:kernel@K,W."""
    return f"{kernel_key}@{schedule[0]},{schedule[1]}"


def traffic_from_profiles(kernel_key, model, n_units, schedule):
    """HBM bytes per launch from committed rocprofv3 counter summaries, valid
    only while the kernel source they were taken from is unchanged and for
    the schedule they were taken with."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(profile_key(kernel_key, schedule))
        sha = kernel_source_sha(model)
        if (not rec or rec.get("source_sha") != sha or rec.get("units") != n_units
                or rec.get("schedule") != list(schedule)):
            return None
        return rec["bytes_per_launch"]
    except Exception:
        return None


# VALU issue: one wave64 instruction occupies a 16-lane SIMD for 4 cycles
# (unpacked float32); 256 CUs x 4 SIMDs at 2.4 GHz.
SIMDS, CLOCK_MHZ, CYCLES_PER_VALU = 1024, 2400.0, 4


def valu_issue_from_profiles(kernel_key, model, schedule, kernel_us):
    """Fraction of the chip's VALU issue rate the kernel used: committed SQ
    counters (VALU instructions per wave, waves per dispatch) over the
    kernel's measured duration; valid only for the sources and schedule the
    counters were taken with."""
    path = os.path.join(ROOT, "profiles", "valu.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(profile_key(kernel_key, schedule))
        if (not rec or rec.get("source_sha") != kernel_source_sha(model)
                or rec.get("schedule") != list(schedule)):
            return None
        issue_us = (rec["waves"] * rec["valu_per_wave"] * CYCLES_PER_VALU
                    / (SIMDS * CLOCK_MHZ))
        return {"valu_per_wave": rec["valu_per_wave"], "waves": rec["waves"],
                "issue_us": round(issue_us, 3), "frac": round(issue_us / kernel_us, 4),
                "profile": rec["profile"],
                "source": "committed rocprofv3 SQ_WAVES/SQ_INSTS_VALU runs over this run's "
                          "kernel duration"}
    except Exception:
        return None


def chain_grad_rel(gpu, ref, off):
    worst = 0.0
    for c in range(len(off) - 1):
        r0, r1 = off[c], off[c + 1]
        if r1 > r0:
            sc = np.max(np.abs(ref[:, r0:r1]))
            d = float(np.max(np.abs(gpu[:, r0:r1] - ref[:, r0:r1])))
            worst = max(worst, d / sc if sc > 0 else d)
    return worst


def cpu_baseline(model, inp, g_np, gpu_coords, gpu_grad, budget_s=12.0, single_budget_s=4.0,
                 quat_coords=None):
    """The FP64 oracle (forward + O(N) adjoint, OpenMP over chains) on the
    full batch, repeated for about budget_s seconds of host time on every
    host core, then on one thread for about single_budget_s seconds (whole
    batches, at least one).  The parity figures compare the GPU output of
    the timed graph with the oracle's on the same float32 inputs."""
    import oracle
    from workloads import BACKBONE_GEOMETRY

    cores = len(os.sched_getaffinity(0))
    off, ang, seq = inp["offsets"], inp["angles"], inp["seq"]
    R = int(off[-1])

    def run(threads):
        if model == "backbone":
            ref = oracle.backbone_forward(off, ang, BACKBONE_GEOMETRY, n_threads=threads)
            gref = oracle.backbone_backward(off, ang, BACKBONE_GEOMETRY, g_np, n_threads=threads)
        else:
            ref, _ = oracle.fullatom_forward(off, seq, ang, BACKBONE_GEOMETRY, n_threads=threads)
            gref = oracle.fullatom_backward(off, seq, ang, BACKBONE_GEOMETRY, g_np,
                                            n_threads=threads)
        return ref, gref

    def timed(threads, budget):
        n, t_total, out = 0, 0.0, None
        while (n == 0 or t_total < budget) and n < 100000:
            t0 = time.perf_counter()
            out = run(threads)
            t_total += time.perf_counter() - t0
            n += 1
        return n, t_total, out

    n, t_total, (ref, gref) = timed(cores, budget_s)
    n1, t1, _ = timed(1, single_budget_s)
    lens = np.diff(off)
    parity = {"max_abs_coord_A": float(np.max(np.abs(gpu_coords - ref))),
              "max_chain_grad_rel": chain_grad_rel(gpu_grad, gref, off),
              "max_chain_len": int(lens.max()) if len(lens) else 0,
              "chains_len_ge_900": int(np.sum(lens >= 900)),
              "compared": "every atom and every angle gradient of the batch"}
    if quat_coords is not None:
        parity["quaternion_state_max_abs_coord_A"] = float(np.max(np.abs(quat_coords - ref)))
    return {"value": n * R / t_total, "unit": "residues/s", "cores": cores, "kind": "oracle",
            "sample": f"full batch ({R} residues) x {n} repeats, FP64 {model} forward + O(N) "
                      f"adjoint, OpenMP over chains",
            "single_thread": {"value": n1 * R / t1, "unit": "residues/s", "cores": 1,
                              "sample": f"full batch x {n1} repeats on one thread"}}, parity


def copy_calibration(torch):
    """A plain device copy of 256 MiB, ten times: under rocprofv3 --pmc its
    FETCH_SIZE / WRITE_SIZE per dispatch give the counters' scale against a
    known byte count."""
    n = 64 * 1024 * 1024
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(10):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 10}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(chains are independent: a multi-GPU run would shard the packed batch by "
              "residue count with no exchange).", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        copy_calibration(torch)
        return

    import paper_1812_01108_amd as a2c
    from workloads import CONFIGS, make_inputs, upstream_grad

    cfg = CONFIGS[args.workload]
    model = cfg.model
    training = args.workload == "ragged_fullatom_512"
    mode = args.mode if args.mode else ("recompute" if training else "coords")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    inp = make_inputs(cfg)
    R = inp["n_res"]
    plan = a2c.Plan(model, offsets=inp["offsets"], seq=inp["seq"], device=dev)
    angles = torch.from_numpy(inp["angles"]).to(dev)
    target = None
    if training:
        # target: the layer on perturbed angles, then a random rigid motion
        # per chain (built once, outside the timed region)
        from workloads import target_perturbation
        pert, quat, trans = target_perturbation(cfg.seed, inp["angles"], inp["n_chains"])
        t_xyz = plan.forward(torch.from_numpy(pert).to(dev))
        ca, _ = plan.atom_offsets()
        counts = torch.from_numpy(np.diff(ca).astype(np.int64)).to(dev)
        q = torch.from_numpy(quat).to(dev, torch.float64)
        w, x, y, z = q.unbind(1)
        rot = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                           2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                           2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
                          1).view(-1, 3, 3).float()
        rot_a = torch.repeat_interleave(rot, counts, dim=0)
        tr_a = torch.repeat_interleave(torch.from_numpy(trans).to(dev).float(), counts, dim=0)
        target = torch.stack([rot_a[:, i, 0] * t_xyz[0] + rot_a[:, i, 1] * t_xyz[1] +
                              rot_a[:, i, 2] * t_xyz[2] + tr_a[:, i] for i in range(3)])
        torch.cuda.synchronize()
    g_np = upstream_grad(cfg.seed, plan.n_atoms)
    grad_up = torch.from_numpy(g_np).to(dev)
    if args.schedule:
        sv = [int(v) for v in args.schedule.split(",")]
        if len(sv) not in (2, 4):
            sys.exit("--schedule takes K,W or K,W,aK,aW")
        if len(sv) == 2:
            plan.set_schedule(sv[0], sv[1])
        else:
            plan.set_forward_schedule(sv[0], sv[1])
            plan.set_adjoint_schedule(sv[2], sv[3])
    elif args.fused:
        plan.autotune(angles, reps=50, mse_target=target)
    else:
        plan.autotune(angles, grad_up, from_coords=mode == "coords", reps=50)

    # scan form, whole step in one graph
    loss = args.loss if training else None
    if args.fused and (not training or loss != "mse"):
        sys.exit("--fused applies to the training-step workload with the squared-distance loss")
    if args.fused:
        fused_xyz = torch.empty((3, plan.n_atoms), dtype=torch.float32, device=dev)
        fused_grad = torch.empty_like(angles)
        fused_loss = torch.zeros(1, device=dev)

        def step():
            plan.mse_step(angles, target, coords=fused_xyz, grad_angles=fused_grad,
                          loss_out=fused_loss)
            return fused_xyz, fused_grad
    else:
        step = make_step(a2c, plan, angles, grad_up, mode, target, loss or "mse")
    gn, g1, outs = capture(step, per_graph=min(args.steps_per_graph, max(args.steps, 1)))
    dt = time_graph((gn, g1), args.steps, args.warmup)
    ms = dt * 1000.0 / args.steps
    value = R * args.steps / dt
    cold = time_cold(step, R)
    copy_gbs = copy_bandwidth_gbs()
    gpu_coords = outs[0].detach().cpu().numpy()
    gpu_grad = outs[1].detach().cpu().numpy()
    lr_info = None
    if training and loss == "mse":
        g_np = 2.0 * (gpu_coords.astype(np.float64) - target.cpu().numpy())
        grad_up = torch.from_numpy(g_np.astype(np.float32)).to(dev)
    elif training:
        # the loss gradient the step fed to the adjoint, and the LRMSD
        # kernels' durations (forward reads both sets: 24 B per atom;
        # backward reads both and writes the gradient: 36 B per atom)
        xyz_t = outs[0].detach()
        ws = plan.lrmsd_workspace()
        lr_out = plan.lrmsd_forward(xyz_t, target, ws)
        ones = torch.ones(plan.n_chains, device=dev)
        grad_up = plan.lrmsd_backward(xyz_t, target, ones, ws)
        lf = kernel_avg_us(lambda: plan.lrmsd_forward(xyz_t, target, ws, lr_out),
                           args.kernel_reps)
        lb = kernel_avg_us(lambda: plan.lrmsd_backward(xyz_t, target, ones, ws, grad_up),
                           args.kernel_reps)
        A = plan.n_atoms
        lr_info = {"forward_us": round(lf, 3), "backward_us": round(lb, 3),
                   "forward_GBs": round(24 * A / (lf * 1e-6) / 1e9, 1),
                   "backward_GBs": round(36 * A / (lb * 1e-6) / 1e9, 1),
                   "mean_lrmsd_A": float(lr_out.mean())}
        torch.cuda.synchronize()

    # per-kernel durations for the roofline
    coords_buf = torch.empty((3, plan.n_atoms), device=dev)
    gang = torch.empty_like(angles)
    plan.forward(angles, coords_buf)
    fwd_us = kernel_avg_us(lambda: plan.forward(angles, coords_buf), args.kernel_reps)
    if mode == "coords":
        bwd_us = kernel_avg_us(lambda: plan.backward(angles, grad_up, coords=coords_buf,
                                                     grad_angles=gang), args.kernel_reps)
        bwd_key = "backward_coords"
    else:
        bwd_us = kernel_avg_us(lambda: plan.backward(angles, grad_up, grad_angles=gang),
                               args.kernel_reps)
        bwd_key = "backward_recompute"
    kern = {"forward": fwd_us, bwd_key: bwd_us}
    if args.fused:
        kern = {"fused_step": kernel_avg_us(step, args.kernel_reps)}
    dom = max(kern, key=kern.get)
    n_chi_total = n_side_used = None
    if model == "fullatom":
        from paper_1812_01108_amd.residues import default_table
        chi_of = np.array(default_table().n_chi)[inp["seq"]]
        n_chi_total = int(np.sum(chi_of))
        n_side_used = int(np.sum(chi_of + (chi_of > 0)))
    if args.fused:
        # angles, codes and offsets, the target (12 B per atom), the
        # coordinates written (12 B per atom) and the angle gradient
        nbytes = (algorithmic_bytes(model, "forward", R, plan.n_atoms, n_chi_total)
                  + 12 * plan.n_atoms + 28 * R)
    else:
        nbytes = algorithmic_bytes(model, dom, R, plan.n_atoms, n_chi_total)
    achieved = nbytes / (kern[dom] * 1e-6) / 1e9
    # the dominant kernel's own schedule (forward, or adjoint / fused step)
    dom_sched = plan.schedule if dom == "forward" else plan.adjoint_schedule
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profiles(
                f"{cfg.name}:{dom}", model, R,
                (dom_sched["res_per_lane"], dom_sched["waves_per_group"])),
            "kernel": dom,
            "kernel_us": {k: round(v, 3) for k, v in kern.items()},
            "bytes_per_launch": nbytes,
            "traffic_source": "committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs "
                              "(profiles/traffic.json), reported only for the kernel sources "
                              "and schedule they were taken on",
            "valu_issue": valu_issue_from_profiles(
                f"{cfg.name}:{dom}", model,
                (dom_sched["res_per_lane"], dom_sched["waves_per_group"]), kern[dom]),
            "copy_GBs": round(copy_gbs, 1),
            "frac_of_copy": round(achieved / copy_gbs, 4)}

    # the inverse map (coordinates -> angles) on the forward's coordinates
    back = torch.empty_like(angles)
    plan.coords_to_angles(coords_buf, out=back)
    inv_us = kernel_avg_us(lambda: plan.coords_to_angles(coords_buf, out=back), args.kernel_reps)
    inv_bytes = algorithmic_bytes(model, "inverse", R, plan.n_atoms, n_chi_total, n_side_used)
    inv_gbs = inv_bytes / (inv_us * 1e-6) / 1e9
    inverse = {"us": round(inv_us, 3), "bytes_per_launch": inv_bytes,
               "GBs": round(inv_gbs, 1), "frac": round(inv_gbs / HBM_PEAK_GBS, 4)}

    plain = None
    if model == "backbone" and not args.no_plain:
        pstep = make_step(a2c, plan, angles, grad_up, "plain")
        psteps = max(3, min(args.steps, 20))
        pgn, pg1, _ = capture(pstep, warm=1, per_graph=min(args.steps_per_graph, psteps))
        pdt = time_graph((pgn, pg1), psteps, 2)
        plain = {"value": R * psteps / pdt, "ms_per_step": pdt * 1000.0 / psteps,
                 "form": "one workgroup per chain, sequential product storing M_i, "
                         "O(atoms x angles) gradient"}

    # the comparison form with the quaternion + translation scan state
    # (forward only): duration on the forward's schedule, error in parity
    quat, quat_np = None, None
    if model == "backbone":
        qbuf = torch.empty_like(coords_buf)
        plan.forward(angles, qbuf, variant="scan_quat")
        q_us = kernel_avg_us(lambda: plan.forward(angles, qbuf, variant="scan_quat"),
                             args.kernel_reps)
        quat_np = qbuf.cpu().numpy()
        quat = {"forward_us": round(q_us, 3), "affine_forward_us": round(fwd_us, 3),
                "GBs": round(algorithmic_bytes(model, "forward", R) / (q_us * 1e-6) / 1e9, 1),
                "state": "unit quaternion + translation (7 floats) in the scans and look-back"}

    cpu, parity = (None, None)
    if not args.no_cpu_baseline:
        if loss == "lrmsd":
            # the oracle's LRMSD gradient of the step's coordinates, fed to
            # the oracle adjoint inside the baseline's parity check
            from oracle import lrmsd as olr
            ca, _ = plan.atom_offsets()
            g_np = olr.lrmsd_grad_batch(target.cpu().numpy().astype(np.float64),
                                        gpu_coords.astype(np.float64), ca,
                                        np.ones(plan.n_chains)).astype(np.float32)
        cpu, parity = cpu_baseline(model, inp, g_np, gpu_coords, gpu_grad, quat_coords=quat_np)

    sched, asched = plan.schedule, plan.adjoint_schedule
    line = {
        "metric": "fwd+bwd residues/sec FP32 (scan vs plain GPU) at <=1e-3 A vs FP64 oracle",
        "value": value, "unit": "residues/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg.name, "model": model, "n_chains": inp["n_chains"],
                   "residues": R, "atoms": plan.n_atoms, "angles": cfg.angles,
                   "adjoint": "fused" if args.fused else mode, "loss_in_graph": loss,
                   "res_per_lane": sched["res_per_lane"],
                   "waves_per_group": sched["waves_per_group"], "tiles": sched["n_tiles"],
                   "adjoint_res_per_lane": asched["res_per_lane"],
                   "adjoint_waves_per_group": asched["waves_per_group"],
                   "adjoint_tiles": asched["n_tiles"], "steps_per_graph": gn[1]},
        "roofline": roof,
        "lrmsd": lr_info,
        "inverse_map": inverse,
        "plain_gpu": plain,
        "quaternion_state": quat,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "cold": cold,
        "cpu_baseline": cpu,
        "parity": parity,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
