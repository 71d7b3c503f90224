"""Host-side logic of bench.py (no GPU): the one-GPU guard, exact step
counting when several steps share a graph, the algorithmic byte counts the
roofline divides by, and the gating of the committed HBM traffic figures."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


class _Graph:
    def __init__(self, steps, log):
        self.steps, self.log = steps, log

    def replay(self):
        self.log.append(self.steps)


@pytest.mark.parametrize("k,n", [(23, 10), (20, 10), (7, 10), (0, 10), (5, 1)])
def test_exactly_k_steps_run(k, n):
    log = []
    bench._run_steps(((_Graph(n, log), n), _Graph(1, log)), k)
    assert sum(log) == k
    assert log.count(n) == (k // n if n > 1 else k)


def test_algorithmic_bytes_per_residue():
    R = 1000
    assert bench.algorithmic_bytes("backbone", "forward", R) == 48 * R
    assert bench.algorithmic_bytes("backbone", "backward_coords", R) == 84 * R
    assert bench.algorithmic_bytes("backbone", "backward_recompute", R) == 60 * R
    A, n_chi = 8350, 1950
    ang, meta = 4 * (3 * R + n_chi), 5 * R
    assert bench.algorithmic_bytes("fullatom", "forward", R, A, n_chi) == ang + meta + 12 * A
    assert (bench.algorithmic_bytes("fullatom", "backward_recompute", R, A, n_chi)
            == ang + meta + 12 * A + 28 * R)
    assert (bench.algorithmic_bytes("fullatom", "backward_coords", R, A, n_chi)
            == meta + 24 * A + 28 * R)


def test_inverse_map_bytes():
    """Backbone: three atoms in, three angles out per residue.  Full-atom: a
    residue with n chi angles reads n + 1 side atoms (none without chi)."""
    import numpy as np
    from paper_1812_01108_amd.residues import default_table
    assert bench.algorithmic_bytes("backbone", "inverse", 10) == 480
    n_chi = np.array(default_table().n_chi)
    seq = np.arange(20)
    used = int(np.sum(n_chi[seq] + (n_chi[seq] > 0)))
    # glycine and alanine have no chi, so 18 residue types read side atoms
    assert used == int(n_chi.sum()) + 18
    assert (bench.algorithmic_bytes("fullatom", "inverse", 20, n_side_used=used)
            == 20 * (36 + 5 + 28) + 12 * used)


def test_traffic_only_for_the_profiled_sources_and_schedule():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    full_key, r = next(iter(rec.items()))
    key = full_key.split("@")[0]   # records are keyed workload:kernel@K,W
    assert full_key == bench.profile_key(key, r["schedule"])
    model = "fullatom" if "fullatom" in key else "backbone"
    got = bench.traffic_from_profiles(key, model, r["units"], tuple(r["schedule"]))
    if r["source_sha"] == bench.kernel_source_sha(model):
        assert got == r["bytes_per_launch"]
    else:
        assert got is None
    K, W = r["schedule"]
    # a schedule of the same kernel with no record of its own
    W2 = next(w for w in range(W + 1, 64) if bench.profile_key(key, (K, w)) not in rec)
    assert bench.traffic_from_profiles(key, model, r["units"], (K, W2)) is None
    assert bench.traffic_from_profiles(key, model, r["units"] + 1, (K, W)) is None
    assert bench.traffic_from_profiles("no_such_workload:forward", model, 1, (K, W)) is None


def test_valu_issue_only_for_the_profiled_sources_and_schedule():
    rec = json.load(open(os.path.join(ROOT, "profiles", "valu.json")))
    full_key, r = next(iter(rec.items()))
    key = full_key.split("@")[0]
    model = "fullatom" if "fullatom" in key else "backbone"
    got = bench.valu_issue_from_profiles(key, model, tuple(r["schedule"]), 10.0)
    if r["source_sha"] == bench.kernel_source_sha(model):
        issue_us = r["waves"] * r["valu_per_wave"] * 4 / (1024 * 2400.0)
        assert got["issue_us"] == round(issue_us, 3)
        assert got["frac"] == round(issue_us / 10.0, 4)
    else:
        assert got is None
    K, W = r["schedule"]
    W2 = next(w for w in range(W + 1, 64) if bench.profile_key(key, (K, w)) not in rec)
    assert bench.valu_issue_from_profiles(key, model, (K, W2), 10.0) is None
    assert bench.valu_issue_from_profiles("no_such_workload:forward", model, (K, W), 10.0) is None
