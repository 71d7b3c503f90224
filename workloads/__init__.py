"""Seeded synthetic inputs for the dihedral-angle -> coordinate map.

This module is shared by the tests, the benchmark and the oracle's callers.
It only draws random numbers and describes workload shapes: it holds none of
the map's arithmetic (no transforms, no coordinates, no gradients).

The paper times its layers on random angles and random sequences (Benchmarks
section, batch 32, random sequences) and measures the FP32 error on random
backbone angles; no structure dataset is involved, so every workload here is
synthetic.
"""
from .generate import (  # noqa: F401
    ALPHABET,
    BACKBONE_GEOMETRY,
    CONFIGS,
    PAPER_LITERAL_GEOMETRY,
    WorkloadConfig,
    chain_lengths,
    make_angles,
    make_inputs,
    mixture_phi_psi,
    offsets_from_lengths,
    random_sequence,
    target_perturbation,
    uniform_angles,
    upstream_grad,
    wrap_angle,
)
