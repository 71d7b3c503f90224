"""Seeded input generators and the five workload shapes.

Everything is drawn with numpy's PCG64 in float64 and cast once to float32, so
the GPU path and the FP64 oracle see identical float32 bits (the oracle
promotes them exactly to float64).

Angles are radians wrapped to (-pi, pi].  Planes are ordered
phi, psi, omega, chi1, chi2, chi3, chi4 (backbone uses the first three).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# One-letter residue codes; the integer code of a residue is its index here.
ALPHABET = "ACDEFGHIKLMNPQRSTVWY"

# Backbone geometry named by the bonded atoms and the angle vertex, as the
# backbone workloads state it.  Bond lengths in Angstrom, angles in degrees.
BACKBONE_GEOMETRY = {
    "bond_N_CA": 1.458,
    "bond_CA_C": 1.525,
    "bond_C_N": 1.329,
    "angle_N_CA_C": 111.2,
    "angle_CA_C_N": 116.2,
    "angle_C_N_CA": 121.7,
}

# The constant list of the paper's "Backbone model" section, read with the
# same vertex naming: the transform placing N uses d = 1.330 and
# theta = pi - 2.1186, the one placing CA d = 1.460 and theta = pi - 1.9391,
# the one placing C d = 1.525 and theta = pi - 2.0610 (angles in radians
# there, in degrees here).
PAPER_LITERAL_GEOMETRY = {
    "bond_C_N": 1.330,
    "angle_CA_C_N": float(np.degrees(2.1186)),
    "bond_N_CA": 1.460,
    "angle_C_N_CA": float(np.degrees(1.9391)),
    "bond_CA_C": 1.525,
    "angle_N_CA_C": float(np.degrees(2.0610)),
}

PI32 = np.float32(np.pi)


def wrap_angle(x):
    """Wrap radians to (-pi, pi]."""
    x = np.asarray(x, dtype=np.float64)
    return np.pi - np.mod(np.pi - x, 2.0 * np.pi)


def uniform_angles(rng: np.random.Generator, n: int) -> np.ndarray:
    """n angles uniform in (-pi, pi] as pi - 2*pi*U[0,1)."""
    return np.pi - 2.0 * np.pi * rng.random(n)


def mixture_phi_psi(rng: np.random.Generator, n: int):
    """Ramachandran-like mixture: 0.5 helix N((-63,-43) deg, 10 deg),
    0.4 sheet N((-120,130) deg, 15 deg), 0.1 uniform; then wrapped."""
    comp = rng.choice(3, size=n, p=[0.5, 0.4, 0.1])
    phi = np.empty(n)
    psi = np.empty(n)
    h = comp == 0
    s = comp == 1
    u = comp == 2
    nh, ns, nu = int(h.sum()), int(s.sum()), int(u.sum())
    d2r = np.pi / 180.0
    phi[h] = rng.normal(-63.0, 10.0, nh) * d2r
    psi[h] = rng.normal(-43.0, 10.0, nh) * d2r
    phi[s] = rng.normal(-120.0, 15.0, ns) * d2r
    psi[s] = rng.normal(130.0, 15.0, ns) * d2r
    phi[u] = uniform_angles(rng, nu)
    psi[u] = uniform_angles(rng, nu)
    return wrap_angle(phi), wrap_angle(psi)


def offsets_from_lengths(lengths) -> np.ndarray:
    lengths = np.asarray(lengths, dtype=np.int64)
    off = np.zeros(len(lengths) + 1, dtype=np.int32)
    off[1:] = np.cumsum(lengths)
    return off


def random_sequence(rng: np.random.Generator, n: int) -> np.ndarray:
    """Residue codes iid uniform over the 20 standard amino acids."""
    return rng.integers(0, len(ALPHABET), size=n).astype(np.uint8)


def upstream_grad(seed: int, n_atoms: int) -> np.ndarray:
    """Upstream coordinate gradient, iid N(0,1) float32, planes [3][n_atoms]."""
    rng = np.random.Generator(np.random.PCG64(seed + 7_000_000))
    return rng.standard_normal((3, n_atoms)).astype(np.float32)


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    model: str            # "backbone" or "fullatom"
    n_chains: int
    lengths: str          # "fixed:<L>", "uniform:<lo>:<hi>", "loguniform:<lo>:<hi>"
    angles: str           # "uniform" or "mixture" for phi/psi
    seed: int
    note: str = ""


CONFIGS = {
    "backbone_16x64": WorkloadConfig(
        "backbone_16x64", "backbone", 16, "fixed:64", "uniform", 1000,
        "16 chains x 64 residues, uniform phi/psi, plain and scan forms"),
    "backbone_256x700": WorkloadConfig(
        "backbone_256x700", "backbone", 256, "fixed:700", "mixture", 1001,
        "256 chains x 700 residues, mixture phi/psi, through autograd"),
    "fullatom_64x300": WorkloadConfig(
        "fullatom_64x300", "fullatom", 64, "fixed:300", "mixture", 1002,
        "64 chains x 300 residues, random sequence, chi uniform"),
    "ragged_backbone_4096": WorkloadConfig(
        "ragged_backbone_4096", "backbone", 4096, "uniform:20:1000", "mixture", 1003,
        "4096 chains, L uniform in [20,1000], packed ragged, one graph"),
    "ragged_fullatom_512": WorkloadConfig(
        "ragged_fullatom_512", "fullatom", 512, "loguniform:50:2000", "mixture", 1004,
        "512 chains, L log-uniform in [50,2000], training-step shape"),
}


def chain_lengths(spec: str, n_chains: int, rng: np.random.Generator) -> np.ndarray:
    kind, *args = spec.split(":")
    if kind == "fixed":
        return np.full(n_chains, int(args[0]), dtype=np.int64)
    if kind == "uniform":
        lo, hi = int(args[0]), int(args[1])
        return rng.integers(lo, hi + 1, size=n_chains).astype(np.int64)
    if kind == "loguniform":
        lo, hi = float(args[0]), float(args[1])
        return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_chains))).astype(np.int64)
    raise ValueError(f"unknown length spec {spec!r}")


def make_angles(rng: np.random.Generator, n_res: int, kind: str, n_planes: int) -> np.ndarray:
    """Angle planes [n_planes][n_res] float32: phi, psi, omega (= fp32 pi),
    then chi1..chi4 uniform (the map ignores chi slots a residue lacks)."""
    if kind == "uniform":
        phi, psi = uniform_angles(rng, n_res), uniform_angles(rng, n_res)
    elif kind == "mixture":
        phi, psi = mixture_phi_psi(rng, n_res)
    else:
        raise ValueError(kind)
    out = np.empty((n_planes, n_res), dtype=np.float32)
    out[0] = phi
    out[1] = psi
    out[2] = PI32
    for p in range(3, n_planes):
        out[p] = uniform_angles(rng, n_res)
    return out


def target_perturbation(seed: int, angles: np.ndarray, n_chains: int):
    """Inputs for the training-step target: angles + N(0, 20 deg) on phi, psi
    and chi (omega kept), plus per chain a uniform random rotation (normalised
    Gaussian quaternion, w,x,y,z) and a translation ~ N(0, 10 A) per axis."""
    rng = np.random.Generator(np.random.PCG64(seed + 9_000_000))
    pert = angles.astype(np.float64).copy()
    sig = 20.0 * np.pi / 180.0
    for p in range(pert.shape[0]):
        if p == 2:
            continue
        pert[p] = wrap_angle(pert[p] + rng.normal(0.0, sig, pert.shape[1]))
    q = rng.standard_normal((n_chains, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    t = rng.normal(0.0, 10.0, (n_chains, 3))
    return pert.astype(np.float32), q, t


def make_inputs(cfg: WorkloadConfig | str, scale_chains: int | None = None,
                max_len: int | None = None):
    """Angles, offsets and (full-atom) sequence for a workload.

    scale_chains / max_len shrink a workload for tests that need a bounded
    oracle run; the generator stream is otherwise the same recipe.
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    n_chains = cfg.n_chains if scale_chains is None else scale_chains
    lengths = chain_lengths(cfg.lengths, n_chains, rng)
    if max_len is not None:
        lengths = np.minimum(lengths, max_len)
    offsets = offsets_from_lengths(lengths)
    n_res = int(offsets[-1])
    n_planes = 3 if cfg.model == "backbone" else 7
    angles = make_angles(rng, n_res, cfg.angles if cfg.angles else "uniform", n_planes)
    seq = random_sequence(rng, n_res) if cfg.model == "fullatom" else None
    return {"config": cfg, "offsets": offsets, "angles": angles, "seq": seq,
            "n_chains": n_chains, "n_res": n_res}
