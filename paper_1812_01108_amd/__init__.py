"""Dihedral angles -> Cartesian coordinates on MI355X (gfx950).

Thin Python binding over the C ABI of libangles2coords.so (include/a2c.h):
argument marshalling only; every step of the map runs in the HIP kernels.
PyTorch supplies device memory and the current stream.

    plan = Plan("backbone", lengths=[700] * 256)
    coords = angles_to_coords(angles, plan)      # angles [3][R] -> coords [3][A]
    coords.backward(grad)                        # angle gradient via the adjoint

The backward keeps the forward's coordinates for the adjoint while they fit
the plan's memory budget (Plan(..., mem_budget_bytes=...)), and otherwise
recomputes the frames from the angles; nothing else is kept between passes.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import A2C_BACKBONE, A2C_FULLATOM, A2C_PLAIN, A2C_SCAN, A2C_SCAN_QUAT, A2CError, check

__all__ = ["Plan", "Angles2Coords", "angles_to_coords", "LRMSD", "lrmsd", "A2CError",
           "library_version", "DEFAULT_GEOMETRY", "PAPER_LITERAL_GEOMETRY"]

DEFAULT_GEOMETRY = {
    "bond_N_CA": 1.458, "bond_CA_C": 1.525, "bond_C_N": 1.329,
    "angle_N_CA_C": 111.2, "angle_CA_C_N": 116.2, "angle_C_N_CA": 121.7,
}

# The constants listed in the paper's "Backbone model" section, kept as data
# for reproducing its numbers: per slot a bond length and theta = pi - angle
# (angles 2.1186, 1.9391 and 2.0610 rad for the transforms placing N, CA and
# C).  Read with the vertex-named convention of a2c_backbone_geometry they
# are attached one slot off the chemical bond angles (C-N-CA comes out
# 111.1 deg, N-CA-C 118.1 deg), which is why the default geometry is the
# standard one above.
_RAD = 180.0 / 3.141592653589793
PAPER_LITERAL_GEOMETRY = {
    "bond_C_N": 1.330, "angle_CA_C_N": 2.1186 * _RAD,     # transform placing N_j
    "bond_N_CA": 1.460, "angle_C_N_CA": 1.9391 * _RAD,    # transform placing CA_j
    "bond_CA_C": 1.525, "angle_N_CA_C": 2.0610 * _RAD,    # transform placing C_j
}

_VARIANTS = {"scan": A2C_SCAN, "plain": A2C_PLAIN, "scan_quat": A2C_SCAN_QUAT}


def library_version() -> str:
    return _lib.load().a2c_version().decode()


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _geometry_struct(geom: dict | None):
    if geom is None:
        return None
    return _lib.BackboneGeometry(geom["bond_N_CA"], geom["bond_CA_C"], geom["bond_C_N"],
                                 geom["angle_N_CA_C"], geom["angle_CA_C_N"],
                                 geom["angle_C_N_CA"])


class Plan:
    """A packed batch of chains: residue offsets, sequence (full-atom), the
    device tables and the scan schedule.  Create once, reuse for every call
    on batches of the same shape."""

    def __init__(self, model: str = "backbone", lengths=None, offsets=None, seq=None,
                 geometry: dict | None = None, table=None, device=None,
                 mem_budget_bytes: int | None = None):
        """mem_budget_bytes: memory the autograd Function may keep between the
        forward and the backward (the coordinates, 12 bytes per atom); None =
        no limit, 0 = always recompute."""
        lib = _lib.load()
        if model not in ("backbone", "fullatom"):
            raise ValueError(f"unknown model {model!r}")
        if (lengths is None) == (offsets is None):
            raise ValueError("give exactly one of lengths or offsets")
        if offsets is None:
            lengths = np.asarray(lengths, dtype=np.int64)
            offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
            offsets[1:] = np.cumsum(lengths)
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        self.model = model
        self.n_chains = len(off) - 1
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.offsets = off
        self.n_planes = 3 if model == "backbone" else 7
        seq_arr = None
        table_struct = None
        if model == "fullatom":
            if seq is None:
                raise ValueError("the full-atom model needs a residue sequence")
            seq_arr = np.ascontiguousarray(seq, dtype=np.uint8)
            if table is None:
                from .residues import default_table
                table = default_table()
            table_struct = table.to_struct() if hasattr(table, "to_struct") else table
        self._seq = seq_arr
        self._table = table_struct
        geom = _geometry_struct(geometry)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.a2c_plan_create(
                ctypes.byref(handle), A2C_BACKBONE if model == "backbone" else A2C_FULLATOM,
                self.n_chains, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                None if seq_arr is None else seq_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                None if geom is None else ctypes.byref(geom),
                None if table_struct is None else ctypes.byref(table_struct),
                _lib.SIZE_MAX if mem_budget_bytes is None else int(mem_budget_bytes),
                _stream_ptr(self.device))
        check(st, "a2c_plan_create")
        self._h = handle
        n_res, n_atoms = ctypes.c_int64(), ctypes.c_int64()
        check(lib.a2c_plan_sizes(self._h, ctypes.byref(n_res), ctypes.byref(n_atoms)),
              "a2c_plan_sizes")
        self.n_res, self.n_atoms = n_res.value, n_atoms.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None and _lib._lib is not None:
            _lib._lib.a2c_plan_destroy(h)
            self._h = None

    # -- plan queries ------------------------------------------------------
    @property
    def keep_coords(self) -> bool:
        """The plan's store-vs-recompute choice: keep the forward's
        coordinates for the adjoint (True) or recompute the frames (False)."""
        k = ctypes.c_int32()
        check(_lib.load().a2c_plan_keep_coords(self._h, ctypes.byref(k)), "a2c_plan_keep_coords")
        return bool(k.value)

    def atom_offsets(self):
        """(chain atom offsets [n_chains+1], residue atom offsets [R+1])."""
        ca = np.zeros(self.n_chains + 1, dtype=np.int32)
        ra = np.zeros(self.n_res + 1, dtype=np.int32)
        check(_lib.load().a2c_plan_atom_offsets(
            self._h, ca.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            ra.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "a2c_plan_atom_offsets")
        return ca, ra

    def workspace_bytes(self, variant: str = "scan") -> int:
        n = ctypes.c_size_t()
        check(_lib.load().a2c_plan_workspace_bytes(self._h, _VARIANTS[variant], ctypes.byref(n)),
              "a2c_plan_workspace_bytes")
        return n.value

    def new_workspace(self, variant: str = "scan"):
        n = self.workspace_bytes(variant)
        if n == 0:
            return None
        return torch.empty(n // 4, dtype=torch.float32, device=self.device)

    @property
    def schedule(self):
        k, w, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(_lib.load().a2c_plan_get_schedule(self._h, ctypes.byref(k), ctypes.byref(w),
                                                ctypes.byref(t)), "a2c_plan_get_schedule")
        return {"res_per_lane": k.value, "waves_per_group": w.value, "n_tiles": t.value}

    @property
    def adjoint_schedule(self):
        """The schedule of the adjoint and the fused step."""
        k, w, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(_lib.load().a2c_plan_get_adjoint_schedule(self._h, ctypes.byref(k),
                                                        ctypes.byref(w), ctypes.byref(t)),
              "a2c_plan_get_adjoint_schedule")
        return {"res_per_lane": k.value, "waves_per_group": w.value, "n_tiles": t.value}

    def set_schedule(self, res_per_lane: int, waves_per_group: int):
        """Both schedules (forward, and adjoint / fused step)."""
        with torch.cuda.device(self.device):
            check(_lib.load().a2c_plan_set_schedule(self._h, res_per_lane, waves_per_group,
                                                    _stream_ptr(self.device)),
                  "a2c_plan_set_schedule")

    def set_forward_schedule(self, res_per_lane: int, waves_per_group: int):
        """The forward's schedule alone (the backbone forward also takes 8
        residues per lane)."""
        with torch.cuda.device(self.device):
            check(_lib.load().a2c_plan_set_forward_schedule(self._h, res_per_lane,
                                                            waves_per_group,
                                                            _stream_ptr(self.device)),
                  "a2c_plan_set_forward_schedule")

    def set_adjoint_schedule(self, res_per_lane: int, waves_per_group: int):
        with torch.cuda.device(self.device):
            check(_lib.load().a2c_plan_set_adjoint_schedule(self._h, res_per_lane,
                                                            waves_per_group,
                                                            _stream_ptr(self.device)),
                  "a2c_plan_set_adjoint_schedule")

    def autotune(self, angles: torch.Tensor, grad_coords: torch.Tensor | None = None,
                 from_coords: bool = True, reps: int = 5, cache_path: str | None = None,
                 mse_target: torch.Tensor | None = None):
        """Time every valid schedule on these buffers and keep the fastest
        forward and the fastest adjoint schedule (synchronises; call before
        capturing a graph).  With mse_target, the fused training step
        (mse_step) is timed as the adjoint.  Returns (forward, adjoint)
        schedules."""
        self._check_tensor(angles, (self.n_planes, self.n_res), "angles")
        coords = torch.empty((3, self.n_atoms), dtype=torch.float32, device=angles.device)
        if grad_coords is None:
            grad_coords = torch.ones_like(coords)
        self._check_tensor(grad_coords, (3, self.n_atoms), "grad_coords")
        grad = torch.empty_like(angles)
        mode = 1 if from_coords else 0
        if mse_target is not None:
            self._check_tensor(mse_target, (3, self.n_atoms), "mse_target")
            grad_coords, mode = mse_target, _lib.A2C_TUNE_MSE_STEP
        k, w = ctypes.c_int32(), ctypes.c_int32()
        with torch.cuda.device(self.device):
            check(_lib.load().a2c_plan_autotune(
                self._h, ctypes.c_void_p(angles.data_ptr()), ctypes.c_void_p(coords.data_ptr()),
                ctypes.c_void_p(grad_coords.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                mode, reps,
                None if cache_path is None else cache_path.encode(), ctypes.byref(k),
                ctypes.byref(w), _stream_ptr(self.device)), "a2c_plan_autotune")
        return self.schedule, self.adjoint_schedule

    # -- raw calls (no autograd) ------------------------------------------
    def _check_tensor(self, t, shape, name):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
                and tuple(t.shape) == tuple(shape)):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape {shape}, "
                             f"got {tuple(t.shape)} {t.dtype} on {t.device}")

    def forward(self, angles: torch.Tensor, coords: torch.Tensor | None = None,
                variant: str = "scan", workspace: torch.Tensor | None = None) -> torch.Tensor:
        self._check_tensor(angles, (self.n_planes, self.n_res), "angles")
        if coords is None:
            coords = torch.empty((3, self.n_atoms), dtype=torch.float32, device=angles.device)
        self._check_tensor(coords, (3, self.n_atoms), "coords")
        check(_lib.load().a2c_forward(
            self._h, _VARIANTS[variant], ctypes.c_void_p(angles.data_ptr()),
            ctypes.c_void_p(coords.data_ptr()),
            None if workspace is None else ctypes.c_void_p(workspace.data_ptr()),
            _stream_ptr(angles.device)), "a2c_forward")
        return coords

    def backward(self, angles: torch.Tensor, grad_coords: torch.Tensor,
                 coords: torch.Tensor | None = None, grad_angles: torch.Tensor | None = None,
                 variant: str = "scan", workspace: torch.Tensor | None = None) -> torch.Tensor:
        self._check_tensor(angles, (self.n_planes, self.n_res), "angles")
        self._check_tensor(grad_coords, (3, self.n_atoms), "grad_coords")
        if coords is not None:
            self._check_tensor(coords, (3, self.n_atoms), "coords")
        if grad_angles is None:
            grad_angles = torch.empty_like(angles)
        self._check_tensor(grad_angles, (self.n_planes, self.n_res), "grad_angles")
        check(_lib.load().a2c_backward(
            self._h, _VARIANTS[variant], ctypes.c_void_p(angles.data_ptr()),
            None if coords is None else ctypes.c_void_p(coords.data_ptr()),
            ctypes.c_void_p(grad_coords.data_ptr()), ctypes.c_void_p(grad_angles.data_ptr()),
            None if workspace is None else ctypes.c_void_p(workspace.data_ptr()),
            _stream_ptr(angles.device)), "a2c_backward")
        return grad_angles


    # -- inverse map ----------------------------------------------------
    def coords_to_angles(self, coords: torch.Tensor,
                         out: torch.Tensor | None = None) -> torch.Tensor:
        """Dihedral angles [K][R] of coordinates [3][A] in the plan's layout."""
        self._check_tensor(coords, (3, self.n_atoms), "coords")
        if out is None:
            out = torch.empty((self.n_planes, self.n_res), dtype=torch.float32,
                              device=coords.device)
        self._check_tensor(out, (self.n_planes, self.n_res), "angles")
        check(_lib.load().a2c_coords_to_angles(
            self._h, ctypes.c_void_p(coords.data_ptr()), ctypes.c_void_p(out.data_ptr()),
            _stream_ptr(coords.device)), "a2c_coords_to_angles")
        return out

    # -- fused training step ------------------------------------------
    def mse_step(self, angles: torch.Tensor, target: torch.Tensor,
                 coords: torch.Tensor | None = None, loss: bool = True,
                 grad_angles: torch.Tensor | None = None,
                 loss_out: torch.Tensor | None = None):
        """One fused pass for L = sum |r - t|^2: returns (L as a 0-dim tensor
        or None, dL/dangles); writes r into `coords` when given.  L is summed
        on the device (a2c_mse_step); with `loss_out` (float32, >= 1 element)
        it lands in loss_out[0] and nothing is allocated, so the call can be
        captured in a graph."""
        self._check_tensor(angles, (self.n_planes, self.n_res), "angles")
        self._check_tensor(target, (3, self.n_atoms), "target")
        if coords is not None:
            self._check_tensor(coords, (3, self.n_atoms), "coords")
        if grad_angles is None:
            grad_angles = torch.empty_like(angles)
        self._check_tensor(grad_angles, (self.n_planes, self.n_res), "grad_angles")
        out = loss_out
        if out is not None:
            if (out.dtype != torch.float32 or not out.is_contiguous()
                    or out.device != angles.device or out.numel() < 1):
                raise ValueError("loss_out: contiguous float32 with >= 1 element on the "
                                 "plan's device")
        elif loss:
            out = torch.empty(1, dtype=torch.float32, device=angles.device)
        check(_lib.load().a2c_mse_step(
            self._h, ctypes.c_void_p(angles.data_ptr()), ctypes.c_void_p(target.data_ptr()),
            None if coords is None else ctypes.c_void_p(coords.data_ptr()),
            None if out is None else ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(grad_angles.data_ptr()), _stream_ptr(angles.device)),
            "a2c_mse_step")
        return (None if out is None else out[0]), grad_angles

    # -- LRMSD loss -------------------------------------------------------
    def lrmsd_workspace(self) -> torch.Tensor | None:
        n = ctypes.c_size_t()
        check(_lib.load().a2c_lrmsd_workspace_bytes(self._h, ctypes.byref(n)),
              "a2c_lrmsd_workspace_bytes")
        if n.value == 0:
            return None
        return torch.empty(n.value // 4, dtype=torch.float32, device=self.device)

    def lrmsd_forward(self, coords: torch.Tensor, target: torch.Tensor, workspace=None,
                      out: torch.Tensor | None = None) -> torch.Tensor:
        """Per-chain LRMSD [n_chains] between coords (input) and target; fills
        `workspace` (from lrmsd_workspace) for lrmsd_backward."""
        self._check_tensor(coords, (3, self.n_atoms), "coords")
        self._check_tensor(target, (3, self.n_atoms), "target")
        if out is None:
            out = torch.empty(self.n_chains, dtype=torch.float32, device=coords.device)
        self._check_tensor(out, (self.n_chains,), "out")
        check(_lib.load().a2c_lrmsd_forward(
            self._h, ctypes.c_void_p(coords.data_ptr()), ctypes.c_void_p(target.data_ptr()),
            ctypes.c_void_p(out.data_ptr()),
            None if workspace is None else ctypes.c_void_p(workspace.data_ptr()),
            _stream_ptr(coords.device)), "a2c_lrmsd_forward")
        return out

    def lrmsd_forward_noalloc(self, coords: torch.Tensor, target: torch.Tensor,
                              out: torch.Tensor) -> torch.Tensor:
        """Per-chain LRMSD into `out` [n_chains] without a workspace: the
        library's fixed per-device scratch holds the intermediate sums (calls
        on one device must not overlap)."""
        self._check_tensor(coords, (3, self.n_atoms), "coords")
        self._check_tensor(target, (3, self.n_atoms), "target")
        self._check_tensor(out, (self.n_chains,), "out")
        check(_lib.load().a2c_lrmsd_forward_noalloc(
            self._h, ctypes.c_void_p(coords.data_ptr()), ctypes.c_void_p(target.data_ptr()),
            ctypes.c_void_p(out.data_ptr()), _stream_ptr(coords.device)),
            "a2c_lrmsd_forward_noalloc")
        return out

    def lrmsd_backward(self, coords: torch.Tensor, target: torch.Tensor,
                       grad_lrmsd: torch.Tensor, workspace,
                       grad_coords: torch.Tensor | None = None) -> torch.Tensor:
        self._check_tensor(coords, (3, self.n_atoms), "coords")
        self._check_tensor(target, (3, self.n_atoms), "target")
        self._check_tensor(grad_lrmsd, (self.n_chains,), "grad_lrmsd")
        if grad_coords is None:
            grad_coords = torch.zeros_like(coords)
        self._check_tensor(grad_coords, (3, self.n_atoms), "grad_coords")
        check(_lib.load().a2c_lrmsd_backward(
            self._h, ctypes.c_void_p(coords.data_ptr()), ctypes.c_void_p(target.data_ptr()),
            ctypes.c_void_p(grad_lrmsd.data_ptr()), ctypes.c_void_p(grad_coords.data_ptr()),
            None if workspace is None else ctypes.c_void_p(workspace.data_ptr()),
            _stream_ptr(coords.device)), "a2c_lrmsd_backward")
        return grad_coords


class LRMSD(torch.autograd.Function):
    """lrmsd = LRMSD.apply(coords, target, plan): per-chain LRMSD [n_chains];
    the gradient flows to coords (the target is a constant)."""

    @staticmethod
    def forward(ctx, coords, target, plan: Plan):
        coords, target = coords.contiguous(), target.contiguous()
        ws = plan.lrmsd_workspace()
        out = plan.lrmsd_forward(coords, target, ws)
        ctx.plan, ctx.ws = plan, ws
        ctx.save_for_backward(coords, target)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        coords, target = ctx.saved_tensors
        g = ctx.plan.lrmsd_backward(coords, target, grad_out.contiguous(), ctx.ws)
        return g, None, None


def lrmsd(coords: torch.Tensor, target: torch.Tensor, plan: Plan) -> torch.Tensor:
    return LRMSD.apply(coords, target, plan)


class Angles2Coords(torch.autograd.Function):
    """coords = Angles2Coords.apply(angles, plan, mode).

    mode "auto" (default): the plan's store-vs-recompute choice
    (Plan.keep_coords: the coordinates fit its memory budget or not);
    mode "coords": the backward reads the forward's coordinates (saved);
    mode "recompute": the backward recomputes every frame from the angles and
    nothing but the angles is kept between the passes;
    mode "plain": the paper's GPU design (stores M_i per atom in a workspace).
    """

    @staticmethod
    def forward(ctx, angles, plan: Plan, mode: str = "auto"):
        if mode == "auto":
            mode = "coords" if plan.keep_coords else "recompute"
        if mode not in ("coords", "recompute", "plain"):
            raise ValueError(f"unknown mode {mode!r}")
        angles = angles.contiguous()
        ws = plan.new_workspace("plain") if mode == "plain" else None
        variant = "plain" if mode == "plain" else "scan"
        coords = plan.forward(angles, variant=variant, workspace=ws)
        ctx.plan = plan
        ctx.mode = mode
        ctx.ws = ws
        if mode == "coords":
            ctx.save_for_backward(angles, coords)
        else:
            ctx.save_for_backward(angles)
        return coords

    @staticmethod
    def backward(ctx, grad_coords):
        plan, mode = ctx.plan, ctx.mode
        saved = ctx.saved_tensors
        angles = saved[0]
        coords = saved[1] if mode == "coords" else None
        variant = "plain" if mode == "plain" else "scan"
        grad = plan.backward(angles, grad_coords.contiguous(), coords=coords, variant=variant,
                             workspace=ctx.ws)
        return grad, None, None


def angles_to_coords(angles: torch.Tensor, plan: Plan, mode: str = "auto") -> torch.Tensor:
    return Angles2Coords.apply(angles, plan, mode)
