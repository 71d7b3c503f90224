"""ctypes declarations of the C ABI in include/a2c.h (argument marshalling only).

The shared library is built in-tree (paper_1812_01108_amd/libangles2coords.so).
There is no fallback: if it is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# A2C_LIB selects another build of the library (the host-sanitizer one)
LIB_PATH = os.environ.get("A2C_LIB", os.path.join(HERE, "libangles2coords.so"))

A2C_OK = 0
STATUS = {0: "A2C_OK", -1: "A2C_ERR_INVALID_ARG", -2: "A2C_ERR_UNSUPPORTED",
          -3: "A2C_ERR_WORKSPACE", -4: "A2C_ERR_HIP", -5: "A2C_ERR_STATE"}
A2C_BACKBONE, A2C_FULLATOM = 0, 1
A2C_SCAN, A2C_PLAIN, A2C_SCAN_QUAT = 0, 1, 2
A2C_TUNE_MSE_STEP = 2
NUM_RESIDUE_TYPES = 20
MAX_SIDE_FRAMES = 4
MAX_RESIDUE_ATOMS = 14
ATOM_ORIGIN, ATOM_AZIMUTH, ATOM_ZMATRIX = 0, 1, 2

# every function include/a2c.h declares
EXPORTS = (
    "a2c_plan_create", "a2c_plan_destroy", "a2c_plan_sizes", "a2c_plan_atom_offsets",
    "a2c_plan_workspace_bytes", "a2c_plan_set_schedule", "a2c_plan_get_schedule",
    "a2c_plan_set_adjoint_schedule", "a2c_plan_get_adjoint_schedule", "a2c_plan_autotune",
    "a2c_forward", "a2c_backward", "a2c_residue_table_info", "a2c_status_string",
    "a2c_last_error", "a2c_version", "a2c_lrmsd_workspace_bytes", "a2c_lrmsd_forward",
    "a2c_lrmsd_backward", "a2c_mse_step", "a2c_coords_to_angles", "a2c_plan_keep_coords",
    "a2c_lrmsd_forward_noalloc", "a2c_plan_set_forward_schedule",
)

SIZE_MAX = 2 ** 64 - 1


class BackboneGeometry(ctypes.Structure):
    _fields_ = [("bond_n_ca", ctypes.c_double), ("bond_ca_c", ctypes.c_double),
                ("bond_c_n", ctypes.c_double), ("angle_n_ca_c", ctypes.c_double),
                ("angle_ca_c_n", ctypes.c_double), ("angle_c_n_ca", ctypes.c_double)]


class SideFrame(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_int32), ("chi", ctypes.c_int32),
                ("pre_rotation_deg", ctypes.c_double), ("bond", ctypes.c_double),
                ("bond_angle_deg", ctypes.c_double)]


class AtomDef(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("ref", ctypes.c_int32 * 3), ("bond", ctypes.c_double),
                ("angle_deg", ctypes.c_double), ("torsion_deg", ctypes.c_double)]


class ResidueDef(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_side_frames", ctypes.c_int32),
                ("frames", SideFrame * MAX_SIDE_FRAMES),
                ("atoms", AtomDef * MAX_RESIDUE_ATOMS)]


class ResidueTable(ctypes.Structure):
    _fields_ = [("residues", ResidueDef * NUM_RESIDUE_TYPES)]


_lib = None


def load():
    """Load the HIP library once.  Raises RuntimeError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
            "g.build()'` (hipcc, gfx950). There is no CPU fallback.")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    P = ctypes.POINTER
    lib.a2c_plan_create.argtypes = [P(vp), ctypes.c_int, i32, P(i32), P(ctypes.c_uint8),
                                    P(BackboneGeometry), P(ResidueTable), sz, vp]
    lib.a2c_plan_create.restype = ctypes.c_int
    lib.a2c_plan_destroy.argtypes = [vp]
    lib.a2c_plan_destroy.restype = None
    lib.a2c_plan_sizes.argtypes = [vp, P(i64), P(i64)]
    lib.a2c_plan_keep_coords.argtypes = [vp, P(i32)]
    lib.a2c_plan_atom_offsets.argtypes = [vp, P(i32), P(i32)]
    lib.a2c_plan_workspace_bytes.argtypes = [vp, ctypes.c_int, P(sz)]
    lib.a2c_plan_set_schedule.argtypes = [vp, i32, i32, vp]
    lib.a2c_plan_get_schedule.argtypes = [vp, P(i32), P(i32), P(i32)]
    lib.a2c_plan_set_adjoint_schedule.argtypes = [vp, i32, i32, vp]
    lib.a2c_plan_set_forward_schedule.argtypes = [vp, i32, i32, vp]
    lib.a2c_plan_get_adjoint_schedule.argtypes = [vp, P(i32), P(i32), P(i32)]
    lib.a2c_plan_autotune.argtypes = [vp, vp, vp, vp, vp, i32, i32, ctypes.c_char_p, P(i32),
                                      P(i32), vp]
    lib.a2c_plan_autotune.restype = ctypes.c_int
    lib.a2c_forward.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    lib.a2c_backward.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp, vp]
    lib.a2c_mse_step.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.a2c_coords_to_angles.argtypes = [vp, vp, vp, vp]
    lib.a2c_lrmsd_workspace_bytes.argtypes = [vp, P(sz)]
    lib.a2c_lrmsd_forward.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.a2c_lrmsd_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.a2c_lrmsd_forward_noalloc.argtypes = [vp, vp, vp, vp, vp]
    for name in ("a2c_plan_sizes", "a2c_plan_keep_coords", "a2c_plan_atom_offsets", "a2c_plan_workspace_bytes",
                 "a2c_plan_set_schedule", "a2c_plan_get_schedule",
                 "a2c_plan_set_adjoint_schedule", "a2c_plan_get_adjoint_schedule", "a2c_forward",
                 "a2c_backward", "a2c_lrmsd_workspace_bytes", "a2c_lrmsd_forward",
                 "a2c_lrmsd_backward", "a2c_mse_step", "a2c_coords_to_angles",
                 "a2c_lrmsd_forward_noalloc", "a2c_plan_set_forward_schedule"):
        getattr(lib, name).restype = ctypes.c_int
    lib.a2c_residue_table_info.argtypes = [P(ResidueTable), P(i32), P(ctypes.c_float)]
    lib.a2c_residue_table_info.restype = ctypes.c_int
    lib.a2c_status_string.argtypes = [ctypes.c_int]
    lib.a2c_status_string.restype = ctypes.c_char_p
    lib.a2c_last_error.argtypes = []
    lib.a2c_last_error.restype = ctypes.c_char_p
    lib.a2c_version.argtypes = []
    lib.a2c_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


class A2CError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}: {detail}")
        self.status = status


def check(status: int, what: str):
    if status != A2C_OK:
        raise A2CError(status, what, load().a2c_last_error().decode())
