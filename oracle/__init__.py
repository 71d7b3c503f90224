"""FP64 CPU oracle for the dihedral-angle -> Cartesian map (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
baseline leg of the benchmark.  The library's product path never imports it.

All inputs are promoted to float64 here (float32 angles promote exactly).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, build

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_U8 = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("A2C_ORACLE_LIB", LIB)  # e.g. the sanitizer build
        if path == LIB and not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(path)
        lib.oracle_transform.argtypes = [ctypes.c_double] * 3 + [_D]
        for name in ("oracle_backbone_forward",):
            getattr(lib, name).argtypes = [ctypes.c_int32, _I32, _D, _D, _D, ctypes.c_int]
        lib.oracle_backbone_backward.argtypes = [ctypes.c_int32, _I32, _D, _D, _D, _D, ctypes.c_int]
        lib.oracle_backbone_backward_direct.argtypes = [ctypes.c_int32, _I32, _D, _D, _D, _D]
        lib.oracle_openmp_enabled.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t):
    return a.ctypes.data_as(t)


def backbone_geometry_vector(geom: dict) -> np.ndarray:
    """Slot-ordered geometry (N, CA, C): bond length to the previous atom and
    the bond angle in degrees at the previous atom."""
    return np.array([geom["bond_C_N"], geom["angle_CA_C_N"],
                     geom["bond_N_CA"], geom["angle_C_N_CA"],
                     geom["bond_CA_C"], geom["angle_N_CA_C"]], dtype=np.float64)


def transform(alpha: float, theta: float, d: float) -> np.ndarray:
    out = np.empty(16)
    _load().oracle_transform(alpha, theta, d, _ptr(out, _D))
    return out.reshape(4, 4)


def backbone_forward(offsets, angles, geom: dict, n_threads: int = 0) -> np.ndarray:
    """coords [3][3R] float64 for angle planes [3][R] (phi, psi, omega)."""
    lib = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    ang = _d(angles)
    R = int(off[-1])
    assert ang.shape == (3, R)
    g = backbone_geometry_vector(geom)
    out = np.empty((3, 3 * R))
    lib.oracle_backbone_forward(len(off) - 1, _ptr(off, _I32), _ptr(ang, _D), _ptr(g, _D),
                                _ptr(out, _D), n_threads)
    return out


def backbone_backward(offsets, angles, geom: dict, grad_coords, n_threads: int = 0,
                      direct: bool = False) -> np.ndarray:
    """Angle gradient [3][R] of L = sum g . r for upstream g [3][3R].

    direct=True evaluates the paper's O(N^2) expression instead of the O(N)
    closed form (small inputs only)."""
    lib = _load()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    ang = _d(angles)
    R = int(off[-1])
    gc = _d(grad_coords)
    assert ang.shape == (3, R) and gc.shape == (3, 3 * R)
    g = backbone_geometry_vector(geom)
    out = np.zeros((3, R))
    if direct:
        rc = lib.oracle_backbone_backward_direct(len(off) - 1, _ptr(off, _I32), _ptr(ang, _D),
                                                 _ptr(g, _D), _ptr(gc, _D), _ptr(out, _D))
    else:
        rc = lib.oracle_backbone_backward(len(off) - 1, _ptr(off, _I32), _ptr(ang, _D),
                                          _ptr(g, _D), _ptr(gc, _D), _ptr(out, _D), n_threads)
    if rc != 0:
        raise MemoryError("oracle backward failed")
    return out


def openmp_enabled() -> bool:
    return bool(_load().oracle_openmp_enabled())


# ---------------------------------------------------------------- full atom
_FA = None


def _load_fa():
    global _FA
    lib = _load()
    if _FA is None:
        from . import residue_table as rt
        P = ctypes.POINTER
        lib.oracle_fullatom_forward.argtypes = [ctypes.c_int32, _I32, _U8, _D, _D,
                                                P(rt.OracleTable), _I32, _D, ctypes.c_int]
        lib.oracle_fullatom_backward.argtypes = [ctypes.c_int32, _I32, _U8, _D, _D,
                                                 P(rt.OracleTable), _I32, _D, _D, ctypes.c_int,
                                                 ctypes.c_int]
        _FA = rt.load()
    return lib, _FA


def load_residue_table():
    """(ctypes table, per-type info) read from the residue data file."""
    return _load_fa()[1]


def fullatom_atom_offsets(seq):
    from . import residue_table as rt
    return rt.atom_offsets(seq, _load_fa()[1][0])


def fullatom_forward(offsets, seq, angles, geom: dict, n_threads: int = 0):
    """coords [3][A] float64 and residue atom offsets [R+1] for angle planes
    [7][R] (phi, psi, omega, chi1..chi4) and residue codes seq[R]."""
    lib, (tab, _) = _load_fa()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    sq = np.ascontiguousarray(seq, dtype=np.uint8)
    ang = _d(angles)
    R = int(off[-1])
    assert ang.shape == (7, R) and sq.shape == (R,)
    aoff = fullatom_atom_offsets(sq)
    A = int(aoff[-1])
    out = np.empty((3, A))
    g = backbone_geometry_vector(geom)
    lib.oracle_fullatom_forward(len(off) - 1, _ptr(off, _I32), _ptr(sq, _U8), _ptr(ang, _D),
                                _ptr(g, _D), ctypes.byref(tab), _ptr(aoff, _I32), _ptr(out, _D),
                                n_threads)
    return out, aoff


def fullatom_backward(offsets, seq, angles, geom: dict, grad_coords, n_threads: int = 0,
                      direct: bool = False):
    """Angle gradient [7][R] of L = sum g . r (chi planes a residue lacks are 0).
    direct=True evaluates Eq. FAMBackward term by term (O(N^2), small inputs)."""
    lib, (tab, _) = _load_fa()
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    sq = np.ascontiguousarray(seq, dtype=np.uint8)
    ang = _d(angles)
    R = int(off[-1])
    aoff = fullatom_atom_offsets(sq)
    gc = _d(grad_coords)
    assert gc.shape == (3, int(aoff[-1]))
    out = np.zeros((7, R))
    g = backbone_geometry_vector(geom)
    rc = lib.oracle_fullatom_backward(len(off) - 1, _ptr(off, _I32), _ptr(sq, _U8),
                                      _ptr(ang, _D), _ptr(g, _D), ctypes.byref(tab),
                                      _ptr(aoff, _I32), _ptr(gc, _D), _ptr(out, _D),
                                      1 if direct else 0, n_threads)
    if rc != 0:
        raise MemoryError("oracle full-atom backward failed")
    return out
