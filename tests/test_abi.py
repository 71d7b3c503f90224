"""The C-ABI library loads on a machine without a GPU and exports every
function include/a2c.h declares; host-side validation rejects bad arguments
before anything touches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "a2c.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(a2c_[a-z_]+)\s*\(", text)))


def test_header_matches_binding_list():
    from paper_1812_01108_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared_functions()


def test_library_exports_every_declared_symbol():
    from paper_1812_01108_amd import _lib
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert lib.a2c_version().decode().startswith("a2c")
    assert lib.a2c_status_string(-1).decode() == "invalid argument"


def test_struct_layouts_match_header():
    from paper_1812_01108_amd import _lib
    # a2c_side_frame: 2 int32 + 3 double; a2c_atom_def: 5 int32 (+pad) + 3 double
    assert ctypes.sizeof(_lib.SideFrame) == 32
    assert ctypes.sizeof(_lib.AtomDef) == 48
    assert ctypes.sizeof(_lib.BackboneGeometry) == 48


@pytest.mark.parametrize("offsets,err", [
    ([1, 3], "h_res_offsets[0] != 0"),
    ([0, 5, 3], "decreases"),
])
def test_bad_offsets_rejected_on_host(offsets, err):
    from paper_1812_01108_amd import _lib
    lib = _lib.load()
    off = np.asarray(offsets, dtype=np.int32)
    h = ctypes.c_void_p()
    st = lib.a2c_plan_create(ctypes.byref(h), 0, len(off) - 1,
                             off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None, None,
                             None, 0, None)
    assert st == -1
    assert err in lib.a2c_last_error().decode()
    assert not h.value


def test_null_arguments_rejected_on_host():
    from paper_1812_01108_amd import _lib
    lib = _lib.load()
    assert lib.a2c_plan_create(None, 0, 0, None, None, None, None, 0, None) == -1
    h = ctypes.c_void_p()
    assert lib.a2c_plan_create(ctypes.byref(h), 0, 1, None, None, None, None, 0, None) == -1
    assert lib.a2c_forward(None, 0, None, None, None, None) == -1
    assert lib.a2c_backward(None, 0, None, None, None, None, None, None) == -1
    # unknown model
    off = np.array([0, 2], dtype=np.int32)
    assert lib.a2c_plan_create(ctypes.byref(h), 7, 1,
                               off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                               None, None, None, 0, None) == -1
    assert lib.a2c_plan_keep_coords(None, None) == -1


@pytest.mark.parametrize("model,limit", [(0, 64 * 64 * 16 * 4), (1, 64 * 64 * 16 * 2)])
def test_too_long_chain_unsupported(model, limit):
    """A chain beyond 64 chunks of the widest schedule is refused on the host,
    before any device call."""
    from paper_1812_01108_amd import _lib
    lib = _lib.load()
    off = np.array([0, limit + 1], dtype=np.int32)
    seq = np.zeros(limit + 1, dtype=np.uint8)
    h = ctypes.c_void_p()
    st = lib.a2c_plan_create(ctypes.byref(h), model, 1,
                             off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             seq.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), None, None,
                             0, None)
    assert st == -2
    assert b"longer than" in lib.a2c_last_error()


def test_bad_geometry_rejected():
    from paper_1812_01108_amd import _lib
    lib = _lib.load()
    off = np.array([0, 5], dtype=np.int32)
    g = _lib.BackboneGeometry(1.458, -1.0, 1.329, 111.2, 116.2, 121.7)
    h = ctypes.c_void_p()
    st = lib.a2c_plan_create(ctypes.byref(h), 0, 1,
                             off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             None, ctypes.byref(g), None, 0, None)
    assert st == -1 and "geometry" in lib.a2c_last_error().decode()


def test_residue_table_rigid_groups_match_oracle():
    """The library's rigid-group coordinates r°, derived from the table's
    internal coordinates by its own code (NeRF vectors), equal the oracle's
    (derived with the paper's 4x4 transforms) to float32 rounding."""
    import oracle
    from paper_1812_01108_amd import _lib
    from paper_1812_01108_amd.residues import default_table
    lib = _lib.load()
    tab = default_table().to_struct()
    n_atoms = (ctypes.c_int32 * 20)()
    xyz = np.zeros((20, 14, 3), dtype=np.float32)
    st = lib.a2c_residue_table_info(ctypes.byref(tab), n_atoms,
                                    xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    assert st == 0, lib.a2c_last_error()
    otab, info = oracle.load_residue_table()
    for t in range(20):
        assert n_atoms[t] == otab.n_atoms[t] == len(info[t]["atoms"])
        for a in range(n_atoms[t]):
            ref = np.array([otab.atom_r[t][a][q] for q in range(3)])
            assert np.max(np.abs(xyz[t, a] - ref)) < 1e-5, (info[t]["name"], a)


@pytest.mark.parametrize("mutate,msg", [
    (lambda rd: setattr(rd.frames[1], "parent", 1), "hang off"),
    (lambda rd: setattr(rd.frames[1], "chi", 3), "chi"),
    (lambda rd: setattr(rd.atoms[8], "ref", (ctypes.c_int32 * 3)(4, 5, 6)), "z-matrix"),
    (lambda rd: setattr(rd.atoms[0], "kind", 1), "atoms 0, 1, 2"),
    (lambda rd: setattr(rd, "n_atoms", 15), "n_atoms"),
])
def test_bad_residue_tables_rejected(mutate, msg):
    from paper_1812_01108_amd import _lib
    from paper_1812_01108_amd.residues import default_table
    lib = _lib.load()
    tab = default_table().to_struct()
    mutate(tab.residues[4])          # PHE: two side frames, z-matrix ring atoms
    st = lib.a2c_residue_table_info(ctypes.byref(tab), None, None)
    assert st == -1
    assert msg in lib.a2c_last_error().decode()
