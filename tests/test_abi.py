"""The C ABI library loads and exports every symbol include/gmg.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmg_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_1408_6497_amd import gmg
    if not os.path.exists(gmg.LIB_PATH):
        pytest.skip("libgmg.so not built (run __graft_entry__.build())")
    return gmg.load()


def test_header_lists_the_boundary():
    names = _declared()
    for required in ("gmg_setup", "gmg_apply", "gmg_vcycle", "gmg_solve"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1408_6497_amd import gmg
    assert sorted(gmg.EXPORTS) == _declared()


def test_invalid_arguments_rejected_before_device_work():
    from paper_1408_6497_amd import gmg
    lib = _lib()
    h = ctypes.c_void_p()
    opts = gmg.GmgOptions()
    # order 17 (beyond Section 2.3.2's 16), n not a power of two, one element for q = 2, too
    # few nodes, order 0, a generic order on a mesh above its size limit, a generic order
    # on an octree mesh
    for order, n in ((17, 8), (2, 6), (2, 1), (1, 2), (0, 8), (5, 128), (3, 0), (16, 0)):
        mesh = gmg.GmgMesh(order=order, n=n, levels=0, reserved=0)
        st = lib.gmg_setup(ctypes.byref(mesh), ctypes.byref(opts), None, ctypes.byref(h))
        assert st == 1, (order, n, st)
    assert lib.gmg_setup(None, None, None, ctypes.byref(h)) == 1
    # too many levels for the mesh; too few (coarsest level above 512 DoFs, or above one
    # element where that element alone has more)
    for order, n, levels in ((2, 8, 5), (2, 8, 1), (5, 4, 4), (5, 4, 2), (16, 2, 1), (9, 4, 2)):
        mesh = gmg.GmgMesh(order=order, n=n, levels=levels, reserved=0)
        assert lib.gmg_setup(ctypes.byref(mesh), ctypes.byref(opts), None, ctypes.byref(h)) == 1, (order, n, levels)
    assert lib.gmg_status_string(5) == b"not converged"
    assert lib.gmg_destroy(None) == 0


def test_invalid_octrees_rejected_before_device_work():
    """Unsorted, incomplete or unbalanced octrees give GMG_E_MESH; q = 4 octrees and empty
    leaf arrays give GMG_E_ARG -- all before any device call."""
    import numpy as np
    from oracle import octree as ot
    from paper_1408_6497_amd import gmg
    lib = _lib()
    h = ctypes.c_void_p()
    opts = gmg.GmgOptions()

    def setup(order, leaves):
        k = np.array([ot.morton(o[1], o[2], o[3]) for o in leaves], dtype=np.uint64)
        l = np.array([o[0] for o in leaves], dtype=np.uint8)
        mesh = gmg.GmgMesh(order=order, n=0, levels=0, reserved=0, n_leaves=k.size,
                           leaf_morton=k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                           leaf_level=l.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return lib.gmg_setup(ctypes.byref(mesh), ctypes.byref(opts), None, ctypes.byref(h))

    u = ot.uniform(2)
    deep = set(u)
    o = (2, 0, 0, 0)
    for _ in range(3):
        deep.remove(o)
        kids = ot.children(o)
        deep.update(kids)
        o = kids[-1]
    assert setup(2, ot.sort_leaves(deep)) == 2   # not 2:1 balanced
    assert setup(2, u[:-1]) == 2                  # incomplete
    assert setup(2, u[::-1]) == 2                 # not in Morton order
    assert setup(2, ot.uniform(1)) == 2           # coarser than the coarsest multigrid level
    assert setup(4, u) == 1                       # octrees take q = 1, 2
    mesh = gmg.GmgMesh(order=2, n=0, levels=0, reserved=0, n_leaves=0)
    assert lib.gmg_setup(ctypes.byref(mesh), ctypes.byref(opts), None, ctypes.byref(h)) == 1
