"""The library's host octree construction (C ABI, no GPU needed) against the oracle: bit-exact leaves."""
import ctypes

import numpy as np
import pytest

from oracle import octree as ot


def _lib():
    from paper_1408_6497_amd import gmg
    try:
        return gmg, gmg.load()
    except (OSError, RuntimeError) as e:  # the library is built by __graft_entry__.build()
        pytest.skip(f"libgmg.so not loadable here: {e}")


def _as_leaves(keys, levels):
    out = []
    for k, l in zip(keys.tolist(), levels.tolist()):
        x = y = z = 0
        for b in range(ot.DMAX):
            x |= ((k >> (3 * b)) & 1) << b
            y |= ((k >> (3 * b + 1)) & 1) << b
            z |= ((k >> (3 * b + 2)) & 1) << b
        out.append((l, x, y, z))
    return out


def _as_arrays(leaves):
    return (np.array([ot.morton(o[1], o[2], o[3]) for o in leaves], dtype=np.uint64),
            np.array([o[0] for o in leaves], dtype=np.uint8))


@pytest.mark.parametrize("seed,count,sigma,base,top", [(0, 4, 1e-3, 3, 9), (5, 3, 2e-2, 2, 7), (9, 1, 5e-3, 3, 8)])
def test_refine_gaussians_matches_oracle(seed, count, sigma, base, top):
    gmg, _ = _lib()
    rng = np.random.default_rng(seed)
    c, s, a = rng.random((count, 3)), np.full(count, sigma), rng.standard_normal(count)
    keys, lev = gmg.octree_refine_gaussians(base, top, c, s, a)
    ref = ot.refine_gaussians(base, top, c, s, a)
    assert _as_leaves(keys, lev) == ref


@pytest.mark.parametrize("base,top,centre,radius,alpha,tol", [
    (2, 4, (0.5, 0.5, 0.5), 0.25, 10.0, 1e-2),
    (3, 5, (0.3, 0.6, 0.9), 0.2, 20.0, 1e-2),
    (2, 5, (0.01, 0.99, 0.5), 0.3, 40.0, 3e-2),   # the layer wraps across three faces
])
def test_refine_sharp_layer_matches_oracle(base, top, centre, radius, alpha, tol):
    gmg, _ = _lib()
    keys, lev = gmg.octree_refine_sharp_layer(base, top, centre, radius, alpha, tol)
    assert _as_leaves(keys, lev) == ot.refine_sharp_layer(base, top, centre, radius, alpha, tol)


def test_refine_sharp_layer_rejects_bad_arguments():
    gmg, lib = _lib()
    cnt = ctypes.c_int64()
    c = np.array([0.5, 0.5, 0.5])
    vp = c.ctypes.data_as(ctypes.c_void_p)
    for args in ((3, 2, vp, 0.25, 10.0, 1e-2), (2, 4, vp, 0.0, 10.0, 1e-2), (2, 4, vp, 0.25, 2.0, 1e-2),
                 (2, 4, None, 0.25, 10.0, 1e-2), (2, 11, vp, 0.25, 10.0, 1e-2)):
        assert lib.gmg_octree_refine_sharp_layer(*args, None, None, 0, ctypes.byref(cnt)) == 1  # GMG_E_ARG
    bad = np.array([0.5, 1.0, 0.5])
    assert lib.gmg_octree_refine_sharp_layer(2, 4, bad.ctypes.data_as(ctypes.c_void_p), 0.25, 10.0, 1e-2,
                                             None, None, 0, ctypes.byref(cnt)) == 1


def test_balance_matches_oracle_and_rejects_incomplete():
    gmg, lib = _lib()
    leaves = set(ot.uniform(2))
    o = (2, 0, 0, 0)
    for _ in range(4):
        leaves.remove(o)
        kids = ot.children(o)
        leaves.update(kids)
        o = kids[-1]
    t = ot.sort_leaves(leaves)
    keys, lev = gmg.octree_balance(*_as_arrays(t))
    assert _as_leaves(keys, lev) == ot.balance(t)
    k, l = _as_arrays(t[:-1])
    cnt = ctypes.c_int64()
    st = lib.gmg_octree_balance(k.ctypes.data_as(ctypes.c_void_p), l.ctypes.data_as(ctypes.c_void_p), k.size,
                                None, None, 0, ctypes.byref(cnt))
    assert st == 2  # GMG_E_MESH
