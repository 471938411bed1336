"""Pins of the oracle's periodic octree and its continuous Q_q space with hanging nodes."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import octree as ot, octree_fe as ofe, operator as op
from oracle.basis import gauss_legendre, lgl_nodes, lagrange

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _refine_at(tree, leaf_pred):
    out = set(tree)
    for o in tree:
        if leaf_pred(o):
            out.remove(o)
            out.update(ot.children(o))
    return ot.sort_leaves(out)


def _corner_tree(base, depth):
    """Uniform base level, one corner leaf refined `depth` more levels (not balanced)."""
    leaves = set(ot.uniform(base))
    o = (base, 0, 0, 0)
    for _ in range(depth):
        leaves.remove(o)
        kids = ot.children(o)
        leaves.update(kids)
        o = kids[-1]
    return ot.sort_leaves(leaves)


def _touch_matrix(leaves):
    """Brute force: do the closed boxes of leaves i, j touch on the periodic cube?"""
    L = np.array([o[0] for o in leaves])
    X = np.array([[o[1], o[2], o[3]] for o in leaves])
    S = np.array([ot.size(l) for l in L])
    U = ot.UNITS
    touch = np.ones((len(leaves), len(leaves)), dtype=bool)
    for k in range(3):
        a1, s1 = X[:, k][:, None], S[:, None]
        a2, s2 = X[:, k][None, :], S[None, :]
        ok = np.zeros_like(touch)
        for m in (-U, 0, U):
            ok |= (a1 <= a2 + m + s2) & (a2 + m <= a1 + s1)
        touch &= ok
    np.fill_diagonal(touch, False)
    return touch, L


def _balanced(leaves):
    touch, L = _touch_matrix(leaves)
    return not np.any(touch & (np.abs(L[:, None] - L[None, :]) > 1))


def _covers(coarse, fine):
    """Every fine leaf lies inside exactly one coarse leaf."""
    loc = ot.Locator(coarse)
    for l, x, y, z in fine:
        c = loc.find(x, y, z)
        if c[0] > l:
            return False
    return True


@pytest.mark.parametrize("base,depth", [(2, 3), (3, 4)])
def test_balance_is_2to1_refining_and_minimal(base, depth):
    t = _corner_tree(base, depth)
    assert ot.is_linear_complete(t) and not _balanced(t)
    b = ot.balance(t)
    assert ot.is_linear_complete(b)
    assert _balanced(b)
    assert _covers(t, b)
    # minimal: merging back any family that balancing created breaks the balance
    bset = set(b)
    tset = set(t)
    fams = {}
    for o in b:
        if o not in tset:
            fams.setdefault(ot.parent(o), []).append(o)
    checked = 0
    for p, kids in fams.items():
        if len(kids) == 8 and all(k in bset for k in kids):
            merged = ot.sort_leaves((bset - set(kids)) | {p})
            assert not _balanced(merged)
            checked += 1
    assert checked > 0


def test_uniform_is_complete_and_balanced_and_morton_sorted():
    u = ot.uniform(3)
    assert len(u) == 512 and ot.is_linear_complete(u) and not ot.violators(u)
    assert ot.morton(1, 0, 0) == 1 and ot.morton(0, 1, 0) == 2 and ot.morton(0, 0, 1) == 4
    assert ot.morton(2, 0, 0) == 8
    assert not ot.is_linear_complete(u[:-1])


def test_refinement_stops_where_the_indicator_says():
    rng = np.random.default_rng(3)
    c, s, a = rng.random((2, 3)), np.full(2, 0.01), rng.standard_normal(2)
    t = ot.refine_by_indicator(2, 6, c, s, a)
    thr = 1e-2 * np.abs(a).sum()
    for o in t:
        assert o[0] == 6 or ot.gradient_indicator(o, c, s, a) <= thr
        if o[0] > 2:
            assert ot.gradient_indicator(ot.parent(o), c, s, a) > thr
    assert max(o[0] for o in t) == 6
    # the distance is periodic: a centre at 0.999 refines leaves at x = 0 too
    t2 = ot.refine_by_indicator(2, 5, np.array([[0.999, 0.5, 0.5]]), np.array([0.01]), np.array([1.0]))
    assert any(o[0] == 5 and o[1] == 0 for o in t2)


def test_periodic_distance_closed_forms():
    assert ot.periodic_box_distance((0.5, 0.5, 0.5), (0.25, 0.25, 0.25), 0.5) == 0.0
    assert abs(ot.periodic_box_distance((0.95, 0.5, 0.5), (0.0, 0.5, 0.5), 0.25) - 0.05) < 1e-15
    assert abs(ot.periodic_box_distance((0.0, 0.0, 0.0), (0.5, 0.5, 0.5), 0.25) - np.sqrt(3) * 0.25) < 1e-15


def test_hierarchy_nests_and_ends_uniform():
    t = ot.balance(_corner_tree(2, 4))
    H = ot.hierarchy(t, 2)
    assert H[0] == ot.uniform(2) and H[-1] == t
    for c, f in zip(H[:-1], H[1:]):
        assert ot.is_linear_complete(c) and _balanced(c) and _covers(c, f)
        assert max(o[0] for o in c) == max(o[0] for o in f) - 1
        # every coarse leaf is a fine leaf or the parent of 8 fine leaves
        fset = set(f)
        for o in c:
            assert o in fset or all(k in fset for k in ot.children(o))


# ---------------------------------------------------------------------------- FE space

def _mixed(q):
    return ofe.OctreeSpace(ot.balance(_corner_tree(2, 2)), q)


@pytest.mark.parametrize("q,level", [(1, 2), (2, 2), (2, 3)])
def test_uniform_octree_reproduces_uniform_operator(q, level):
    S = ofe.OctreeSpace(ot.uniform(level), q)
    A = op.assemble(q, 1 << level)
    assert S.ndof == A.shape[0] and not S.hanging_src
    assert abs(S.A - A).max() <= 1e-14 * abs(A).max()
    assert abs(S.M - op.assemble(q, 1 << level, "mass")).max() <= 1e-15


@pytest.mark.parametrize("q", [1, 2])
def test_null_space_symmetry_definiteness(q):
    S = _mixed(q)
    A = S.A.toarray()
    assert len(S.hanging_src) > 0
    assert np.abs(A @ np.ones(S.ndof)).max() < 1e-13 * np.abs(A).max()
    assert np.abs(A - A.T).max() < 1e-15 * np.abs(A).max()
    w = np.linalg.eigvalsh(A)
    assert abs(w[0]) < 1e-12 * w[-1] and w[1] > 1e-6 * w[-1]
    M = S.M.toarray()
    assert np.linalg.eigvalsh(M)[0] > 0
    assert abs(M.sum() - 1.0) < 1e-13  # the basis sums to one and the cube has volume 1


def _face_points(S, rng, per_face=2):
    """Random points on the faces of random leaves, with the leaf on each side."""
    out = []
    for e in rng.choice(S.E, min(S.E, 40), replace=False):
        l, x, y, z = S.leaves[e]
        h = 1.0 / (1 << l)
        lo = np.array([x, y, z]) / ot.UNITS
        for ax in range(3):
            for side in (0, 1):
                for _ in range(per_face):
                    p = lo + rng.random(3) * h
                    p[ax] = lo[ax] + side * h
                    out.append((e, p % 1.0, ax, side))
    return out


def _eval_in_leaf(S, e, x, p):
    """The polynomial of leaf e (through its constrained nodal values) at point p of its closed box."""
    m1 = S.m1
    ue = (S.C @ x).reshape(S.E, m1 ** 3)[e]
    l, ax, ay, az = S.leaves[e]
    h = 1.0 / (1 << l)
    # local coordinate in [0, 1] (a point on the upper face of the leaf is at 1)
    t = np.array([((p[k] - (ax, ay, az)[k] / ot.UNITS) % 1.0) / h for k in range(3)])
    assert np.all(t <= 1.0 + 1e-9), t
    B = lagrange(lgl_nodes(S.q), t)
    phi = np.einsum("a,b,c->cba", B[:, 0], B[:, 1], B[:, 2]).ravel()
    return phi @ ue


@pytest.mark.parametrize("q", [1, 2])
def test_fe_functions_are_continuous_across_faces(q):
    """A wrong hanging weight, sign or index shows up as a jump across a coarse-fine face."""
    S = ofe.OctreeSpace(ot.balance(_corner_tree(2, 3)), q)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(S.ndof)
    n = 0
    for e, p, ax, side in _face_points(S, rng):
        # the neighbour across the face: the leaf holding a point just beyond it
        eps = np.zeros(3)
        eps[ax] = (1 if side else -1) * 1e-9
        q_ = (p + eps) % 1.0
        o = S.loc.find(*[int(np.floor(c * ot.UNITS)) % ot.UNITS for c in q_])
        f = S.leaf_index()[o]
        if f == e:
            continue
        # evaluate the neighbour at the same point: local coordinate 0 or 1 on its side
        pa = p.copy()
        v_e = _eval_in_leaf(S, e, x, pa)
        v_f = _eval_in_leaf(S, f, x, pa)
        assert abs(v_e - v_f) <= 1e-12 * max(1.0, abs(v_e)), (S.leaves[e], o, p)
        n += 1
    assert n > 100


def test_hanging_weights_are_rows_of_the_1d_prolongation():
    g = GOLDEN["q2_quarter_point_prolongation"]
    one_d = {0.0: (1.0, 0.0, 0.0), 0.25: tuple(g["row_at_1_4"]), 0.5: (0.0, 1.0, 0.0),
             0.75: tuple(g["row_at_3_4"]), 1.0: (0.0, 0.0, 1.0)}
    S = _mixed(2)
    m1 = 3
    checked = 0
    for p, o in S.hanging_src.items():
        e = S.leaf_index()[o]
        nodes = [tuple(S.pos[e, a]) for a in range(27)]
        if any(nd in S.hanging_src for nd in nodes):
            continue  # a chained constraint; covered by continuity
        s = ot.size(o[0])
        t = [tk / (2.0 * s) for tk in S.local(o, p)]
        w = S.expand(p)
        for a in range(27):
            ia, ib, ic = a % m1, (a // m1) % m1, a // (m1 * m1)
            want = one_d[t[0]][ia] * one_d[t[1]][ib] * one_d[t[2]][ic]
            assert w.get(S.dof[nodes[a]], 0.0) == want
        checked += 1
    assert checked > 10


@pytest.mark.parametrize("q", [1, 2])
def test_prolongation_nests_and_galerkin_identity(q):
    H = ot.hierarchy(ot.balance(_corner_tree(2, 2)), 2)
    coarse, fine = ofe.OctreeSpace(H[-2], q), ofe.OctreeSpace(H[-1], q)
    P = ofe.prolongation(coarse, fine)
    rng = np.random.default_rng(11)
    xc = rng.standard_normal(coarse.ndof)
    pts = rng.random((200, 3))
    assert np.allclose(coarse.evaluate(xc, pts), fine.evaluate(P @ xc, pts), atol=1e-12, rtol=0)
    assert np.allclose(P @ np.ones(coarse.ndof), 1.0, atol=1e-14)
    G = (P.T @ fine.A @ P).toarray()
    assert np.abs(G - coarse.A.toarray()).max() <= 1e-13 * np.abs(G).max()


def _l2_error(S, u, exact):
    """sqrt(sum_e int_e (u_h - u)^2) with (q+2)^3 Gauss points per leaf."""
    t, w = gauss_legendre(S.q + 2)
    B = lagrange(lgl_nodes(S.q), t)  # (m1, g)
    phi = np.einsum("ai,bj,ck->ijkcba", B, B, B).reshape(len(t) ** 3, -1)
    W = np.einsum("i,j,k->ijk", w, w, w).ravel()
    T = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)  # (i, j, k) = (x, y, z)
    ue = (S.C @ u).reshape(S.E, -1)
    err = 0.0
    for e, (l, x, y, z) in enumerate(S.leaves):
        h = 1.0 / (1 << l)
        pts = np.array([x, y, z]) / ot.UNITS + h * T
        err += h ** 3 * np.sum(W * (phi @ ue[e] - exact(pts)) ** 2)
    return np.sqrt(err)


@pytest.mark.parametrize("q", [1, 2])
def test_l2_convergence_on_graded_octrees(q):
    """sin(2 pi x) sin(2 pi y) sin(2 pi z): the L2 error falls by 2^(q+1) per refinement."""
    exact = lambda p: np.sin(2 * np.pi * p[:, 0]) * np.sin(2 * np.pi * p[:, 1]) * np.sin(2 * np.pi * p[:, 2])
    base = ot.balance(_corner_tree(2, 2))
    errs = []
    first = 1 if q == 1 else 0
    for k in range(first, first + 2):
        tree = base
        for _ in range(k):
            tree = ot.sort_leaves([c for o in tree for c in ot.children(o)])
        S = ofe.OctreeSpace(tree, q)
        b = ofe.rhs(S, 12 * np.pi ** 2 * exact(S.coords()))
        A = S.A.tocsr()
        u = np.zeros(S.ndof)
        u[1:] = spla.spsolve(A[1:, 1:].tocsc(), b[1:])
        u = ofe.normalize_mean(S, u)
        errs.append(_l2_error(S, u, exact))
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - (q + 1)) < 0.35, (errs, rate)


def test_octree_vcycle_is_symmetric_and_pcg_converges():
    from oracle import krylov, multigrid as mg
    H = ot.hierarchy(ot.balance(_corner_tree(2, 3)), 2)
    MG = ofe.OctreeHierarchy(H, 2, mg.Options(seed=3))
    assert MG.L == len(H) == 4
    S = MG.spaces[-1]
    rng = np.random.default_rng(1)
    x, y = mg.project(rng.standard_normal(S.ndof)), mg.project(rng.standard_normal(S.ndof))
    Vx, Vy = MG.vcycle(x), MG.vcycle(y)
    assert abs(y @ Vx - x @ Vy) <= 1e-12 * abs(x @ Vy)
    assert x @ Vx > 0
    b = ofe.rhs(S, rng.standard_normal(S.ndof))
    u, info = krylov.pcg(S.A, b, MG.vcycle, 1e-10, 50)
    assert info.converged and info.iters <= 12
    assert np.linalg.norm(b - S.A @ u) <= 1e-10 * np.linalg.norm(b) * 1.001


# ---------------------------------------------------------------- sharp layer (test case 2)

def test_sharp_layer_profile_is_minus_the_radial_laplacian():
    """f = -(u'' + 2 u'/r) for u = exp(-(r/R)^alpha), and f' is the derivative of f:
    both against central differences of the plain definitions, across the layer."""
    R, alpha = 0.25, 10.0
    u = lambda r: math.exp(-((r / R) ** alpha))
    h = 1e-5
    for r in np.linspace(0.05, 0.45, 41):
        f, fp = ot.sharp_layer_profile(r, R, alpha)
        upp = (u(r + h) - 2.0 * u(r) + u(r - h)) / (h * h)
        up = (u(r + h) - u(r - h)) / (2.0 * h)
        assert abs(f + upp + 2.0 * up / r) <= 1e-4 * 400.0
        fdf = (ot.sharp_layer_profile(r + h, R, alpha)[0] - ot.sharp_layer_profile(r - h, R, alpha)[0]) / (2 * h)
        assert abs(fp - fdf) <= 1e-5 * max(1.0, abs(fp))
    assert ot.sharp_layer_profile(0.0, R, alpha) == (0.0, 0.0)


def test_periodic_box_distance_range_brackets_every_point():
    rng = np.random.default_rng(3)
    for _ in range(300):
        c = rng.random(3)
        l = int(rng.integers(1, 5))
        h = 1.0 / (1 << l)
        lo = rng.integers(0, 1 << l, 3) * h
        dmin, dmax = ot.periodic_box_distance_range(c, lo, h)
        pts = lo + h * rng.random((400, 3))
        d = np.abs(pts - c) % 1.0
        d = np.minimum(d, 1.0 - d)
        r = np.sqrt((d * d).sum(1))
        assert r.min() >= dmin - 1e-12 and r.max() <= dmax + 1e-12
        # the corners and the box's nearest point attain the range up to the sampling
        assert dmin == pytest.approx(ot.periodic_box_distance(c, lo, h), abs=1e-15)
        assert r.max() >= dmax - 2 * h


def test_sharp_layer_refinement_concentrates_on_the_sphere():
    """Leaves cut by the sphere r = R reach the finest level, every finest leaf lies in a band
    around the sphere, and the tree is complete and 2:1 balanced."""
    centre, R, alpha, top = (0.5, 0.5, 0.5), 0.25, 10.0, 5
    tree = ot.refine_sharp_layer(2, top, centre, R, alpha, 1e-2)
    assert ot.is_linear_complete(tree) and not ot.violators(tree)
    finest = 0
    for l, x, y, z in tree:
        h = 1.0 / (1 << l)
        dmin, dmax = ot.periodic_box_distance_range(centre, (x / ot.UNITS, y / ot.UNITS, z / ot.UNITS), h)
        if dmin <= R <= dmax:
            assert l == top
        if l == top:
            finest += 1
        if dmin > 0.4:  # exp(-(0.4/R)**alpha) < 1e-50: the source and its slope vanish there
            assert l < top
    assert finest > len(tree) // 2


def _assert_refines(coarse, fine):
    """Every leaf of `fine` lies inside some leaf of `coarse` (fine refines coarse)."""
    cells = {(l, x, y, z) for l, x, y, z in coarse}
    for l, x, y, z in fine:
        hit = False
        for lc in range(l, -1, -1):
            m = ot.UNITS >> lc
            if (lc, x - x % m, y - y % m, z - z % m) in cells:
                hit = True
                break
        assert hit


def test_sharp_layer_smaller_tolerance_refines_the_tree():
    """The criterion h * max|f'| > tol * max|f| only switches on more cells as tol falls, so the
    tree for a smaller tolerance refines the tree for a larger one."""
    centre, R, alpha = (0.5, 0.5, 0.5), 0.25, 10.0
    loose = ot.refine_sharp_layer(2, 5, centre, R, alpha, 1e-1)
    tight = ot.refine_sharp_layer(2, 5, centre, R, alpha, 1e-2)
    assert len(tight) > len(loose)
    _assert_refines(loose, tight)
