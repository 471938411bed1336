"""Octree levels on the GPU (gather / element apply / gather kernels, CSR transfers) vs the FP64 oracle.

Same bars as the uniform path: FP64 applies within 1e-12 relative l2, FP32
within 2e-5; the hierarchy (leaves of every level), the DoF numbering and the
DoF coordinates are integer / exact and compared exactly.
"""
import functools

import numpy as np
import pytest

from tests.gpu_common import FP32_TOL, FP64_TOL, mean_free_normal, rel_l2, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _corner_tree(base, depth):
    from oracle import octree as ot
    leaves = set(ot.uniform(base))
    o = (base, 0, 0, 0)
    for _ in range(depth):
        leaves.remove(o)
        kids = ot.children(o)
        leaves.update(kids)
        o = kids[-1]
    return ot.balance(ot.sort_leaves(leaves))


def _arrays(leaves):
    from oracle import octree as ot
    return (np.array([ot.morton(o[1], o[2], o[3]) for o in leaves], dtype=np.uint64),
            np.array([o[0] for o in leaves], dtype=np.uint8))


@functools.lru_cache(maxsize=None)
def _oracle(q, case, seed=0):
    from oracle import octree as ot, octree_fe as ofe, multigrid as mg
    tree = _tree(case)
    return ofe.OctreeHierarchy(ot.hierarchy(tree, 2), q, mg.Options(seed=seed))


@functools.lru_cache(maxsize=None)
def _tree(case):
    from oracle import octree as ot
    if case == "corner":
        return tuple(_corner_tree(2, 3))
    if case == "gauss":
        rng = np.random.default_rng(21)
        return tuple(ot.refine_gaussians(3, 6, rng.random((4, 3)), np.full(4, 1e-2), rng.standard_normal(4)))
    raise KeyError(case)


def _ctx(q, case, **kw):
    torch_cuda()
    from paper_1408_6497_amd import Context
    return Context(q, 0, leaves=_arrays(_tree(case)), **kw)


CASES = [(1, "corner"), (2, "corner"), (2, "gauss")]


@pytest.mark.parametrize("q,case", CASES)
def test_hierarchy_numbering_and_coordinates(q, case):
    from oracle import octree as ot
    ctx = _ctx(q, case)
    MG = _oracle(q, case)
    assert ctx.levels == MG.L
    for l in range(ctx.levels):
        keys, lev = ctx.level_leaves(l)
        ref = MG.spaces[l].leaves
        assert [(int(b), *(_dec(int(a)))) for a, b in zip(keys, lev)] == [tuple(o) for o in ref]
        assert ctx.num_dofs(l) == MG.spaces[l].ndof
        assert ctx.num_elements(l) == len(ref)
        assert np.array_equal(ctx.dof_coords(l), MG.spaces[l].coords())
    print(f"[octree] q={q} {case}: levels {ctx.levels}, DoFs {[ctx.num_dofs(l) for l in range(ctx.levels)]}",
          flush=True)


def _dec(k):
    x = y = z = 0
    for b in range(10):
        x |= ((k >> (3 * b)) & 1) << b
        y |= ((k >> (3 * b + 1)) & 1) << b
        z |= ((k >> (3 * b + 2)) & 1) << b
    return x, y, z


@pytest.mark.parametrize("q,case", CASES)
def test_apply_mass_diagonal_parity(q, case):
    torch = torch_cuda()
    ctx = _ctx(q, case)
    MG = _oracle(q, case)
    for l in range(ctx.levels):
        S = MG.spaces[l]
        x = mean_free_normal(S.ndof, 100 + l)
        for prec, dt, tol in ((0, torch.float64, FP64_TOL), (1, torch.float32, FP32_TOL)):
            xd = to_dev(x, dt)
            yd = torch.empty_like(xd)
            ctx.apply(l, xd, yd)
            md = torch.empty_like(xd)
            ctx.mass(l, xd, md)
            torch.cuda.synchronize()
            xr = to_host(xd)
            ea, em = rel_l2(to_host(yd), S.A @ xr), rel_l2(to_host(md), S.M @ xr)
            assert ea <= tol and em <= tol, (l, prec, ea, em)
        d = torch.empty(S.ndof, dtype=torch.float64, device="cuda")
        ctx.diagonal(l, d)
        torch.cuda.synchronize()
        assert rel_l2(to_host(d), S.A.diagonal()) <= 1e-14


@pytest.mark.parametrize("q,case", CASES)
def test_transfers_parity(q, case):
    torch = torch_cuda()
    ctx = _ctx(q, case)
    MG = _oracle(q, case)
    for l in range(1, ctx.levels):
        P = MG.levels[l].transfer.P
        xf = mean_free_normal(P.shape[0], 7 + l)
        xc = mean_free_normal(P.shape[1], 8 + l)
        for dt, tol in ((torch.float64, 1e-14), (torch.float32, 1e-6)):
            rc = torch.empty(P.shape[1], dtype=dt, device="cuda")
            ctx.restrict(l, to_dev(xf, dt), rc)
            uf = to_dev(xf, dt)
            ctx.prolong(l, to_dev(xc, dt), uf)
            torch.cuda.synchronize()
            xf_r, xc_r = to_host(to_dev(xf, dt)), to_host(to_dev(xc, dt))
            assert rel_l2(to_host(rc), P.T @ xf_r) <= tol
            assert rel_l2(to_host(uf), xf_r + P @ xc_r) <= tol


@pytest.mark.parametrize("q,case", CASES)
def test_lambda_smoother_vcycle_parity(q, case):
    torch = torch_cuda()
    ctx = _ctx(q, case)
    MG = _oracle(q, case)
    for l in range(ctx.levels):
        assert abs(ctx.lam(l) - MG.levels[l].lam) <= 1e-10 * MG.levels[l].lam
    l = ctx.levels - 1
    lev = MG.levels[l]
    b = mean_free_normal(lev.size, 31)
    u0 = mean_free_normal(lev.size, 32)
    ud = to_dev(u0, torch.float64)
    ctx.smooth(l, to_dev(b, torch.float64), ud, 2)
    torch.cuda.synchronize()
    assert rel_l2(to_host(ud), MG.smooth(lev, b, u0, 2)) <= 1e-12
    zd = torch.empty(lev.size, dtype=torch.float64, device="cuda")
    ctx.vcycle(to_dev(b, torch.float64), zd)
    z32 = torch.empty(lev.size, dtype=torch.float32, device="cuda")
    ctx.vcycle(to_dev(b, torch.float32), z32)
    torch.cuda.synchronize()
    z = MG.vcycle(b)
    assert rel_l2(to_host(zd), z) <= 1e-11
    assert rel_l2(to_host(z32), z) <= 1e-4


@pytest.mark.parametrize("q,case", [(1, "corner"), (2, "gauss")])
def test_solves_reach_tolerance_on_the_oracle_operator(q, case):
    torch = torch_cuda()
    from oracle import multigrid as mg
    from paper_1408_6497_amd import GMG_FP32, GMG_FP64
    from workloads import gaussian_params, gaussian_source_points
    MG = _oracle(q, case)
    S = MG.spaces[-1]
    params = gaussian_params(3, 4, 0.01, 0.05)
    f = gaussian_source_points(S.coords(), params)
    b = mg.project(S.M @ f)
    for prec in (GMG_FP64, GMG_FP32):
        ctx = _ctx(q, case, vcycle_prec=prec)
        fd = torch.from_numpy(f).cuda()
        u = torch.empty_like(fd)
        info = ctx.solve(fd, u, 1e-8)
        torch.cuda.synchronize()
        uh = to_host(u)
        res = b - S.A @ uh
        rel = np.linalg.norm(res - res.mean()) / np.linalg.norm(b)
        w = S.M @ np.ones(S.ndof)
        print(f"[octree-solve] q={q} {case} prec={prec}: iters {info.inner_iters} rel {rel:.2e} "
              f"mean {w @ uh:.1e}", flush=True)
        assert rel <= 1e-8 * 1.001
        assert abs(w @ uh) <= 1e-10 * np.abs(uh).max()


def test_invalid_octrees_are_rejected():
    torch_cuda()
    from oracle import octree as ot
    from paper_1408_6497_amd import Context, GmgError
    # not 2:1 balanced: one corner leaf refined three levels below its neighbours
    leaves = set(ot.uniform(2))
    o = (2, 0, 0, 0)
    for _ in range(3):
        leaves.remove(o)
        kids = ot.children(o)
        leaves.update(kids)
        o = kids[-1]
    bad = ot.sort_leaves(leaves)
    for arrays in (_arrays(bad), _arrays(ot.uniform(2)[:-1]), _arrays(ot.uniform(2)[::-1])):
        with pytest.raises(GmgError) as e:
            Context(2, 0, leaves=arrays)
        assert e.value.status == 2  # GMG_E_MESH


def test_adaptive_workload_full_size():
    """The adaptive workload at its full size: 4 Gaussians (sigma 1e-3, seed 0) refined by the
    gradient bound from level 3 to level 9, Q2; the library's tree equals the oracle's, and the
    plain FP64 and the FP32-cycle solves reach 1e-8 on the oracle's assembled operator."""
    torch = torch_cuda()
    from oracle import octree as ot, octree_fe as ofe, multigrid as mg
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64, octree_refine_gaussians
    from workloads import gaussian_params, gaussian_source_points
    p = gaussian_params(0, 4, 1e-3, 1e-3)
    keys, lev = octree_refine_gaussians(3, 9, p["centres"], p["sigma"], p["amps"])
    tree = ot.refine_gaussians(3, 9, p["centres"], p["sigma"], p["amps"])
    assert [(int(b), *_dec(int(a))) for a, b in zip(keys, lev)] == [tuple(o) for o in tree]
    S = ofe.OctreeSpace(tree, 2)
    f = gaussian_source_points(S.coords(), p)
    b = mg.project(S.M @ f)
    for prec in (GMG_FP64, GMG_FP32):
        ctx = Context(2, 0, leaves=(keys, lev), vcycle_prec=prec)
        assert ctx.num_dofs() == S.ndof and np.array_equal(ctx.dof_coords(), S.coords())
        fd = torch.from_numpy(f).cuda()
        u = torch.empty_like(fd)
        info = ctx.solve(fd, u, 1e-8)
        torch.cuda.synchronize()
        res = b - S.A @ to_host(u)
        rel = np.linalg.norm(res - res.mean()) / np.linalg.norm(b)
        print(f"[c5] leaves {len(tree)} DoFs {S.ndof} levels {ctx.levels} prec {prec}: iters {info.inner_iters} "
              f"rel {rel:.2e} t_solve {info.t_solve * 1e3:.2f} ms", flush=True)
        assert rel <= 1e-8 * 1.001


@pytest.mark.parametrize("prec", [0, 1])
def test_octree_graph_replay_matches_eager(prec):
    """Octree V-cycles replayed from a captured HIP graph give the bits of the eager launches,
    replay after replay, with unrelated eager work in between."""
    torch = torch_cuda()
    from workloads import gaussian_params, gaussian_source_points
    eager = _ctx(2, "gauss", seed=2, vcycle_prec=prec, no_graphs=1)
    graph = _ctx(2, "gauss", seed=2, vcycle_prec=prec)
    f = torch.from_numpy(gaussian_source_points(eager.dof_coords(), gaussian_params(3, 4, 0.01, 0.05))).cuda()
    ue, ug = torch.empty_like(f), torch.empty_like(f)
    for rep in range(3):
        ie = eager.solve(f, ue, 1e-8)
        scratch = torch.randn_like(f) * 3.0
        ig = graph.solve(f, ug, 1e-8)
        torch.cuda.synchronize()
        assert ie.inner_iters == ig.inner_iters
        assert torch.equal(ue, ug), f"replay {rep} differs"
        del scratch


@functools.lru_cache(maxsize=None)
def _sharp_oracle(q, top):
    """Oracle space, exact solution, source and a converged sparse-CG solution for the
    sharp-layer case (alpha 10, radius 0.25, centre (0.5, 0.5, 0.5)) on levels 2..top."""
    import scipy.sparse.linalg as spl
    from oracle import octree as ot, octree_fe as ofe, multigrid as mg
    from workloads import sharp_layer
    tree = ot.refine_sharp_layer(2, top, (0.5, 0.5, 0.5), 0.25, 10.0, 1e-2)
    S = ofe.OctreeSpace(tree, q)
    ue, f = sharp_layer(S.coords())
    b = mg.project(S.M @ f)
    x, info = spl.cg(S.A.tocsr(), b, rtol=1e-12, maxiter=50000)
    assert info == 0
    return tree, S, ue, f, b, x


def _err_mod_const(u, ue):
    """max-norm distance of u to ue + c, minimised over the constant c (the periodic
    solution is fixed only up to a constant)."""
    e = u - ue
    return 0.5 * (e.max() - e.min())


@pytest.mark.parametrize("q", [1, 2])
def test_sharp_layer_solve_matches_oracle_and_converges(q):
    """The sharp-layer test solution u = exp(-(r/R)^alpha): the library's refinement equals the
    oracle's, both V-cycle precisions drive the residual on the oracle's assembled operator to
    1e-8, the nodal max-norm error matches the oracle's own sparse solve, and it falls as the
    maximum level grows."""
    torch = torch_cuda()
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64, octree_refine_sharp_layer
    errs = []
    for top in (4, 5):
        tree, S, ue, f, b, x = _sharp_oracle(q, top)
        keys, lev = octree_refine_sharp_layer(2, top, (0.5, 0.5, 0.5), 0.25, 10.0, 1e-2)
        assert [(int(l), *_dec(int(k))) for k, l in zip(keys, lev)] == [tuple(o) for o in tree]
        e_oracle = _err_mod_const(x, ue)
        for prec in (GMG_FP64, GMG_FP32):
            ctx = Context(q, 0, leaves=(keys, lev), vcycle_prec=prec)
            assert ctx.num_dofs() == S.ndof and np.array_equal(ctx.dof_coords(), S.coords())
            fd = torch.from_numpy(f).cuda()
            u = torch.empty_like(fd)
            info = ctx.solve(fd, u, 1e-8)
            torch.cuda.synchronize()
            uh = to_host(u)
            res = b - S.A @ uh
            rel = np.linalg.norm(res - res.mean()) / np.linalg.norm(b)
            e = _err_mod_const(uh, ue)
            print(f"[sharp] q={q} top={top} DoFs {S.ndof} prec {prec}: iters {info.inner_iters} rel {rel:.2e} "
                  f"err {e:.3e} (oracle {e_oracle:.3e})", flush=True)
            assert rel <= 1e-8 * 1.001
            # the algebraic error left at 1e-8 is far below the discretisation error
            assert abs(e - e_oracle) <= 1e-3 * e_oracle
        errs.append(e_oracle)
    assert errs[1] < 0.25 * errs[0]


def test_learned_correction_on_the_uniform_levels_of_an_octree_hierarchy():
    """An octree level whose leaves all have one level is the uniform lattice in lattice order:
    the learned correction runs there (the lattice convolution is defined) and gives the bits of
    the uniform context's correction on the same lattice; a learned solve uses it on that level
    and reaches 1e-8 on the oracle's operator.  Coarsening merges every complete family at once,
    so a hierarchy has uniform levels above the coarsest only when its tree is uniform: here the
    level-4 tree (levels of 32^3, 16^3 and 8^3 Q2 nodes).  (The adaptive workload's hierarchy has
    no uniform level but the coarsest, so its learned solve runs no net.)"""
    torch = torch_cuda()
    import os
    from oracle import octree as ot, octree_fe as ofe, multigrid as mg
    from paper_1408_6497_amd import Context
    from paper_1408_6497_amd import train as T
    from workloads import gaussian_params, gaussian_source_points
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    w = T.load(os.path.join(root, "paper_1408_6497_amd", "weights", "q2_depth0.gmgw"))["w"]
    from oracle import octree as ot_
    tree = ot_.sort_leaves(ot_.uniform(4))
    ctx = Context(2, 0, leaves=_arrays(tree), use_learned=1, learned_min_depth=1, timing=1)
    ctx.net_set_weights(0, w)
    sizes = [ctx.num_dofs(l) for l in range(ctx.levels)]
    l1 = sizes.index(16 ** 3)          # the uniform level-3 mesh
    assert l1 < ctx.levels - 1
    uni = Context(2, 8, 0)
    uni.net_set_weights(0, w)
    assert np.array_equal(ctx.dof_coords(l1), uni.dof_coords(uni.levels - 1))
    r = torch.from_numpy(np.random.default_rng(4).standard_normal(16 ** 3)).float().cuda()
    e_oct, e_uni = torch.empty_like(r), torch.empty_like(r)
    ctx.net_correction(l1, r, e_oct)
    uni.net_correction(uni.levels - 1, r, e_uni)
    torch.cuda.synchronize()
    assert torch.equal(e_oct, e_uni)
    S = ofe.OctreeSpace(tree, 2)
    p = gaussian_params(3, 4, 0.01, 0.05)
    f = gaussian_source_points(S.coords(), p)
    b = mg.project(S.M @ f)
    fd = torch.from_numpy(f).cuda()
    u = torch.empty_like(fd)
    ctx.timing_reset()
    info = ctx.solve(fd, u, 1e-8)
    torch.cuda.synchronize()
    used = ctx.timing(l1, Context.KIND_LEARNED, 1)[0]
    others = sum(ctx.timing(l, Context.KIND_LEARNED, 1)[0] for l in range(ctx.levels) if l != l1)
    res = b - S.A @ to_host(u)
    rel = np.linalg.norm(res - res.mean()) / np.linalg.norm(b)
    print(f"[octree-learned] level sizes {sizes}: iters {info.inner_iters} fallbacks {info.fallbacks} learned "
          f"corrections on the uniform level {used}, elsewhere {others}; rel {rel:.2e}", flush=True)
    assert used > 0 and others == 0
    assert rel <= 1e-8 * 1.001
