"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances: FP64 apply 1e-12 relative (l2), FP32 apply 2e-5; composite steps
(smoother, V-cycle) accumulate a few applies, so they use 1e-11 (FP64) and
1e-4 (FP32); solves are judged by the oracle's own CSR residual of the GPU
solution (<= tolerance) and the distance to the oracle's solution is reported.
"""
import math

import numpy as np
import pytest

from tests.gpu_common import (FP32_TOL, FP64_TOL, mean_free_normal, oracle_hierarchy, rel_l2, to_dev, to_host,
                              torch_cuda)

pytestmark = pytest.mark.gpu

CASES = [(1, 4), (1, 8), (1, 32), (2, 2), (2, 4), (2, 8), (2, 16), (4, 2), (4, 4), (4, 8)]


def _ctx(q, n, levels=0, **kw):
    torch_cuda()
    from paper_1408_6497_amd import Context
    return Context(q, n, levels, **kw)


def _levels_for(ctx):
    return ctx.levels


@pytest.mark.parametrize("q,n", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_apply_parity(q, n, prec):
    torch = torch_cuda()
    from oracle import operator as op
    print(f"[apply] q={q} n={n} prec={prec}", flush=True)
    ctx = _ctx(q, n, 0)
    A = op.assemble(q, n)
    x = mean_free_normal(A.shape[0], seed=100 + q * 10 + n)
    dt = torch.float64 if prec == "fp64" else torch.float32
    xd = to_dev(x, dt)
    yd = torch.empty_like(xd)
    ctx.apply(ctx.levels - 1, xd, yd)
    torch.cuda.synchronize()
    y_gpu = to_host(yd)
    y_orc = A @ to_host(xd)   # the oracle sees the same (rounded) input
    err = rel_l2(y_gpu, y_orc)
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    print(f"  rel_l2={err:.3e}", flush=True)
    assert err <= tol
    assert np.max(np.abs(y_gpu - y_orc)) <= 10 * tol * np.max(np.abs(y_orc))


@pytest.mark.parametrize("q,n", [(1, 8), (2, 8), (4, 4)])
def test_mass_diagonal_coords(q, n):
    torch = torch_cuda()
    from oracle import operator as op
    ctx = _ctx(q, n, 0)
    top = ctx.levels - 1
    assert np.max(np.abs(ctx.dof_coords_1d(top) - op.dof_coords_1d(q, n))) < 1e-15
    M = op.assemble(q, n, "mass")
    x = mean_free_normal(M.shape[0], seed=7)
    xd = to_dev(x, torch.float64)
    yd = torch.empty_like(xd)
    ctx.mass(top, xd, yd)
    d = torch.empty_like(xd)
    ctx.diagonal(top, d)
    torch.cuda.synchronize()
    assert rel_l2(to_host(yd), M @ x) <= FP64_TOL
    assert rel_l2(to_host(d), op.assemble(q, n).diagonal()) <= 1e-14


@pytest.mark.parametrize("q,n", [(1, 16), (2, 8), (4, 4)])
def test_lanczos_lambda_parity(q, n):
    torch_cuda()
    ctx = _ctx(q, n, 0, seed=11)
    H = oracle_hierarchy(q, n, ctx.levels, seed=11)
    for l in range(ctx.levels):
        assert abs(ctx.lam(l) - H.levels[l].lam) <= 1e-10 * H.levels[l].lam, (l, ctx.lam(l), H.levels[l].lam)


@pytest.mark.parametrize("q,n", [(1, 16), (2, 8), (4, 4)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_smoother_parity(q, n, prec):
    torch = torch_cuda()
    ctx = _ctx(q, n, 0, seed=3)
    H = oracle_hierarchy(q, n, ctx.levels, seed=3)
    lev = H.finest
    dt = torch.float64 if prec == "fp64" else torch.float32
    b = to_dev(mean_free_normal(lev.size, 21), dt)
    u = to_dev(np.random.default_rng(22).standard_normal(lev.size), dt)
    u0 = to_host(u)
    ctx.smooth(ctx.levels - 1, b, u, 2)
    torch.cuda.synchronize()
    ref = H.smooth(lev, to_host(b), u0, 2)
    err = rel_l2(to_host(u), ref)
    print(f"[smooth] q={q} n={n} {prec} rel={err:.2e}", flush=True)
    assert err <= (1e-11 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("q,n", [(1, 8), (2, 4), (2, 8), (4, 4), (1, 64), (2, 32), (4, 8), (1, 128)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_transfer_parity(q, n, prec):
    torch = torch_cuda()
    from oracle import transfer
    ctx = _ctx(q, n, 2) if q * n // 2 <= 8 else _ctx(q, n, 0)  # the finest transfer of the hierarchy
    lv = ctx.levels - 1
    P = transfer.prolongation(q, n // 2)
    dt = torch.float64 if prec == "fp64" else torch.float32
    tol = 1e-14 if prec == "fp64" else 1e-6
    rf = to_dev(np.random.default_rng(5).standard_normal(P.shape[0]), dt)
    rc = torch.empty(P.shape[1], dtype=dt, device="cuda")
    ctx.restrict(lv, rf, rc)
    ec = to_dev(np.random.default_rng(6).standard_normal(P.shape[1]), dt)
    uf = to_dev(np.random.default_rng(7).standard_normal(P.shape[0]), dt)
    uf0 = to_host(uf)
    ctx.prolong(lv, ec, uf)
    torch.cuda.synchronize()
    assert rel_l2(to_host(rc), P.T @ to_host(rf)) <= tol
    assert rel_l2(to_host(uf), uf0 + P @ to_host(ec)) <= tol


@pytest.mark.parametrize("q,n", [(1, 8), (2, 4), (4, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coarse_solve_parity(q, n, prec):
    torch = torch_cuda()
    ctx = _ctx(q, n, 1)
    H = oracle_hierarchy(q, n, 1)
    dt = torch.float64 if prec == "fp64" else torch.float32
    b = to_dev(np.random.default_rng(8).standard_normal(H.levels[0].size), dt)   # not mean-free on purpose
    x = torch.empty_like(b)
    ctx.coarse_solve(b, x)
    torch.cuda.synchronize()
    ref = H.coarse_solve(to_host(b))
    assert rel_l2(to_host(x), ref) <= (1e-12 if prec == "fp64" else 1e-6)


# (1, 64), (2, 32), (4, 16): the finest level (64 nodes a side) runs the streaming column
# kernel, including the fused first two smoother steps from the zero guess
@pytest.mark.parametrize("q,n,levels", [(1, 16, 3), (1, 32, 4), (2, 8, 0), (2, 16, 0), (4, 4, 0), (4, 8, 0),
                                        (1, 64, 0), (2, 32, 0), (4, 16, 0)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_vcycle_parity(q, n, levels, prec):
    torch = torch_cuda()
    ctx = _ctx(q, n, levels, seed=5)
    H = oracle_hierarchy(q, n, ctx.levels, seed=5, form="kron" if q * n >= 64 else "csr")
    dt = torch.float64 if prec == "fp64" else torch.float32
    r = to_dev(mean_free_normal(H.finest.size, 31), dt)
    z = torch.empty_like(r)
    ctx.vcycle(r, z)
    torch.cuda.synchronize()
    ref = H.vcycle(to_host(r))
    err = rel_l2(to_host(z), ref)
    print(f"[vcycle] q={q} n={n} L={ctx.levels} {prec} rel={err:.2e}", flush=True)
    assert err <= (1e-11 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("q,n", [(1, 16), (2, 8), (2, 16), (4, 4)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fused_tail_level_parity(q, n, prec):
    """The 16^3-node level next to the coarsest runs its cycle in two one-workgroup
    launches (LDS-resident smoothing, residual and transfers); with the fusion on and
    off the V-cycle matches the oracle, and the two agree to rounding."""
    torch = torch_cuda()
    dt = torch.float64 if prec == "fp64" else torch.float32
    fused = _ctx(q, n, 0, seed=5)
    plain = _ctx(q, n, 0, seed=5, no_fused_tail=1, timing=1)
    H = oracle_hierarchy(q, n, fused.levels, seed=5)
    r = to_dev(mean_free_normal(H.finest.size, 41), dt)
    zf, zp = torch.empty_like(r), torch.empty_like(r)
    fused.vcycle(r, zf)
    plain.vcycle(r, zp)
    torch.cuda.synchronize()
    ref = H.vcycle(to_host(r))
    tol = 1e-11 if prec == "fp64" else 1e-4
    ef, ep, efp = rel_l2(to_host(zf), ref), rel_l2(to_host(zp), ref), rel_l2(to_host(zf), to_host(zp))
    print(f"[tail] q={q} n={n} {prec}: fused {ef:.2e} separate {ep:.2e} between {efp:.2e}", flush=True)
    assert ef <= tol and ep <= tol and efp <= tol
    # the separate path really ran separate kernels on that level
    from paper_1408_6497_amd import Context
    assert plain.timing(1, Context.KIND_TAIL, 0 if prec == "fp64" else 1)[0] == 0
    fused_t = _ctx(q, n, 0, seed=5, timing=1)
    fused_t.vcycle(r, zf)
    fused_used = fused_t.timing(1, Context.KIND_TAIL, 0 if prec == "fp64" else 1)[0] > 0
    assert fused_used == (fused.levels >= 2 and q * n // (1 << (fused.levels - 2)) == 16
                          and not (q == 4 and prec == "fp64"))


@pytest.mark.parametrize("q,n", [(1, 16), (1, 64), (2, 8), (2, 32)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_paper_jacobi_v21_vcycle_parity(q, n, prec):
    """The paper's own cycle (Section 3 runs): damped Jacobi, omega = 2/3, two pre- and one
    post-smoothing sweep, on the column-kernel levels, the fused 16^3 level and the point kernel."""
    torch = torch_cuda()
    from oracle import multigrid as mg
    dt = torch.float64 if prec == "fp64" else torch.float32
    ctx = _ctx(q, n, 0, seed=5, smoother=1, jacobi_omega=2.0 / 3.0, nu_pre=2, nu_post=1)
    opts = mg.Options(seed=5, smoother="jacobi", jacobi_omega=2.0 / 3.0, nu_pre=2, nu_post=1)
    H = mg.Hierarchy(q, n, ctx.levels, opts, form="kron" if q * n >= 64 else "csr")
    r = to_dev(mean_free_normal(H.finest.size, 51), dt)
    z = torch.empty_like(r)
    ctx.vcycle(r, z)
    torch.cuda.synchronize()
    err = rel_l2(to_host(z), H.vcycle(to_host(r)))
    print(f"[jacobi-v21] q={q} n={n} {prec} rel={err:.2e}", flush=True)
    assert err <= (1e-11 if prec == "fp64" else 1e-4)


def test_paper_jacobi_v21_solve():
    """PCG with the Jacobi V(2,1) cycle reaches 1e-10 on the oracle's operator (C1 sizes)."""
    torch = torch_cuda()
    from oracle import multigrid as mg, operator as op
    from workloads import gaussian_params, gaussian_source
    q, n = 1, 32
    ctx = _ctx(q, n, 4, seed=1, smoother=1, jacobi_omega=2.0 / 3.0, nu_pre=2, nu_post=1)
    f = gaussian_source(ctx.dof_coords_1d(), gaussian_params(0, 32, 0.02, 0.1)).cuda()
    u = torch.empty_like(f)
    info = ctx.solve(f, u, 1e-10)
    torch.cuda.synchronize()
    b = mg.rhs(q, n, to_host(f))
    res = b - op.assemble(q, n) @ to_host(u)
    res -= res.mean()
    rel = np.linalg.norm(res) / np.linalg.norm(b)
    print(f"[jacobi-v21-solve] iters={info.inner_iters} rel={rel:.2e}", flush=True)
    assert rel <= 1e-10 * 1.001


def _oracle_residual(q, n, u, b):
    from oracle import operator as op
    A = op.assemble(q, n)
    r = b - A @ u
    r -= r.mean()
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_solve_c1_closed_form():
    """Q1, 32^3, 4 levels, f = 12 pi^2 sin sin sin, plain FP64 to 1e-10."""
    torch = torch_cuda()
    from workloads import sin_source, sin_exact
    from oracle import multigrid as mg, krylov
    q, n = 1, 32
    ctx = _ctx(q, n, 4)
    x1 = ctx.dof_coords_1d()
    f = sin_source(x1).cuda()
    u = torch.empty_like(f)
    info = ctx.solve(f, u, 1e-10)
    torch.cuda.synchronize()
    ug = to_host(u)
    b = mg.rhs(q, n, to_host(f))
    res = _oracle_residual(q, n, ug, b)
    th, h = 2 * math.pi / n, 1.0 / n
    amp = 4 * math.pi ** 2 * (h * (4 + 2 * math.cos(th)) / 6) / ((2 - 2 * math.cos(th)) / h)
    closed = amp * sin_exact(x1)
    print(f"[c1] iters={info.inner_iters} gpu_rel={info.rel_residual_f64:.2e} oracle_res={res:.2e} "
          f"err_vs_closed={np.max(np.abs(ug - closed)):.2e}", flush=True)
    assert info.rel_residual_f64 <= 1e-10
    assert res <= 1e-10 * (1 + 1e-3)
    assert np.max(np.abs(ug - closed)) < 1e-9


@pytest.mark.parametrize("q,n,prec", [(2, 16, "fp64"), (2, 16, "fp32"), (4, 8, "fp32"), (1, 32, "fp32")])
def test_solve_gaussian_source(q, n, prec):
    """Gaussian-sum source, FP64 PCG or FP32 V-cycle + FP64 refinement, to 1e-8."""
    torch = torch_cuda()
    from workloads import gaussian_params, gaussian_source
    from oracle import multigrid as mg, krylov
    from paper_1408_6497_amd import GMG_FP32, GMG_FP64
    vp = GMG_FP32 if prec == "fp32" else GMG_FP64
    ctx = _ctx(q, n, 0, seed=1, vcycle_prec=vp)
    params = gaussian_params(0, 32, 0.02, 0.1)
    f = gaussian_source(ctx.dof_coords_1d(), params).cuda()
    u = torch.empty_like(f)
    info = ctx.solve(f, u, 1e-8)
    torch.cuda.synchronize()
    ug = to_host(u)
    b = mg.rhs(q, n, to_host(f))
    res = _oracle_residual(q, n, ug, b)
    H = oracle_hierarchy(q, n, ctx.levels, seed=1)
    uo, oinfo = krylov.pcg(H.finest.A, b, H.vcycle, 1e-12)
    uo = krylov.normalize_mean(uo, q, n)
    diff = rel_l2(ug, uo)
    print(f"[solve] q={q} n={n} {prec} outer={info.outer_iters} inner={info.inner_iters} "
          f"gpu_rel={info.rel_residual_f64:.2e} oracle_res={res:.2e} |u-u_orc|/|u_orc|={diff:.2e}", flush=True)
    assert info.rel_residual_f64 <= 1e-8
    assert res <= 1e-8 * (1 + 1e-3)
    assert diff <= 1e-5


def test_error_paths_on_device():
    torch = torch_cuda()
    from paper_1408_6497_amd import GmgError
    ctx = _ctx(2, 8, 0, max_iters=1)
    f = torch.from_numpy(mean_free_normal(16 ** 3, 3)).cuda()
    u = torch.empty_like(f)
    with pytest.raises(GmgError) as e:
        ctx.solve(f, u, 1e-12)
    assert e.value.status == 5          # GMG_E_NOCONV
    f[5] = float("nan")
    ctx2 = _ctx(2, 8, 0)
    with pytest.raises(GmgError) as e:
        ctx2.solve(f, u, 1e-8)
    assert e.value.status == 6          # GMG_E_BREAKDOWN
    with pytest.raises(ValueError):
        ctx2.apply(-1, f, f[:10])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_matches_eager(prec):
    """The V-cycle replayed from a captured HIP graph gives the bits of the eager launches."""
    torch = torch_cuda()
    from workloads import gaussian_params, gaussian_source
    from paper_1408_6497_amd import GMG_FP32, GMG_FP64
    vp = GMG_FP32 if prec == "fp32" else GMG_FP64
    q, n = 2, 16
    eager = _ctx(q, n, 0, seed=2, vcycle_prec=vp, no_graphs=1)
    graph = _ctx(q, n, 0, seed=2, vcycle_prec=vp)
    f = gaussian_source(eager.dof_coords_1d(), gaussian_params(3, 32, 0.02, 0.1)).cuda()
    ue, ug = torch.empty_like(f), torch.empty_like(f)
    for rep in range(3):
        ie = eager.solve(f, ue, 1e-8)
        scratch = torch.randn_like(f) * 3.0          # eager work between replays
        ig = graph.solve(f, ug, 1e-8)
        torch.cuda.synchronize()
        assert ie.inner_iters == ig.inner_iters and ie.outer_iters == ig.outer_iters
        assert torch.equal(ue, ug), f"replay {rep} differs"
        del scratch


def test_phase_timing_fills_info():
    """With launch timing on, the solve reports its smoother, transfer and coarsest-solve
    seconds, each positive and together below the solve's own time."""
    torch = torch_cuda()
    from workloads import gaussian_params, gaussian_source
    from paper_1408_6497_amd import Context
    ctx = _ctx(2, 16, 0, seed=1, timing=1)
    f = gaussian_source(ctx.dof_coords_1d(), gaussian_params(0, 32, 0.02, 0.1)).cuda()
    u = torch.empty_like(f)
    info = ctx.solve(f, u, 1e-8)
    parts = (info.t_smooth, info.t_transfer, info.t_coarse)
    print(f"[phases] solve {info.t_solve * 1e3:.3f} ms: smooth {parts[0] * 1e3:.3f} transfer {parts[1] * 1e3:.3f} "
          f"coarse {parts[2] * 1e3:.3f} ms", flush=True)
    assert all(p > 0 for p in parts) and info.t_learned == 0.0
    assert sum(parts) < info.t_solve
    c, s = ctx.timing(0, Context.KIND_COARSE, 0)
    assert c == info.inner_iters + 1 or c >= info.inner_iters
    plain = _ctx(2, 16, 0, seed=1)
    assert plain.solve(f, u, 1e-8).t_smooth == 0.0


def test_speculative_cycles_give_the_same_bits():
    """FP32 cycles in FP64 flexible CG enqueue the next cycle while the residual norm is read
    back; the kernels and their order on the stream are those of the waiting solve, so the
    solution and the iteration count are the same bits either way, over repeated solves."""
    torch = torch_cuda()
    from workloads import gaussian_params, gaussian_source
    from paper_1408_6497_amd import GMG_FP32
    for q, n in ((2, 32), (1, 64)):
        spec = _ctx(q, n, 0, seed=3, vcycle_prec=GMG_FP32)
        wait = _ctx(q, n, 0, seed=3, vcycle_prec=GMG_FP32, no_speculation=1)
        f = gaussian_source(spec.dof_coords_1d(), gaussian_params(4, 32, 0.02, 0.1)).cuda()
        us, uw = torch.empty_like(f), torch.empty_like(f)
        for rep in range(2):
            i_s = spec.solve(f, us, 1e-9)
            i_w = wait.solve(f, uw, 1e-9)
            torch.cuda.synchronize()
            print(f"[spec] q={q} n={n} rep {rep}: iters {i_s.inner_iters} / {i_w.inner_iters} "
                  f"rel {i_s.rel_residual_f64:.2e}", flush=True)
            assert i_s.inner_iters == i_w.inner_iters and i_s.rel_residual_f64 == i_w.rel_residual_f64
            assert torch.equal(us, uw)


@pytest.mark.parametrize("q,n,precs", [(1, 128, ("fp64", "fp32")), (2, 64, ("fp64", "fp32")), (2, 128, ("fp64", "fp32")),
                                       (1, 512, ("fp32",)), (2, 256, ("fp32",))])
def test_fused_restriction_is_the_axis_passes(q, n, precs):
    """The one-pass restriction gives the bits of the three one-axis passes on every level
    of the hierarchy (it runs for q <= 2 onto coarse grids of 64 to 256 nodes a side:
    several tiles and z chunks), in both precisions."""
    torch = torch_cuda()
    fused = _ctx(q, n, 0)
    axis = _ctx(q, n, 0, no_fused_transfer=1)
    for prec in precs:
        dt = torch.float64 if prec == "fp64" else torch.float32
        for lv in range(1, fused.levels):
            size_f = fused.num_dofs(lv)
            size_c = fused.num_dofs(lv - 1)
            g = torch.Generator(device="cuda").manual_seed(100 + lv)
            rf = torch.randn(size_f, dtype=dt, device="cuda", generator=g)
            rc1 = torch.full((size_c,), float("nan"), dtype=dt, device="cuda")
            rc2 = torch.full((size_c,), float("nan"), dtype=dt, device="cuda")
            fused.restrict(lv, rf, rc1)
            axis.restrict(lv, rf, rc2)
            torch.cuda.synchronize()
            print(f"[restrict3] q={q} n={n} {prec} level {lv}: {size_f} -> {size_c}", flush=True)
            assert torch.equal(rc1, rc2), f"level {lv} differs"
            del rf, rc1, rc2
    fused.close()
    axis.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("q,n,precs", [(1, 16, ("fp64", "fp32")), (2, 8, ("fp64", "fp32")), (2, 128, ("fp64", "fp32")),
                                       (1, 512, ("fp32",)), (2, 256, ("fp32",))])
def test_fused_prolongation_is_the_axis_passes(q, n, precs):
    """The one-pass prolongation adds the bits of the three one-axis passes into the fine
    vector on every level of the hierarchy (it runs for q <= 2 from coarse grids of 2q up
    to 256 nodes a side), in both precisions."""
    torch = torch_cuda()
    fused = _ctx(q, n, 0)
    axis = _ctx(q, n, 0, no_fused_transfer=1)
    for prec in precs:
        dt = torch.float64 if prec == "fp64" else torch.float32
        for lv in range(1, fused.levels):
            g = torch.Generator(device="cuda").manual_seed(200 + lv)
            ec = torch.randn(fused.num_dofs(lv - 1), dtype=dt, device="cuda", generator=g)
            uf1 = torch.randn(fused.num_dofs(lv), dtype=dt, device="cuda", generator=g)
            uf2 = uf1.clone()
            fused.prolong(lv, ec, uf1)
            axis.prolong(lv, ec, uf2)
            torch.cuda.synchronize()
            print(f"[prolong3] q={q} n={n} {prec} level {lv}: {ec.numel()} -> {uf1.numel()}", flush=True)
            assert torch.equal(uf1, uf2), f"level {lv} differs"
            del ec, uf1, uf2
    fused.close()
    axis.close()
    torch.cuda.empty_cache()
