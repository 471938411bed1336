"""Learned smoother on the GPU vs the FP64 oracle with BF16 emulation.

Tolerances (reading of the learned-smoother definition): forward outputs 1e-2
relative l2, gradients 1e-3 relative l2 -- the GPU accumulates in FP32 in a
different order, and BF16 rounding of an activation or gradient can flip where
the FP32 and FP64 sums straddle a rounding boundary.
"""
import numpy as np
import pytest

from tests.gpu_common import mean_free_normal, rel_l2, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _ctx(q, n, **kw):
    torch_cuda()
    from paper_1408_6497_amd import Context
    return Context(q, n, 0, **kw)


def _weights(seed, scale=0.25):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(7776) * scale
    return w.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("q,n", [(2, 8), (1, 16), (2, 16)])
def test_net_forward_backward_parity(q, n):
    torch = torch_cuda()
    from oracle import learned
    ctx = _ctx(q, n)
    N = q * n
    w = _weights(1)
    ctx.net_set_weights(0, w)
    x = np.random.default_rng(2).standard_normal(N ** 3)
    xd = to_dev(x, torch.float32)
    yd = torch.empty_like(xd)
    cache = ctx.net_cache(0)
    ctx.net_forward(0, xd, yd, cache)
    y_ref, cache_ref = learned.forward(w, to_host(xd).reshape(N, N, N))
    err_y = rel_l2(to_host(yd), y_ref.ravel())
    gy = np.random.default_rng(3).standard_normal(N ** 3)
    gyd = to_dev(gy, torch.float32)
    gw = torch.zeros(7776, dtype=torch.float32, device="cuda")
    gin = torch.empty_like(xd)
    ctx.net_backward(0, gyd, cache, gw, gin)
    torch.cuda.synchronize()
    g_ref, gin_ref = learned.backward(cache_ref, to_host(gyd).reshape(N, N, N), want_gin=True)
    err_w = rel_l2(to_host(gw), g_ref)
    err_in = rel_l2(to_host(gin), gin_ref.ravel())
    parts = [rel_l2(to_host(gw)[a:b], g_ref[a:b]) for a, b in ((0, 432), (432, 7344), (7344, 7776))]
    print(f"[net] q={q} n={n} fwd={err_y:.2e} gw={err_w:.2e} parts={parts} gin={err_in:.2e}", flush=True)
    assert err_y <= 1e-2
    assert err_w <= 1e-3 and max(parts) <= 1e-3
    assert err_in <= 1e-3


@pytest.mark.parametrize("n", [64, 256])
def test_net_forward_sampled_at_production_lattices(n):
    """The forward kernels at the lattices the solves and the bench run them on (128^3 voxels:
    the depth-2 level of the headline problem; 512^3: its finest level, where the bench times one
    application), in the same launch configuration, on 96 sampled voxels: a voxel's output
    depends on the 7^3 input neighbourhood around it only, so the oracle's forward pass on that
    7^3 patch (its periodic wrap never reaches the centre's dependencies) gives the exact
    reference value at the patch centre."""
    torch = torch_cuda()
    from oracle import learned
    ctx = _ctx(2, n)
    N = 2 * n
    assert ctx.lattice(ctx.levels - 1) == N
    w = _weights(11)
    ctx.net_set_weights(0, w)
    g = torch.Generator(device="cuda").manual_seed(12)
    xd = torch.randn(N ** 3, device="cuda", dtype=torch.float32, generator=g)
    yd = torch.empty_like(xd)
    cache = ctx.net_cache(0)
    print(f"[net sampled] N={N}", flush=True)
    ctx.net_forward(0, xd, yd, cache)
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    # samples on brick edges and corners as well as inside (bricks are 16 x 8 x 4 and 16 x 8 x 8)
    pts = [(0, 0, 0), (N - 1, N - 1, N - 1), (15, 7, 3), (16, 8, 4), (N - 1, 0, 7)]
    pts += [tuple(int(v) for v in rng.integers(0, N, 3)) for _ in range(91)]
    ys, refs = [], []
    ar = np.arange(-3, 4)
    for (i, j, k) in pts:
        iz, iy, ix = (k + ar) % N, (j + ar) % N, (i + ar) % N
        idx = (iz[:, None, None] * N + iy[None, :, None]) * N + ix[None, None, :]
        patch = to_host(xd[torch.from_numpy(idx.ravel()).cuda()]).reshape(7, 7, 7)
        y_ref, _ = learned.forward(w, patch)
        refs.append(y_ref[3, 3, 3])
        ys.append(float(yd[(k * N + j) * N + i]))
    err = rel_l2(np.array(ys), np.array(refs))
    print(f"[net sampled] N={N}: rel l2 over {len(pts)} voxels {err:.2e}", flush=True)
    assert err <= 1e-2
    del cache, xd, yd
    ctx.close()


def test_net_correction_parity_and_jacobi_special_case():
    torch = torch_cuda()
    from oracle import learned, operator as op
    q, n = 2, 8
    ctx = _ctx(q, n)
    N = q * n
    A = op.assemble(q, n)
    dinv = (1.0 / A.diagonal()).reshape(N, N, N)
    r = mean_free_normal(N ** 3, 4)
    rd = to_dev(r, torch.float32)
    e = torch.empty_like(rd)
    # identity weights: the learned correction is damped Jacobi (up to BF16 input rounding)
    omega = 0.625  # a BF16 value
    ctx.net_set_weights(0, learned.jacobi_weights(omega))
    ctx.net_correction(-1, rd, e)
    torch.cuda.synchronize()
    jac = omega * dinv.ravel() * to_host(rd)
    assert np.max(np.abs(to_host(e) - jac)) <= 2 ** -8 * np.max(np.abs(jac))
    ref, _ = learned.correction(learned.jacobi_weights(omega), to_host(rd).reshape(N, N, N), dinv)
    assert rel_l2(to_host(e), ref.ravel()) <= 1e-5
    # random weights
    w = _weights(5)
    ctx.net_set_weights(0, w)
    ctx.net_correction(-1, rd, e)
    torch.cuda.synchronize()
    ref, _ = learned.correction(w, to_host(rd).reshape(N, N, N), dinv)
    assert rel_l2(to_host(e), ref.ravel()) <= 1e-2


def test_adam_step_matches_definition():
    torch = torch_cuda()
    ctx = _ctx(2, 8)
    w0 = _weights(7).astype(np.float32)
    ctx.net_set_weights(0, w0)
    rng = np.random.default_rng(8)
    m = np.zeros(7776, np.float32)
    v = np.zeros(7776, np.float32)
    w = w0.copy()
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    for step in (1, 2, 3):
        g = rng.standard_normal(7776).astype(np.float32)
        ctx.adam_step(0, torch.from_numpy(g).cuda(), lr, step)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        w = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    got = ctx.net_get_weights(0)
    assert np.max(np.abs(got - w)) <= 1e-6 * np.max(np.abs(w))


def test_learned_solve_converges_and_fallback_fires():
    """A learned solve reaches the tolerance; adversarial weights trigger the fallback every cycle."""
    torch = torch_cuda()
    from oracle import learned, multigrid as mg, operator as op
    from workloads import gaussian_params, gaussian_source
    q, n = 2, 16
    f = None
    for name, w in (("jacobi", learned.jacobi_weights(0.625)), ("adversarial", -50.0 * learned.jacobi_weights(1.0))):
        ctx = _ctx(q, n, seed=4, use_learned=1)
        ctx.net_set_weights(0, w)
        if f is None:
            f = gaussian_source(ctx.dof_coords_1d(), gaussian_params(2, 32, 0.02, 0.1)).cuda()
        u = torch.empty_like(f)
        info = ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        b = mg.rhs(q, n, to_host(f))
        A = op.assemble(q, n)
        res = b - A @ to_host(u)
        res -= res.mean()
        rel = np.linalg.norm(res) / np.linalg.norm(b)
        print(f"[learned-solve] {name}: iters={info.inner_iters} fallbacks={info.fallbacks} rel={rel:.2e}", flush=True)
        assert rel <= 1e-8 * 1.001
        if name == "adversarial":
            assert info.fallbacks >= info.inner_iters - 1 and info.fallbacks >= 1
        # the recorded tests follow the fallback rule: kept iff rho_L <= reference,
        # and a rejection makes the plain cycle's contraction the next reference
        hist = ctx.history(1)
        rejected = np.isfinite(hist[:, 2])
        assert len(hist) >= info.inner_iters - 1 and rejected.sum() == info.fallbacks
        assert np.all((hist[:, 0] <= hist[:, 1]) == ~rejected)
        for k in range(len(hist) - 1):
            assert hist[k + 1, 1] == (hist[k, 2] if rejected[k] else hist[k, 1])
        res = ctx.history(0)
        assert len(res) >= info.inner_iters + 1 and res[-1] <= 1e-8 * res[0]


def test_learned_min_depth_keeps_the_finest_levels_plain():
    """learned_min_depth = 2: the two finest levels keep the Chebyshev smoother (no net
    launches there), the coarser levels with at least 16 nodes a side use the net, and the
    solve still reaches the tolerance on the oracle's operator."""
    torch = torch_cuda()
    from oracle import learned, multigrid as mg, operator as op
    from paper_1408_6497_amd import Context, GMG_FP32
    from workloads import gaussian_params, gaussian_source
    q, n = 2, 32   # levels of 64, 32, 16 and 8 nodes a side
    ctx = _ctx(q, n, seed=4, use_learned=1, learned_min_depth=2, timing=1)
    ctx.net_set_weights(0, learned.jacobi_weights(0.625))
    f = gaussian_source(ctx.dof_coords_1d(), gaussian_params(2, 32, 0.02, 0.1)).cuda()
    u = torch.empty_like(f)
    info = ctx.solve(f, u, 1e-8)
    torch.cuda.synchronize()
    L = ctx.levels
    used = [ctx.timing(l, Context.KIND_LEARNED, GMG_FP32)[0] for l in range(L)]
    print(f"[learned-min-depth] levels {L}: learned launches per level {used}, iters {info.inner_iters}", flush=True)
    assert used[L - 1] == 0 and used[L - 2] == 0      # depths 0 and 1
    assert used[L - 3] > 0                            # depth 2: 16 nodes a side
    b = mg.rhs(q, n, to_host(f))
    res = b - op.assemble(q, n) @ to_host(u)
    res -= res.mean()
    assert np.linalg.norm(res) / np.linalg.norm(b) <= 1e-8 * 1.001


@pytest.mark.parametrize("kind", ["energy", "residual"])
def test_loss_gradient_parity(kind):
    """gmg_net_loss_grad (forward, A e~, loss, backward through A and the net) vs the oracle."""
    torch = torch_cuda()
    from oracle import learned, operator as op
    from paper_1408_6497_amd import LOSS_ENERGY, LOSS_RESIDUAL
    q, n = 2, 8
    ctx = _ctx(q, n)
    N = q * n
    A = op.assemble(q, n)
    dinv = (1.0 / A.diagonal()).reshape(N, N, N)
    w = _weights(9, scale=0.2)
    ctx.net_set_weights(0, w)
    r = mean_free_normal(N ** 3, 10)
    rd = to_dev(r, torch.float32)
    r = to_host(rd)
    e = np.linalg.lstsq(A.toarray(), r, rcond=None)[0]
    e -= e.mean()
    ed = to_dev(e, torch.float32)
    e = to_host(ed)
    cache = ctx.net_cache(0)
    gw = torch.zeros(7776, dtype=torch.float32, device="cuda")
    k = LOSS_ENERGY if kind == "energy" else LOSS_RESIDUAL
    loss = ctx.net_loss_grad(0, rd, ed if kind == "energy" else None, cache, gw, scale=0.5, kind=k)
    torch.cuda.synchronize()
    loss_ref, g_ref = learned.loss_and_gradient(w, A, dinv, r.reshape(N, N, N), e.reshape(N, N, N), kind)
    err = rel_l2(to_host(gw), 0.5 * g_ref)
    print(f"[loss-grad] {kind}: loss gpu={loss:.6f} oracle={loss_ref:.6f} grad rel={err:.2e}", flush=True)
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref)
    assert err <= 1e-3


def test_trained_net_gain_on_held_out_sources():
    """What the shipped trained net (paper_1408_6497_amd/weights/q2_depth0.gmgw, made by
    `python -m paper_1408_6497_amd.train --n 64 --sources 2500 --cycles 4 --loss residual`)
    gains over the Chebyshev application it replaces, on sources it never saw.

    Per application: the residual contraction ||r - A e~||^2 / ||r||^2 at the replaced
    positions of plain cycles (lower is better).  Per solve: iterations and fallbacks of
    the learned FP32 solve against the plain FP32 solve, both to 1e-8."""
    torch = torch_cuda()
    import os
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64, LOSS_RESIDUAL
    from paper_1408_6497_amd import train as T
    from workloads import grf
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    w = T.load(os.path.join(here, "paper_1408_6497_amd", "weights", "q2_depth0.gmgw"))
    assert (w["order"], w["depth"]) == (2, 0)
    ctx = Context(2, 32, 0, seed=0, vcycle_prec=GMG_FP64)
    cctx = Context(2, 16, 0, seed=0, vcycle_prec=GMG_FP64)
    pm = T.PairMaker(ctx, cctx)
    ctx.net_set_weights(0, w["w"])
    cache = ctx.net_cache(0)
    tmp = (torch.empty_like(pm.r32), torch.empty_like(pm.r32))
    net, cheb = [], []
    for seed in range(30000, 30004):
        pm.source(seed)
        for cyc in range(4):
            if cyc:
                pm.next_cycle()
            for pos in ("pre", "post"):
                r, _ = pm.pair(pos, need_e=False)
                net.append(ctx.net_loss_grad(0, r, None, cache, kind=LOSS_RESIDUAL))
                cheb.append(T.chebyshev_loss(ctx, r, None, tmp, LOSS_RESIDUAL))
    net, cheb = float(np.mean(net)), float(np.mean(cheb))
    out = {}
    for name, kw in (("plain", dict(vcycle_prec=GMG_FP32)), ("learned", dict(use_learned=1))):
        c = Context(2, 32, 0, seed=0, **kw)
        if name == "learned":
            c.net_set_weights(0, w["w"])
        f, _ = grf(c.lattice(), 30000, device="cuda")
        u = torch.empty_like(f)
        info = c.solve(f, u, 1e-8)
        out[name] = (info.inner_iters, info.fallbacks, info.rel_residual_f64)
    print(f"[gain] held-out contraction: net {net:.4f} vs Chebyshev {cheb:.4f}; solves {out}", flush=True)
    assert net < cheb
    assert out["learned"][2] <= 1e-8 and out["learned"][0] <= out["plain"][0]


def test_learned_test_norms_fused_into_the_residual():
    """The per-cycle test of a learned cycle takes ||r32 - A z32||^2 and ||r32||^2 in the FP32
    residual's epilogue on uniform levels of more than 32 nodes (the residual itself is not
    stored); with no_fused_test_norms it stores the residual and reduces both norms in a pass of
    its own.  At 32^3 Q2 elements the top level (64 nodes a side) takes the fused form.  The two
    forms compute the residual by the same FP32 expression and differ in the order of the FP64
    sums (and at most in one FP32 rounding per entry where the compiler contracts differently),
    so the contractions agree to 1e-7 relative, the keep-or-fall-back decisions are the same,
    and so is every cycle's output and the solution."""
    torch = torch_cuda()
    import os
    from paper_1408_6497_amd import Context
    from paper_1408_6497_amd import train as T
    from workloads import grf
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    w = T.load(os.path.join(here, "paper_1408_6497_amd", "weights", "q2_depth0.gmgw"))["w"]
    out = {}
    for fused in (True, False):
        c = Context(2, 32, 0, seed=0, use_learned=1, no_fused_test_norms=0 if fused else 1)
        c.net_set_weights(0, w)
        f, _ = grf(c.lattice(), 30001, device="cuda")
        u = torch.empty_like(f)
        info = c.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        out[fused] = (info.inner_iters, info.fallbacks, c.history(1), to_host(u))
        c.close()
    (i1, f1, h1, u1), (i0, f0, h0, u0) = out[True], out[False]
    print(f"[test norms] iterations {i1} / {i0}, fallbacks {f1} / {f0}, rho {h1[:, 0]}", flush=True)
    assert (i1, f1) == (i0, f0) and h1.shape == h0.shape
    fin = np.isfinite(h0)
    assert np.array_equal(fin, np.isfinite(h1))
    assert np.allclose(h1[fin], h0[fin], rtol=1e-7, atol=0.0)
    assert rel_l2(u1, u0) <= 1e-12


@pytest.mark.parametrize("depth", [2, 3, 4, 5])
def test_per_depth_nets_beat_chebyshev_on_their_levels(depth):
    """The shipped net of each depth of the headline hierarchy (Q2 on 256^3 elements; depth d is
    the finest level of the 256 / 2^d-element mesh, trained there on 10 000 GRF sources by
    `python -m paper_1408_6497_amd.train --n 256 --depth d --sources 10000`) against the Chebyshev
    application it replaces, on held-out sources, at both replaced positions of two plain cycles:
    mean residual contraction ||r - A e~||^2 / ||r||^2 (lower is better)."""
    torch = torch_cuda()
    import os
    from paper_1408_6497_amd import Context, GMG_FP64, LOSS_RESIDUAL
    from paper_1408_6497_amd import train as T
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    w = T.load(os.path.join(here, "paper_1408_6497_amd", "weights", f"q2_depth{depth}.gmgw"))
    nd = 256 >> depth
    assert (w["order"], w["depth"], w["n"]) == (2, depth, nd)
    ctx = Context(2, nd, 0, seed=0, vcycle_prec=GMG_FP64)
    cctx = Context(2, nd // 2, 0, seed=0, vcycle_prec=GMG_FP64)
    pm = T.PairMaker(ctx, cctx)
    ctx.net_set_weights(0, w["w"])
    cache = ctx.net_cache(0)
    tmp = (torch.empty_like(pm.r32), torch.empty_like(pm.r32))
    net, cheb = [], []
    for seed in range(30000, 30003):
        pm.source(seed)
        for cyc in range(2):
            if cyc:
                pm.next_cycle()
            for pos in ("pre", "post"):
                r, _ = pm.pair(pos, need_e=False)
                net.append(ctx.net_loss_grad(0, r, None, cache, kind=LOSS_RESIDUAL))
                cheb.append(T.chebyshev_loss(ctx, r, None, tmp, LOSS_RESIDUAL))
    net, cheb = float(np.mean(net)), float(np.mean(cheb))
    print(f"[depth {depth}] lattice {2 * nd}: held-out contraction net {net:.4f} vs Chebyshev {cheb:.4f}",
          flush=True)
    assert net < cheb
    ctx.close()
    cctx.close()


def test_training_stops_and_resumes_on_the_same_bits(tmp_path):
    """A run stopped twice (mid-source) and resumed from its version-2 checkpoints ends on the
    same weights, bit for bit, as the uninterrupted run: optimizer moments, step count and the
    position in the pair stream all travel in the file, and every training kernel is
    deterministic (fixed-order reductions)."""
    torch_cuda()
    from paper_1408_6497_amd import train as T
    kw = dict(n=16, sources=3, batch=3, val=2, cycles=2, positions=("pre", "post"), loss="residual",
              log=lambda *a: None)
    straight = T.train(**kw)
    assert straight["step"] == 4
    ck1, ck2 = str(tmp_path / "a.gmgw"), str(tmp_path / "b.gmgw")
    T.train(**kw, stop_after=1, out=ck1)
    c1 = T.load(ck1)
    assert c1["version"] == 2 and c1["step"] == 1 and c1["extra"]["stream"] == {"src": 0, "cyc": 1, "pos": 1}
    T.train(resume=ck1, stop_after=1, out=ck2, log=lambda *a: None)
    assert T.load(ck2)["extra"]["stream"] == {"src": 1, "cyc": 1, "pos": 0}
    resumed = T.train(resume=ck2, log=lambda *a: None)
    assert resumed["step"] == 4
    assert np.array_equal(resumed["w"], straight["w"])
