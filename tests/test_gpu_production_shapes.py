"""The operator kernels at the launch shapes the solves run, element by element against the oracle.

The hierarchies are the ones the solves use:
  * Q2 on 128^3 elements (levels of 256^3 and 128^3 nodes): the column kernel with one
    x-row group per tile (G = 1) streaming several element layers per block on the
    finest level, and on the 128^3-node level the instance the device's occupancy picks
    (the one that loads all planes of a one-layer z chunk at once, where it fits);
  * Q4 on 64^3 elements and Q1 on 256^3 elements (256^3 nodes).
Every single-level operation is run through the C ABI (apply, residual, nu = 1 and 2
smoother applications from a random guess and from zero, restriction, prolongation)
and compared with the oracle's Kronecker-form operator, smoother and transfers on the
same input.  Inputs are FP32-representable, so the FP64 and FP32 runs see the same
values and the oracle result serves both.  The launch shape each operation takes is
read back (gmg_launch_shape) and checked against the instance named above.

Bars (relative l2, and a max-abs bound of 10x that on the largest reference entry):
apply and residual 1e-12 (FP64) / 2e-5 (FP32); smoother 1e-11 / 1e-4; transfers
1e-14 / 1e-6 (the same bars as the small-lattice parity tests).
"""
import functools

import numpy as np
import pytest

from tests.gpu_common import rel_l2, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

# lambda_hat handed to both sides: the closed forms of lambda_max(D^-1 A) for Q1 and Q2 and
# the Q4 value of the block symbol, so that the Chebyshev interval is the production one
LAMBDA = {1: 1.5, 2: 75.0 / 56.0, 4: 2.199326}

# (q, n, level offset from the finest): the levels under test
CASES = [(2, 128, 0), (2, 128, 1), (4, 64, 0), (1, 256, 0)]


def _case_id(c):
    q, n, off = c
    return f"q{q}_n{n}_N{q * (n >> off)}"


@functools.lru_cache(maxsize=2)
def _ctx(q, n):
    torch_cuda()
    from paper_1408_6497_amd import Context
    return Context(q, n, 0, seed=0, lambda_override=LAMBDA[q])


@functools.lru_cache(maxsize=2)
def _oracle(q, n, levels):
    from oracle import multigrid as mg
    return mg.Hierarchy(q, n, levels, mg.Options(lambda_override=LAMBDA[q]), form="kron")


def _f32_normal(size, seed, mean_free=True):
    v = np.random.default_rng(seed).standard_normal(size)
    if mean_free:
        v -= v.mean()
    return v.astype(np.float32).astype(np.float64)


def _check(got, ref, tol, what):
    err = rel_l2(got, ref)
    amax = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"  {what}: rel_l2 {err:.2e}  max-abs/max {amax:.2e}", flush=True)
    assert err <= tol, what
    assert amax <= 10 * tol, what


def _shape(ctx, level, prec, op):
    s = ctx.launch_shape(level, prec, op)
    print(f"  shape {op} level {level} prec {prec}: {s}", flush=True)
    return s


def _assert_production_instance(q, N, prec, shape):
    kernel, G, TZ, blocks = shape
    assert kernel in ("column", "column_preload"), shape
    if q == 2 and N >= 128:
        assert G == 1, shape
    if kernel == "column_preload":
        assert TZ == 1 and prec == 1 and q <= 2, shape
    if q == 2 and N == 256 and prec == 1:
        # the streaming loop (several element layers per block) of the 256^3-node level
        assert kernel == "column" and TZ > 1, shape


@pytest.mark.parametrize("case", CASES, ids=_case_id)
def test_apply_and_residual_production_shapes(case):
    torch = torch_cuda()
    from paper_1408_6497_amd import GMG_FP32, GMG_FP64
    q, n, off = case
    ctx = _ctx(q, n)
    lvl = ctx.levels - 1 - off
    H = _oracle(q, n, ctx.levels)
    lev = H.levels[lvl]
    N = lev.N
    print(f"[prod apply] q={q} n={n} level {lvl} N={N}", flush=True)
    x = _f32_normal(lev.size, 1000 + N + q)
    b = _f32_normal(lev.size, 2000 + N + q)
    y_ref = lev.A @ x
    r_ref = b - y_ref
    for prec, dt, tol in ((GMG_FP64, torch.float64, 1e-12), (GMG_FP32, torch.float32, 2e-5)):
        _assert_production_instance(q, N, prec, _shape(ctx, lvl, prec, "apply"))
        _assert_production_instance(q, N, prec, _shape(ctx, lvl, prec, "residual"))
        xd, bd = to_dev(x, dt), to_dev(b, dt)
        yd, rd = torch.empty_like(xd), torch.empty_like(xd)
        ctx.apply(lvl, xd, yd)
        ctx.residual(lvl, bd, xd, rd)
        torch.cuda.synchronize()
        _check(to_host(yd), y_ref, tol, f"apply prec {prec}")
        _check(to_host(rd), r_ref, tol, f"residual prec {prec}")
        del xd, bd, yd, rd


@pytest.mark.parametrize("case", CASES, ids=_case_id)
@pytest.mark.parametrize("start", ["random", "zero"])
def test_smoother_production_shapes(case, start):
    """nu = 1 and 2 Chebyshev(3) applications; from a random guess every step is the
    Chebyshev epilogue, from zero the first two steps are the fused zero-start pass."""
    torch = torch_cuda()
    from paper_1408_6497_amd import GMG_FP32, GMG_FP64
    q, n, off = case
    ctx = _ctx(q, n)
    lvl = ctx.levels - 1 - off
    H = _oracle(q, n, ctx.levels)
    lev = H.levels[lvl]
    N = lev.N
    print(f"[prod smooth] q={q} n={n} level {lvl} N={N} start={start}", flush=True)
    b = _f32_normal(lev.size, 3000 + N + q)
    u0 = _f32_normal(lev.size, 4000 + N + q, mean_free=False) if start == "random" else np.zeros(lev.size)
    ref1 = H.smooth(lev, b, u0, 1)
    ref2 = H.smooth(lev, b, ref1, 1)
    for prec, dt, tol in ((GMG_FP64, torch.float64, 1e-11), (GMG_FP32, torch.float32, 1e-4)):
        _assert_production_instance(q, N, prec, _shape(ctx, lvl, prec, "smooth"))
        if start == "zero":
            _assert_production_instance(q, N, prec, _shape(ctx, lvl, prec, "smooth_zero"))
        bd = to_dev(b, dt)
        for nu, ref in ((1, ref1), (2, ref2)):
            if start == "random":
                ud = to_dev(u0, dt)
                ctx.smooth(lvl, bd, ud, nu)
            else:
                ud = torch.full_like(bd, float("nan"))   # not read: a zero guess is implied
                ctx.smooth_zero(lvl, bd, ud, nu)
            torch.cuda.synchronize()
            _check(to_host(ud), ref, tol, f"smooth nu={nu} prec {prec}")
            del ud
        del bd


@pytest.mark.parametrize("case", CASES, ids=_case_id)
def test_transfers_production_shapes(case):
    """Restriction onto and prolongation from the next coarser level; on Q1 and Q2 with
    64 to 256 coarse nodes a side these are the one-pass kernels."""
    torch = torch_cuda()
    from paper_1408_6497_amd import GMG_FP32, GMG_FP64
    q, n, off = case
    ctx = _ctx(q, n)
    lvl = ctx.levels - 1 - off
    H = _oracle(q, n, ctx.levels)
    lev = H.levels[lvl]
    Nc = H.levels[lvl - 1].N
    print(f"[prod transfer] q={q} n={n} level {lvl} N={lev.N} -> {Nc}", flush=True)
    rf = _f32_normal(lev.size, 5000 + lev.N + q, mean_free=False)
    ec = _f32_normal(Nc ** 3, 6000 + lev.N + q, mean_free=False)
    uf = _f32_normal(lev.size, 7000 + lev.N + q, mean_free=False)
    rc_ref = lev.transfer.restrict(rf)
    uf_ref = uf + lev.transfer.prolong(ec)
    for prec, dt, tol in ((GMG_FP64, torch.float64, 1e-14), (GMG_FP32, torch.float32, 1e-6)):
        rk = _shape(ctx, lvl, prec, "restrict")[0]
        pk = _shape(ctx, lvl, prec, "prolong")[0]
        assert rk == ("transfer_fused" if q <= 2 and 64 <= Nc <= 256 else "transfer_axis")
        assert pk == ("transfer_fused" if q <= 2 and 2 * q <= Nc <= 256 else "transfer_axis")
        rfd = to_dev(rf, dt)
        rcd = torch.empty(Nc ** 3, dtype=dt, device="cuda")
        ecd, ufd = to_dev(ec, dt), to_dev(uf, dt)
        ctx.restrict(lvl, rfd, rcd)
        ctx.prolong(lvl, ecd, ufd)
        torch.cuda.synchronize()
        _check(to_host(rcd), rc_ref, tol, f"restrict prec {prec}")
        _check(to_host(ufd), uf_ref, tol, f"prolong prec {prec}")
        del rfd, rcd, ecd, ufd
