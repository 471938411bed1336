"""The matrix-core form of the FP32 q = 4 column kernel (option q4_mfma) against the oracle.

With q4_mfma the x and z passes of the sum factorization run as 4x4x1 FP32 MFMA outer
products (the y pass, the vertex's taps into the left element and the shared top plane stay
on the vector unit); it is the same operator to FP32 rounding.  Checked element by element
against the oracle's Kronecker-form operator and smoother on Q4 levels of 64, 128 and 256
nodes a side (one, two and four wavefronts per x row; the 256^3-node level is the production
C3 level), for the apply, the residual and the smoother step from a random guess and from
zero, with the launch shape read back to confirm the matrix-core instance ran.  Bars as the
FP32 parity tests: apply and residual 2e-5, smoother 1e-4 relative l2 (and max-abs 10x that
on the largest reference entry).  A Q4 solve with it reaches the FP64 tolerance.
"""
import numpy as np
import pytest

from tests.gpu_common import to_dev, to_host, torch_cuda
from tests.test_gpu_production_shapes import LAMBDA, _check, _f32_normal, _oracle

pytestmark = pytest.mark.gpu


def _ctx(n, **kw):
    torch_cuda()
    from paper_1408_6497_amd import Context
    return Context(4, n, 0, seed=0, lambda_override=LAMBDA[4], q4_mfma=1, **kw)


@pytest.mark.parametrize("n", [16, 32, 64])
def test_q4_mfma_apply_residual_smoother(n):
    torch = torch_cuda()
    from paper_1408_6497_amd import GMG_FP32
    ctx = _ctx(n)
    lvl = ctx.levels - 1
    H = _oracle(4, n, ctx.levels)
    lev = H.levels[lvl]
    N = lev.N
    print(f"[q4 mfma] n={n} N={N}", flush=True)
    for op in ("apply", "residual", "smooth", "smooth_zero"):
        shape = ctx.launch_shape(lvl, GMG_FP32, op)
        print(f"  shape {op}: {shape}", flush=True)
        assert shape[0] == "column_mfma", shape
    x = _f32_normal(lev.size, 5000 + N)
    b = _f32_normal(lev.size, 6000 + N)
    y_ref = lev.A @ x
    xd, bd = to_dev(x, torch.float32), to_dev(b, torch.float32)
    yd, rd = torch.empty_like(xd), torch.empty_like(xd)
    ctx.apply(lvl, xd, yd)
    ctx.residual(lvl, bd, xd, rd)
    torch.cuda.synchronize()
    _check(to_host(yd), y_ref, 2e-5, "apply")
    _check(to_host(rd), b - y_ref, 2e-5, "residual")
    u0 = _f32_normal(lev.size, 7000 + N, mean_free=False)
    ref1 = H.smooth(lev, b, u0, 1)
    ud = to_dev(u0, torch.float32)
    ctx.smooth(lvl, bd, ud, 1)
    torch.cuda.synchronize()
    _check(to_host(ud), ref1, 1e-4, "smooth nu=1 from a random guess")
    z1 = H.smooth(lev, b, np.zeros(lev.size), 1)
    z2 = H.smooth(lev, b, z1, 1)
    for nu, ref in ((1, z1), (2, z2)):
        ud = torch.full_like(bd, float("nan"))
        ctx.smooth_zero(lvl, bd, ud, nu)
        torch.cuda.synchronize()
        _check(to_host(ud), ref, 1e-4, f"smooth nu={nu} from zero")
    ctx.close()


def test_q4_mfma_solve_reaches_tolerance():
    """The Q4 FP32-cycle solve with the matrix-core form: the FP64 residual meets 1e-8 and
    the iteration count is the vector form's."""
    torch = torch_cuda()
    from paper_1408_6497_amd import Context, GMG_FP32
    from workloads import gaussian_params, gaussian_source
    params = gaussian_params(0, 8, 1e-3, 1e-2, log_uniform=True)
    out = {}
    for mf in (0, 1):
        ctx = Context(4, 32, 0, seed=0, vcycle_prec=GMG_FP32, q4_mfma=mf)
        f = gaussian_source(ctx.dof_coords_1d(), params, device="cuda")
        u = torch.empty_like(f)
        info = ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        out[mf] = (info.inner_iters, info.rel_residual_f64)
        ctx.close()
    print(f"[q4 mfma solve] vector {out[0]}, matrix cores {out[1]}", flush=True)
    assert out[1][1] <= 1e-8
    assert out[1][0] == out[0][0]
