"""gmg_dot_noalloc (the entry point for callers that cannot allocate) against gmg_dot.

Both run the same kernels in the same order, so the FP64 results must be the same bits;
they are also checked against the exact sum of the inputs (math.fsum of the products of
the values as stored, each product exact in FP64 for FP32 inputs).  Two calls in a row on
one device share the static scratch: the second, on a smaller input, must not see the
first call's partials.
"""
import math

import numpy as np
import pytest

from tests.gpu_common import torch_cuda

pytestmark = pytest.mark.gpu


def _ctx():
    torch_cuda()
    from paper_1408_6497_amd import Context
    return Context(2, 8, 0, seed=0)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_dot_noalloc_matches_gmg_dot_on_two_calls(dtype):
    torch = torch_cuda()
    ctx = _ctx()
    dt = getattr(torch, dtype)
    g = torch.Generator(device="cuda").manual_seed(17)
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    # a large first call (1024 partials in use), then a smaller one (fewer partials)
    for n in (3_000_001, 777):
        print(f"[noalloc] dtype={dtype} n={n}", flush=True)
        x = torch.randn(n, dtype=dt, device="cuda", generator=g)
        y = torch.randn(n, dtype=dt, device="cuda", generator=g)
        ref = ctx.dot(x, y)
        ctx.dot_noalloc(x, y, out)
        torch.cuda.synchronize()
        got = float(out.item())
        xs, ys = x.double().cpu().numpy(), y.double().cpu().numpy()
        exact = math.fsum((xs * ys).tolist()) if dtype == "float32" else math.fsum(np.multiply(xs, ys).tolist())
        print(f"  gmg_dot {ref!r} noalloc {got!r} exact {exact!r}", flush=True)
        assert got == ref
        assert abs(got - exact) <= 1e-12 * math.fsum(np.abs(xs * ys).tolist())
    # n = 0 gives 0
    e = torch.empty(0, dtype=dt, device="cuda")
    ctx.dot_noalloc(e, e, out)
    torch.cuda.synchronize()
    assert float(out.item()) == 0.0


def test_dot_noalloc_two_contexts_share_the_device_scratch():
    """A second context on the same device uses the same array; results stay exact."""
    torch = torch_cuda()
    a, b = _ctx(), _ctx()
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    x = torch.arange(1, 1001, dtype=torch.float64, device="cuda")
    a.dot_noalloc(x, x, out[0:1])
    torch.cuda.synchronize()
    b.dot_noalloc(x[:10], x[:10], out[1:2])
    torch.cuda.synchronize()
    assert out.tolist() == [sum(i * i for i in range(1, 1001)), sum(i * i for i in range(1, 11))]
