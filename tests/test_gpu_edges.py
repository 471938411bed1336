"""Edge cases on the GPU: degenerate sources, the smallest meshes, the largest meshes.

The largest meshes (Q1 and Q2 on 512^3 elements, Q4 on 256^3: about 10^9 DoFs) are
checked on sampled rows: the oracle computes (A x)_i for each sampled DoF from the rows
of its periodic 1D matrices, (A x)_ijk = sum K1[i,i'] M1[j,j'] M1[k,k'] x + (two more
terms), with the input gathered from the device vector around the DoF.
"""
import numpy as np
import pytest

from tests.gpu_common import FP32_TOL, FP64_TOL, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _ctx(q, n, levels=0, **kw):
    torch_cuda()
    from paper_1408_6497_amd import Context
    return Context(q, n, levels, **kw)


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_and_constant_sources_give_zero(prec):
    """f = 0 returns u = 0 without iterating.  On Q1 every node has the same basis integral,
    so a constant f projects to a zero load (up to the rounding of the mean) and u ~ 0; on Q2
    the node classes integrate differently and the projected load of a constant is not zero."""
    torch = torch_cuda()
    ctx = _ctx(2, 8, vcycle_prec=prec)
    f = torch.zeros(ctx.num_dofs(), dtype=torch.float64, device="cuda")
    u = torch.full_like(f, 7.0)
    info = ctx.solve(f, u, 1e-8)
    torch.cuda.synchronize()
    assert float(u.abs().max()) == 0.0 and info.inner_iters == 0
    ctx1 = _ctx(1, 16, vcycle_prec=prec)
    f = torch.full((ctx1.num_dofs(),), 3.0, dtype=torch.float64, device="cuda")
    u = torch.full_like(f, 7.0)
    ctx1.solve(f, u, 1e-8, raise_on_noconv=False)
    torch.cuda.synchronize()
    assert float(u.abs().max()) <= 1e-12


@pytest.mark.parametrize("q,n", [(1, 4), (2, 2), (4, 2)])
def test_smallest_meshes_solve(q, n):
    """q n = 4 or 8 nodes per direction: a single level, solved by the dense coarsest solve
    inside CG; checked on the assembled oracle matrix."""
    torch = torch_cuda()
    from oracle import operator as op, multigrid as mg
    from workloads import normal_vector
    ctx = _ctx(q, n)
    assert ctx.levels == 1
    N = q * n
    f = normal_vector(N ** 3, 4)
    fd = torch.from_numpy(f).cuda()
    u = torch.empty_like(fd)
    info = ctx.solve(fd, u, 1e-10)
    torch.cuda.synchronize()
    b = mg.rhs(q, n, f)
    r = b - op.assemble(q, n) @ to_host(u)
    assert np.linalg.norm(r - r.mean()) <= 1e-10 * np.linalg.norm(b) * 1.001
    assert info.inner_iters <= 2


def _sampled_rows(q, n, x_dev, idx):
    """(A x)_i for the sampled flat indices, from the oracle's 1D rows."""
    from oracle import operator as op
    K1, M1 = op.assemble_1d(q, n)
    N = q * n
    X = x_dev.view(N, N, N)  # [k][j][i]
    out = np.empty(len(idx))
    for t, flat in enumerate(idx):
        i, j, k = flat % N, (flat // N) % N, flat // (N * N)
        ri, rj, rk = K1.getrow(i), K1.getrow(j), K1.getrow(k)
        ci, cj, ck = ri.indices, rj.indices, rk.indices   # same pattern as the M1 rows
        Ki, Kj, Kk = ri.toarray()[0, ci], rj.toarray()[0, cj], rk.toarray()[0, ck]
        Mi, Mj, Mk = (M1.getrow(i).toarray()[0, ci], M1.getrow(j).toarray()[0, cj], M1.getrow(k).toarray()[0, ck])
        import torch
        blk = X[torch.as_tensor(ck, device=X.device)][:, torch.as_tensor(cj, device=X.device)][
            :, :, torch.as_tensor(ci, device=X.device)].double().cpu().numpy()
        out[t] = (np.einsum("c,b,a,cba->", Mk, Mj, Ki, blk) + np.einsum("c,b,a,cba->", Mk, Kj, Mi, blk)
                  + np.einsum("c,b,a,cba->", Kk, Mj, Mi, blk))
    return out


@pytest.mark.parametrize("q,n", [(1, 512), (2, 512), (4, 256)])
def test_largest_meshes_apply_on_sampled_rows(q, n):
    torch = torch_cuda()
    ctx = _ctx(q, n, lambda_override=1.0)
    N = q * n
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.integers(0, N ** 3, 200), [0, N - 1, N * N - 1, N ** 3 - 1]])
    g = torch.Generator(device="cuda").manual_seed(6)
    for dt, tol in ((torch.float64, FP64_TOL), (torch.float32, FP32_TOL)):
        x = torch.randn(N ** 3, dtype=dt, device="cuda", generator=g)
        y = torch.empty_like(x)
        ctx.apply(-1, x, y)
        torch.cuda.synchronize()
        ref = _sampled_rows(q, n, x, idx)
        got = y[torch.as_tensor(idx, device="cuda")].double().cpu().numpy()
        # per-row bound: FP32 rounding of ~(2q+1)^3 terms of size |A_ij x_j|
        scale = np.abs(ref).max()
        err = np.abs(got - ref).max() / scale
        print(f"[max] q={q} n={n} {dt}: {N ** 3} DoFs, sampled max rel err {err:.2e}", flush=True)
        assert err <= 20 * tol
        del x, y
        torch.cuda.empty_cache()
