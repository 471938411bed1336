"""FFT solve of the uniform Q1, Q2 and Q4 systems (gmg_fft_solve) against the oracle.

The oracle's assembled Kronecker operator checks the residual of the FFT solution (an
exact solve: within rounding, 1e-12 relative); the C1 source has the closed-form discrete
solution amp * sin sin sin (the oracle's pin); the multigrid solve of the same load vector
agrees to its own tolerance; errors are reported for other orders.
"""
import math

import numpy as np
import pytest

from tests.gpu_common import to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _ctx(q, n, levels=0, **kw):
    torch_cuda()
    from paper_1408_6497_amd import Context
    return Context(q, n, levels, **kw)


@pytest.mark.parametrize("q,n", [(1, 8), (1, 32), (2, 4), (2, 16), (4, 4)])
def test_fft_solve_residual_on_the_oracle_operator(q, n):
    torch = torch_cuda()
    from oracle import operator as op
    ctx = _ctx(q, n, 2 if q * n <= 8 else 0)
    b = np.random.default_rng(11).standard_normal((q * n) ** 3)
    b -= b.mean()
    bd = to_dev(b, torch.float64)
    b0 = bd.clone()
    u = torch.empty_like(bd)
    ctx.fft_solve(bd, u)
    torch.cuda.synchronize()
    uh = to_host(u)
    A = op.assemble(q, n)
    rel = np.linalg.norm(b - A @ uh) / np.linalg.norm(b)
    print(f"[fft] q={q} n={n}: residual {rel:.2e}, mean {uh.mean():.1e}", flush=True)
    assert rel <= 1e-12
    if q == 1:
        assert abs(uh.mean()) <= 1e-12 * np.abs(uh).max()
    assert torch.equal(bd, b0)  # the load vector is left as it was


@pytest.mark.parametrize("q,n", [(1, 128), (2, 64), (2, 128), (4, 32), (4, 64)])
def test_fft_solve_residual_large_on_the_kronecker_operator(q, n):
    """The exact-to-rounding claim at the workloads' sizes (128^3 and 256^3 nodes): the
    smallest pencil eigenvalues vanish like t^2 there, which an FP64 evaluation of the
    determinant or of the Q4 eigen-decomposition would lose digits to."""
    torch = torch_cuda()
    from oracle import operator as op
    ctx = _ctx(q, n, 0)
    N = q * n
    b = np.random.default_rng(12).standard_normal(N ** 3)
    b -= b.mean()
    bd = to_dev(b, torch.float64)
    u = torch.empty_like(bd)
    ctx.fft_solve(bd, u)
    torch.cuda.synchronize()
    uh = to_host(u)
    del bd, u
    rel = np.linalg.norm(b - op.KroneckerOperator(q, n) @ uh) / np.linalg.norm(b)
    print(f"[fft-large] q={q} n={n}: residual {rel:.2e}", flush=True)
    assert rel <= 1e-12


def _accurate_kron_sin_load(q, n):
    """b = A v for v = sin(2 pi x) sin(2 pi y) sin(2 pi z) at the DoFs, each entry to a few ulp.

    A = K (x) M (x) M + M (x) K (x) M + M (x) M (x) K with the oracle's 1D matrices, and v a
    tensor product, so A v = (K s)(x)(M s)(x)(M s) + ...  The 1D product K s cancels (the rows of
    K sum to zero and s is smooth); it is taken as (K s)_i = Im(e^{i th_i} sum_j K_ij
    (e^{i (th_j - th_i)} - 1)), th = 2 pi x, with e^{i d} - 1 = -2 sin^2(d/2) + i sin d, which
    keeps every digit (and reads the rows as summing to zero exactly)."""
    from oracle import operator as op
    x = op.dof_coords_1d(q, n)
    K1, M1 = op.assemble_1d(q, n)
    K1 = K1.tocoo()
    th = 2 * np.pi * x
    d = x[K1.col] - x[K1.row]
    d -= np.round(d)
    dth = 2 * np.pi * d
    em1 = -2 * np.sin(dth / 2) ** 2 + 1j * np.sin(dth)
    acc = np.zeros(x.size, dtype=complex)
    np.add.at(acc, K1.row, K1.data * em1)
    ks = np.imag(np.exp(1j * th) * acc)
    s = np.sin(th)
    ms = M1 @ s
    b = (np.einsum("k,j,i->kji", ms, ms, ks) + np.einsum("k,j,i->kji", ms, ks, ms)
         + np.einsum("k,j,i->kji", ks, ms, ms)).ravel()
    return np.einsum("k,j,i->kji", s, s, s).ravel(), b


@pytest.mark.parametrize("q,n", [(2, 64), (2, 128), (4, 32), (4, 64)])
def test_fft_solve_recovers_a_smooth_mode(q, n):
    """b = A v for the smooth v = sin(2 pi x) sin(2 pi y) sin(2 pi z) (zero integral), computed to
    a few ulp per entry: the FFT solve returns v.  The lowest wavenumbers dominate u here and
    their pencil eigenvalues vanish like t^2, so an eigenvalue with relative error d shows as
    an error d in u (an FP64 determinant of the Q2 pencil gave d = 4.7e-13 at n = 128); the
    transforms' own rounding stays near 1e-15."""
    torch = torch_cuda()
    ctx = _ctx(q, n, 0)
    v, b = _accurate_kron_sin_load(q, n)
    bd = to_dev(b, torch.float64)
    u = torch.empty_like(bd)
    ctx.fft_solve(bd, u)
    torch.cuda.synchronize()
    err = np.linalg.norm(to_host(u) - v) / np.linalg.norm(v)
    print(f"[fft-smooth] q={q} n={n}: relative error {err:.2e}", flush=True)
    assert err <= 1e-14


def test_fft_solve_c1_closed_form():
    """f = 12 pi^2 sin sin sin on 64^3 Q1 nodes: the discrete solution is the closed form."""
    torch = torch_cuda()
    from workloads import sin_source, sin_exact
    from oracle import multigrid as mg
    q, n = 1, 64
    ctx = _ctx(q, n)
    x1 = ctx.dof_coords_1d()
    b = to_dev(mg.rhs(q, n, to_host(sin_source(x1))), torch.float64)
    u = torch.empty_like(b)
    ctx.fft_solve(b, u)
    torch.cuda.synchronize()
    th, h = 2 * math.pi / n, 1.0 / n
    amp = 4 * math.pi ** 2 * (h * (4 + 2 * math.cos(th)) / 6) / ((2 - 2 * math.cos(th)) / h)
    err = np.max(np.abs(to_host(u) - amp * sin_exact(x1)))
    print(f"[fft-c1] max error against the closed form {err:.2e}", flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("q,n", [(1, 128), (2, 64), (4, 32)])
def test_fft_solve_matches_multigrid(q, n):
    """The FFT solution and the multigrid solution of one load vector agree (128^3 nodes): both
    take the zero-integral solution."""
    torch = torch_cuda()
    from workloads import gaussian_params, gaussian_source
    ctx = _ctx(q, n)
    f = gaussian_source(ctx.dof_coords_1d(), gaussian_params(0, 32, 0.02, 0.1), device="cuda")
    b = torch.empty_like(f)
    ctx.rhs(f, b)
    uf, ug = torch.empty_like(b), torch.empty_like(b)
    ctx.fft_solve(b, uf)
    info = ctx.solve_rhs(b, ug, 1e-11)
    torch.cuda.synchronize()
    d = (uf - ug).norm().item() / ug.norm().item()
    print(f"[fft-mg] relative difference {d:.2e} (multigrid to {info.rel_residual_f64:.1e})", flush=True)
    assert d <= 1e-7


def test_fft_solve_rejects_octrees_and_aliasing():
    torch = torch_cuda()
    from oracle import octree as ot
    from paper_1408_6497_amd import Context, GmgError
    tree = ot.uniform(2)
    keys = np.array([ot.morton(o[1], o[2], o[3]) for o in tree], dtype=np.uint64)
    lev = np.array([o[0] for o in tree], dtype=np.uint8)
    ctx = Context(2, 0, leaves=(keys, lev))
    b = torch.zeros(ctx.num_dofs(), dtype=torch.float64, device="cuda")
    u = torch.empty_like(b)
    with pytest.raises(GmgError) as e:
        ctx.fft_solve(b, u)
    assert e.value.status == 1  # GMG_E_ARG
    c1 = _ctx(1, 8, 2)
    b1 = torch.zeros(c1.num_dofs(), dtype=torch.float64, device="cuda")
    with pytest.raises(GmgError):
        c1.fft_solve(b1, b1)
