"""Solves at the workloads' full sizes, checked with the oracle's own FP64 operator.

The oracle applies A in its Kronecker-of-1D-CSR form (no assembled matrix), builds
b = M f - mean from the same nodal source, and recomputes the relative residual of
the GPU solution: ||b - A u - mean|| / ||b|| must be at most the solve tolerance.
"""
import numpy as np
import pytest

from tests.gpu_common import to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle_rel_residual(q, n, f_host, u_host):
    from oracle import operator as op, multigrid as mg
    b = mg.rhs(q, n, f_host, form="kron")
    r = b - op.operator(q, n, "kron") @ u_host
    r -= r.mean()
    return float(np.linalg.norm(r) / np.linalg.norm(b))


@pytest.mark.parametrize("case", ["q2_128_gaussians", "q4_64_sharp"])
def test_full_size_solves_on_the_oracle_operator(case):
    """256^3 DoFs: Q2 on 128^3 elements with 32 Gaussians (sigma U[0.02, 0.1], seed 0), and Q4 on
    64^3 elements with 8 Gaussians (sigma log-uniform in [1e-3, 1e-2], seed 0); plain FP64 CG
    and FP32 cycles in FP64 flexible CG, to 1e-8."""
    torch = torch_cuda()
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64
    from workloads import gaussian_params, gaussian_source
    if case == "q2_128_gaussians":
        q, n, params = 2, 128, gaussian_params(0, 32, 0.02, 0.1)
    else:
        q, n, params = 4, 64, gaussian_params(0, 8, 1e-3, 1e-2, log_uniform=True)
    f_host = None
    for prec in (GMG_FP64, GMG_FP32):
        ctx = Context(q, n, 0, seed=0, vcycle_prec=prec)
        f = gaussian_source(ctx.dof_coords_1d(), params, device="cuda")
        u = torch.empty_like(f)
        info = ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        if f_host is None:
            f_host = to_host(f)
        rel = _oracle_rel_residual(q, n, f_host, to_host(u))
        print(f"[full] {case} prec={prec}: iters {info.inner_iters} gpu {info.rel_residual_f64:.2e} "
              f"oracle {rel:.2e} t_solve {info.t_solve * 1e3:.2f} ms", flush=True)
        assert rel <= 1e-8 * 1.001
        ctx.close()
        del f, u
        torch.cuda.empty_cache()


def test_learned_solve_full_size():
    """Q2 on 256^3 elements (512^3 DoFs), GRF source of the held-out seed 30000, the shipped net
    in every learned cycle with the per-cycle fallback, to 1e-8 on the oracle's operator."""
    torch = torch_cuda()
    import os
    from paper_1408_6497_amd import Context
    from paper_1408_6497_amd import train as T
    from workloads import grf
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    w = T.load(os.path.join(root, "paper_1408_6497_amd", "weights", "q2_depth0.gmgw"))["w"]
    q, n = 2, 256
    ctx = Context(q, n, 0, seed=0, use_learned=1)
    ctx.net_set_weights(0, w)
    f, _ = grf(ctx.lattice(), 30000, device="cuda")
    u = torch.empty_like(f)
    info = ctx.solve(f, u, 1e-8)
    torch.cuda.synchronize()
    f_host, u_host = to_host(f), to_host(u)
    ctx.close()
    del f, u
    torch.cuda.empty_cache()
    rel = _oracle_rel_residual(q, n, f_host, u_host)
    print(f"[full] learned 512^3: iters {info.inner_iters} fallbacks {info.fallbacks} "
          f"gpu {info.rel_residual_f64:.2e} oracle {rel:.2e}", flush=True)
    assert rel <= 1e-8 * 1.001


def test_nested_refinement_solve_full_size():
    """ir_mode = 1 (FP64 residual and update around FP32 flexible CG solves) on the Q2 128^3-element
    Gaussian workload, to 1e-8 on the oracle's operator, with its outer and inner counts."""
    torch = torch_cuda()
    from paper_1408_6497_amd import Context, GMG_FP32
    from workloads import gaussian_params, gaussian_source
    q, n = 2, 128
    ctx = Context(q, n, 0, seed=0, vcycle_prec=GMG_FP32, ir_mode=1)
    f = gaussian_source(ctx.dof_coords_1d(), gaussian_params(0, 32, 0.02, 0.1), device="cuda")
    u = torch.empty_like(f)
    info = ctx.solve(f, u, 1e-8)
    torch.cuda.synchronize()
    rel = _oracle_rel_residual(q, n, to_host(f), to_host(u))
    print(f"[full] nested refinement: outer {info.outer_iters} inner {info.inner_iters} "
          f"gpu {info.rel_residual_f64:.2e} oracle {rel:.2e}", flush=True)
    assert rel <= 1e-8 * 1.001
    assert info.outer_iters >= 2 and info.inner_iters > info.outer_iters
    # the distance to the default flexible-CG form's solution
    ctx0 = Context(q, n, 0, seed=0, vcycle_prec=GMG_FP32)
    u0 = torch.empty_like(f)
    ctx0.solve(f, u0, 1e-8)
    torch.cuda.synchronize()
    d = float((u - u0).norm() / u0.norm())
    print(f"  distance to the ir_mode 0 solution {d:.2e} (reported; bounded by kappa x tol)", flush=True)
