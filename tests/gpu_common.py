"""Shared helpers of the GPU parity tests (oracle side and device side kept apart)."""
import functools

import numpy as np

FP64_TOL = 1e-12   # relative l2 error of an FP64 apply
FP32_TOL = 2e-5    # relative l2 error of an FP32 apply


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(x, dtype):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def to_host(t):
    return t.detach().double().cpu().numpy()


@functools.lru_cache(maxsize=None)
def oracle_hierarchy(q, n, levels, seed=0, smoother="chebyshev", form="csr"):
    from oracle import multigrid as mg
    opts = mg.Options(seed=seed, smoother=smoother)
    return mg.Hierarchy(q, n, levels, opts, form=form)


def mean_free_normal(size, seed):
    from workloads import normal_vector
    v = normal_vector(size, seed)
    return v - v.mean()
