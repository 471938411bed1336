"""The spectral FFT Poisson solve (gmg_spectral_*, Section 2.1) against the oracle.

The oracle (numpy FFT in FP64, itself pinned to written-out trigonometric solutions
and an explicit DFT) gives the reference on the same seeded source; the GPU path's
transforms are its own kernels.  Bars: 1e-13 relative l2 against the oracle (a few
hundred FP64 roundings per point through five transform passes), and for test case 1
of Section 3 (u = sin(2 pi k x) sin(2 pi k y) sin(2 pi k z) with 2k < N points a side)
the exact u to 1e-13 absolute.
"""
import math

import numpy as np
import pytest

from tests.gpu_common import rel_l2, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _solver(N):
    torch_cuda()
    from paper_1408_6497_amd import SpectralSolver
    return SpectralSolver(N)


@pytest.mark.parametrize("N", [16, 32, 64, 128, 256])
def test_spectral_solve_matches_oracle(N):
    torch = torch_cuda()
    from oracle import spectral
    print(f"[spectral] N={N}", flush=True)
    f = np.random.default_rng(N).standard_normal(N ** 3)
    fd = to_dev(f, torch.float64)
    u = torch.empty_like(fd)
    sp = _solver(N)
    sp.solve(fd, u)
    torch.cuda.synchronize()
    ref = spectral.solve(f, N)
    err = rel_l2(to_host(u), ref)
    print(f"  rel_l2 {err:.2e}  mean {float(u.mean()):.1e}", flush=True)
    assert err <= 1e-13
    assert abs(float(u.mean())) <= 1e-14 * float(u.abs().max())
    assert torch.equal(fd, to_dev(f, torch.float64))   # the source is left as it was


@pytest.mark.parametrize("k,N", [(1, 16), (16, 64), (32, 128), (100, 512)])
def test_spectral_solve_oscillatory_test_case(k, N):
    """Test case 1 of Section 3 at frequency k: exact to rounding once N > 2k."""
    torch = torch_cuda()
    print(f"[spectral-sin] k={k} N={N}", flush=True)
    x = torch.arange(N, dtype=torch.float64, device="cuda") / N
    s = torch.sin(2 * math.pi * k * x)
    ue = (s[:, None, None] * s[None, :, None] * s[None, None, :]).reshape(-1)
    f = 12 * math.pi ** 2 * k * k * ue
    u = torch.empty_like(f)
    sp = _solver(N)
    sp.solve(f, u)
    torch.cuda.synchronize()
    err = float((u - ue).abs().max())
    print(f"  max error {err:.2e}", flush=True)
    assert err <= 1e-13


def test_spectral_solve_in_place_and_sizes():
    """f and u may alias; sizes outside 16..1024 or not a power of two are refused."""
    torch = torch_cuda()
    from oracle import spectral
    from paper_1408_6497_amd import GmgError
    N = 32
    f = np.random.default_rng(9).standard_normal(N ** 3)
    fd = to_dev(f, torch.float64)
    sp = _solver(N)
    sp.solve(fd, fd)
    torch.cuda.synchronize()
    assert rel_l2(to_host(fd), spectral.solve(f, N)) <= 1e-13
    for bad in (8, 48, 2048):
        with pytest.raises(GmgError):
            _solver(bad)
