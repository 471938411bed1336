"""The spectral FFT Poisson solve of the oracle against what fixes it (Section 2.1)."""
import math

import numpy as np
import pytest

from oracle import spectral


def _trig(N, terms):
    """f and the exact u of -Laplace(u) = f for f = sum a cos(2 pi m.x + phi), written out."""
    x = spectral.grid(N)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    f = np.zeros((N, N, N))
    u = np.zeros((N, N, N))
    for a, (mx, my, mz), phi in terms:
        ph = 2 * math.pi * (mx * X + my * Y + mz * Z) + phi
        f += a * np.cos(ph)
        u += a / (4 * math.pi ** 2 * (mx * mx + my * my + mz * mz)) * np.cos(ph)
    return f.ravel(), u.ravel()


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_trigonometric_polynomial_is_solved_exactly(N):
    terms = [(1.0, (1, 0, 0), 0.3), (-0.7, (1, 2, -1), 1.1), (0.25, (N // 2 - 1, 1, 0), -0.4),
             (2.0, (0, 0, N // 2 - 1), 0.0)]
    f, u = _trig(N, terms)
    got = spectral.solve(f + 3.5, N)           # the constant of f is dropped
    assert np.max(np.abs(got - u)) <= 1e-14 * max(1.0, np.max(np.abs(u))) * N


def test_sin_product_source():
    """Test case 1 of Section 3 (frequency k): f = 12 pi^2 k^2 sss -> u = sss, exact on 2k+ points."""
    for k, N in ((1, 8), (4, 16), (7, 16)):
        x = spectral.grid(N)
        s = np.sin(2 * math.pi * k * x)
        u = np.einsum("k,j,i->kji", s, s, s).ravel()
        f = 12 * math.pi ** 2 * k * k * u
        assert np.max(np.abs(spectral.solve(f, N) - u)) <= 1e-13


@pytest.mark.parametrize("N", [2, 4, 6])
def test_matches_explicit_dft(N):
    f = np.random.default_rng(N).standard_normal(N ** 3)
    a, b = spectral.solve(f, N), spectral.solve_dft(f, N)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


def test_nyquist_and_mean():
    """The Nyquist component enters as (N/2)^2: cos(pi N x) on the grid is (-1)^i, an
    eigenvector of the band-limited Laplacian with eigenvalue -4 pi^2 (N/2)^2 per axis."""
    N = 8
    i = np.arange(N)
    alt = (-1.0) ** i
    f = np.einsum("k,j,i->kji", np.ones(N), np.ones(N), alt).ravel()
    u = spectral.solve(f, N)
    assert np.max(np.abs(u - f / (4 * math.pi ** 2 * (N // 2) ** 2))) <= 1e-15
    g = np.random.default_rng(3).standard_normal(N ** 3)
    assert abs(spectral.solve(g, N).mean()) <= 1e-16
