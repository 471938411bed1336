"""Seeded synthetic inputs shared by the oracle tests, the HIP-path tests and the bench.

This module holds input generation only -- none of the solver's arithmetic.  It
knows nothing about basis functions, operators or grids: callers pass the 1D
coordinate lists (or points) at which a source is sampled, computed by their own
side.

Sources (shapes of the paper's workloads, Section 3):
  * sin_source        f = 12 pi^2 sin(2 pi x) sin(2 pi y) sin(2 pi z), whose
                      periodic solution is u = sin sin sin (the oscillatory
                      test case at frequency 1).
  * gaussian_params / gaussian_source
                      sums of periodized Gaussians with seeded centres, widths
                      and amplitudes, minus their exact mean (smooth but
                      localized sources, and the sharp-layer regime at small
                      widths).
  * sharp_layer       u = exp(-(r/R)^alpha), r the periodic distance to a centre,
                      and f = -Laplace(u) in closed form (the paper's second
                      time-to-solution test, a sharp internal layer on the sphere
                      r = R).
  * grf               Gaussian random fields with power spectrum |k|^-alpha.
  * normal_vector     seeded N(0, 1) vectors for operator-level parity.
"""
import math

import numpy as np


def normal_vector(n, seed):
    """Seeded N(0, 1) float64 vector of length n."""
    return np.random.default_rng(seed).standard_normal(n)


def gaussian_params(seed, count, sigma_lo, sigma_hi, log_uniform=False):
    """Centres (count, 3) ~ U[0,1)^3, widths, amplitudes ~ N(0,1), drawn in that order."""
    rng = np.random.default_rng(seed)
    centres = rng.random((count, 3))
    if log_uniform:
        sigma = 10.0 ** rng.uniform(math.log10(sigma_lo), math.log10(sigma_hi), count)
    else:
        sigma = rng.uniform(sigma_lo, sigma_hi, count)
    amps = rng.standard_normal(count)
    return {"centres": centres, "sigma": sigma, "amps": amps}


def _periodic_gauss_1d(x, c, s):
    """sum over images m in {-1, 0, 1} of exp(-(x - c - m)^2 / (2 s^2))."""
    out = np.zeros_like(x)
    for m in (-1.0, 0.0, 1.0):
        out += np.exp(-((x - c - m) ** 2) / (2.0 * s * s))
    return out


def gaussian_source(x1d, params, device=None, dtype=None):
    """Mean-free sum of periodized Gaussians on the tensor grid x1d^3 (x fastest).

    f(x) = sum_i a_i [ prod_d g_id(x_d) - (2 pi s_i^2)^{3/2} ], where g_id sums the
    three nearest periodic images along axis d.  Returned as a torch tensor of
    shape (N^3,) on `device` (CPU numpy-backed if None).
    """
    import torch
    x1d = np.asarray(x1d, dtype=np.float64)
    N = len(x1d)
    dev = torch.device("cpu") if device is None else torch.device(device)
    f = torch.zeros((N, N, N), dtype=torch.float64, device=dev)
    for c, s, a in zip(params["centres"], params["sigma"], params["amps"]):
        gx = torch.from_numpy(_periodic_gauss_1d(x1d, c[0], s)).to(dev)
        gy = torch.from_numpy(_periodic_gauss_1d(x1d, c[1], s)).to(dev)
        gz = torch.from_numpy(_periodic_gauss_1d(x1d, c[2], s)).to(dev)
        f += a * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
        f -= a * (2.0 * math.pi * s * s) ** 1.5
    f = f.reshape(-1)
    return f if dtype is None else f.to(dtype)


def gaussian_source_points(points, params):
    """The same source at arbitrary points (P, 3), as a float64 numpy array."""
    pts = np.asarray(points, dtype=np.float64)
    f = np.zeros(len(pts))
    for c, s, a in zip(params["centres"], params["sigma"], params["amps"]):
        g = np.ones(len(pts))
        for d in range(3):
            g *= _periodic_gauss_1d(pts[:, d], c[d], s)
        f += a * (g - (2.0 * math.pi * s * s) ** 1.5)
    return f


def sharp_layer(points, centre=(0.5, 0.5, 0.5), radius=0.25, alpha=10.0):
    """(u, f) at points (P, 3): u = exp(-s), s = (r/R)^alpha with r the nearest-image
    distance to centre on the unit torus, and f = -Laplace(u) = e^-s (alpha s / r^2)
    (alpha + 1 - alpha s) (radial Laplacian u'' + 2 u' / r; f -> 0 as r -> 0 for
    alpha > 2).  u and f are not periodic, but for radius <= 0.3 and alpha >= 10 they
    and their derivatives vanish to below 1e-14 at the faces."""
    pts = np.asarray(points, dtype=np.float64)
    d = np.abs(pts - np.asarray(centre, dtype=np.float64)[None, :]) % 1.0
    d = np.minimum(d, 1.0 - d)
    r = np.sqrt(np.sum(d * d, axis=1))
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(r > 0.0, np.exp(alpha * np.log(np.where(r > 0.0, r, 1.0) / radius)), 0.0)
        rr = np.where(r > 0.0, r * r, 1.0)
        f = np.where(r > 0.0, np.exp(-s) * (alpha * s / rr) * (alpha + 1.0 - alpha * s), 0.0)
    return np.exp(-s), f


def sin_source(x1d, device=None):
    """12 pi^2 sin(2 pi x) sin(2 pi y) sin(2 pi z) on the tensor grid x1d^3 (x fastest)."""
    import torch
    s = torch.from_numpy(np.sin(2.0 * math.pi * np.asarray(x1d, dtype=np.float64)))
    if device is not None:
        s = s.to(device)
    f = 12.0 * math.pi ** 2 * (s[:, None, None] * s[None, :, None] * s[None, None, :])
    return f.reshape(-1)


def sin_exact(x1d):
    """u = sin(2 pi x) sin(2 pi y) sin(2 pi z) on the tensor grid (numpy, x fastest)."""
    s = np.sin(2.0 * math.pi * np.asarray(x1d, dtype=np.float64))
    return (s[:, None, None] * s[None, :, None] * s[None, None, :]).ravel()


def grf(N, seed, alpha_lo=2.0, alpha_hi=4.0, device=None):
    """Gaussian random field on the N^3 lattice, power spectrum |k|^-alpha, unit RMS.

    alpha ~ U[alpha_lo, alpha_hi]; coefficients (xi1 + i xi2) |2 pi k|^(-alpha/2) for
    integer wavevectors k != 0 inside the lattice band; the real part of the
    inverse FFT, scaled to unit RMS.  Returns (field (N^3,), alpha).
    """
    import torch
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(alpha_lo, alpha_hi)
    dev = torch.device("cpu") if device is None else torch.device(device)
    gen = torch.Generator(device=dev).manual_seed(int(seed))
    re = torch.randn((N, N, N), generator=gen, dtype=torch.float64, device=dev)
    im = torch.randn((N, N, N), generator=gen, dtype=torch.float64, device=dev)
    k = torch.fft.fftfreq(N, d=1.0 / N, dtype=torch.float64, device=dev)
    kk = (k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    kk[0, 0, 0] = 1.0
    amp = (2.0 * math.pi) ** (-alpha / 2.0) * kk ** (-alpha / 4.0)
    amp[0, 0, 0] = 0.0
    field = torch.fft.ifftn(torch.complex(re * amp, im * amp)).real
    field = field / torch.sqrt(torch.mean(field * field))
    return field.reshape(-1), alpha
