"""Spectral FFT Poisson solve on a uniform periodic grid (Section 2.1, last paragraph).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's FFT method discretises -Laplace(u) = f spectrally: transform f, scale each
Fourier coefficient by the inverse of the Laplacian's diagonal form in the Fourier basis
(a Hadamard product), transform back.  On the N^3 grid x = (i, j, k) / N of the unit
periodic cube the Laplacian's eigenvalue for the integer wavevector m is -4 pi^2 |m|^2,
so u_hat(m) = f_hat(m) / (4 pi^2 |m|^2).

Readings (the paper gives only the three steps):
  * wavevector components m_d in {-N/2, ..., N/2 - 1} (the FFT's band; the Nyquist
    component -N/2 enters |m|^2 as (N/2)^2);
  * m = 0 is dropped: the solution has zero mean, and the mean of f (which has no
    periodic solution) is ignored;
  * f and u are real; layout x fastest, index i + N (j + N k).

Pins (tests/test_oracle_spectral.py): a trigonometric polynomial inside the band is
solved exactly (its solution is written out term by term, no transform); the solve
equals an explicit DFT-matrix evaluation of the same formula on tiny grids; the output
has zero mean and is real.
"""
import numpy as np


def wavenumbers(N):
    """Integer wavevector component of each FFT index, in {-N/2, ..., N/2 - 1}."""
    return np.fft.fftfreq(N, d=1.0 / N)


def solve(f, N):
    """u with -Laplace(u) = f - mean(f) spectrally on the N^3 grid (FP64, numpy FFT)."""
    F = np.fft.fftn(np.asarray(f, dtype=np.float64).reshape(N, N, N))   # axes [z, y, x]
    m = wavenumbers(N)
    mm = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    scale = np.zeros_like(mm)
    nz = mm > 0
    scale[nz] = 1.0 / (4.0 * np.pi ** 2 * mm[nz])
    return np.fft.ifftn(F * scale).real.ravel()


def solve_dft(f, N):
    """The same formula with explicit DFT matrices (tiny N; no FFT)."""
    idx = np.arange(N)
    W = np.exp(-2j * np.pi * np.outer(idx, idx) / N)
    X = np.asarray(f, dtype=np.float64).reshape(N, N, N).astype(complex)
    F = np.einsum("az,by,cx,zyx->abc", W, W, W, X)
    m = wavenumbers(N)
    out = np.zeros((N, N, N), dtype=complex)
    for a in range(N):
        for b in range(N):
            for c in range(N):
                mm = m[a] ** 2 + m[b] ** 2 + m[c] ** 2
                if mm > 0:
                    out[a, b, c] = F[a, b, c] / (4.0 * np.pi ** 2 * mm)
    Wi = np.conj(W) / N
    return np.einsum("za,yb,xc,abc->zyx", Wi, Wi, Wi, out).real.ravel()


def grid(N):
    """Grid coordinates of one axis: i / N."""
    return np.arange(N) / N
