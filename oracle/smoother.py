"""Chebyshev-accelerated Jacobi smoother and the eigenvalue estimate it needs.

Paper: Section 2.3.3 -- a Chebyshev-accelerated Jacobi smoother is used for high
orders; it needs the largest eigenvalue of the system, estimated in the setup
phase with 10 iterations of a Krylov eigenvalue method (Arnoldi in the paper).

Readings (the paper gives no formulas):
  * The polynomial is the classical Chebyshev acceleration of D^-1 A on the
    interval [alpha, beta] (Saad, Iterative Methods for Sparse Linear Systems,
    2nd ed., Section 12.3), with theta = (beta+alpha)/2, delta = (beta-alpha)/2,
    sigma = theta/delta and the two-term recurrence written out in chebyshev().
  * [alpha, beta] = [0.1, 1.1] * lambda_hat, lambda_hat the largest Ritz value.
  * D^-1/2 A D^-1/2 is symmetric, so the Krylov method is Lanczos (the symmetric
    case of Arnoldi), started from a SplitMix64 vector made orthogonal to the
    null vector D^1/2 1.

Pins (tests/test_oracle_smoother.py): the Chebyshev error factor on a Fourier
mode of Q1 (where D is a multiple of I) equals T_d((theta - lambda)/delta) /
T_d(sigma); the Lanczos estimate reaches 3/2 (Q1), 75/56 (Q2).
"""
import numpy as np


def lanczos_lambda_max(A, diag, v0, steps=10):
    """Largest Ritz value of `steps` Lanczos steps on S = D^-1/2 A D^-1/2.

    v0 is the raw start vector; it is projected onto the complement of the null
    vector D^1/2 1 and normalized.  The recurrence stops early if the Krylov
    space becomes invariant (beta <= 1e-12 times the largest |alpha| so far).
    """
    s = 1.0 / np.sqrt(diag)
    w0 = np.sqrt(diag)
    v = v0 - (v0 @ w0) / (w0 @ w0) * w0
    v = v / np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    beta = 0.0
    alphas, betas = [], []
    for j in range(steps):
        w = s * (A @ (s * v)) - beta * v_prev
        alpha = w @ v
        w = w - alpha * v
        alphas.append(alpha)
        beta_new = np.linalg.norm(w)
        if j == steps - 1 or beta_new <= 1e-12 * max(abs(a) for a in alphas):
            break
        betas.append(beta_new)
        v_prev, v = v, w / beta_new
        beta = beta_new
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    return float(np.max(np.linalg.eigvalsh(T)))


def chebyshev(A, dinv, b, x, alpha, beta, degree):
    """One application of the degree-`degree` Chebyshev-Jacobi polynomial.

    r0 = b - A x0;  rho0 = 1/sigma;  d0 = D^-1 r0 / theta;
    for j = 0 .. degree-1:
        x_{j+1} = x_j + d_j
        r_{j+1} = r_j - A d_j
        rho_{j+1} = 1 / (2 sigma - rho_j)
        d_{j+1} = rho_{j+1} rho_j d_j + (2 rho_{j+1} / delta) D^-1 r_{j+1}
    returns x_degree.
    """
    theta = 0.5 * (beta + alpha)
    delta = 0.5 * (beta - alpha)
    sigma = theta / delta
    r = b - A @ x
    rho = 1.0 / sigma
    d = dinv * r / theta
    for _ in range(degree):
        x = x + d
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * dinv * r
        rho = rho_new
    return x


def jacobi(A, dinv, b, x, omega, sweeps):
    """Damped point Jacobi, x <- x + omega D^-1 (b - A x), `sweeps` times (Section 2.3.3)."""
    for _ in range(sweeps):
        x = x + omega * dinv * (b - A @ x)
    return x
