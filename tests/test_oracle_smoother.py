"""Pins of the oracle's Chebyshev-Jacobi smoother and Lanczos estimate (Section 2.3.3)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import operator as op, smoother, rng as orng

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _cheb_T(d, y):
    return math.cos(d * math.acos(y)) if abs(y) <= 1 else math.cosh(d * math.acosh(abs(y))) * (np.sign(y) ** d)


@pytest.mark.parametrize("mode", [(1, 0, 0), (2, 3, 1), (4, 4, 4), (3, 0, 2)])
def test_chebyshev_error_factor_on_q1_fourier_mode(mode):
    # Q1: D = 8h/3 I, so cosine modes are eigenvectors of D^-1 A.  With b = 0 the
    # error is x, and one degree-d application multiplies it by
    # T_d((theta - lambda)/delta) / T_d(sigma).
    n = 8
    h = 1.0 / n
    A = op.assemble(1, n)
    D = A.diagonal()
    I = np.arange(n)
    th = [2 * np.pi * m / n for m in mode]
    v = (np.cos(th[2] * I)[:, None, None] * np.cos(th[1] * I)[None, :, None] * np.cos(th[0] * I)[None, None, :]).ravel()
    ks = lambda t: (2 - 2 * np.cos(t)) / h
    ms = lambda t: h * (4 + 2 * np.cos(t)) / 6
    lam = (ks(th[0]) * ms(th[1]) * ms(th[2]) + ms(th[0]) * ks(th[1]) * ms(th[2]) + ms(th[0]) * ms(th[1]) * ks(th[2])) / (8 * h / 3)
    assert np.max(np.abs(A @ v / D - lam * v)) < 1e-12
    alpha, beta, deg = 0.15, 1.65, 3
    x = smoother.chebyshev(A, 1.0 / D, np.zeros_like(v), v.copy(), alpha, beta, deg)
    theta, delta = (beta + alpha) / 2, (beta - alpha) / 2
    factor = _cheb_T(deg, (theta - lam) / delta) / _cheb_T(deg, theta / delta)
    assert np.max(np.abs(x - factor * v)) < 1e-12


def _q2_block_symbol_lambda_max():
    # Independent of the oracle: textbook Q2 element matrices, 2-node periodic cell.
    g = GOLD["q2_element_1d"]
    Kh = np.array(g["Khat_times_3"], float) / 3
    Mh = np.array(g["Mhat_times_30"], float) / 30
    best = 0.0
    dK = np.array([Kh[0, 0] + Kh[2, 2], Kh[1, 1]])   # real-space diagonal per node class
    dM = np.array([Mh[0, 0] + Mh[2, 2], Mh[1, 1]])
    d = (np.kron(np.kron(dM, dM), dK) + np.kron(np.kron(dM, dK), dM) + np.kron(np.kron(dK, dM), dM))

    def sym(Xh, t):
        # unknowns of cell c: vertex v_c (node 2c) and midpoint m_c (node 2c+1);
        # element c couples (v_c, m_c, v_{c+1})
        S = np.zeros((2, 2), complex)
        S[0, 0] = Xh[0, 0] + Xh[2, 2] + Xh[0, 2] * np.exp(1j * t) + Xh[2, 0] * np.exp(-1j * t)
        S[0, 1] = Xh[0, 1] + Xh[2, 1] * np.exp(-1j * t)
        S[1, 0] = Xh[1, 0] + Xh[1, 2] * np.exp(1j * t)
        S[1, 1] = Xh[1, 1]
        return S

    for tx, ty, tz in itertools.product(np.linspace(0, 2 * np.pi, 25), repeat=3):
        Kx, Mx = sym(Kh, tx), sym(Mh, tx)
        Ky, My = sym(Kh, ty), sym(Mh, ty)
        Kz, Mz = sym(Kh, tz), sym(Mh, tz)
        A = np.kron(np.kron(Mz, My), Kx) + np.kron(np.kron(Mz, Ky), Mx) + np.kron(np.kron(Kz, My), Mx)
        S = A / np.sqrt(np.outer(d, d))
        best = max(best, np.linalg.eigvalsh(S).max())
    return best


def test_q2_lambda_max_from_block_symbol():
    lam_sym = _q2_block_symbol_lambda_max()
    assert abs(lam_sym - GOLD["lambda_max_dinv_a"]["q2"]) < 1e-12
    A = op.assemble(2, 4)
    D = A.diagonal()
    ev = np.linalg.eigvalsh(A.toarray() / np.sqrt(np.outer(D, D)))
    assert abs(ev.max() - lam_sym) < 1e-12


@pytest.mark.parametrize("q,n,lam", [(1, 4, 1.5), (2, 4, 75 / 56)])
def test_lanczos_estimate(q, n, lam):
    A = op.assemble(q, n)
    D = A.diagonal()
    v0 = orng.lanczos_start(7, 0, A.shape[0])
    est10 = smoother.lanczos_lambda_max(A, D, v0, 10)
    assert 0.9 * lam <= est10 <= lam * (1 + 1e-12)
    # Krylov space exhausted: the estimate is the exact largest eigenvalue
    est = smoother.lanczos_lambda_max(A, D, v0, A.shape[0] - 1)
    assert abs(est - lam) < 1e-10


def test_jacobi_special_case_of_chebyshev_degree_1():
    # Degree-1 Chebyshev is damped Jacobi with omega = 1/theta.
    A = op.assemble(2, 4)
    D = A.diagonal()
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    x0 = np.random.default_rng(1).standard_normal(A.shape[0])
    alpha, beta = 0.2, 1.3
    x1 = smoother.chebyshev(A, 1 / D, b, x0, alpha, beta, 1)
    x2 = smoother.jacobi(A, 1 / D, b, x0, 2 / (alpha + beta), 1)
    assert np.max(np.abs(x1 - x2)) < 1e-13
