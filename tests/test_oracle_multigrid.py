"""Pins of the oracle's coarse solve and V-cycle (Algorithm 2.1)."""
import math

import numpy as np
import pytest

from oracle import operator as op, multigrid as mg, transfer


def test_coarse_solve_is_pseudo_inverse():
    H = mg.Hierarchy(2, 4, 2)
    A0 = H.levels[0].A.toarray()
    b = mg.project(np.random.default_rng(2).standard_normal(A0.shape[0]))
    x = H.coarse_solve(b)
    assert np.max(np.abs(x - np.linalg.pinv(A0) @ b)) < 1e-12 * np.max(np.abs(x))
    assert abs(x.sum()) < 1e-12 * np.abs(x).sum()
    assert np.linalg.norm(A0 @ x - b) < 1e-13 * np.linalg.norm(b)


def _vcycle_matrix(H):
    n = H.finest.size
    V = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        V[:, j] = H.vcycle(e)
    return V


@pytest.mark.parametrize("q,n,levels", [(1, 4, 2), (2, 4, 2), (1, 8, 3)])
def test_vcycle_symmetric_positive(q, n, levels):
    H = mg.Hierarchy(q, n, levels)
    rng = np.random.default_rng(4)
    x = mg.project(rng.standard_normal(H.finest.size))
    y = mg.project(rng.standard_normal(H.finest.size))
    xVy, yVx = x @ H.vcycle(y), y @ H.vcycle(x)
    assert abs(xVy - yVx) < 1e-13 * math.sqrt(abs(x @ H.vcycle(x)) * abs(y @ H.vcycle(y)))
    for s in range(5):
        z = mg.project(np.random.default_rng(10 + s).standard_normal(H.finest.size))
        assert z @ H.vcycle(z) > 0


def _cheb_poly_matrix(X, alpha, beta, deg):
    """T_deg((theta I - X)/delta) / T_deg(sigma) by the Chebyshev three-term polynomial recurrence."""
    theta, delta = (beta + alpha) / 2, (beta - alpha) / 2
    Y = (theta * np.eye(len(X)) - X) / delta
    T0, T1 = np.eye(len(X)), Y
    t0, t1 = 1.0, theta / delta
    for _ in range(deg - 1):
        T0, T1 = T1, 2 * Y @ T1 - T0
        t0, t1 = t1, 2 * (theta / delta) * t1 - t0
    return T1 / t1


def test_two_level_cycle_error_propagator():
    # I - V A = G (I - P C P^T A) G, G = p(D^-1 A)^nu with p the Chebyshev error
    # polynomial in closed form and C the coarse pseudo-inverse with projection.
    q, n = 1, 4
    H = mg.Hierarchy(q, n, 2)
    f, c = H.levels[1], H.levels[0]
    A = f.A.toarray()
    X = A / f.D[:, None]
    p = _cheb_poly_matrix(X, f.alpha, f.beta, 3)
    G = np.linalg.matrix_power(p, 2)
    P = transfer.prolongation(q, n // 2).toarray()
    Nc = P.shape[1]
    Ac = c.A.toarray()
    C = np.linalg.inv(Ac + np.ones((Nc, Nc)) / Nc) @ (np.eye(Nc) - np.ones((Nc, Nc)) / Nc)
    E = G @ (np.eye(len(A)) - P @ C @ P.T @ A) @ G
    V = _vcycle_matrix(H)
    assert np.max(np.abs((np.eye(len(A)) - V @ A) - E)) < 1e-12


def test_rhs_projection_and_mass():
    q, n = 2, 4
    x1 = op.dof_coords_1d(q, n)
    f = np.ones(len(x1) ** 3)
    b_raw = op.assemble(q, n, "mass") @ f
    assert abs(b_raw.sum() - 1.0) < 1e-14          # 1^T M 1 = volume of the cube
    b = mg.rhs(q, n, f)
    assert abs(b.sum()) < 1e-16 * 100                    # b is orthogonal to the null vector
    # l2 projection of M 1: for Q2 the vertex/edge/face/interior rows of M 1 differ
    Mh = np.array([1 / 3, 2 / 3])                    # assembled 1D mass row sums (h = 1): vertex, midpoint
    cls = np.arange(q * n) % 2
    m1 = Mh[cls] / n
    Mone = (m1[:, None, None] * m1[None, :, None] * m1[None, None, :]).ravel()
    assert np.max(np.abs(b - (Mone - Mone.mean()))) < 1e-15
