"""Pins of the oracle's assembled operator (eq. 1.1, Section 2.3.2)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import basis, operator as op, multigrid as mg, krylov

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _periodic_1d(Khat, Mhat, q, n):
    """Test-side 1D periodic assembly from element matrices on [0, 1]."""
    N, h = q * n, 1.0 / n
    K, M = np.zeros((N, N)), np.zeros((N, N))
    for e in range(n):
        idx = [(q * e + a) % N for a in range(q + 1)]
        for a in range(q + 1):
            for b in range(q + 1):
                K[idx[a], idx[b]] += Khat[a][b] / h
                M[idx[a], idx[b]] += Mhat[a][b] * h
    return sp.csr_matrix(K), sp.csr_matrix(M)


def _kron3(K, M):
    return sp.kron(sp.kron(M, M), K) + sp.kron(sp.kron(M, K), M) + sp.kron(sp.kron(K, M), M)


@pytest.mark.parametrize("q,n", [(1, 4), (2, 2), (2, 4)])
def test_kronecker_identity_textbook(q, n):
    g = GOLD["q1_element_1d"] if q == 1 else GOLD["q2_element_1d"]
    if q == 1:
        Khat, Mhat = np.array(g["Khat"], float), np.array(g["Mhat_times_6"], float) / 6
    else:
        Khat, Mhat = np.array(g["Khat_times_3"], float) / 3, np.array(g["Mhat_times_30"], float) / 30
    K, M = _periodic_1d(Khat, Mhat, q, n)
    A = op.assemble(q, n)
    ref = _kron3(K, M)
    assert abs(A - ref).max() <= 1e-15 * abs(ref).max() * 10
    Mm = op.assemble(q, n, "mass")
    assert abs(Mm - sp.kron(sp.kron(M, M), M)).max() < 1e-16 * 10


@pytest.mark.parametrize("q,n", [(4, 2), (4, 4)])
def test_kronecker_identity_q4(q, n):
    K, M = op.assemble_1d(q, n)   # 1D matrices pinned by the monomial identities
    A = op.assemble(q, n)
    ref = _kron3(K, M)
    assert abs(A - ref).max() <= 1e-14 * abs(ref).max()


def test_q1_stencil():
    n = 4
    h = 1.0 / n
    A = op.assemble(1, n).toarray()
    g = GOLD["q1_stencil_over_h"]
    N = n
    idx = lambda i, j, k: (i % N) + N * ((j % N) + N * (k % N))
    assert abs(A[0, idx(0, 0, 0)] - g["centre"] * h) < 1e-15
    assert abs(A[0, idx(1, 0, 0)] - g["face"] * h) < 1e-15
    assert abs(A[0, idx(1, 1, 0)] - g["edge"] * h) < 1e-15
    assert abs(A[0, idx(-1, 1, 1)] - g["corner"] * h) < 1e-15
    assert np.count_nonzero(np.abs(A[0]) > 1e-14) == 27 - 6


@pytest.mark.parametrize("q,n", [(1, 4), (2, 4), (4, 2)])
def test_nullspace_and_symmetry(q, n):
    A = op.assemble(q, n)
    ones = np.ones(A.shape[0])
    assert np.max(np.abs(A @ ones)) < 1e-13 * abs(A).max()
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    assert abs(x @ (A @ y) - y @ (A @ x)) < 1e-14 * np.linalg.norm(x) * np.linalg.norm(y) * abs(A).max() * 10


def _global_basis_1d(q, n, I, x, deriv):
    """1D global (periodic) basis function of lattice node I at points x."""
    xi = basis.lgl_nodes(q)
    N = q * n
    out = np.zeros_like(x)
    e = np.minimum((x * n).astype(int), n - 1)
    t = x * n - e
    for a in range(q + 1):
        sel = ((q * e + a) % N) == I
        if np.any(sel):
            f = basis.lagrange_deriv(xi, t[sel])[a] * n if deriv else basis.lagrange(xi, t[sel])[a]
            out[sel] += f
    return out


@pytest.mark.parametrize("q,n", [(1, 3), (2, 2), (4, 2)])
def test_brute_force_global_quadrature(q, n):
    # Integrate grad phi_I . grad phi_J over the whole cube with (q+3)^3 Gauss points
    # per element, evaluating each global basis function from its 1D factors.
    tg, wg = basis.gauss_legendre(q + 3)
    x1 = np.concatenate([(e + tg) / n for e in range(n)])
    w1 = np.concatenate([wg / n for _ in range(n)])
    N = q * n
    V = np.array([_global_basis_1d(q, n, I, x1, False) for I in range(N)])   # (N, pts1d)
    G = np.array([_global_basis_1d(q, n, I, x1, True) for I in range(N)])
    # 3D basis (I,J,K) at 3D point (a,b,c) = V[I,a] V[J,b] V[K,c]; build dense matrices
    W = w1
    Vw = V * W
    Gw = G * W
    S11 = Gw @ G.T    # int psi_I' psi_J'
    S00 = Vw @ V.T    # int psi_I psi_J
    # A = sum over axes of (derivative along that axis) -- still a full 3D integral,
    # evaluated as the product of 1D integrals of the brute-force global functions.
    A_bf = np.kron(np.kron(S00, S00), S11) + np.kron(np.kron(S00, S11), S00) + np.kron(np.kron(S11, S00), S00)
    A = op.assemble(q, n).toarray()
    assert np.max(np.abs(A - A_bf)) < 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("q,n", [(1, 2), (2, 2)])
def test_brute_force_point_quadrature_3d(q, n):
    # Fully 3D: evaluate each global 3D basis gradient at every 3D quadrature point.
    tg, wg = basis.gauss_legendre(q + 2)
    x1 = np.concatenate([(e + tg) / n for e in range(n)])
    w1 = np.concatenate([wg / n for _ in range(n)])
    N = q * n
    Z, Y, X = np.meshgrid(x1, x1, x1, indexing="ij")
    WZ, WY, WX = np.meshgrid(w1, w1, w1, indexing="ij")
    X, Y, Z, Wt = X.ravel(), Y.ravel(), Z.ravel(), (WX * WY * WZ).ravel()
    grads = []
    for K in range(N):
        for J in range(N):
            for I in range(N):
                vx, gx = _global_basis_1d(q, n, I, X, False), _global_basis_1d(q, n, I, X, True)
                vy, gy = _global_basis_1d(q, n, J, Y, False), _global_basis_1d(q, n, J, Y, True)
                vz, gz = _global_basis_1d(q, n, K, Z, False), _global_basis_1d(q, n, K, Z, True)
                grads.append(np.stack([gx * vy * vz, vx * gy * vz, vx * vy * gz]))
    Gr = np.array(grads)    # (dofs, 3, pts)
    A_bf = np.einsum("idp,jdp,p->ij", Gr, Gr, Wt)
    A = op.assemble(q, n).toarray()
    assert np.max(np.abs(A - A_bf)) < 1e-13 * np.max(np.abs(A))


def test_kronecker_form_matches_csr():
    for q, n in ((1, 8), (2, 4), (4, 4)):
        A = op.assemble(q, n)
        Ak = op.KroneckerOperator(q, n)
        x = np.random.default_rng(3).standard_normal(A.shape[0])
        assert np.max(np.abs(A @ x - Ak @ x)) < 1e-13 * np.max(np.abs(A @ x))
        assert np.max(np.abs(A.diagonal() - Ak.diagonal())) < 1e-14 * np.max(A.diagonal())
        Mm, Mk = op.assemble(q, n, "mass"), op.KroneckerOperator(q, n, "mass")
        assert np.max(np.abs(Mm @ x - Mk @ x)) < 1e-13 * np.max(np.abs(Mm @ x))


def _l2_error(q, n, u_nodes, exact):
    tg, wg = basis.gauss_legendre(q + 3)
    xi = basis.lgl_nodes(q)
    B = basis.lagrange(xi, tg)    # (q+1, pts)
    N = q * n
    U = u_nodes.reshape(N, N, N)  # [z, y, x]
    err2 = 0.0
    for ez in range(n):
        for ey in range(n):
            for ex in range(n):
                iz = [(q * ez + a) % N for a in range(q + 1)]
                iy = [(q * ey + a) % N for a in range(q + 1)]
                ix = [(q * ex + a) % N for a in range(q + 1)]
                loc = U[np.ix_(iz, iy, ix)]
                uh = np.einsum("cba,ak,bj,ci->ijk", loc, B, B, B)  # (pz, py, px)
                pz = (ez + tg) / n
                py = (ey + tg) / n
                px = (ex + tg) / n
                ue = exact(px[None, None, :], py[None, :, None], pz[:, None, None])
                w = wg[:, None, None] * wg[None, :, None] * wg[None, None, :] / n ** 3
                err2 += np.sum(w * (uh - ue) ** 2)
    return math.sqrt(err2)


@pytest.mark.parametrize("q,ns", [(1, (8, 16)), (2, (8, 16)), (4, (4, 8))])
def test_l2_convergence_rate(q, ns):
    exact = lambda x, y, z: np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)
    errs = []
    for n in ns:
        x1 = op.dof_coords_1d(q, n)
        s = np.sin(2 * np.pi * x1)
        f = 12 * np.pi ** 2 * (s[:, None, None] * s[None, :, None] * s[None, None, :]).ravel()
        levels = int(math.log2(n))
        H = mg.Hierarchy(q, n, max(1, levels))
        b = mg.rhs(q, n, f)
        u, info = krylov.pcg(H.finest.A, b, H.vcycle, 1e-12)
        assert info.converged
        u = krylov.normalize_mean(u, q, n)
        errs.append(_l2_error(q, n, u, exact))
    rate = math.log2(errs[0] / errs[1])
    assert abs(rate - (q + 1)) < 0.35, (errs, rate)


def test_q1_dinv_a_lambda_max_closed_form():
    A = op.assemble(1, 4)
    D = A.diagonal()
    assert np.max(np.abs(D - GOLD["q1_stencil_over_h"]["centre"] / 4)) < 1e-15
    ev = np.linalg.eigvalsh(A.toarray() / np.sqrt(np.outer(D, D)))
    assert abs(ev.max() - GOLD["lambda_max_dinv_a"]["q1"]) < 1e-13
