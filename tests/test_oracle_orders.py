"""Pins of the oracle at the paper's other orders (Section 2.3.2: 1 <= q <= 16; Table 10 uses
q = 4, 5, 6, 8) and on the single periodic element the coarsening ends with (Section 2.3.1).

What fixes them: the LGL nodes are the end points and the roots of P_q' (closed forms for
q = 3, 5, 6); the element matrices integrate monomials exactly; the assembled operator is
the Kronecker sum of its 1D matrices, symmetric, with the constants as its null space; the
L2 error of the sin solution converges at rate q + 1; the prolongation reproduces the
constants and satisfies the Galerkin identity P^T A_f P = A_c, also from one element; the
V-cycle is symmetric and positive on the complement of the constants.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import basis, multigrid as mg, operator as op, transfer

ORDERS = [3, 5, 6, 8]


def test_lgl_nodes_closed_forms_q3_q5_q6():
    # interior roots of P_q' on [-1, 1]
    cases = {
        3: [-1 / math.sqrt(5), 1 / math.sqrt(5)],
        5: sorted([s * math.sqrt(1 / 3 + t * 2 * math.sqrt(7) / 21) for s in (-1, 1) for t in (-1, 1)]),
        6: sorted([0.0] + [s * math.sqrt((15 + t * 2 * math.sqrt(15)) / 33) for s in (-1, 1) for t in (-1, 1)]),
    }
    for q, inner in cases.items():
        ref = 0.5 * (np.array([-1.0] + inner + [1.0]) + 1.0)
        assert np.max(np.abs(basis.lgl_nodes(q) - ref)) < 1e-15, q


@pytest.mark.parametrize("q", [8, 14, 16])
def test_lgl_interior_nodes_are_roots_of_the_legendre_derivative(q):
    from numpy.polynomial import legendre as L
    c = np.zeros(q + 1)
    c[q] = 1.0
    x = 2 * basis.lgl_nodes(q)[1:-1] - 1
    assert np.max(np.abs(L.legval(x, L.legder(c)))) < 1e-11 * q * q
    assert np.all(np.diff(basis.lgl_nodes(q)) > 0)


@pytest.mark.parametrize("q", ORDERS + [14, 16])
def test_element_matrices_integrate_monomials_exactly(q):
    Khat, Mhat = basis.element_matrices_1d(q)
    xi = basis.lgl_nodes(q)
    for m in range(q + 1):
        for k in range(q + 1):
            vm, vk = xi ** m, xi ** k
            kex = 0.0 if (m == 0 or k == 0) else m * k / (m + k - 1)
            mex = 1.0 / (m + k + 1)
            assert abs(vm @ Khat @ vk - kex) < 1e-12
            assert abs(vm @ Mhat @ vk - mex) < 1e-13


@pytest.mark.parametrize("q,n", [(3, 2), (5, 1), (5, 2), (6, 1), (8, 1)])
def test_operator_kronecker_null_space_symmetry(q, n):
    A = op.assemble(q, n)
    K1, M1 = op.assemble_1d(q, n)
    Ak = sp.kron(sp.kron(M1, M1), K1) + sp.kron(sp.kron(M1, K1), M1) + sp.kron(sp.kron(K1, M1), M1)
    scale = abs(A).max()
    assert abs(A - Ak).max() <= 1e-13 * scale
    assert np.max(np.abs(A @ np.ones(A.shape[0]))) <= 1e-12 * scale
    assert abs(A - A.T).max() <= 1e-14 * scale
    x = np.random.default_rng(q).standard_normal(A.shape[0])
    x -= x.mean()
    assert x @ (A @ x) > 0


@pytest.mark.parametrize("q,ns", [(3, (2, 4, 8)), (5, (1, 2, 4))])
def test_l2_convergence_rate(q, ns):
    """L2 error of -Laplace u = 12 pi^2 sss solved on the oracle's operator (Gauss rule with q + 3
    points per direction) decays like h^(q+1)."""
    errs = []
    for n in ns:
        A = op.assemble(q, n)
        M = op.assemble(q, n, "mass")
        x = op.dof_coords_1d(q, n)
        s = np.sin(2 * np.pi * x)
        f = 12 * np.pi ** 2 * np.einsum("k,j,i->kji", s, s, s).ravel()
        b = mg.project(M @ f)
        u, info = spla.cg(A, b, rtol=1e-13, atol=0.0, maxiter=20000)   # consistent singular system
        assert info == 0
        u -= u.mean()
        # L2 error by a q+3 point Gauss rule per element and direction
        t, w = basis.gauss_legendre(q + 3)
        B = basis.lagrange(basis.lgl_nodes(q), t)          # (q+1, npts)
        U = u.reshape(q * n, q * n, q * n)
        h = 1.0 / n
        err2 = 0.0
        idx = lambda e: [(q * e + a) % (q * n) for a in range(q + 1)]
        for ez in range(n):
            for ey in range(n):
                for ex in range(n):
                    Ue = U[np.ix_(idx(ez), idx(ey), idx(ex))]
                    uq = np.einsum("cz,by,ax,cba->zyx", B, B, B, Ue)
                    xs = (ex + t) * h
                    ys = (ey + t) * h
                    zs = (ez + t) * h
                    ue = np.einsum("z,y,x->zyx", np.sin(2 * np.pi * zs), np.sin(2 * np.pi * ys), np.sin(2 * np.pi * xs))
                    err2 += h ** 3 * np.einsum("z,y,x,zyx->", w, w, w, (uq - ue) ** 2)
        errs.append(math.sqrt(err2))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] >= q + 1 - 0.35, (errs, rates)


@pytest.mark.parametrize("q,n_c", [(3, 1), (3, 2), (5, 1), (6, 1), (8, 1)])
def test_prolongation_galerkin_and_constants(q, n_c):
    P = transfer.prolongation(q, n_c)
    P1 = transfer.prolongation_1d(q, n_c)
    assert np.max(np.abs(P @ np.ones(P.shape[1]) - 1.0)) < 1e-13
    assert abs(P - sp.kron(sp.kron(P1, P1), P1)).max() < 1e-14
    Af = op.assemble(q, 2 * n_c).toarray()
    Ac = op.assemble(q, n_c).toarray()
    G = (P.T @ Af @ P)
    assert np.max(np.abs(G - Ac)) < 1e-13 * np.max(np.abs(Ac)) * q


@pytest.mark.parametrize("q", [14, 16])
def test_high_orders_1d_factors(q):
    """Orders 14 and 16 (Table 7's GMG-14, Section 3's GMG-16) through the 1D factors that the
    operator and the prolongation are Kronecker products of: K symmetric with the constants as
    its null space and positive elsewhere, M symmetric positive definite with total mass 1 (the
    unit interval), P1 reproducing the constants and satisfying P1^T K_f P1 = K_c and
    P1^T M_f P1 = M_c from one coarse element (every 3D identity is a product of these)."""
    for n in (1, 2):
        K1, M1 = (m.toarray() for m in op.assemble_1d(q, n))
        N = q * n
        assert np.max(np.abs(K1 - K1.T)) <= 1e-13 * np.max(np.abs(K1))
        assert np.max(np.abs(K1 @ np.ones(N))) <= 1e-12 * np.max(np.abs(K1))
        ev = np.linalg.eigvalsh(K1)
        assert abs(ev[0]) <= 1e-10 * ev[-1] and ev[1] > 1e-6 * ev[-1]
        assert np.min(np.linalg.eigvalsh(M1)) > 0 and abs(M1.sum() - 1.0) < 1e-13
    P1 = transfer.prolongation_1d(q, 1).toarray()
    assert np.max(np.abs(P1 @ np.ones(q) - 1.0)) < 1e-12
    Kf, Mf = (m.toarray() for m in op.assemble_1d(q, 2))
    Kc, Mc = (m.toarray() for m in op.assemble_1d(q, 1))
    assert np.max(np.abs(P1.T @ Kf @ P1 - Kc)) < 1e-11 * np.max(np.abs(Kc))
    assert np.max(np.abs(P1.T @ Mf @ P1 - Mc)) < 1e-13


def test_single_element_prolongation_sums_the_identified_end_nodes():
    """On one periodic element the coarse node 0 is local nodes 0 and q together: its
    prolongation row at a fine node is phi_0 + phi_q there."""
    q = 5
    P1 = transfer.prolongation_1d(q, 1).toarray()     # (2q, q)
    xi = basis.lgl_nodes(q)
    for b in range(2 * q):
        e, a = divmod(b, q)
        t = (e + xi[a]) / 2
        phi = basis.lagrange(xi, [t])[:, 0]
        assert abs(P1[b, 0] - (phi[0] + phi[q])) < 1e-14
        assert np.max(np.abs(P1[b, 1:] - phi[1:q])) < 1e-14


@pytest.mark.parametrize("q,n,levels", [(3, 4, 3), (5, 2, 2), (6, 2, 2)])
def test_vcycle_symmetric_positive_down_to_one_element(q, n, levels):
    H = mg.Hierarchy(q, n, levels, mg.Options(seed=1))
    assert H.levels[0].n == n >> (levels - 1)
    size = H.finest.size
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(size), rng.standard_normal(size)
    x -= x.mean()
    y -= y.mean()
    vx, vy = H.vcycle(x), H.vcycle(y)
    assert abs(x @ vy - y @ vx) <= 1e-11 * abs(x @ vy)
    assert x @ vx > 0
