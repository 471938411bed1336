"""LGL nodal basis and Gauss-Legendre quadrature on the unit interval.

Paper: Section 2.3.2 -- the GMG discretization uses Legendre-Gauss-Lobatto (LGL)
nodal basis functions of order q, tensorized on hexahedra.

All arrays are float64.  The reference element is [0, 1]; an element of width h
maps t -> x = x0 + h t.

Pins (tests/test_oracle_basis.py): closed-form LGL nodes for q = 1, 2, 4;
Lagrange cardinality; 1D element matrices reproduce the exact integrals of
monomials; textbook Q1 and Q2 element matrices.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def lgl_nodes(q):
    """The q+1 LGL nodes on [0, 1] (Section 2.3.2).

    They are the end points of [-1, 1] together with the roots of P_q', mapped
    affinely onto [0, 1], in increasing order.  The interior roots are polished
    by Newton's method on P_q' so that they are accurate to rounding.
    """
    if q < 1:
        raise ValueError("order q must be >= 1")
    interior = np.zeros(0)
    if q >= 2:
        c = np.zeros(q + 1)
        c[q] = 1.0
        d1 = npleg.legder(c)
        d2 = npleg.legder(d1)
        r = np.sort(npleg.legroots(d1).real)
        for _ in range(4):
            r = r - npleg.legval(r, d1) / npleg.legval(r, d2)
        interior = r
    x = np.concatenate([[-1.0], interior, [1.0]])
    return 0.5 * (x + 1.0)


def gauss_legendre(m):
    """m-point Gauss-Legendre rule on [0, 1]: points and weights (exact to degree 2m-1)."""
    x, w = npleg.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(nodes, t):
    """phi[a, p] = prod_{b != a} (t_p - x_b) / (x_a - x_b): the nodal basis at points t."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    m = len(nodes)
    phi = np.ones((m, len(t)))
    for a in range(m):
        for b in range(m):
            if b != a:
                phi[a] *= (t - nodes[b]) / (nodes[a] - nodes[b])
    return phi


def lagrange_deriv(nodes, t):
    """dphi[a, p] = d/dt phi_a(t_p), by the product rule applied to lagrange()."""
    nodes = np.asarray(nodes, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    m = len(nodes)
    dphi = np.zeros((m, len(t)))
    for a in range(m):
        for k in range(m):
            if k == a:
                continue
            term = np.full(len(t), 1.0 / (nodes[a] - nodes[k]))
            for b in range(m):
                if b != a and b != k:
                    term = term * (t - nodes[b]) / (nodes[a] - nodes[b])
            dphi[a] += term
    return dphi


def element_matrices_1d(q):
    """Reference 1D stiffness and mass on [0, 1] for the order-q LGL basis.

    Khat[a, b] = int_0^1 phi_a' phi_b' dt,  Mhat[a, b] = int_0^1 phi_a phi_b dt,
    evaluated with q+1 Gauss-Legendre points (exact: the integrands have degree
    at most 2q).  An element of width h has K = Khat / h and M = h Mhat.
    """
    xi = lgl_nodes(q)
    t, w = gauss_legendre(q + 1)
    B = lagrange(xi, t)
    D = lagrange_deriv(xi, t)
    Khat = (D * w) @ D.T
    Mhat = (B * w) @ B.T
    return Khat, Mhat
