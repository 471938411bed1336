"""Intergrid transfers between nested uniform periodic meshes.

Paper: Section 2.3.4, eqs. (2.1)-(2.2): the coarse space is a subspace of the
fine space, so the prolongation has entries P(i, j) = phi_j^{k-1}(p_i), the
coarse shape function j evaluated at fine node p_i; the restriction is R = P^T.

The coarse mesh has n_c >= 1 elements per direction, the fine mesh n_f = 2 n_c,
both of order q.  P is built by visiting each coarse element and, in it, each fine
node of its half-open extent [E, E+1) (so every fine node once), evaluating the
coarse element's tensor-product basis (q+1 LGL nodes per direction) there, and
adding the value into the entry of the global coarse node each local node is.
Continuity makes the half-open choice immaterial.  On a single periodic element
(n_c = 1) the element's two end nodes are one global node, whose basis function is
the sum of the two local ones; the sum is what the adding gives (for n_c >= 2 no
two local nodes of an element share a global node).

Pins (tests/test_oracle_transfer.py): P 1 = 1; P equals the Kronecker cube of
its 1D version and reproduces polynomials of degree <= q locally; the Galerkin
identity P^T A_f P = A_c; the Q2 quarter-point rows (3/8, 3/4, -1/8).
"""
import numpy as np
import scipy.sparse as sp

from .basis import lgl_nodes, lagrange


def _child_coords(q):
    """Reference coordinate in the coarse element of fine node b = 0 .. 2q of its closure."""
    xi = lgl_nodes(q)
    t = np.empty(2 * q + 1)
    for b in range(2 * q):
        e, a = divmod(b, q)
        t[b] = (e + xi[a]) / 2.0
    t[2 * q] = 1.0
    return t


def prolongation_1d(q, n_c):
    """1D periodic P1 (N_f x N_c) by eq. (2.2)."""
    Nf, Nc = 2 * q * n_c, q * n_c
    xi = lgl_nodes(q)
    phi = lagrange(xi, _child_coords(q))   # (q+1, 2q+1)
    rows, cols, vals = [], [], []
    for E in range(n_c):
        for b in range(2 * q):                 # the half-open extent: each fine node once
            for a in range(q + 1):
                v = phi[a, b]
                if abs(v) < 1e-15:
                    continue
                rows.append((2 * q * E + b) % Nf)
                cols.append((q * E + a) % Nc)
                vals.append(v)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(Nf, Nc)).tocsr()   # duplicates (n_c = 1) summed
    P.sum_duplicates()
    return P


def prolongation(q, n_c):
    """3D periodic P (N_f^3 x N_c^3), P(i, j) = phi_j^coarse(p_i), eq. (2.2)."""
    Nf, Nc = 2 * q * n_c, q * n_c
    xi = lgl_nodes(q)
    phi = lagrange(xi, _child_coords(q))   # phi[a, b]: coarse 1D node a at child node b
    m = 2 * q
    # fine nodes of the element's half-open extent (bx, by, bz) and coarse element nodes (a1, a2, a3)
    bx, by, bz = [g.ravel() for g in np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")]
    a1, a2, a3 = [g.ravel() for g in np.meshgrid(np.arange(q + 1), np.arange(q + 1), np.arange(q + 1), indexing="ij")]
    val = phi[a1][:, bx] * phi[a2][:, by] * phi[a3][:, bz]          # (coarse local, fine local)
    keep = np.abs(val) > 1e-15
    ci, fi = np.nonzero(keep)
    v = val[ci, fi]
    rows, cols, vals = [], [], []
    for Ez in range(n_c):
        for Ey in range(n_c):
            for Ex in range(n_c):
                I = (2 * q * Ex + bx[fi]) % Nf
                J = (2 * q * Ey + by[fi]) % Nf
                K = (2 * q * Ez + bz[fi]) % Nf
                cI = (q * Ex + a1[ci]) % Nc
                cJ = (q * Ey + a2[ci]) % Nc
                cK = (q * Ez + a3[ci]) % Nc
                rows.append(I + Nf * (J + Nf * K))
                cols.append(cI + Nc * (cJ + Nc * cK))
                vals.append(v)
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Nf ** 3, Nc ** 3)).tocsr()      # duplicates (n_c = 1) summed
    P.sum_duplicates()
    return P


class KroneckerProlongation:
    """P = P1 (x) P1 (x) P1 applied by 1D passes (same matrix as prolongation())."""

    def __init__(self, q, n_c):
        self.P1 = prolongation_1d(q, n_c)
        self.Nc = q * n_c
        self.Nf = 2 * q * n_c

    def prolong(self, xc):
        from .operator import apply_along
        X = np.asarray(xc, dtype=np.float64).reshape(self.Nc, self.Nc, self.Nc)
        for ax in (2, 1, 0):
            X = apply_along(self.P1, X, ax)
        return X.ravel()

    def restrict(self, xf):
        from .operator import apply_along
        X = np.asarray(xf, dtype=np.float64).reshape(self.Nf, self.Nf, self.Nf)
        PT = self.P1.T.tocsr()
        for ax in (2, 1, 0):
            X = apply_along(PT, X, ax)
        return X.ravel()


class MatrixProlongation:
    def __init__(self, q, n_c):
        self.P = prolongation(q, n_c)
        self.PT = self.P.T.tocsr()

    def prolong(self, xc):
        return self.P @ xc

    def restrict(self, xf):
        return self.PT @ xf
