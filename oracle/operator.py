"""Assembled operator of the periodic Q_q finite-element Laplacian.

Paper: eq. (1.1) -- -Laplace(u) = f, u periodic on the unit cube; Section 2.3.2 --
continuous Galerkin discretization with the tensorized LGL nodal basis of order q
on a uniform hexahedral mesh; Section 2.3.6 -- unit cube, periodic boundaries,
constant element metric.

Definitions used here (the paper does not name its quadrature rule; the reading
taken is exact Galerkin integration):
  A_ij = int_[0,1]^3 grad(phi_i) . grad(phi_j) dx,   M_ij = int phi_i phi_j dx,
over the continuous periodic Q_q space with n elements per direction.  Lattice
nodes per direction: N = q n; lattice node I sits at x = (e + xi_a) / n with
e = I div q, a = I mod q.  Nodes at x = 0 and x = 1 are the same node.  Global
index of lattice node (I, J, K) is I + N (J + N K): x fastest.

Element matrices are integrated in 3D with (q+1)^3 Gauss points, without using
their tensor structure; the global matrix is the sum of element matrices
scattered through the periodic element-to-node map (CSR, int64 indices).
The Kronecker form (three 1D passes) is a second route to the same matrix,
used only where the CSR matrix would not fit in host memory; the tests check
the two against each other.

Pins (tests/test_oracle_operator.py): Kronecker identity against textbook 1D
matrices; Q1 stencil values; A 1 = 0; symmetry; brute-force global quadrature
on 2^3 / 3^3 meshes; L2 convergence at rate q+1; the Q1 Fourier eigenvalue.
"""
import numpy as np
import scipy.sparse as sp

from .basis import lgl_nodes, gauss_legendre, lagrange, lagrange_deriv, element_matrices_1d


def lattice_size(q, n):
    return q * n


def dof_coords_1d(q, n):
    """Coordinates of the N = q n lattice nodes along one axis, in [0, 1)."""
    xi = lgl_nodes(q)
    e = np.repeat(np.arange(n), q)
    a = np.tile(np.arange(q), n)
    return (e + xi[a]) / n


def dof_coords(q, n):
    """(N^3, 3) coordinates of all DoFs, x fastest."""
    x = dof_coords_1d(q, n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def element_matrices_3d(q, n):
    """Element stiffness and mass of one cube of width h = 1/n.

    Local node (a, b, c) has local index a + (q+1)(b + (q+1)c).  Each basis
    function is phi_a(t1) phi_b(t2) phi_c(t3) and its gradient is evaluated at
    each of the (q+1)^3 Gauss points; then
        Ke = h^3 sum_p w_p grad phi_i(p) . grad phi_j(p)   (grad = grad_t / h),
        Me = h^3 sum_p w_p phi_i(p) phi_j(p).
    """
    h = 1.0 / n
    xi = lgl_nodes(q)
    t, w = gauss_legendre(q + 1)
    B = lagrange(xi, t)          # (q+1, npts)
    D = lagrange_deriv(xi, t)
    m1 = q + 1
    # node index -> (a, b, c); point index -> (i, j, k); both with first fastest
    a, b, c = np.meshgrid(np.arange(m1), np.arange(m1), np.arange(m1), indexing="ij")
    a, b, c = a.transpose(2, 1, 0).ravel(), b.transpose(2, 1, 0).ravel(), c.transpose(2, 1, 0).ravel()
    i, j, k = a, b, c  # same enumeration for points
    W = w[i] * w[j] * w[k]                                  # (npts,)
    phi = B[a][:, i] * B[b][:, j] * B[c][:, k]              # (nodes, npts)
    gx = D[a][:, i] * B[b][:, j] * B[c][:, k] / h
    gy = B[a][:, i] * D[b][:, j] * B[c][:, k] / h
    gz = B[a][:, i] * B[b][:, j] * D[c][:, k] / h
    vol = h ** 3
    Ke = vol * ((gx * W) @ gx.T + (gy * W) @ gy.T + (gz * W) @ gz.T)
    Me = vol * ((phi * W) @ phi.T)
    return Ke, Me


def element_dofs(q, n):
    """(n^3, (q+1)^3) periodic element-to-node map, elements with x fastest."""
    N = q * n
    m1 = q + 1
    ez, ey, ex = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    la, lb, lc = np.meshgrid(np.arange(m1), np.arange(m1), np.arange(m1), indexing="ij")
    la, lb, lc = la.transpose(2, 1, 0).ravel(), lb.transpose(2, 1, 0).ravel(), lc.transpose(2, 1, 0).ravel()
    I = (q * ex[:, None] + la[None, :]) % N
    J = (q * ey[:, None] + lb[None, :]) % N
    K = (q * ez[:, None] + lc[None, :]) % N
    return (I + N * (J + N * K)).astype(np.int64)


def assemble(q, n, which="stiffness"):
    """Global periodic CSR matrix (stiffness or mass), duplicates summed."""
    Ke, Me = element_matrices_3d(q, n)
    Ae = Ke if which == "stiffness" else Me
    dofs = element_dofs(q, n)
    E, m = dofs.shape
    rows = np.repeat(dofs, m, axis=1).ravel()
    cols = np.tile(dofs, (1, m)).ravel()
    vals = np.tile(Ae.ravel(), E)
    Nt = (q * n) ** 3
    A = sp.coo_matrix((vals, (rows, cols)), shape=(Nt, Nt)).tocsr()
    A.sum_duplicates()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int64)
    return A


def assemble_1d(q, n):
    """Periodic 1D stiffness K1 and mass M1 (N x N, N = q n) on [0, 1)."""
    Khat, Mhat = element_matrices_1d(q)
    h = 1.0 / n
    N = q * n
    rows, cols, kv, mv = [], [], [], []
    for e in range(n):
        idx = [(q * e + a) % N for a in range(q + 1)]
        for a in range(q + 1):
            for b in range(q + 1):
                rows.append(idx[a])
                cols.append(idx[b])
                kv.append(Khat[a, b] / h)
                mv.append(Mhat[a, b] * h)
    K1 = sp.coo_matrix((kv, (rows, cols)), shape=(N, N)).tocsr()
    M1 = sp.coo_matrix((mv, (rows, cols)), shape=(N, N)).tocsr()
    return K1, M1


def apply_along(mat, X, axis):
    """Apply a sparse (M x N) matrix along one axis (of length N) of the 3D array X[z, y, x]."""
    Xm = np.moveaxis(X, axis, -1)
    shp = Xm.shape
    Y = (mat @ Xm.reshape(-1, shp[-1]).T).T.reshape(shp[:-1] + (mat.shape[0],))
    return np.moveaxis(Y, -1, axis)


class KroneckerOperator:
    """A = K (x) M (x) M + M (x) K (x) M + M (x) M (x) K applied by 1D passes.

    Same matrix as assemble(q, n); used where the CSR matrix exceeds host memory.
    ``which`` selects the stiffness or the mass (M (x) M (x) M).
    """

    def __init__(self, q, n, which="stiffness"):
        self.q, self.n, self.N = q, n, q * n
        self.K1, self.M1 = assemble_1d(q, n)
        self.which = which
        self.shape = (self.N ** 3, self.N ** 3)

    def __matmul__(self, x):
        N = self.N
        X = np.asarray(x, dtype=np.float64).reshape(N, N, N)  # [z, y, x]
        K1, M1 = self.K1, self.M1
        if self.which == "mass":
            Y = apply_along(M1, apply_along(M1, apply_along(M1, X, 2), 1), 0)
            return Y.ravel()
        Y = apply_along(K1, apply_along(M1, apply_along(M1, X, 0), 1), 2)
        Y += apply_along(M1, apply_along(K1, apply_along(M1, X, 0), 1), 2)
        Y += apply_along(M1, apply_along(M1, apply_along(K1, X, 0), 1), 2)
        return Y.ravel()

    def diagonal(self):
        N = self.N
        kd, md = self.K1.diagonal(), self.M1.diagonal()
        if self.which == "mass":
            return np.einsum("k,j,i->kji", md, md, md).ravel()
        return (np.einsum("k,j,i->kji", md, md, kd) + np.einsum("k,j,i->kji", md, kd, md)
                + np.einsum("k,j,i->kji", kd, md, md)).ravel()


def operator(q, n, form="csr"):
    """The stiffness matrix in CSR form or in Kronecker form."""
    return assemble(q, n) if form == "csr" else KroneckerOperator(q, n)


def mass(q, n, form="csr"):
    return assemble(q, n, "mass") if form == "csr" else KroneckerOperator(q, n, "mass")


def diagonal(A):
    return A.diagonal()
