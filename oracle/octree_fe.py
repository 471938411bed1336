"""Continuous Q_q finite elements on a periodic 2:1-balanced octree (oracle, test infrastructure).

Paper: Section 2.3 (continuous Galerkin discretization on octree meshes;
Section 2.3.1, meshing turns the octree into element-to-node data), Section 4
(nodes that are not independent degrees of freedom -- hanging nodes -- raise
the cost of the mesh lookup), Section 2.3.4 with eqs. (2.1)-(2.2) (the coarse
space is a subspace of the fine one and P(i, j) = phi_j^{k-1}(p_i), R = P^T).
The method for hanging nodes is in references the paper cites but does not
reproduce; the reading here is the standard conforming one.

Readings:
  * Node lattice: positions in units of 2^-(DMAX+1) ("ticks"); a leaf of level l
    has width 2 s ticks (s = 2^(DMAX-l)) and its order-q LGL nodes at anchor +
    2 s xi_a (q = 1, 2 only: their LGL nodes are multiples of 1/2).
  * A node position p is an independent degree of freedom iff it is a node of
    every leaf whose closed box contains it (equivalently, of the coarsest such
    leaf).  Otherwise it is hanging, and its value is the coarsest containing
    leaf's Q_q interpolant at p: u(p) = sum_j phi_j(p) u(node_j), recursively
    resolved when node_j hangs itself.  The discrete space is then the
    continuous piecewise-Q_q functions on the leaves.
  * A = C^T blockdiag(A_e) C with C the (element node) x (DoF) constraint
    matrix and A_e the element stiffness of width 2^-l; M likewise.
  * DoFs are numbered by increasing x + T (y + T z) of their tick coordinates
    (T = 2^(DMAX+1)), which for a uniform octree is the lattice order i + N(j + N k).
  * P between nested octrees: row p of P is the coarse interpolant at p, taken
    in the coarse leaf that holds the tick cell [p, p+1)^3.

Pins (tests/test_oracle_octree.py): continuity of random FE functions across
every face between two leaves; a uniform octree reproduces the uniform
operator exactly; A 1 = 0, symmetry and a one-dimensional null space; hanging
weights equal the rows of the 1D prolongation; nestedness (P x_c agrees with
the coarse function at random points) and the Galerkin identity P^T A_f P = A_c;
L2 convergence at rate q+1 on graded octrees.

Not a product path: only the tests, the smoke check and the CPU baseline use it.
"""
import numpy as np
import scipy.sparse as sp

from .basis import lgl_nodes, lagrange
from .octree import DMAX, UNITS, Locator, size
from .operator import element_matrices_3d
from . import multigrid as mg
from .rng import lanczos_start
from .smoother import lanczos_lambda_max

TICKS = 2 * UNITS


def node_ticks(q):
    """Node offsets in units of s (half the leaf width in ticks) : 2 xi_a."""
    xi = lgl_nodes(q)
    t = np.rint(2.0 * xi).astype(int)
    assert np.allclose(2.0 * xi, t), "only orders whose LGL nodes are multiples of 1/2"
    return t


class OctreeSpace:
    """Element-node constraint map, DoF numbering and assembled operators of one octree."""

    def __init__(self, leaves, q):
        self.q = q
        self.leaves = list(leaves)
        self.E = len(self.leaves)
        self.m1 = q + 1
        self.loc = Locator(self.leaves)
        off = node_ticks(q)
        self.off = off
        m1 = self.m1
        # element node positions (E, m1^3, 3) in ticks, local index a + m1 (b + m1 c)
        pos = np.zeros((self.E, m1 ** 3, 3), dtype=np.int64)
        for e, (l, x, y, z) in enumerate(self.leaves):
            s = size(l)
            for c in range(m1):
                for b in range(m1):
                    for a in range(m1):
                        pos[e, a + m1 * (b + m1 * c)] = ((2 * x + s * off[a]) % TICKS,
                                                         (2 * y + s * off[b]) % TICKS,
                                                         (2 * z + s * off[c]) % TICKS)
        self.pos = pos
        points = {tuple(p) for p in pos.reshape(-1, 3)}
        self.hanging_src = {}
        indep = []
        for p in points:
            E = self.coarsest_containing(p)
            if self.is_node(E, p):
                indep.append(p)
            else:
                self.hanging_src[p] = E
        indep.sort(key=lambda p: p[0] + TICKS * (p[1] + TICKS * p[2]))
        self.dof = {p: i for i, p in enumerate(indep)}
        self.points = np.array(indep, dtype=np.int64).reshape(-1, 3)
        self.ndof = len(indep)
        self._memo = {}
        rows, cols, vals = [], [], []
        for e in range(self.E):
            for a in range(m1 ** 3):
                for k, w in self.expand(tuple(pos[e, a])).items():
                    rows.append(e * m1 ** 3 + a)
                    cols.append(k)
                    vals.append(w)
        self.C = sp.csr_matrix((vals, (rows, cols)), shape=(self.E * m1 ** 3, self.ndof))
        self._A = None
        self._M = None

    # -- geometry
    def containing(self, p):
        """Leaves whose closed box holds tick point p (at most 8, no repeats)."""
        out = []
        for dz in (-1, 0):
            for dy in (-1, 0):
                for dx in (-1, 0):
                    o = self.loc.find((p[0] + dx) // 2, (p[1] + dy) // 2, (p[2] + dz) // 2)
                    if o not in out:
                        out.append(o)
        return out

    def coarsest_containing(self, p):
        cands = self.containing(p)
        lmin = min(o[0] for o in cands)
        from .octree import morton
        return min((o for o in cands if o[0] == lmin), key=lambda o: morton(o[1], o[2], o[3]))

    def local(self, o, p):
        """Tick offsets of p from leaf o's anchor, in [0, 2 s] per axis."""
        l, x, y, z = o
        t = tuple((pk - 2 * ak) % TICKS for pk, ak in zip(p, (x, y, z)))
        assert all(0 <= tk <= 2 * size(l) for tk in t)
        return t

    def is_node(self, o, p):
        s = size(o[0])
        return all(tk % s == 0 and (tk // s) in set(self.off.tolist()) for tk in self.local(o, p))

    def basis_at(self, o, p):
        """phi_a(p) for the m1^3 local nodes of leaf o (tensor-product LGL Lagrange)."""
        s = size(o[0])
        t = np.array(self.local(o, p), dtype=np.float64) / (2.0 * s)
        xi = lgl_nodes(self.q)
        B = lagrange(xi, t)  # (m1, 3)
        m1 = self.m1
        phi = np.zeros(m1 ** 3)
        for c in range(m1):
            for b in range(m1):
                for a in range(m1):
                    phi[a + m1 * (b + m1 * c)] = B[a, 0] * B[b, 1] * B[c, 2]
        return phi

    def leaf_index(self):
        if not hasattr(self, "_lidx"):
            self._lidx = {o: e for e, o in enumerate(self.leaves)}
        return self._lidx

    def expand(self, p):
        """{dof: weight} of the value at node position p."""
        if p in self.dof:
            return {self.dof[p]: 1.0}
        if p in self._memo:
            return self._memo[p]
        o = self.hanging_src[p]
        e = self.leaf_index()[o]
        phi = self.basis_at(o, p)
        out = {}
        for a in np.nonzero(phi)[0]:
            for k, w in self.expand(tuple(self.pos[e, a])).items():
                out[k] = out.get(k, 0.0) + phi[a] * w
        out = {k: w for k, w in out.items() if w != 0.0}
        self._memo[p] = out
        return out

    # -- operators
    def _assemble(self, which):
        blocks = []
        cache = {}
        for l, *_ in self.leaves:
            if l not in cache:
                Ke, Me = element_matrices_3d(self.q, 1 << l)
                cache[l] = sp.csr_matrix(Ke if which == 0 else Me)
            blocks.append(cache[l])
        Ahat = sp.block_diag(blocks, format="csr")
        A = (self.C.T @ Ahat @ self.C).tocsr()
        A.sum_duplicates()
        return A

    @property
    def A(self):
        if self._A is None:
            self._A = self._assemble(0)
        return self._A

    @property
    def M(self):
        if self._M is None:
            self._M = self._assemble(1)
        return self._M

    def coords(self):
        """(ndof, 3) DoF coordinates in [0, 1)."""
        return self.points.astype(np.float64) / TICKS

    def evaluate(self, x, pts):
        """FE function with DoF vector x at points (P, 3) in [0, 1) (leaf holding the point)."""
        m1 = self.m1
        ue = (self.C @ x).reshape(self.E, m1 ** 3)
        lidx = self.leaf_index()
        out = np.zeros(len(pts))
        for i, pt in enumerate(pts):
            # the leaf holding the unit cell of the point (a point on a face picks the upper side)
            cell = [int(np.floor(c * UNITS)) % UNITS for c in pt]
            o = self.loc.find(*cell)
            l, ax, ay, az = o
            h = 1.0 / (1 << l)
            t = [((pt[k] - (ax, ay, az)[k] / UNITS) % 1.0) / h for k in range(3)]
            B = lagrange(lgl_nodes(self.q), np.array(t))
            phi = np.einsum("a,b,c->cba", B[:, 0], B[:, 1], B[:, 2]).ravel()
            out[i] = phi @ ue[lidx[o]]
        return out


def prolongation(coarse, fine):
    """P (fine ndof x coarse ndof): coarse interpolant at every fine DoF position (eq. 2.2)."""
    rows, cols, vals = [], [], []
    lidx = coarse.leaf_index()
    m1 = coarse.m1
    Cc = coarse.C
    for i, p in enumerate(map(tuple, fine.points)):
        o = coarse.loc.find(p[0] // 2, p[1] // 2, p[2] // 2)
        e = lidx[o]
        phi = coarse.basis_at(o, p)
        row = {}
        for a in np.nonzero(phi)[0]:
            r = e * m1 ** 3 + a
            for k, w in zip(Cc.indices[Cc.indptr[r]:Cc.indptr[r + 1]], Cc.data[Cc.indptr[r]:Cc.indptr[r + 1]]):
                row[k] = row.get(k, 0.0) + phi[a] * w
        for k, w in row.items():
            if w != 0.0:
                rows.append(i)
                cols.append(k)
                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(fine.ndof, coarse.ndof))


class _Transfer:
    def __init__(self, P):
        self.P = P
        self.PT = P.T.tocsr()

    def prolong(self, xc):
        return self.P @ xc

    def restrict(self, xf):
        return self.PT @ xf


class _OctLevel:
    def __init__(self, space, index, opts):
        self.space = space
        self.index = index
        self.size = space.ndof
        self.A = space.A
        self.D = self.A.diagonal()
        self.dinv = 1.0 / self.D
        if opts.lambda_override > 0:
            self.lam = opts.lambda_override
        else:
            v0 = lanczos_start(opts.seed, index, self.size)
            self.lam = lanczos_lambda_max(self.A, self.D, v0, min(opts.lanczos_steps, self.size - 1))
        self.alpha = opts.cheb_lo * self.lam
        self.beta = opts.cheb_hi * self.lam
        self.transfer = None


class OctreeHierarchy(mg.Hierarchy):
    """Algorithm 2.1 on the octree hierarchy: trees[0] coarsest .. trees[-1] finest."""

    def __init__(self, trees, q, opts=None):
        if opts is None:
            opts = mg.Options()
        self.q, self.opts = q, opts
        self.L = len(trees)
        self.spaces = [OctreeSpace(t, q) for t in trees]
        self.levels = []
        for l, S in enumerate(self.spaces):
            lev = _OctLevel(S, l, opts)
            if l > 0:
                lev.transfer = _Transfer(prolongation(self.spaces[l - 1], S))
            self.levels.append(lev)
        A0 = self.levels[0].A.toarray()
        N0 = A0.shape[0]
        self.coarse_inv = np.linalg.inv(A0 + np.ones((N0, N0)) / N0)


def rhs(space, f_nodal):
    """Load vector b = M f_I projected onto 1-perp (as on uniform meshes)."""
    return mg.project(space.M @ f_nodal)


def normalize_mean(space, u):
    """Shift u by a constant so that its integral vanishes: 1^T M u = 0."""
    w = space.M @ np.ones(space.ndof)
    return u - (w @ u) / w.sum()
