"""Multigrid hierarchy and V-cycle for the periodic Q_q Poisson problem.

Paper: Algorithm 2.1 (V-cycle: pre-smooth, residual, restrict, recurse,
correct, post-smooth) with a direct solve on the coarsest level (Section 2.3);
Section 2.3.1 (every coarse element is the parent of 8 fine ones: on a uniform
mesh the hierarchy halves n per level); Section 2.3.4 (R = P^T, coarse
operators rediscretized on nested spaces); Section 2.3.3 (smoother).

Readings:
  * Zero initial guess on every level; the same smoother, nu applications of
    the degree-3 Chebyshev polynomial, before and after the correction, so the
    cycle is symmetric (the paper's own runs use an unsymmetric V(2,1) inside CG).
  * The coarse direct solve (SuperLU in the paper) is the pseudo-inverse on the
    complement of the constants: x = (A_0 + 1 1^T / N_0)^-1 (b - mean(b) 1),
    which is the mean-zero solution of A_0 x = b - mean(b) 1.
  * Level l has n_l = n / 2^(L-1-l) elements per direction; level 0 is coarsest.
    The recursion may go down to a single periodic element (n_0 = 1): the paper
    stops coarsening when no further coarsening is possible (Section 2.3.1).

Pins (tests/test_oracle_multigrid.py): coarse solve against numpy's
pseudo-inverse; V-cycle symmetry and positive definiteness on 1-perp; a
two-level cycle against its dense-matrix expression.
"""
import numpy as np

from . import operator as op
from .transfer import MatrixProlongation, KroneckerProlongation
from .smoother import lanczos_lambda_max, chebyshev, jacobi
from .rng import lanczos_start


class Options:
    def __init__(self, cheb_degree=3, nu_pre=2, nu_post=2, cheb_lo=0.1, cheb_hi=1.1,
                 lanczos_steps=10, seed=0, lambda_override=0.0, smoother="chebyshev",
                 jacobi_omega=2.0 / 3.0):
        self.cheb_degree = cheb_degree
        self.nu_pre = nu_pre
        self.nu_post = nu_post
        self.cheb_lo = cheb_lo
        self.cheb_hi = cheb_hi
        self.lanczos_steps = lanczos_steps
        self.seed = seed
        self.lambda_override = lambda_override
        self.smoother = smoother
        self.jacobi_omega = jacobi_omega


class Level:
    def __init__(self, q, n, index, opts, form):
        self.q, self.n, self.index = q, n, index
        self.N = q * n
        self.size = self.N ** 3
        self.A = op.operator(q, n, form)
        self.D = self.A.diagonal()
        self.dinv = 1.0 / self.D
        if opts.lambda_override > 0:
            self.lam = opts.lambda_override
        else:
            v0 = lanczos_start(opts.seed, index, self.size)
            self.lam = lanczos_lambda_max(self.A, self.D, v0, min(opts.lanczos_steps, self.size - 1))
        self.alpha = opts.cheb_lo * self.lam
        self.beta = opts.cheb_hi * self.lam
        self.transfer = None   # prolongation from level index-1 to this level


class Hierarchy:
    """Levels 0 (coarsest) .. L-1 (finest) for order q and n elements per direction."""

    def __init__(self, q, n, levels, opts=None, form="csr"):
        if opts is None:
            opts = Options()
        if n < 1 or (n & (n - 1)) != 0:
            raise ValueError("n must be a power of two")
        if levels < 1 or (n >> (levels - 1)) < 1:
            raise ValueError("too many levels")
        self.q, self.n, self.L, self.opts = q, n, levels, opts
        self.levels = []
        for l in range(levels):
            nl = n >> (levels - 1 - l)
            lev = Level(q, nl, l, opts, form)
            if l > 0:
                lev.transfer = (MatrixProlongation(q, nl // 2) if form == "csr"
                                else KroneckerProlongation(q, nl // 2))
            self.levels.append(lev)
        A0 = self.levels[0].A
        A0d = A0.toarray() if hasattr(A0, "toarray") else _dense(A0)
        N0 = A0d.shape[0]
        self.coarse_inv = np.linalg.inv(A0d + np.ones((N0, N0)) / N0)

    @property
    def finest(self):
        return self.levels[-1]

    def coarse_solve(self, b):
        """Mean-zero solution of A_0 x = b - mean(b) (Section 2.3, direct coarsest solve)."""
        return self.coarse_inv @ (b - np.mean(b))

    def smooth(self, lev, b, u, nu):
        o = self.opts
        for _ in range(nu):
            if o.smoother == "jacobi":
                u = jacobi(lev.A, lev.dinv, b, u, o.jacobi_omega, 1)
            else:
                u = chebyshev(lev.A, lev.dinv, b, u, lev.alpha, lev.beta, o.cheb_degree)
        return u

    def vcycle(self, b, l=None):
        """Algorithm 2.1 on level l (default: finest) with zero initial guess."""
        if l is None:
            l = self.L - 1
        if l == 0:
            return self.coarse_solve(b)
        lev = self.levels[l]
        u = np.zeros_like(b)
        u = self.smooth(lev, b, u, self.opts.nu_pre)          # pre-smooth
        r = b - lev.A @ u                                      # residual
        bc = lev.transfer.restrict(r)                          # restrict, R = P^T
        ec = self.vcycle(bc, l - 1)                            # recurse
        u = u + lev.transfer.prolong(ec)                       # correct
        u = self.smooth(lev, b, u, self.opts.nu_post)         # post-smooth
        return u


def _dense(Aop):
    n = Aop.shape[0]
    out = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        out[:, j] = Aop @ e
        e[j] = 0.0
    return out


def project(v):
    """l2 projection onto the complement of the constants: v - mean(v) 1."""
    return v - np.mean(v)


def rhs(q, n, f_nodal, form="csr"):
    """Load vector b = M f_I, projected onto 1-perp (reading: the paper does not
    say how f is discretized; f_I is f at the DoFs, M the consistent mass)."""
    M = op.mass(q, n, form)
    return project(M @ f_nodal)
