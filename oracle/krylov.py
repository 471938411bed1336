"""CG and flexible CG, each preconditioned by one multigrid V-cycle.

Paper: Section 2.3 -- every multigrid run is CG preconditioned by a single
V-cycle; Section 3 -- the relative residual is driven to a fixed tolerance.

Readings (the paper does not define the norm or the null-space handling):
  * Relative residual = ||b - A u||_2 / ||b||_2 with b the projected load.
  * r and z are projected onto 1-perp every iteration (periodic null space).
  * The recursive residual triggers the stop; the true residual b - A u is
    then recomputed, and if it is above tolerance it replaces r and the
    iteration restarts from it (direction reset to the preconditioned residual).
  * Flexible CG is Notay's FCG truncated to one direction, FCG(1):
    beta = -<z_{k+1}, A p_k> / <p_k, A p_k>, alpha = <p_k, r_k> / <p_k, A p_k>.
    With a fixed SPD preconditioner it reproduces the CG iterates.

Pins (tests/test_oracle_krylov.py): FCG(1) == PCG for a fixed SPD V; plain CG
terminates in at most (number of distinct eigenvalues) steps; the Q1 discrete
closed-form solution of the sin source.
"""
import numpy as np

from .multigrid import project


class SolveInfo:
    def __init__(self):
        self.iters = 0
        self.converged = False
        self.rel_residual = np.inf
        self.history = []


def _true_rel(A, b, u, nb):
    return np.linalg.norm(project(b - A @ u)) / nb


def pcg(A, b, precond, rtol, maxit=200, flexible=False):
    """Preconditioned CG (Hestenes-Stiefel) or FCG(1); u0 = 0."""
    info = SolveInfo()
    nb = np.linalg.norm(b)
    u = np.zeros_like(b)
    if nb == 0.0:
        info.converged, info.rel_residual = True, 0.0
        return u, info
    r = project(b.copy())

    def restart(r):
        z = project(precond(r))
        return z, z.copy(), r @ z

    z, p, rz = restart(r)
    while True:
        rel = np.linalg.norm(r) / nb
        info.history.append(rel)
        if rel <= rtol:
            true = _true_rel(A, b, u, nb)
            if true <= rtol:
                info.converged, info.rel_residual = True, true
                break
            r = project(b - A @ u)
            z, p, rz = restart(r)
            continue
        if info.iters >= maxit:
            info.rel_residual = _true_rel(A, b, u, nb)
            break
        w = A @ p
        pw = p @ w
        alpha = (p @ r) / pw if flexible else rz / pw
        u = u + alpha * p
        r = project(r - alpha * w)
        z = project(precond(r))
        if flexible:
            beta = -(z @ w) / pw
        else:
            rz_new = r @ z
            beta = rz_new / rz
            rz = rz_new
        p = z + beta * p
        info.iters += 1
    return u, info


def normalize_mean(u, q, n, form="csr"):
    """Shift u by a constant so that its integral vanishes: 1^T M u = 0."""
    from . import operator as op
    M = op.mass(q, n, form)
    w = M @ np.ones_like(u)
    return u - (w @ u) / (w @ np.ones_like(u))
