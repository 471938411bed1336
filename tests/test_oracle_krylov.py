"""Pins of the oracle's Krylov solvers (Section 2.3: CG preconditioned by one V-cycle)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import operator as op, multigrid as mg, krylov

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def test_fcg1_equals_pcg_for_fixed_spd_preconditioner():
    H = mg.Hierarchy(2, 8, 3)
    b = mg.project(np.random.default_rng(6).standard_normal(H.finest.size))
    u1, i1 = krylov.pcg(H.finest.A, b, H.vcycle, 1e-12, flexible=False)
    u2, i2 = krylov.pcg(H.finest.A, b, H.vcycle, 1e-12, flexible=True)
    assert i1.iters == i2.iters
    k = min(5, len(i1.history))
    assert np.max(np.abs(np.array(i1.history[:k]) - np.array(i2.history[:k]))) < 1e-10
    assert np.max(np.abs(u1 - u2)) < 1e-10 * np.max(np.abs(u1))


def test_cg_terminates_in_distinct_eigenvalue_count():
    A = op.assemble(1, 2)    # 8 DoFs
    ev = np.linalg.eigvalsh(A.toarray())
    distinct = len(np.unique(np.round(ev[ev > 1e-12], 10)))
    b = mg.project(np.random.default_rng(0).standard_normal(8))
    u, info = krylov.pcg(A, b, lambda r: r.copy(), 1e-12, maxit=20)
    assert info.converged and info.iters <= distinct


def test_c1_closed_form_solution():
    # Q1, n = 32, f = 12 pi^2 sin sin sin, 4 levels, tolerance 1e-10.
    q, n = 1, 32
    x1 = op.dof_coords_1d(q, n)
    s = np.sin(2 * np.pi * x1)
    sss = (s[:, None, None] * s[None, :, None] * s[None, None, :]).ravel()
    H = mg.Hierarchy(q, n, 4)
    b = mg.rhs(q, n, 12 * np.pi ** 2 * sss)
    u, info = krylov.pcg(H.finest.A, b, H.vcycle, 1e-10)
    assert info.converged and info.rel_residual <= 1e-10
    u = krylov.normalize_mean(u, q, n)
    amp = GOLD["c1_discrete_amplitude_n32"]["value"]
    th, h = 2 * np.pi / n, 1.0 / n
    amp_formula = 4 * np.pi ** 2 * (h * (4 + 2 * np.cos(th)) / 6) / ((2 - 2 * np.cos(th)) / h)
    assert abs(amp - amp_formula) < 1e-10
    assert np.max(np.abs(u - amp_formula * sss)) < 1e-9
    # plausibility: the paper's GMG-1 needs about 6 CG iterations to 1e-13
    assert info.iters <= 12
