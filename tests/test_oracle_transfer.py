"""Pins of the oracle's intergrid transfers (Section 2.3.4, eqs. 2.1-2.2)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import basis, operator as op, transfer

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


@pytest.mark.parametrize("q", [1, 2, 4])
def test_prolongation_partition_of_unity_and_kronecker(q):
    P = transfer.prolongation(q, 2)
    P1 = transfer.prolongation_1d(q, 2)
    assert np.max(np.abs(P @ np.ones(P.shape[1]) - 1.0)) < 1e-14
    assert abs(P - sp.kron(sp.kron(P1, P1), P1)).max() < 1e-15


@pytest.mark.parametrize("q", [1, 2, 4])
def test_prolongation_reproduces_local_polynomials(q):
    # Inside one coarse element the coarse interpolant of t^m (m <= q) is exact,
    # so P maps its nodal values to t^m at the fine nodes (closure of the 2 children).
    n_c = 4
    P1 = transfer.prolongation_1d(q, n_c).toarray()
    xi = basis.lgl_nodes(q)
    E = 1
    for m in range(q + 1):
        vc = np.zeros(q * n_c)
        vc[q * E: q * E + q + 1] = xi ** m
        vf = P1 @ vc
        # fine nodes strictly inside coarse element E and its right end point
        for b in range(2 * q + 1):
            e, a = divmod(b, q)
            t = 1.0 if b == 2 * q else (e + xi[a]) / 2.0
            i = 2 * q * E + b
            assert abs(vf[i] - t ** m) < 1e-13


def test_q2_quarter_point_rows():
    P1 = transfer.prolongation_1d(2, 4).toarray()
    g = GOLD["q2_quarter_point_prolongation"]
    # fine node 1 (x = 1/4 of coarse element 0) and 3 (x = 3/4)
    assert np.max(np.abs(P1[1, 0:3] - g["row_at_1_4"])) < 1e-15
    assert np.max(np.abs(P1[3, 0:3] - g["row_at_3_4"])) < 1e-15


@pytest.mark.parametrize("q,n_c", [(1, 2), (2, 2), (4, 2), (2, 4)])
def test_galerkin_identity(q, n_c):
    P = transfer.prolongation(q, n_c)
    Af = op.assemble(q, 2 * n_c)
    Ac = op.assemble(q, n_c)
    G = (P.T @ Af @ P).toarray()
    assert np.max(np.abs(G - Ac.toarray())) < 1e-14 * 10 * np.max(np.abs(Ac.toarray()))


def test_kronecker_transfer_matches_matrix():
    q, n_c = 2, 4
    Pm = transfer.MatrixProlongation(q, n_c)
    Pk = transfer.KroneckerProlongation(q, n_c)
    rng = np.random.default_rng(5)
    xc = rng.standard_normal((q * n_c) ** 3)
    xf = rng.standard_normal((2 * q * n_c) ** 3)
    assert np.max(np.abs(Pm.prolong(xc) - Pk.prolong(xc))) < 1e-13
    assert np.max(np.abs(Pm.restrict(xf) - Pk.restrict(xf))) < 1e-12
