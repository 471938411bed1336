"""Pins of the oracle's LGL basis and 1D element matrices (Section 2.3.2)."""
import json
import os

import numpy as np
import pytest

from oracle import basis

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def test_lgl_nodes_closed_forms():
    assert np.allclose(basis.lgl_nodes(1), [0.0, 1.0], atol=0, rtol=0)
    assert np.allclose(basis.lgl_nodes(2), [0.0, 0.5, 1.0], atol=1e-16)
    s = GOLD["lgl_q4_interior_offset"]["value"]
    ref = 0.5 * (np.array([-1.0, -s, 0.0, s, 1.0]) + 1.0)
    assert np.max(np.abs(basis.lgl_nodes(4) - ref)) < 1e-15


@pytest.mark.parametrize("q", [1, 2, 3, 4, 6, 8])
def test_lagrange_cardinal_and_partition_of_unity(q):
    xi = basis.lgl_nodes(q)
    assert np.max(np.abs(basis.lagrange(xi, xi) - np.eye(q + 1))) < 1e-13
    t = np.linspace(0, 1, 17)
    assert np.max(np.abs(basis.lagrange(xi, t).sum(axis=0) - 1.0)) < 1e-12
    assert np.max(np.abs(basis.lagrange_deriv(xi, t).sum(axis=0))) < 1e-10


@pytest.mark.parametrize("q", [1, 2, 4])
def test_element_matrices_integrate_monomials_exactly(q):
    # Interpolation of t^m (m <= q) is exact, so v_m^T Khat v_k = int m k t^(m+k-2)
    # and v_m^T Mhat v_k = int t^(m+k) over [0, 1].
    Khat, Mhat = basis.element_matrices_1d(q)
    xi = basis.lgl_nodes(q)
    for m in range(q + 1):
        for k in range(q + 1):
            vm, vk = xi ** m, xi ** k
            kex = 0.0 if (m == 0 or k == 0) else m * k / (m + k - 1)
            mex = 1.0 / (m + k + 1)
            assert abs(vm @ Khat @ vk - kex) < 1e-13
            assert abs(vm @ Mhat @ vk - mex) < 1e-14


def test_textbook_q1_q2_element_matrices():
    K1, M1 = basis.element_matrices_1d(1)
    assert np.max(np.abs(K1 - np.array(GOLD["q1_element_1d"]["Khat"]))) < 1e-15
    assert np.max(np.abs(6 * M1 - np.array(GOLD["q1_element_1d"]["Mhat_times_6"]))) < 1e-14
    K2, M2 = basis.element_matrices_1d(2)
    assert np.max(np.abs(3 * K2 - np.array(GOLD["q2_element_1d"]["Khat_times_3"]))) < 1e-13
    assert np.max(np.abs(30 * M2 - np.array(GOLD["q2_element_1d"]["Mhat_times_30"]))) < 1e-13


def test_splitmix64_published_vector():
    from oracle.rng import splitmix64
    out = splitmix64(1234567, 5)
    assert [int(v) for v in out] == [int(s) for s in GOLD["splitmix64_key_1234567"]["first_outputs"]]
