"""Pins for the oracle's collocation data (Sec. 3.1): textbook closed forms and identities."""
import math

import numpy as np
import pytest

from oracle.collocation import Collocation, doolittle

S6 = math.sqrt(6.0)


def test_radau_nodes_closed_forms():
    # Hairer & Wanner, Solving ODEs II, Sec. IV.5 (Radau IIA tableaux)
    assert np.allclose(Collocation(1).tau, [1.0], atol=0, rtol=0)
    assert np.allclose(Collocation(2).tau, [1 / 3, 1.0], rtol=0, atol=1e-15)
    assert np.allclose(Collocation(3).tau, [(4 - S6) / 10, (4 + S6) / 10, 1.0], rtol=0, atol=1e-15)
    assert np.allclose(Collocation(4).tau,
                       [0.088587959512704, 0.4094668644407346, 0.7876594617608471, 1.0],
                       rtol=0, atol=1e-14)


def test_nodes_are_radau_right_points():
    # roots of P_M(2t-1) - P_{M-1}(2t-1), checked with scipy's Legendre evaluation
    from scipy.special import eval_legendre
    for M in range(2, 8):
        t = Collocation(M).tau
        x = 2 * t - 1
        assert np.max(np.abs(eval_legendre(M, x) - eval_legendre(M - 1, x))) < 1e-13
        assert t[-1] == 1.0 and np.all(np.diff(t) > 0) and t[0] > 0


def test_Q_matches_butcher_tableaux():
    Q2 = np.array([[5 / 12, -1 / 12], [3 / 4, 1 / 4]])
    assert np.allclose(Collocation(2).Q, Q2, rtol=0, atol=1e-15)
    Q3 = np.array([
        [(88 - 7 * S6) / 360, (296 - 169 * S6) / 1800, (-2 + 3 * S6) / 225],
        [(296 + 169 * S6) / 1800, (88 + 7 * S6) / 360, (-2 - 3 * S6) / 225],
        [(16 - S6) / 36, (16 + S6) / 36, 1 / 9],
    ])
    assert np.allclose(Collocation(3).Q, Q3, rtol=0, atol=1e-15)


@pytest.mark.parametrize("M", [2, 3, 4, 5])
def test_Q_polynomial_exactness(M):
    c = Collocation(M)
    for deg in range(0, 2 * M):
        f = c.tau ** deg
        exact = c.tau ** (deg + 1) / (deg + 1)
        got = c.Q @ f
        if deg <= M - 1:          # interpolatory: every row exact
            assert np.allclose(got, exact, rtol=0, atol=1e-14)
        if deg <= 2 * M - 2:      # Radau quadrature: the end point row exact
            assert abs(got[-1] - exact[-1]) < 1e-14
    # degree 2M-1 is not integrated exactly by the end point row
    f = c.tau ** (2 * M - 1)
    assert abs((c.Q @ f)[-1] - 1 / (2 * M)) > 1e-6


@pytest.mark.parametrize("M", [2, 3, 4, 5])
def test_QI_lu_trick(M):
    c = Collocation(M)
    QI = c.QI
    assert np.all(np.triu(QI, 1) == 0.0)
    L, U = doolittle(c.Q.T)
    assert np.allclose(L @ U, c.Q.T, rtol=0, atol=1e-15)
    assert np.allclose(np.diag(L), 1.0) and np.all(np.triu(L, 1) == 0)
    # stiff-limit nilpotency: QI^{-1} Q = L^T is unit upper triangular
    E = np.eye(M) - np.linalg.solve(QI, c.Q)
    assert np.max(np.abs(np.linalg.matrix_power(E, M))) < 1e-13
    assert np.max(np.abs(np.linalg.matrix_power(E, M - 1))) > 1e-3


def test_QI_diagonals():
    assert np.allclose(np.diag(Collocation(2).QI), [5 / 12, 2 / 5], atol=1e-15)
    assert np.allclose(np.diag(Collocation(3).QI), [0.19681548, 0.42340844, 0.2], atol=1e-8)
    assert np.allclose(np.diag(Collocation(4).QI), [0.11299948, 0.29050213, 0.30825766, 2 / 17], atol=1e-8)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_QE_forward_euler_structure(M):
    c = Collocation(M)
    assert np.all(np.triu(c.QE) == 0.0)
    # row m of QE integrates a constant from tau_0 to tau_m
    assert np.allclose(c.QE.sum(axis=1), c.tau - c.tau[0], atol=1e-15)
    for m in range(1, M):
        assert np.allclose(c.QE[m, :m], np.diff(c.tau)[:m])
