"""Collocation data for SDC on Radau-IIA nodes (oracle; test infrastructure).

Sec. 3.1 of the paper: on one step [0, dt] the collocation grid
0 < tau_1 < ... < tau_M = 1 (scaled to the unit interval) holds the Radau-IIA
points, which exclude the start point and include the end point (L-stable,
order 2M-1).  The paper writes the quadrature node-to-node (S_i, eq. "SDC
Integration"); we use the equivalent zero-to-node form

    Q[m, j] = integral_0^{tau_m} l_j(s) ds,      S_i = Q_i - Q_{i-1},

with l_j the Lagrange basis on tau_1..tau_M.  For Radau-IIA no basis function
sits at tau_0 = 0, so the paper's S_{i0} column vanishes.

Lower-triangular approximations used by the sweep (eq. (SDC)):

* QI, the "LU trick" the paper cites for S-hat (Weiser 2015): factor
  Q^T = L U (Doolittle, L unit lower triangular, no pivoting) and take
  QI = U^T.  The paper cites this choice without stating it; this is our
  reading, pinned by the stiff-limit nilpotency (I - QI^{-1} Q)^M = 0.
* QE, forward Euler between consecutive nodes for the explicit (reaction)
  part of the implicit-explicit operator splitting (Sec. 3.2):
  QE[m, j] = tau_{j+1} - tau_j for j < m, zero otherwise.  Its F(z_0) column
  cancels in the correction and is dropped.

Indices in code are 0-based: node m = 0..M-1, tau[M-1] = 1.
"""
import numpy as np
from numpy.polynomial import legendre as _leg
from numpy.polynomial import polynomial as _poly


def radau_iia_nodes(M):
    """Right Radau points on [0, 1]: roots of P_M(2t-1) - P_{M-1}(2t-1).

    The end point t = 1 is a root of that combination; it is set exactly.
    Roots are polished by Newton's method on the Legendre combination.
    """
    if M < 1:
        raise ValueError("M >= 1 required")
    if M == 1:
        return np.array([1.0])
    c = np.zeros(M + 1)
    c[M] = 1.0
    c[M - 1] = -1.0
    x = np.sort(np.real(_leg.legroots(c)))
    dc = _leg.legder(c)
    for _ in range(3):
        x = x - _leg.legval(x, c) / _leg.legval(x, dc)
    tau = (x + 1.0) / 2.0
    tau[-1] = 1.0
    return tau


def lagrange_basis(tau, j):
    """Power-series coefficients of the Lagrange polynomial l_j on nodes tau."""
    others = np.delete(tau, j)
    coeffs = _poly.polyfromroots(others)
    return coeffs / _poly.polyval(tau[j], coeffs)


def integration_matrix(tau):
    """Q[m, j] = integral from 0 to tau[m] of l_j (zero-to-node quadrature)."""
    M = len(tau)
    Q = np.zeros((M, M))
    for j in range(M):
        antideriv = _poly.polyint(lagrange_basis(tau, j))
        for m in range(M):
            Q[m, j] = _poly.polyval(tau[m], antideriv) - _poly.polyval(0.0, antideriv)
    return Q


def doolittle(Mat):
    """Doolittle LU without pivoting: Mat = L U, L unit lower triangular."""
    n = Mat.shape[0]
    L = np.eye(n)
    U = np.zeros((n, n))
    for i in range(n):
        for k in range(i, n):
            U[i, k] = Mat[i, k] - sum(L[i, s] * U[s, k] for s in range(i))
        for k in range(i + 1, n):
            L[k, i] = (Mat[k, i] - sum(L[k, s] * U[s, i] for s in range(i))) / U[i, i]
    return L, U


def lu_trick(Q):
    """QI = U^T where Q^T = L U (the LU trick S-hat of Sec. 3.1)."""
    _, U = doolittle(Q.T)
    return U.T.copy()


def explicit_euler_matrix(tau):
    """QE[m, j] = tau[j+1] - tau[j] for j < m (forward Euler between nodes)."""
    M = len(tau)
    QE = np.zeros((M, M))
    for m in range(M):
        for j in range(m):
            QE[m, j] = tau[j + 1] - tau[j]
    return QE


class Collocation:
    """All collocation matrices for M Radau-IIA nodes."""

    def __init__(self, M):
        self.M = M
        self.tau = radau_iia_nodes(M)
        self.Q = integration_matrix(self.tau)
        self.QI = lu_trick(self.Q)
        self.QE = explicit_euler_matrix(self.tau)
