"""Tangent-linear model of the adaptive SDC step (oracle; test infrastructure).

Forward-mode differentiation of the step in :mod:`oracle.sdc` (Sec. 3,
eq. final-sdc, with the IMEX reading documented there), with respect to the
step's initial state (v0, w0), the nodal conductivity multipliers sigma and
the Aliev-Panfilov parameter a (Sec. 5.1).  The active index sets of every
sweep are held fixed (replayed), so the step is a smooth map; each linear
solve is differentiated as an exact solve of its restricted system:

    H dv = b   =>   H dv' = b' - H' dv,   H' = dt QI[m,m] A'(sigma'),

on the rows of the active set (zero tangent off the set).  Each line below
is the tangent of the corresponding line of ``SDC.sweep``; a primed name
holds the tangent of the unprimed quantity.

The solves here are direct (sparse LU of the principal submatrix) so that
the tangent is exact to rounding; the forward uses the same direct solves
when called through this module.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from . import ionic
from .assembly import lumped_mass, stiffness, stiffness_sigma_derivative
from .collocation import Collocation


class TLMProblem:
    """Data of a (possibly multi-instance) monodomain problem for differentiation."""

    def __init__(self, problem):
        P = problem
        self.P = P
        self.N = P.N
        self.ML = lumped_mass(P.coords, P.elems, P.N)
        self.col = Collocation(P.M)
        self.M, self.dt = P.M, P.dt
        self.inst_of = np.repeat(np.arange(P.n_inst), np.diff(P.node_off))

    def A(self, sigma):
        P = self.P
        return stiffness(P.coords, P.elems, P.elem_tensor, sigma, P.N)

    def dA(self, dsigma):
        P = self.P
        return stiffness_sigma_derivative(P.coords, P.elems, P.elem_tensor, P.N, dsigma)

    def params(self, a):
        """[6, N] Aliev-Panfilov parameters with per-instance a."""
        p = np.repeat(self.P.ionic, np.diff(self.P.node_off), axis=0).T.copy()
        p[1] = np.asarray(a, dtype=np.float64)[self.inst_of]
        return p


def _reaction(v, w, p, dv, dw, da):
    """(I, R) and their tangents in direction (dv, dw, da)."""
    I = ionic.current(v, w, p)
    R = ionic.rate(v, w, p)
    Iv, Iw, Ia = ionic.current_partials(v, w, p)
    Rv, Rw, Ra = ionic.rate_partials(v, w, p)
    return I, R, Iv * dv + Iw * dw + Ia * da, Rv * dv + Rw * dw + Ra * da


def step(tp, sigma, a, v0, w0, sets, dsigma=None, da=None, dv0=None, dw0=None):
    """One step with the given active sets; returns (v1, w1, v1', w1').

    sets[k] is the ascending row list of sweep k (sets[0] = all rows).
    Tangent directions default to zero.
    """
    N, M, dt = tp.N, tp.M, tp.dt
    Q, QI, QE = tp.col.Q, tp.col.QI, tp.col.QE
    ML = tp.ML
    A = tp.A(sigma)
    dsigma = np.zeros(N) if dsigma is None else dsigma
    dA = tp.dA(dsigma)
    p = tp.params(a)
    da_node = np.zeros(N) if da is None else np.asarray(da, dtype=np.float64)[tp.inst_of]
    dv0 = np.zeros(N) if dv0 is None else dv0
    dw0 = np.zeros(N) if dw0 is None else dw0

    I0, R0, I0t, R0t = _reaction(v0, w0, p, dv0, dw0, da_node)
    v = np.tile(v0, (M, 1)); vt = np.tile(dv0, (M, 1))
    w = np.tile(w0, (M, 1)); wt = np.tile(dw0, (M, 1))
    I = np.tile(I0, (M, 1)); It = np.tile(I0t, (M, 1))
    R = np.tile(R0, (M, 1)); Rt = np.tile(R0t, (M, 1))

    for idx in sets:
        idx = np.asarray(idx, dtype=np.int64)
        F = np.zeros((M, N)); Ft = np.zeros((M, N))
        for j in range(M):
            F[j, idx] = -(A @ v[j])[idx] - ML[idx] * I[j, idx]
            Ft[j, idx] = -(dA @ v[j] + A @ vt[j])[idx] - ML[idx] * It[j, idx]
        Phi = np.zeros((M, N)); Phit = np.zeros((M, N))
        Gam = np.zeros((M, N)); Gamt = np.zeros((M, N))
        for m in range(M):
            Phi[m, idx] = ML[idx] * (v0[idx] - v[m, idx]) + dt * (Q[m, :] @ F[:, idx])
            Phit[m, idx] = ML[idx] * (dv0[idx] - vt[m, idx]) + dt * (Q[m, :] @ Ft[:, idx])
            Gam[m, idx] = w0[idx] - w[m, idx] + dt * (Q[m, :] @ R[:, idx])
            Gamt[m, idx] = dw0[idx] - wt[m, idx] + dt * (Q[m, :] @ Rt[:, idx])
        dv = np.zeros((M, N)); dvt = np.zeros((M, N))
        dI = np.zeros((M, N)); dIt = np.zeros((M, N))
        dR = np.zeros((M, N)); dRt = np.zeros((M, N))
        for m in range(M):
            dw = Gam[m, idx].copy(); dwt = Gamt[m, idx].copy()
            rhs = Phi[m, idx].copy(); rhst = Phit[m, idx].copy()
            y = np.zeros(N); yt = np.zeros(N)
            for j in range(m):
                dw += dt * QE[m, j] * dR[j, idx]; dwt += dt * QE[m, j] * dRt[j, idx]
                rhs -= dt * QE[m, j] * ML[idx] * dI[j, idx]; rhst -= dt * QE[m, j] * ML[idx] * dIt[j, idx]
                y += dt * QI[m, j] * dv[j]; yt += dt * QI[m, j] * dvt[j]
            rhs -= (A @ y)[idx]
            rhst -= (dA @ y + A @ yt)[idx]
            c = dt * QI[m, m]
            x = np.zeros(N); xt = np.zeros(N)
            if idx.size:
                H = (sp.diags(ML) + c * A).tocsr()[idx][:, idx].tocsc()
                lu = splu(H)
                x[idx] = lu.solve(rhs)
                Hdot_x = c * (dA @ x)[idx]
                xt[idx] = lu.solve(rhst - Hdot_x)
            dv[m] = x; dvt[m] = xt
            v[m, idx] += x[idx]; vt[m, idx] += xt[idx]
            w[m, idx] += dw; wt[m, idx] += dwt
            In, Rn, Int, Rnt = _reaction(v[m, idx], w[m, idx], p[:, idx], vt[m, idx], wt[m, idx], da_node[idx])
            dI[m, idx] = In - I[m, idx]; dIt[m, idx] = Int - It[m, idx]
            dR[m, idx] = Rn - R[m, idx]; dRt[m, idx] = Rnt - Rt[m, idx]
            I[m, idx] = In; It[m, idx] = Int
            R[m, idx] = Rn; Rt[m, idx] = Rnt
    return v[-1].copy(), w[-1].copy(), vt[-1].copy(), wt[-1].copy()


def run(tp, sigma, a, v, w, n_steps, sets_per_step, stimuli=(), t0=0.0,
        dsigma=None, da=None, dv=None, dw=None):
    """Several steps (stimulus overwrites clear the tangent on their nodes)."""
    v = np.array(v, dtype=np.float64); w = np.array(w, dtype=np.float64)
    vt = np.zeros(tp.N) if dv is None else np.array(dv, dtype=np.float64)
    wt = np.zeros(tp.N) if dw is None else np.array(dw, dtype=np.float64)
    for n in range(n_steps):
        t = t0 + n * tp.dt
        for t_on, nodes, value in stimuli:
            if t - 1e-9 * tp.dt <= t_on < t + tp.dt - 1e-9 * tp.dt:
                v[np.asarray(nodes, dtype=np.int64)] = value
                vt[np.asarray(nodes, dtype=np.int64)] = 0.0
        v, w, vt, wt = step(tp, sigma, a, v, w, sets_per_step[n], dsigma, da, vt, wt)
    return v, w, vt, wt
