"""Dense Newton solve of the full collocation system (oracle; test infrastructure).

Sec. 3.1: the collocation solution on one step satisfies, at every node m,

    ML (v_m - v0) = dt sum_j Q[m,j] (-A v_j - ML I(v_j, w_j))
       w_m - w0   = dt sum_j Q[m,j] R(v_j, w_j),

which couples all M nodes.  Newton's method with the full (dense) Jacobian
of size 2NM is the expensive reference the SDC sweeps approximate; here it
is only used on tiny meshes to pin the fixed point of the sweeps.
"""
import numpy as np

from . import ionic
from .collocation import Collocation


def solve(model, M, dt, v0, w0, tol=1e-14, maxit=50):
    col = Collocation(M)
    Q = col.Q
    N = model.N
    ML = model.ML
    A = model.A.toarray()
    p = model.p
    V = np.tile(v0, (M, 1))
    W = np.tile(w0, (M, 1))

    def residual(V, W):
        I = ionic.current(V, W, p)
        R = ionic.rate(V, W, p)
        F = -(V @ A.T) - ML * I
        rv = ML * (V - v0) - dt * (Q @ F)
        rw = (W - w0) - dt * (Q @ R)
        return np.concatenate([rv.ravel(), rw.ravel()])

    for _ in range(maxit):
        r = residual(V, W)
        if np.max(np.abs(r)) < tol:
            break
        dIv, dIw, _ = ionic.current_partials(V, W, p)
        dRv, dRw, _ = ionic.rate_partials(V, W, p)
        J = np.zeros((2 * M * N, 2 * M * N))
        for m in range(M):
            rv = slice(m * N, (m + 1) * N)
            rw = slice(M * N + m * N, M * N + (m + 1) * N)
            J[rv, rv] += np.diag(ML)
            J[rw, rw] += np.eye(N)
            for j in range(M):
                cv = slice(j * N, (j + 1) * N)
                cw = slice(M * N + j * N, M * N + (j + 1) * N)
                J[rv, cv] += dt * Q[m, j] * (A + np.diag(ML * dIv[j]))
                J[rv, cw] += dt * Q[m, j] * np.diag(ML * dIw[j])
                J[rw, cv] -= dt * Q[m, j] * np.diag(dRv[j])
                J[rw, cw] -= dt * Q[m, j] * np.diag(dRw[j])
        d = np.linalg.solve(J, -r)
        V = V + d[:M * N].reshape(M, N)
        W = W + d[M * N:].reshape(M, N)
    else:
        raise RuntimeError("collocation Newton did not converge")
    return V, W
