"""Jacobi-preconditioned CG on a principal submatrix (oracle; test infrastructure).

Sec. 4.2: the linear systems of each sweep are solved only on the active
index set I_k, i.e. with the principal submatrix H[I_k, I_k] (homogeneous
Dirichlet values on the complement, Sec. 4.1), by CG with a Jacobi
preconditioner because it needs no setup when the submatrix changes.

Stopping rule (a reading; the paper stops at an estimated energy-error
reduction of 1e-3): ||r||_2 <= rtol * ||b||_2 over the active rows, x0 = 0.
A zero right-hand side or an empty index set returns x = 0 after 0
iterations.  ``fixed_iters`` replays a given iteration count instead.

Optional energy-error stop (Sec. 5.1 names an estimated energy-error
reduction; the estimator is a reading).  With x0 = 0, CG step j reduces the
squared energy error by exactly t_j = alpha_j (r_j . z_j) (z = the
preconditioned residual), so
    ||x - x_n||_A^2 = sum_{j >= n} t_j   and   ||x||_A^2 - ||x - x_n||_A^2 = sum_{j < n} t_j.
After n >= d steps the last d terms, sum_{j=n-d}^{n-1} t_j, are a lower
estimate of the squared error of x_{n-d} (the estimate of Hestenes and
Stiefel, with the delay d of Strakos and Tichy), and sum_{j<n} t_j is the
squared energy of x_n.  The solve stops after step n when the residual test
holds or when n >= d and
    sum_{j=n-d}^{n-1} t_j <= energy_tol^2 * sum_{j<n} t_j,
i.e. an estimated relative energy error of at most energy_tol; x_n is
returned.  Both sums are formed left to right in j.  energy_tol = 0 (the
default) leaves only the residual test.
"""
import numpy as np


class CGNotConverged(RuntimeError):
    pass


def jacobi_pcg(H, b, idx, rtol, maxit=1000, fixed_iters=None, energy_tol=0.0, delay=0):
    """Solve H[idx, idx] x = b[idx]; return (x full-length, zero off idx; iterations)."""
    if energy_tol > 0.0 and delay < 1:
        raise ValueError("the energy-error stop needs a delay d >= 1")
    n = H.shape[0]
    x_full = np.zeros(n)
    idx = np.asarray(idx, dtype=np.int64)
    if idx.size == 0:
        return x_full, 0
    Hs = H[idx][:, idx]
    bs = np.asarray(b, dtype=np.float64)[idx]
    bnorm = np.sqrt(bs @ bs)
    if bnorm == 0.0:
        return x_full, 0
    dinv = 1.0 / Hs.diagonal()
    x = np.zeros_like(bs)
    r = bs.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    terms = []   # t_j = alpha_j (r_j . z_j), the energy-error reduction of step j
    limit = maxit if fixed_iters is None else fixed_iters
    while it < limit:
        q = Hs @ p
        alpha = rz / (p @ q)
        terms.append(alpha * rz)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if fixed_iters is None and np.sqrt(r @ r) <= rtol * bnorm:
            break
        if fixed_iters is None and energy_tol > 0.0 and it >= delay:
            if sum(terms[it - delay:]) <= energy_tol ** 2 * sum(terms):
                break
        z = dinv * r
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    else:
        if fixed_iters is None:
            raise CGNotConverged(f"PCG: no convergence in {maxit} iterations")
    x_full[idx] = x
    return x_full, it


def stop_rule_values(H, b, idx, n, delay=0):
    """The two quantities the stopping rules of jacobi_pcg compare, after each
    step j = 1..n of the restricted solve from x0 = 0 (textbook PCG):
    res[j] = ||r_j||_2 / ||b||_2 (against rtol) and, for j >= delay >= 1,
    en[j] = sum_{i=j-d}^{j-1} t_i / sum_{i<j} t_i (against energy_tol^2),
    t_i = alpha_i (r_i . z_i); en[j] = inf where the rule does not apply.
    Index 0 of both arrays is the start (res 1, en inf).  For checking a step
    count that another implementation of CG chose against the rules."""
    idx = np.asarray(idx, dtype=np.int64)
    res = np.full(n + 1, np.inf)
    en = np.full(n + 1, np.inf)
    Hs = H[idx][:, idx]
    bs = np.asarray(b, dtype=np.float64)[idx]
    bnorm = np.sqrt(bs @ bs)
    res[0] = 1.0
    dinv = 1.0 / Hs.diagonal()
    r = bs.copy()
    z = dinv * r
    p = z.copy()
    rz = r @ z
    terms = []
    for j in range(1, n + 1):
        q = Hs @ p
        alpha = rz / (p @ q)
        terms.append(alpha * rz)
        r = r - alpha * q
        res[j] = np.sqrt(r @ r) / bnorm
        if delay >= 1 and j >= delay:
            en[j] = sum(terms[j - delay:]) / sum(terms)
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return res, en
