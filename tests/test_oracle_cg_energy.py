"""Pins of the oracle's optional energy-error stop of the Jacobi-PCG.

The paper stops its CG at an estimated energy-error reduction (Sec. 5.1)
without naming the estimator; the oracle's reading uses the step terms
t_j = alpha_j (r_j . z_j) (see oracle.pcg).  What the mathematics fixes,
checked here against dense solves and the iterates themselves rather than
the terms the solver forms:
- with x0 = 0, sum_{j=n-d}^{n-1} t_j = e_{n-d} - e_n and
  sum_{j<n} t_j = e_0 - e_n, e_n = ||x - x_n||_A^2, so the stopping step is
  the first n >= d with e_{n-d} - e_n <= tol^2 (e_0 - e_n) (brute force over
  the iterates and the exact solution);
- the window is a lower estimate: e_{n-d} >= e_{n-d} - e_n at the stop;
- a vanishing tolerance, or a delay beyond the solve's length, leaves the
  residual stop bit for bit.
"""
import numpy as np
import pytest

from oracle.pcg import jacobi_pcg
from oracle.sdc import build, run
from workloads import config0, config1


def _system(n, seed, frac, s=3e4):
    """ML + s A of the anisotropic 2D workload on an n x n grid: a P1 system
    of the sweep's form, with s large enough that CG takes tens of steps."""
    P = config1(n=n, theta=1e-7)
    m = build(P).model
    H = np.diag(m.ML) + s * m.A.toarray()
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(P.N, int(frac * P.N), replace=False)) if frac < 1 else np.arange(P.N)
    b = rng.standard_normal(P.N)
    return H, b, idx


def _energies(H, b, idx, n_max):
    """e_n = ||x - x_n||_A^2 of the restricted system for n = 0..n_max, from
    the exact solution and the iterates x_n (replayed step counts)."""
    Hs = H[np.ix_(idx, idx)]
    x = np.linalg.solve(Hs, b[idx])
    e = []
    for n in range(n_max + 1):
        xn = jacobi_pcg(H, b, idx, 1e-12, fixed_iters=n)[0][idx] if n else np.zeros(idx.size)
        d = x - xn
        e.append(d @ Hs @ d)
    return np.array(e)


@pytest.mark.parametrize("n,seed,frac,tol,delay", [
    (13, 1, 1.0, 1e-3, 4), (17, 2, 0.6, 1e-3, 3), (17, 3, 1.0, 1e-2, 1), (21, 4, 0.4, 1e-4, 5),
    # loose and early: the last term is a sizeable share of the running sum
    (13, 6, 1.0, 0.3, 1), (17, 7, 0.5, 0.2, 2), (15, 8, 1.0, 0.22, 1),
    (13, 12, 1.0, 0.4, 1), (13, 13, 1.0, 0.4, 2), (13, 11, 1.0, 0.3, 2)])
def test_stop_step_is_the_first_step_the_exact_errors_satisfy(n, seed, frac, tol, delay):
    H, b, idx = _system(n, seed, frac)
    _, it = jacobi_pcg(H, b, idx, 1e-14, maxit=500, energy_tol=tol, delay=delay)
    _, it_full = jacobi_pcg(H, b, idx, 1e-14, maxit=500)
    assert delay <= it < it_full
    e = _energies(H, b, idx, it + 2)
    want = next(k for k in range(delay, it + 3) if e[k - delay] - e[k] <= tol ** 2 * (e[0] - e[k]))
    assert it == want
    # not a near tie: the exact ratio at the stop and one step earlier is clear of tol^2
    ratio = [(e[k - delay] - e[k]) / (e[0] - e[k]) for k in (it - 1, it) if k >= delay]
    assert ratio[-1] < 0.999 * tol ** 2 and (len(ratio) == 1 or ratio[0] > 1.001 * tol ** 2)
    # the window estimates the error of x_{n-d} from below
    assert e[it - delay] >= e[it - delay] - e[it]


def test_vanishing_tolerance_or_long_delay_is_the_residual_stop():
    H, b, idx = _system(17, 5, 0.7)
    xr, ir = jacobi_pcg(H, b, idx, 1e-12)
    for kw in (dict(energy_tol=1e-40, delay=3), dict(energy_tol=1e-3, delay=ir + 1)):
        x, i = jacobi_pcg(H, b, idx, 1e-12, **kw)
        assert i == ir and np.array_equal(x, xr)
    with pytest.raises(ValueError):
        jacobi_pcg(H, b, idx, 1e-12, energy_tol=1e-3, delay=0)


def test_sdc_run_with_the_energy_stop_takes_fewer_steps_and_replays_itself():
    P = config0(n=128, theta=1e-6, n_steps=30)
    std = build(P)
    vs, _, ls = run(std, P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    eng = build(P, cg_energy_tol=1e-3, cg_delay=4)
    ve, we, le = run(eng, P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    its_s = sum(sum(sw["cg_iters"]) for step in ls for sw in step)
    its_e = sum(sum(sw["cg_iters"]) for step in le for sw in step)
    assert its_e < 0.7 * its_s
    # the loose solves move the state by far less than the SDC correction sizes
    assert 0 < np.abs(ve - vs).max() < 1e-3
    # replaying the sets and step counts on the residual-stop integrator
    # reproduces the run bit for bit
    v, w, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli,
                  idx_replay=[[sw["idx"] for sw in step] for step in le],
                  cg_replay=[[sw["cg_iters"] for sw in step] for step in le])
    assert np.array_equal(v, ve) and np.array_equal(w, we)


def test_stop_rule_values_reproduce_the_stop_decisions():
    """stop_rule_values gives the quantities the two rules test: the step
    where jacobi_pcg stops is the first at which one of them passes."""
    from oracle.pcg import stop_rule_values
    for seed, tol, d in ((3, 1e-3, 4), (7, 1e-2, 2), (11, 1e-12, 3)):
        H, b, idx = _system(17, seed, 0.6)
        x, n = jacobi_pcg(H, b, idx, 1e-12, energy_tol=tol, delay=d)
        res, en = stop_rule_values(H, b, idx, n, d)
        passes = (res <= 1e-12) | (en <= tol ** 2)
        assert passes[n] and not passes[:n].any()
