"""Pins for the oracle's SDC step, PCG and index-set rule (Secs. 3-4).

Each pin is independent of the oracle's own formulas: a forward Euler loop,
a dense collocation Newton solve, the Radau-IIA stability function (Pade
approximant), scipy's Radau integrator, dense linear solves, and the
structural facts the paper states (nested index sets, rest state).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.integrate import solve_ivp

from oracle import ionic
from oracle.collocation_newton import solve as collocation_solve
from oracle.pcg import jacobi_pcg
from oracle.sdc import SDC, Monodomain, build, run, select
from oracle.assembly import lumped_mass, stiffness
from workloads import AP_PARAMS, config0, meshes


def _line_model(n, D=1e-3, params=AP_PARAMS, L=1.0):
    coords, elems = meshes.line_mesh(n, L)
    ML = lumped_mass(coords, elems, n)
    A = stiffness(coords, elems, np.full((n - 1, 1, 1), D), np.ones(n), n)
    return Monodomain(ML, A, params), coords[:, 0]


def pade_radau(M, z):
    """Radau IIA stability function = (M-1, M) Pade approximant of exp(z)."""
    k, j = M - 1, M
    num = sum(math.factorial(k + j - i) * math.factorial(k) /
              (math.factorial(k + j) * math.factorial(i) * math.factorial(k - i)) * z ** i
              for i in range(k + 1))
    den = sum(math.factorial(k + j - i) * math.factorial(j) /
              (math.factorial(k + j) * math.factorial(i) * math.factorial(j - i)) * (-z) ** i
              for i in range(j + 1))
    return num / den


def test_pade_closed_forms():
    z = -1.3
    assert np.isclose(pade_radau(3, z), (1 + 2 * z / 5 + z * z / 20) / (1 - 3 * z / 5 + 3 * z * z / 20 - z ** 3 / 60),
                      rtol=1e-15)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_first_sweep_without_diffusion_is_forward_euler_over_nodes(M):
    n = 6
    ML = np.linspace(0.5, 1.5, n)
    model = Monodomain(ML, sp.csr_matrix((n, n)), AP_PARAMS)
    dt = 0.3
    s = SDC(model, M, dt, theta=0.0, cg_rtol=1e-15)
    rng = np.random.default_rng(1)
    v0 = rng.uniform(0, 1, n)
    w0 = rng.uniform(0, 1, n)
    st = s.spread(v0, w0)
    s.sweep(st, np.arange(n))
    # independent forward Euler across 0 = tau_0' < tau_1 < ... < tau_M
    p = np.array(AP_PARAMS)
    tau = np.concatenate([[0.0], s.col.tau])
    v, w = v0.copy(), w0.copy()
    for m in range(M):
        h = (tau[m + 1] - tau[m]) * dt
        v, w = v - h * ionic.current(v, w, p), w + h * ionic.rate(v, w, p)
        assert np.allclose(st["v"][m], v, rtol=1e-13, atol=1e-15)
        assert np.allclose(st["w"][m], w, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_converged_sweeps_reach_collocation_solution(M):
    model, x = _line_model(12, D=1e-2)
    v0 = np.where(x < 0.3, 1.0, 0.0) + 0.05 * np.sin(7 * x)
    w0 = 0.1 * np.cos(3 * x) ** 2
    dt = 0.1
    s = SDC(model, M, dt, theta=0.0, cg_rtol=1e-15)
    V, W = collocation_solve(model, M, dt, v0, w0)
    st = s.spread(v0, w0)
    idx = np.arange(model.N)
    for _ in range(50):
        s.sweep(st, idx)
    assert np.max(np.abs(st["v"] - V)) < 1e-12
    assert np.max(np.abs(st["w"] - W)) < 1e-12
    # a single sweep is far from it, and the contraction is well below 1 (paper: rho < 0.6)
    st2 = s.spread(v0, w0)
    errs = []
    for _ in range(4):
        s.sweep(st2, idx)
        errs.append(np.max(np.abs(st2["v"] - V)))
    assert errs[0] > 1e-6
    assert max(errs[i + 1] / errs[i] for i in range(3)) < 0.6


def _heat_mode(n, kappa, D):
    model, x = _line_model(n, D=D, params=(0.0, 0.15, 0.002, 0.2, 0.3, 0.25))
    h = x[1] - x[0]
    lam = 4 * D / h ** 2 * np.sin(kappa * np.pi * h / 2) ** 2
    return model, np.cos(kappa * np.pi * x), lam


def test_heat_mode_is_generalized_eigenvector():
    model, v, lam = _heat_mode(33, 3, 1e-3)
    assert np.max(np.abs(model.A @ v - lam * model.ML * v)) < 1e-15 * 1e3


@pytest.mark.parametrize("M", [2, 3, 4])
def test_converged_heat_mode_follows_radau_stability_function(M):
    model, v0, lam = _heat_mode(33, 5, 1e-3)
    dt = 0.5
    s = SDC(model, M, dt, theta=0.0, cg_rtol=1e-15)
    st = s.spread(v0, np.zeros_like(v0))
    idx = np.arange(model.N)
    for _ in range(60):
        s.sweep(st, idx)
    r = pade_radau(M, -lam * dt)
    assert np.max(np.abs(st["v"][-1] - r * v0)) < 1e-13
    assert np.all(st["w"] == 0.0)


def test_heat_mode_decay_order():
    # converged steps approximate exp(-lam t) with error O(dt^(2M-1))
    M = 3
    model, v0, lam = _heat_mode(17, 2, 1e-3)
    T = 4.0
    errs = []
    for nsteps in (4, 8, 16):
        s = SDC(model, M, T / nsteps, theta=0.0, cg_rtol=1e-15)
        v = v0.copy()
        for _ in range(nsteps):
            v, _, _ = s.step(v, np.zeros_like(v), 30)
        errs.append(np.max(np.abs(v - np.exp(-lam * T) * v0)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(4.6 < r < 5.4 for r in rates), rates


@pytest.mark.parametrize("M", [2, 3, 4])
def test_stiff_limit_lu_trick_exact_after_M_sweeps(M):
    # for z -> -inf, QI = U^T (Q^T = LU) makes the sweep error operator nilpotent:
    # M sweeps reach the collocation stage values up to O(1/|z|), M-1 do not.
    # Stage values of the heat mode: (I - zQ)^{-1} 1 with the pinned Q.
    model, v0, lam = _heat_mode(9, 4, 1.0)
    z = -1e5
    s = SDC(model, M, -z / lam, theta=0.0, cg_rtol=1e-15)
    stages = np.linalg.solve(np.eye(M) - z * s.col.Q, np.ones(M))
    assert np.isclose(stages[-1], pade_radau(M, z), rtol=1e-10)
    st = s.spread(v0, np.zeros_like(v0))
    idx = np.arange(model.N)
    errs = []
    for _ in range(M):
        s.sweep(st, idx)
        errs.append(np.max(np.abs(st["v"] - np.outer(stages, v0))))
    assert errs[M - 1] < 1e-5
    assert errs[M - 2] > 1e-2


def test_pure_reaction_order_2M_minus_1(root):
    M = 3   # the paper's three Radau points, order five
    model = Monodomain(np.ones(1), sp.csr_matrix((1, 1)), AP_PARAMS)
    p = np.array(AP_PARAMS)
    v0, w0, T = np.array([0.35]), np.array([0.05]), 2.0

    def f(t, y):
        return [-ionic.current(y[0], y[1], p), ionic.rate(y[0], y[1], p)]

    ref = solve_ivp(f, (0, T), [v0[0], w0[0]], method="Radau", rtol=1e-13, atol=1e-15).y[:, -1]
    errs = []
    for nsteps in (8, 16, 32):
        s = SDC(model, M, T / nsteps, theta=0.0, cg_rtol=1e-15)
        v, w = v0.copy(), w0.copy()
        for _ in range(nsteps):
            v, w, _ = s.step(v, w, 30)
        errs.append(max(abs(v[0] - ref[0]), abs(w[0] - ref[1])))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(4.4 < r < 5.6 for r in rates), (errs, rates)


def test_pcg_matches_dense_principal_submatrix_solve():
    rng = np.random.default_rng(7)
    coords, elems = meshes.square_tri_mesh(9, 8, 1.0, 1.0)
    N = coords.shape[0]
    E = elems.shape[0]
    A = stiffness(coords, elems, np.broadcast_to(np.diag([2.0, 0.5]), (E, 2, 2)), np.ones(N), N)
    H = (sp.diags(lumped_mass(coords, elems, N)) + 0.3 * A).tocsr()
    for trial in range(5):
        idx = np.sort(rng.choice(N, size=rng.integers(1, N), replace=False))
        b = rng.standard_normal(N)
        x, it = jacobi_pcg(H, b, idx, 1e-14)
        Hd = H.toarray()[np.ix_(idx, idx)]
        ref = np.linalg.solve(Hd, b[idx])
        assert np.linalg.norm(x[idx] - ref) <= 1e-12 * np.linalg.norm(ref)
        mask = np.ones(N, bool)
        mask[idx] = False
        assert np.all(x[mask] == 0.0)
        assert 0 < it <= idx.size + 5
    x, it = jacobi_pcg(H, np.zeros(N), np.arange(N), 1e-12)
    assert it == 0 and np.all(x == 0)
    x, it = jacobi_pcg(H, np.ones(N), np.array([], dtype=np.int64), 1e-12)
    assert it == 0 and np.all(x == 0)


def test_restricted_solve_discrete_maximum_principle():
    # Thm. 1 (discrete form): with an M-matrix, the error of the restricted solve
    # (zero Dirichlet values off the subset) is bounded by the dropped values next to it.
    model, x = _line_model(41, D=1e-3)
    H = (sp.diags(model.ML) + 0.05 * model.A).tocsr()
    b = np.exp(-((x - 0.5) / 0.05) ** 2) * model.ML
    full, _ = jacobi_pcg(H, b, np.arange(41), 1e-15)
    for lo, hi in ((10, 31), (15, 26), (18, 23)):
        sub = np.arange(lo, hi)
        xs, _ = jacobi_pcg(H, b, sub, 1e-15)
        err = np.max(np.abs(full[sub] - xs[sub]))
        bound = max(abs(full[lo - 1]), abs(full[hi]))
        assert err <= bound * (1 + 1e-12)


def test_selection_rule_brute_force():
    rng = np.random.default_rng(5)
    amax = np.abs(rng.standard_normal(100)) * 1e-6
    amax[7] = 1e-6          # exactly at the threshold is kept (">=")
    idx = np.sort(rng.choice(100, 60, replace=False))
    if 7 not in idx:
        idx = np.sort(np.append(idx, 7))
    got = select(idx, amax, 1e-6)
    ref = np.array([i for i in idx if amax[i] >= 1e-6])
    assert np.array_equal(got, ref) and 7 in got
    assert np.array_equal(select(idx, amax, 0.0), idx)
    assert np.array_equal(select(idx, amax, -1.0), idx)


def test_adaptive_sets_are_nested_and_first_sweep_is_full():
    P = config0(n=64, theta=1e-6, n_steps=40)
    s = build(P)
    _, _, log = run(s, P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    saw_drop = False
    for infos in log:
        assert infos[0]["n_active"] == 64
        for a, b in zip(infos[:-1], infos[1:]):
            assert set(b["idx"].tolist()) <= set(a["idx"].tolist())
            assert np.all(np.diff(b["idx"]) > 0)
            saw_drop |= b["n_active"] < a["n_active"]
    assert saw_drop


def test_theta_nonpositive_and_all_rows_replay_equal_nonadaptive():
    P = config0(n=48, theta=0.0, n_steps=20)
    base = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    P2 = config0(n=48, theta=-1.0, n_steps=20)
    neg = run(build(P2), P2.v_init, P2.w_init, P2.n_steps, P2.K, P2.stimuli)
    P3 = config0(n=48, theta=1e-6, n_steps=20)
    allrows = [[np.arange(48)] * P3.K for _ in range(P3.n_steps)]
    rep = run(build(P3), P3.v_init, P3.w_init, P3.n_steps, P3.K, P3.stimuli, idx_replay=allrows)
    for other in (neg, rep):
        assert np.array_equal(base[0], other[0]) and np.array_equal(base[1], other[1])


def test_rest_state_stays_exactly_at_rest():
    P = config0(n=32, theta=1e-6, n_steps=3)
    s = build(P)
    v, w, infos = s.step(np.zeros(32), np.zeros(32), 4)
    assert np.all(v == 0) and np.all(w == 0)
    assert infos[0]["n_active"] == 32 and infos[1]["n_active"] == 0
    assert all(i == 0 for i in infos[0]["cg_iters"])


def test_jacobi_preconditioner_properties():
    # a diagonal system is solved in one iteration; Jacobi PCG is invariant
    # under symmetric diagonal scaling (same iterates up to rounding)
    rng = np.random.default_rng(11)
    n = 30
    Hd = sp.diags(rng.uniform(0.5, 3.0, n)).tocsr()
    b = rng.standard_normal(n)
    x, it = jacobi_pcg(Hd, b, np.arange(n), 1e-14)
    assert it == 1 and np.allclose(x, b / Hd.diagonal(), rtol=1e-15)
    coords, elems = meshes.square_tri_mesh(8, 8, 1.0, 1.0)
    N, E = coords.shape[0], elems.shape[0]
    A = stiffness(coords, elems, np.broadcast_to(np.eye(2), (E, 2, 2)), np.ones(N), N)
    H = (sp.diags(lumped_mass(coords, elems, N)) + 0.5 * A).tocsr()
    Dg = sp.diags(rng.uniform(0.1, 10.0, N))
    b = rng.standard_normal(N)
    idx = np.arange(5, N - 3)
    x1, it1 = jacobi_pcg(H, b, idx, 1e-10)
    x2, it2 = jacobi_pcg((Dg @ H @ Dg).tocsr(), Dg @ b, idx, 1e-10)
    assert abs(it1 - it2) <= 1


def test_selection_uses_max_correction_over_nodes():
    import copy
    P = config0(n=64, theta=1e-4, n_steps=1)
    s = build(P)
    v0 = np.where(np.arange(64) < 20, 1.0, 0.0)
    idx = np.arange(64)
    st1 = s.spread(v0, np.zeros(64))
    s.sweep(st1, idx)                      # the second sweep's corrections are not monotone in m
    _, info = s.sweep(copy.deepcopy(st1), idx)
    dv = info["dv"]
    big = np.abs(dv).max(axis=0)
    last = np.abs(dv[-1])
    # pick a threshold that separates "max over nodes" from "last node only"
    i = int(np.argmax(big / np.maximum(last, 1e-300)))
    assert big[i] > 2 * last[i]
    s.theta = 0.5 * (big[i] + last[i])
    nxt, _ = s.sweep(copy.deepcopy(st1), idx)
    brute = np.array([r for r in idx if max(abs(dv[m, r]) for m in range(s.M)) >= s.theta])
    assert np.array_equal(nxt, brute) and i in nxt


# ---------------------------------------------------------------- energy-norm termination (Sec. 3.2)

def _sdc_energy_setup():
    model, x = _line_model(12, D=1e-2)
    v0 = np.where(x < 0.3, 1.0, 0.0) + 0.05 * np.sin(7 * x)
    w0 = 0.1 * np.cos(3 * x) ** 2
    return model, v0, w0


@pytest.mark.parametrize("tol", [1e-4, 1e-7])
def test_energy_termination_meets_its_tolerance(tol):
    # the criterion estimates the remaining error by the geometric series
    # rho/(1-rho) ||delta^k||: with rho at least the actual contraction, the
    # last node's value is within tol of the collocation solution in the H norm
    model, v0, w0 = _sdc_energy_setup()
    M, dt = 3, 0.1
    V, _ = collocation_solve(model, M, dt, v0, w0)
    s = SDC(model, M, dt, theta=0.0, cg_rtol=1e-15, tol_sdc=tol, rho=0.6)
    v_end, _, infos = s.step(v0, w0, 60)
    assert 1 < len(infos) < 60
    e = v_end - V[-1]
    assert np.sqrt(e @ (s.H[M - 1] @ e)) <= tol
    # one sweep earlier the criterion did not hold
    thr = ((1 - 0.6) / 0.6 * tol) ** 2
    assert infos[-2]["energy"][0] > thr >= infos[-1]["energy"][0]


def test_energy_termination_extremes_equal_fixed_sweep_counts():
    model, v0, w0 = _sdc_energy_setup()
    fixed = SDC(model, 3, 0.1, theta=0.0)
    v4, w4, _ = fixed.step(v0, w0, 4)
    v2, w2, _ = fixed.step(v0, w0, 2)
    tiny = SDC(model, 3, 0.1, theta=0.0, tol_sdc=1e-300)
    vt, wt, it = tiny.step(v0, w0, 4)
    assert len(it) == 4 and np.array_equal(vt, v4) and np.array_equal(wt, w4)
    huge = SDC(model, 3, 0.1, theta=0.0, tol_sdc=1e10, K_min=2)
    vh, wh, ih = huge.step(v0, w0, 4)
    assert len(ih) == 2 and np.array_equal(vh, v2) and np.array_equal(wh, w2)


def test_energy_termination_is_per_instance():
    # batched instances stop independently: each equals its own run alone
    from workloads import config4
    from workloads.configs import Problem
    P = config4(n_inst=3, sizes=(10, 18), n_steps=3)
    # no stimulus in instance 0: it stays at rest and stops after one sweep
    lo1 = P.node_off[1]
    P.stimuli = [(t, nodes[nodes >= lo1], val) for t, nodes, val in P.stimuli]
    tol = 3e-6
    batched = build(P, tol_sdc=tol, rho=0.3, K_min=1)
    vb, wb, logb = run(batched, P.v_init, P.w_init, 3, 8, P.stimuli)
    n_sweeps = set()
    for i in range(P.n_inst):
        lo, hi = int(P.node_off[i]), int(P.node_off[i + 1])
        e0, e1 = int(P.elem_off[i]), int(P.elem_off[i + 1])
        stim = [(t, nodes[(nodes >= lo) & (nodes < hi)] - lo, val) for t, nodes, val in P.stimuli]
        sub = Problem(name="inst", dim=P.dim, coords=P.coords[lo:hi], elems=P.elems[e0:e1] - lo,
                      elem_tensor=P.elem_tensor[e0:e1], node_sigma=P.node_sigma[lo:hi],
                      node_off=np.array([0, hi - lo]), elem_off=np.array([0, e1 - e0]),
                      ionic=P.ionic[i:i + 1], M=P.M, K=P.K, dt=P.dt, n_steps=3, theta=P.theta,
                      stimuli=stim, v_init=P.v_init[lo:hi], w_init=P.w_init[lo:hi])
        alone = build(sub, tol_sdc=tol, rho=0.3, K_min=1)
        va, wa, loga = run(alone, sub.v_init, sub.w_init, 3, 8, sub.stimuli)
        assert np.abs(vb[lo:hi] - va).max() <= 1e-12 * max(np.abs(va).max(), 1.0)
        n_sweeps.add(tuple(len(st) for st in loga))
    assert len(n_sweeps) > 1          # the instances did stop at different sweeps


def test_batched_instances_are_stepped_as_if_alone():
    """Independent instances in one state vector (block-diagonal A, one CG per
    instance): every instance's state, active sets and CG step counts equal
    those of the instance integrated alone.  A single CG over the stacked
    system would couple the instances through its shared scalars and its
    stopping test (a common step count, the residual over all instances)."""
    from workloads import config4
    P = config4(n_inst=3, sizes=(9, 17), n_steps=3)
    orc = build(P)
    vb, wb, lb = run(orc, P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    for i in range(P.n_inst):
        lo, hi = int(P.node_off[i]), int(P.node_off[i + 1])
        e0, e1 = int(P.elem_off[i]), int(P.elem_off[i + 1])
        ML = lumped_mass(P.coords[lo:hi], P.elems[e0:e1] - lo, hi - lo)
        A = stiffness(P.coords[lo:hi], P.elems[e0:e1] - lo, P.elem_tensor[e0:e1], P.node_sigma[lo:hi], hi - lo)
        solo = SDC(Monodomain(ML, A, P.ionic[i]), P.M, P.dt, P.theta, P.cg_rtol, P.cg_maxit)
        stim = [(t, np.asarray(n)[(n >= lo) & (n < hi)] - lo, val) for t, n, val in P.stimuli]
        v, w, ls = run(solo, P.v_init[lo:hi], P.w_init[lo:hi], P.n_steps, P.K, stim)
        assert np.abs(v - vb[lo:hi]).max() <= 1e-14 and np.abs(w - wb[lo:hi]).max() <= 1e-14
        for sb, s in zip(lb, ls):
            for kb, k in zip(sb, s):
                assert np.array_equal(kb["idx"][(kb["idx"] >= lo) & (kb["idx"] < hi)] - lo, k["idx"])
                assert [int(c[i]) for c in kb["cg_iters_inst"]] == k["cg_iters"]
    # the instances take different step counts somewhere in the run
    assert any(len(set(c.tolist())) > 1 for s in lb for k in s for c in k["cg_iters_inst"])
