"""Pins of the oracle's a-priori drop tolerance (Sec. 4.1, eqs. subset and
drop-tolerance; Thms. 1 and 2).

- r is the iteration count of eq. (r-condition): the closed form
  ceil(log((1 - rho) TOL / c) / log rho), and 0 when c <= (1 - rho) TOL;
- TOL_drop = exp(-eta T) (1 - rho) / (r + 1) TOL on hand-worked values;
- eta = max(0, -min dI/dv): dI/dv against central differences of I, and
  the minimum over v at w = 0 against its closed form k (a - (1 + a)^2 / 3);
- an instance at rest (no correction, dI/dv = k a > 0) gets (1 - rho) TOL
  and keeps no row; a stimulated one gets a smaller tolerance;
- Thm. 2: r + 1 sweeps with the a-priori drop tolerance reach the
  collocation solution within TOL.
"""
import math

import numpy as np
import pytest

from oracle import ionic
from oracle.sdc import SDC, apply_stimuli, apriori_drop_tolerance, build, sweeps_needed
from workloads import config0, config4

P_AP = np.array([8.0, 0.15, 0.002, 0.2, 0.3, 0.25])


def test_sweeps_needed_is_the_r_condition():
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(2000):
        c = 10.0 ** rng.uniform(-8, 1)
        rho = rng.uniform(0.01, 0.9)
        tol = 10.0 ** rng.uniform(-7, -2)
        x = math.log((1 - rho) * tol / c) / math.log(rho)
        if abs(x - round(x)) < 1e-6:
            continue   # the two forms may round differently at an exact integer
        assert sweeps_needed(c, rho, tol) == max(0, math.ceil(x))
        checked += 1
    assert checked > 1900
    assert sweeps_needed(0.0, 0.3, 1e-4) == 0
    assert sweeps_needed(0.7e-4, 0.3, 1e-4) == 0
    assert sweeps_needed(0.71e-4, 0.3, 1e-4) == 1


def test_drop_tolerance_hand_values():
    # c = 1e-2, rho = 0.1, TOL = 1e-4: (1 - rho) TOL = 9e-5; c rho^r = 1e-2, 1e-3, 1e-4, 1e-5 -> r = 3
    tol_drop, r = apriori_drop_tolerance(1e-2, 2.0, 0.1, 0.1, 1e-4)
    assert r == 3
    assert tol_drop == pytest.approx(math.exp(-0.2) * 0.9 / 4 * 1e-4, rel=1e-15)
    # no correction: r = 0 and, with eta = 0, (1 - rho) TOL
    tol_drop, r = apriori_drop_tolerance(0.0, 0.0, 0.1, 0.05, 1e-3)
    assert r == 0 and tol_drop == pytest.approx(0.95e-3, rel=1e-15)


def test_eta_from_the_current_derivative():
    v = np.linspace(-0.2, 1.2, 57)
    w = np.linspace(0.0, 2.0, 57)
    h = 1e-6
    fd = (ionic.current(v + h, w, P_AP) - ionic.current(v - h, w, P_AP)) / (2 * h)
    assert np.allclose(ionic.current_partials(v, w, P_AP)[0], fd, rtol=1e-8, atol=1e-8)
    k, a = P_AP[0], P_AP[1]
    vs = (1 + a) / 3
    assert ionic.current_partials(vs, 0.0, P_AP)[0] == pytest.approx(k * (a - (1 + a) ** 2 / 3), rel=1e-14)
    # the oracle's eta over a state that contains the minimiser
    P = config0(n=16)
    s = SDC(build(P).model, P.M, P.dt, 0.0, tol_sdc=1e-4, rho=0.3, drop="apriori")
    st = s.spread(np.full(P.N, 0.0), np.zeros(P.N))
    st["v"][1, 5] = vs
    theta, r, c, eta = s.drop_tolerances(st, np.zeros(P.N), np.arange(P.N))
    assert eta[0] == pytest.approx(-k * (a - (1 + a) ** 2 / 3), rel=1e-14)
    assert r[0] == 0 and theta[0] == pytest.approx(math.exp(-eta[0] * P.dt) * 0.7e-4, rel=1e-14)


def test_rest_instance_and_stimulated_instance():
    P = config4(n_inst=2, sizes=(10, 14), n_steps=1)
    lo1 = P.node_off[1]
    P.stimuli = [(t, nodes[nodes >= lo1], val) for t, nodes, val in P.stimuli]   # instance 0 at rest
    tol, rho = 1e-4, 0.2
    s = build(P, tol_sdc=tol, rho=rho, K_min=10, drop="apriori")
    v = P.v_init.copy()
    apply_stimuli(v, 0.0, P.dt, P.stimuli)
    _, _, infos = s.step(v, P.w_init.copy(), 3, keep=True)
    theta, c = infos[0]["drop_tol"], infos[0]["drop_c"]
    assert c[0] == 0.0 and theta[0] == pytest.approx((1 - rho) * tol, rel=1e-15)
    assert c[1] > (1 - rho) * tol and theta[1] < theta[0]
    # the sets use each instance's own tolerance: nothing of instance 0 stays active
    nxt = infos[1]["idx"]
    assert np.all(nxt >= lo1)
    amax = infos[0]["amax"]
    hi1 = P.node_off[2]
    assert np.array_equal(nxt, np.arange(lo1, hi1)[amax[lo1:hi1] >= theta[1]])


@pytest.mark.parametrize("rho,tol", [(0.5, 1e-4), (0.3, 1e-3)])
def test_theorem_2_accuracy(rho, tol):
    """r + 1 sweeps (r from the first sweep's correction) with the a-priori
    drop tolerance stay within TOL of the collocation solution of the step."""
    P = config0(theta=0.0)
    ref = build(P)
    v, w = P.v_init.copy(), P.w_init.copy()
    worst = 0.0
    for n in range(25):
        apply_stimuli(v, n * P.dt, P.dt, P.stimuli)
        vr, wr, _ = ref.step(v, w, 30)            # converged sweeps, all rows
        probe = SDC(ref.model, P.M, P.dt, 0.0, P.cg_rtol, P.cg_maxit, tol_sdc=tol, rho=rho, K_min=1000,
                    drop="apriori")
        _, _, inf = probe.step(v, w, 1, keep=True)
        r = int(inf[0]["drop_r"][0])
        va, _, infa = probe.step(v, w, r + 1)
        assert any(x["n_active"] < P.N for x in infa) or r == 0
        worst = max(worst, np.abs(va - vr).max())
        v, w = vr, wr
    assert worst <= tol
