"""Pins of the oracle's linearized scheme, the paper's basic scheme (eq.
final-sdc: lumped reaction Jacobian in the implicit operator, gating by
Gauss-Seidel with implicit dR/dw).

- one node (M = 1) without diffusion: one sweep is a linearized implicit
  Euler step, v1 = v0 - dt I / (1 + dt I_v), then
  w1 = w0 + dt R(v1, w0) / (1 - dt R_w(v1, w0)) (closed form);
- a linear reaction and a linear gating rate: the first sweep is the
  LU-trick SDC iteration y + (1 - dt mu QI)^-1 (y0 1 - y + dt mu Q y) of
  y' = mu y, for v and for w (dense formula written out);
- without reaction (I = R = 0) it is the IMEX scheme;
- converged sweeps reach the dense Newton solution of the collocation
  system (the same fixed point as the IMEX scheme);
- on a stiff reaction it contracts faster than the IMEX scheme.
"""
import numpy as np
import pytest

from oracle import ionic
from oracle.assembly import lumped_mass, stiffness
from oracle.collocation import Collocation
from oracle.collocation_newton import solve as collocation_solve
from oracle.sdc import SDC, Monodomain
from workloads import AP_PARAMS, meshes


def _line_model(n, D, params=AP_PARAMS):
    coords, elems = meshes.line_mesh(n, 1.0)
    ML = lumped_mass(coords, elems, n)
    A = stiffness(coords, elems, np.full((n - 1, 1, 1), D), np.ones(n), n)
    return Monodomain(ML, A, params), coords[:, 0]


def test_one_node_without_diffusion_is_linearized_implicit_euler():
    model, x = _line_model(9, D=0.0)
    p = np.asarray(AP_PARAMS, dtype=np.float64)
    v0 = np.linspace(-0.1, 1.1, 9)
    w0 = np.linspace(0.0, 1.5, 9)
    dt = 0.3
    s = SDC(model, 1, dt, 0.0, cg_rtol=1e-15, scheme="linearized")
    st = s.spread(v0, w0)
    s.sweep(st, np.arange(9))
    dIv = ionic.current_partials(v0, w0, p)[0]
    v1 = v0 - dt * ionic.current(v0, w0, p) / (1.0 + dt * dIv)
    Rw = ionic.rate_partials(v1, w0, p)[1]
    w1 = w0 + dt * ionic.rate(v1, w0, p) / (1.0 - dt * Rw)
    assert np.allclose(st["v"][0], v1, rtol=1e-13, atol=1e-15)
    assert np.allclose(st["w"][0], w1, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_linear_reaction_and_gating_first_sweep_is_lu_sdc(M):
    # k = 0, mu1 = 0: I = v w (linear in v while w is the spread value),
    # R = -s eps0 w (linear in w, independent of v)
    params = (0.0, 0.15, 0.05, 0.0, 0.3, 0.5)
    model, x = _line_model(7, D=0.0, params=params)
    v0 = 0.3 + 0.5 * x
    wc = 0.8
    dt = 0.7
    s = SDC(model, M, dt, 0.0, cg_rtol=1e-15, scheme="linearized")
    st = s.spread(v0, np.full(7, wc))
    s.sweep(st, np.arange(7))
    col = Collocation(M)
    one = np.ones(M)

    def lu_sdc(y0, mu):
        y = y0 * one
        return y + np.linalg.solve(np.eye(M) - dt * mu * col.QI, y0 * one - y + dt * mu * col.Q @ y)

    for i in range(7):
        assert np.allclose(st["v"][:, i], lu_sdc(v0[i], -wc), rtol=1e-13, atol=1e-15)
        assert np.allclose(st["w"][:, i], lu_sdc(wc, -params[5] * params[2]), rtol=1e-13, atol=1e-15)


def test_without_reaction_equals_imex():
    params = (0.0, 0.15, 0.002, 0.2, 0.3, 0.25)   # k = 0 and w = 0: I = R = 0
    model, x = _line_model(40, D=1e-2, params=params)
    v0 = np.exp(-((x - 0.3) / 0.1) ** 2)
    w0 = np.zeros(40)
    for theta in (0.0, 1e-4):
        a = SDC(model, 3, 0.2, theta, cg_rtol=1e-14)
        b = SDC(model, 3, 0.2, theta, cg_rtol=1e-14, scheme="linearized")
        va, wa, ia = a.step(v0, w0, 4)
        vb, wb, ib = b.step(v0, w0, 4)
        assert [x["n_active"] for x in ia] == [x["n_active"] for x in ib]
        assert np.allclose(va, vb, rtol=0, atol=1e-14) and np.all(wb == 0.0)


@pytest.mark.parametrize("M", [2, 3])
def test_converged_sweeps_reach_collocation_solution(M):
    model, x = _line_model(12, D=1e-2)
    v0 = np.where(x < 0.3, 1.0, 0.0) + 0.05 * np.sin(7 * x)
    w0 = 0.1 * np.cos(3 * x) ** 2
    dt = 0.1
    s = SDC(model, M, dt, 0.0, cg_rtol=1e-15, scheme="linearized")
    V, W = collocation_solve(model, M, dt, v0, w0)
    st = s.spread(v0, w0)
    idx = np.arange(model.N)
    for _ in range(40):
        s.sweep(st, idx)
    assert np.max(np.abs(st["v"] - V)) < 1e-12
    assert np.max(np.abs(st["w"] - W)) < 1e-12


def test_stiff_reaction_contracts_faster_than_imex():
    params = (40.0, 0.15, 0.002, 0.2, 0.3, 0.25)   # five times the usual k
    model, x = _line_model(12, D=1e-3, params=params)
    v0 = np.clip(1.2 - 2 * x, 0.0, 1.0)
    w0 = np.zeros(12)
    dt, M = 0.2, 3
    V, W = collocation_solve(model, M, dt, v0, w0)
    err = {}
    for scheme in ("imex", "linearized"):
        s = SDC(model, M, dt, 0.0, cg_rtol=1e-15, scheme=scheme)
        st = s.spread(v0, w0)
        for _ in range(4):
            s.sweep(st, np.arange(12))
        err[scheme] = np.max(np.abs(st["v"] - V))
    assert err["linearized"] < 0.1 * err["imex"]
