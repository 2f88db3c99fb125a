"""Pins of the cell-by-cell (EMI) oracle against what the model and the mathematics fix.

- the lumped membrane, gap-face and outer-boundary measures, computed by
  the oracle from the mesh's facets, equal their closed forms site by site
  (half of each adjacent boundary segment) and agree with the workload's
  arrays (which the library takes as input);
- the membrane jump mass annihilates constants and gives each cell's
  indicator the energy C_m x (cell perimeter);
- A maps constants to the Robin term only (eps x outer perimeter in total)
  and annihilates affine functions on interior rows of every subdomain;
- converged sweeps reproduce the Radau-IIA collocation solution of the DAE
  (independent Newton solve of the collocation equations);
- the collocation solution conserves charge: the Robin-weighted mean of the
  potential on the outer boundary vanishes at every node (M 1 = 0, the ionic
  currents cancel pairwise, A 1 = eps * robin);
- in the lumped limit (huge conductivities and Robin coefficient) one cell
  obeys the membrane ODE C_m v' = -I(v, w), w' = R(v, w) (SciPy's Radau);
- restriction: rows outside the active set and sites with an inactive
  intracellular node keep their values; the sets are nested.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import ionic
from oracle.emi import EMI, EmiSDC, build, collocation_solution, lumped_measures, run
from workloads.emi import config3


def small(**kw):
    base = dict(nc=3, nr=2, nx=5, ny=4)
    base.update(kw)
    return config3(**base)


def test_lumped_measures_per_site():
    """Cells of nx x ny nodes with spacings hx = 100 um / (nx - 1) and
    hy = 16 um / (ny - 1): a corner site carries (hx + hy) / 2, a site inside
    a long side hx, inside a short side hy; a gap-junction node hy at a face
    end, else hy... halved at the ends; an outer-boundary node half of its two
    boundary segments (from the sorted node positions on each side)."""
    nx, ny = 5, 4
    P = small(nx=nx, ny=ny)
    mod = EMI(P)
    hx, hy = 100e-4 / (nx - 1), 16e-4 / (ny - 1)
    xy = P.coords[P.mem_intra]
    cell = P.node_cell[P.mem_intra]
    for c in np.unique(cell):
        s = cell == c
        lo, hi = xy[s].min(axis=0), xy[s].max(axis=0)
        on_x = np.isclose(xy[s, 0], lo[0], rtol=0, atol=1e-12) | np.isclose(xy[s, 0], hi[0], rtol=0, atol=1e-12)
        on_y = np.isclose(xy[s, 1], lo[1], rtol=0, atol=1e-12) | np.isclose(xy[s, 1], hi[1], rtol=0, atol=1e-12)
        want = np.where(on_x & on_y, 0.5 * (hx + hy), np.where(on_y, hx, hy))
        assert np.allclose(mod.mem_len[s], want, rtol=1e-13, atol=0)
    gy = P.coords[P.gap_a, 1]
    cy = P.node_cell[P.gap_a] // 3
    end = np.isclose(gy - (2e-4 + cy * 18e-4), 0, atol=1e-12) | np.isclose(gy - (2e-4 + cy * 18e-4 + 16e-4), 0, atol=1e-12)
    assert np.allclose(mod.gap_len, np.where(end, 0.5 * hy, hy), rtol=1e-13, atol=0)
    # outer boundary: every box side, nodes sorted along it
    W = 3 * (100e-4 + 2e-4) + 2e-4
    Hb = 2 * (16e-4 + 2e-4) + 2e-4
    want = np.zeros(P.N)
    ext = P.node_cell < 0
    for ax, val in ((1, 0.0), (1, Hb), (0, 0.0), (0, W)):
        on = np.nonzero(ext & np.isclose(P.coords[:, ax], val, rtol=0, atol=1e-12))[0]
        t = P.coords[on, 1 - ax]
        o = np.argsort(t)
        seg = np.diff(t[o])
        share = np.zeros(len(on))
        share[:-1] += seg / 2
        share[1:] += seg / 2
        want[on[o]] += share
    assert np.allclose(mod.robin_len, want, rtol=1e-13, atol=0)
    assert abs(mod.robin_len.sum() - 2 * (W + Hb)) <= 1e-15
    # the workload's arrays (the library's input) carry the same measures
    for a, b in ((mod.mem_len, P.mem_len), (mod.gap_len, P.gap_len), (mod.robin_len, P.robin_len)):
        assert np.allclose(a, b, rtol=1e-13, atol=0)


def test_membrane_mass():
    P = small()
    mod = EMI(P)
    Mm = mod.M.toarray()
    assert np.allclose(Mm, Mm.T, atol=0)
    assert np.abs(Mm @ np.ones(P.N)).max() <= 1e-15 * np.abs(Mm).max()
    assert np.linalg.eigvalsh(Mm).min() > -1e-15 * P.N * np.abs(Mm).max()   # eigensolver rounding
    perim = 2 * (100e-4 + 16e-4)
    for c in range(3 * 2):
        ind = (P.node_cell == c).astype(float)
        assert abs(ind @ Mm @ ind - P.cm * perim) <= 1e-12 * perim


def test_stiffness_constants_and_affine_functions():
    P = small()
    mod = EMI(P)
    A = mod.A
    assert abs(A - A.T).max() == 0.0
    # row sums of the element part cancel to rounding (entries up to |A|max)
    assert np.allclose(A @ np.ones(P.N), P.eps * mod.robin_len, rtol=0, atol=1e-15 * 16 * abs(A).max())
    W = 3 * (100e-4 + 2e-4) + 2e-4
    H = 2 * (16e-4 + 2e-4) + 2e-4
    # the element part cancels to rounding of the nnz entries
    assert abs(np.ones(P.N) @ A @ np.ones(P.N) - P.eps * 2 * (W + H)) <= 1e-15 * A.nnz * abs(A).max()
    x, y = P.coords[:, 0], P.coords[:, 1]
    u = 2 * x - 3 * y
    interior = np.ones(P.N, dtype=bool)
    interior[P.mem_intra] = False
    interior[P.mem_extra] = False
    interior[mod.robin_len > 0] = False
    interior[P.gap_a] = False
    interior[P.gap_b] = False
    assert interior.sum() > 20
    assert np.abs((A @ u)[interior]).max() <= 1e-12 * np.abs(A).max() * np.abs(u).max()
    # a cell's indicator only feels the gap junctions of its end faces:
    # g_gap * cell height per neighbour in its row
    for c in range(3 * 2):
        ind = (P.node_cell == c).astype(float)
        n_nb = (c % 3 > 0) + (c % 3 < 2)
        assert abs(ind @ (A @ ind) - P.g_gap * 16e-4 * n_nb) <= 1e-12 * abs(A).max() * A.nnz * 1e-3


@pytest.mark.parametrize("M", [2, 3])
def test_converged_sweeps_equal_collocation_solution(M):
    P = config3(nc=2, nr=1, nx=3, ny=3, M=M, dt=0.05, theta=0.0)
    u0 = np.zeros(P.N)
    u0[P.stimuli[0][1]] = 1.0
    w0 = np.full(len(P.mem_intra), 0.05)
    sdc = build(P, direct=True)
    st = sdc.spread(u0, w0)
    idx = np.arange(P.N)
    for _ in range(60):
        sdc.sweep(st, idx)
    Uc, Wc = collocation_solution(sdc.model, M, P.dt, u0, w0)
    d = st["u"] - Uc
    si, se = sdc.model.si, sdc.model.se
    # the constant mode of the potentials is fixed only by the weak Robin
    # term (eigenvalue ~ dt eps |boundary|), so it carries rounding amplified
    # by the condition number; the transmembrane voltage, the gating and the
    # mean-free potential are well conditioned
    assert np.abs(d[:, si] - d[:, se]).max() <= 1e-12
    assert np.abs(d - d.mean(axis=1, keepdims=True)).max() <= 1e-12 * np.abs(Uc).max()
    assert np.abs(d).max() <= 1e-8 * np.abs(Uc).max()
    assert np.abs(st["w"] - Wc).max() <= 1e-12 * max(np.abs(Wc).max(), 1.0)
    # charge conservation of the collocation solution: robin^T u_m = 0 at every
    # node (to the accuracy of the constant mode)
    rl = sdc.model.robin_len
    for m in range(M):
        assert abs(rl @ Uc[m]) <= 1e-8 * rl.sum() * np.abs(Uc).max()
        assert abs(rl @ st["u"][m]) <= 1e-8 * rl.sum() * np.abs(Uc).max()


def test_single_cell_lumped_limit_follows_membrane_ode():
    big = 1e6
    P = config3(nc=1, nr=1, nx=4, ny=3, sigma_i=big, sigma_e=big, eps=big, M=3, dt=0.02, theta=0.0)
    sdc = build(P, direct=True)
    u = np.zeros(P.N)
    u[P.node_cell == 0] = 0.3          # transmembrane voltage 0.3 above the threshold a = 0.15
    w = np.zeros(len(P.mem_intra))
    n_steps, K = 25, 12
    u, w, _ = run(sdc, u, w, n_steps, K)
    p = np.asarray(P.ionic[0])

    def rhs(t, y):
        v, g = y
        return [-ionic.current(v, g, p) / P.cm, ionic.rate(v, g, p)]

    ref = solve_ivp(rhs, (0.0, n_steps * P.dt), [0.3, 0.0], method="Radau", rtol=1e-12, atol=1e-14)
    v_end = u[P.mem_intra] - u[P.mem_extra]
    assert np.abs(v_end - ref.y[0, -1]).max() <= 1e-5
    assert np.abs(w - ref.y[1, -1]).max() <= 1e-5
    assert abs(v_end.mean() - 0.3) > 0.05          # the voltage moved


def test_restriction_freezes_inactive_rows_and_sites():
    P = small(theta=1e-3)
    sdc = build(P)
    u0 = np.zeros(P.N)
    u0[P.stimuli[0][1]] = 1.0
    w0 = np.zeros(len(P.mem_intra))
    st = sdc.spread(u0, w0)
    idx, _ = sdc.sweep(st, np.arange(P.N))
    assert 0 < idx.size < P.N
    before = {k: st[k].copy() for k in ("u", "w", "I", "R")}
    nxt, info = sdc.sweep(st, idx)
    assert np.all(np.isin(nxt, idx))
    off = np.setdiff1d(np.arange(P.N), idx)
    assert np.array_equal(st["u"][:, off], before["u"][:, off])
    active = np.zeros(P.N, dtype=bool)
    active[idx] = True
    frozen = ~active[sdc.model.si]
    for k in ("w", "I", "R"):
        assert np.array_equal(st[k][:, frozen], before[k][:, frozen])
    assert np.all(info["du"][:, off] == 0.0)


def test_adaptive_run_tracks_nonadaptive():
    P = small(theta=1e-8)
    u0 = np.zeros(P.N)
    w0 = np.zeros(len(P.mem_intra))
    ua, wa, loga = run(build(P), u0, w0, 4, P.K, P.stimuli)
    P0 = small(theta=0.0)
    un, wn, _ = run(build(P0), u0, w0, 4, P0.K, P0.stimuli)
    assert any(info["n_active"] < P.N for step in loga for info in step)
    assert np.abs(ua - un).max() <= 1e-5 * np.abs(un).max()


@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_energy_termination_meets_its_tolerance(tol):
    """Sec. 3.2 for the cell-by-cell model: with rho at least the actual
    contraction, the terminated step's last node lies within tol of the
    collocation solution in the H norm (the gauge mode of the potentials
    carries no energy: H annihilates it up to the weak Robin term)."""
    P = config3(nc=2, nr=1, nx=3, ny=3, M=3, dt=0.05, theta=0.0)
    u0 = np.zeros(P.N)
    u0[P.stimuli[0][1]] = 1.0
    w0 = np.full(len(P.mem_intra), 0.05)
    sdc = build(P, direct=True, tol_sdc=tol, rho=0.6)
    Uc, _ = collocation_solution(sdc.model, P.M, P.dt, u0, w0)
    u_end, _, infos = sdc.step(u0, w0, 60)
    assert 1 < len(infos) < 60
    e = u_end - Uc[-1]
    assert np.sqrt(e @ (sdc.H[P.M - 1] @ e)) <= tol
    thr = ((1 - 0.6) / 0.6 * tol) ** 2
    assert infos[-2]["energy"] > thr >= infos[-1]["energy"]


def test_energy_termination_extremes_equal_fixed_sweep_counts():
    P = small(theta=1e-8)
    u0 = np.zeros(P.N)
    u0[P.stimuli[0][1]] = 1.0
    w0 = np.zeros(len(P.mem_intra))
    fixed = build(P)
    u4, w4, _ = fixed.step(u0, w0, 4)
    u2, w2, _ = fixed.step(u0, w0, 2)
    tiny = build(P, tol_sdc=1e-300)
    ut, wt, it = tiny.step(u0, w0, 4)
    assert len(it) == 4 and np.array_equal(ut, u4) and np.array_equal(wt, w4)
    huge = build(P, tol_sdc=1e10, K_min=2)
    uh, wh, ih = huge.step(u0, w0, 4)
    assert len(ih) == 2 and np.array_equal(uh, u2) and np.array_equal(wh, w2)
