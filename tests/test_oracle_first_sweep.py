"""Pins of the heuristic first-sweep set (oracle).

The paper (Sec. 6) names a heuristic a-priori subset for the first sweep as
a way past the full first sweep, which bounds the speedup, and fixes no
rule; the rule here is a reading (the rows the previous step carried after
its first sweep and this step's stimulated rows, grown by mesh neighbours).
What the mathematics fixes about it:
- one ring of growth adds exactly the mesh neighbours: on a path the set
  grown r times from row i is [i - r, i + r]; on the grid split along the
  (i, j)-(i+1, j+1) diagonals it is the hexagonal ball |dx| <= r,
  |dy| <= r, |dx - dy| <= r, clipped to the grid;
- carried and stimulated rows are always in the set, and growth is monotone;
- a full first sweep on every step, or growth that covers the mesh, gives
  the standard run bit for bit;
- the set a step carries is the one its second sweep uses.
"""
import numpy as np
import pytest

from oracle.sdc import (FirstSweepSubset, build, first_sweep_set, mesh_adjacency, run, select)
from workloads import config0, meshes


def test_growth_on_a_path_is_an_interval():
    coords, elems = meshes.line_mesh(40, 1.0)
    N = coords.shape[0]
    adj = mesh_adjacency(elems, N)
    for i in (0, 7, N - 1):
        for r in (1, 2, 5):
            got = first_sweep_set(adj, [i], [], r)
            assert got.tolist() == list(range(max(0, i - r), min(N, i + r + 1)))


@pytest.mark.parametrize("ij", [(6, 5), (0, 0), (10, 1)])
def test_growth_on_the_split_grid_is_a_hexagonal_ball(ij):
    nx, ny = 11, 9
    coords, elems = meshes.square_tri_mesh(nx, ny, 1.0, 1.0)
    adj = mesh_adjacency(elems, nx * ny)
    i0, j0 = ij
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    ids, di, dj = (J * nx + I).ravel(), (I - i0).ravel(), (J - j0).ravel()
    for r in (1, 2, 3):
        ball = ids[(np.abs(di) <= r) & (np.abs(dj) <= r) & (np.abs(di - dj) <= r)]
        assert first_sweep_set(adj, [j0 * nx + i0], [], r).tolist() == sorted(ball.tolist())


def test_carried_and_forced_rows_are_kept_and_growth_is_monotone():
    coords, elems = meshes.square_tri_mesh(15, 12, 1.0, 1.0)
    N = coords.shape[0]
    adj = mesh_adjacency(elems, N)
    rng = np.random.default_rng(5)
    carried = np.sort(rng.choice(N, 9, replace=False))
    forced = rng.choice(N, 4, replace=False)
    prev = None
    for r in (1, 2, 3):
        got = first_sweep_set(adj, carried, forced, r)
        assert np.all(np.diff(got) > 0)
        assert np.isin(carried, got).all() and np.isin(forced, got).all()
        if prev is not None:
            assert np.isin(prev, got).all() and got.size > prev.size
        prev = got
    assert first_sweep_set(adj, [], [], 3).size == 0


def _standard_and_heuristic(first, n_steps=40):
    P = config0(n=64, theta=1e-6, n_steps=n_steps)
    sdc = build(P)
    std = run(sdc, P.v_init, P.w_init, n_steps, P.K, P.stimuli)
    heu = run(sdc, P.v_init, P.w_init, n_steps, P.K, P.stimuli,
              first=first(mesh_adjacency(P.elems, P.N), P.N))
    return P, std, heu


def test_full_first_sweep_every_step_equals_the_standard_run_bitwise():
    P, (vs, ws, _), (vh, wh, lh) = _standard_and_heuristic(lambda adj, N: FirstSweepSubset(adj, 2, 1))
    assert np.array_equal(vs, vh) and np.array_equal(ws, wh)
    assert all(step[0]["n_active"] == P.N for step in lh)


def test_growth_covering_the_mesh_equals_the_standard_run_bitwise():
    P, (vs, ws, ls), (vh, wh, lh) = _standard_and_heuristic(lambda adj, N: FirstSweepSubset(adj, N, 0))
    # the front keeps a carried set non-empty, so every grown set is all rows
    assert all(step[0]["n_active"] == P.N for step in lh)
    assert np.array_equal(vs, vh) and np.array_equal(ws, wh)


def test_heuristic_set_is_used_after_the_first_step():
    P, _, (vh, wh, lh) = _standard_and_heuristic(lambda adj, N: FirstSweepSubset(adj, 2, 10), n_steps=25)
    first = [step[0]["n_active"] for step in lh]
    assert first[0] == P.N and first[10] == P.N and first[20] == P.N
    assert all(0 < f < P.N for n, f in enumerate(first) if n % 10)


def test_carried_set_is_the_second_sweeps_set():
    P = config0(n=64, theta=1e-6)
    sdc = build(P)
    v = P.v_init.copy()
    v[P.stimuli[0][1]] = P.stimuli[0][2]
    st = sdc.spread(v, P.w_init)
    nxt, _ = sdc.sweep(st, np.arange(P.N))
    sdc.step(v, P.w_init, P.K)
    assert np.array_equal(sdc.carried, nxt)
    # one sweep per step: the first sweep's own set
    sdc.step(v, P.w_init, 1, idx_replay=[np.arange(5, 30)])
    assert sdc.carried.tolist() == list(range(5, 30))
    # a replayed second set is the carried one
    sdc.step(v, P.w_init, 2, idx_replay=[None, np.arange(3, 9)])
    assert sdc.carried.tolist() == list(range(3, 9))
    assert np.array_equal(select(np.arange(P.N), np.ones(P.N), 0.5), np.arange(P.N))


def test_heuristic_run_stays_as_close_to_the_non_adaptive_run_as_the_standard_one():
    """An observed property, not a bound the paper states: with growth that
    covers the front's advance per step (4 rings against about 1.3 rows per
    step here), the heuristic run is no farther from the non-adaptive run
    (theta = 0) than the standard adaptive run is (1D workload, 200 steps,
    the front half way)."""
    P = config0(theta=1e-6, n_steps=200)
    sdc = build(P)
    vs, _, _ = run(sdc, P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    full = build(P)
    full.theta = 0.0
    vn, _, _ = run(full, P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    vh, _, lh = run(sdc, P.v_init, P.w_init, P.n_steps, P.K, P.stimuli,
                    first=FirstSweepSubset(mesh_adjacency(P.elems, P.N), 4, 10))
    assert np.abs(vh - vn).max() <= np.abs(vs - vn).max()
    assert sum(step[0]["n_active"] for step in lh) < 0.95 * P.n_steps * P.N
