"""Graph-captured sweeps (sdc_set_graph): every sweep of a step is one HIP
graph with a fixed launch sequence sized to the all-rows capacity, the sets
and CG outcomes stay on the device, one host synchronisation per step.

Checked against host-launched steps with the same CG launches
(small_set_rows = -1: no one-workgroup solves, which graph steps never use):
states bitwise equal after every step and the same per-sweep statistics, on
1D, 2D, 3D, batched and non-adaptive runs.  Every step after the first
capture replays the graphs, with the host's own work and synchronisations
between replays; the first step takes the synchronous loop (no budget
history yet), and later ones the graphs.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from workloads import config0, config1, config2, config3, config4  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(P, **kw):
    from paper_2311_07206_amd import Solver
    return Solver.from_problem(P, small_set_rows=-1, **kw)


def _steps(P, s, n_steps):
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    states, stats = [], []
    for n in range(n_steps):
        st = s.step(v, w, n * P.dt, stats=True)
        states.append((v.cpu().numpy().copy(), w.cpu().numpy().copy()))
        stats.append([(x["n_active"], x["nnz_active"], x["cg_iters_max"], x["cg_row_iters"]) for x in st])
    return states, stats


@pytest.mark.parametrize("case", ["1d", "2d", "3d", "batched", "batched_chunks", "nonadaptive"])
def test_graph_steps_equal_host_launched_steps_bitwise(case):
    if case == "1d":
        P, n = config0(n=160, theta=1e-6), 14
    elif case == "2d":
        P, n = config1(n=48, theta=1e-7), 10
    elif case == "3d":
        P, n = config2(n=14, theta=1e-7), 5
    elif case == "batched":
        P, n = config4(n_inst=4, sizes=(12, 30)), 8
    elif case == "batched_chunks":
        # maps long enough for full rounds of XCD chunks (90 blocks, chunk 4):
        # the graph sweeps take that order over their grids
        P, n = config4(n_inst=8, sizes=(40, 56)), 6
    else:
        P, n = config1(n=40, theta=0.0), 6
    print(f"[graph {case}] N={P.N}, {n} steps", flush=True)
    ref = _solver(P)
    g = _solver(P)
    g.set_graph(True)
    rs, rst = _steps(P, ref, n)
    gs, gst = _steps(P, g, n)
    info = g.info()
    print(f"   graph steps {info['graph_steps']}, captures {info['graph_captures']}, "
          f"redone {info['graph_redone']}", flush=True)
    for q in range(n):
        assert np.array_equal(rs[q][0], gs[q][0]) and np.array_equal(rs[q][1], gs[q][1]), q
        assert rst[q] == gst[q], q
    assert info["graph_steps"] >= n - 2 and info["graph_steps"] - info["graph_redone"] >= n // 2
    assert info["graph_captures"] >= 1
    assert ref.info()["graph_steps"] == 0
    if case == "batched_chunks":
        # a listed sweep's grid (the entries its set had, a quarter more and
        # 16) spans at least one full round of 8 XCD chunks
        chunk = info["xcd_chunk"]
        rows = g.active().cpu().numpy()
        cnt = np.diff(np.searchsorted(rows, P.node_off))
        entries = int(np.sum((cnt + 255) // 256))
        print(f"   chunk {chunk}, last set {rows.size} rows in {entries} entries", flush=True)
        assert chunk == 4 and entries + entries // 4 + 16 >= 8 * chunk
    # the set the last sweep used is the host mirror's: the same rows either way
    assert np.array_equal(ref.active().cpu().numpy(), g.active().cpu().numpy())
    ref.close()
    g.close()


def test_graph_mode_off_again_and_rejections():
    from paper_2311_07206_amd import SDCError
    P = config1(n=30, theta=1e-7)
    s = _solver(P)
    s.set_graph(True)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    for n in range(3):
        s.step(v, w, n * P.dt)
    s.set_graph(False)
    steps = s.info()["graph_steps"]
    s.step(v, w, 3 * P.dt)
    assert s.info()["graph_steps"] == steps
    with pytest.raises(SDCError, match="graph"):
        _solver(config1(n=12, theta=1e-7), scheme="linearized").set_graph(True)
    with pytest.raises(SDCError, match="graph"):
        _solver(config3(nc=2, nr=1, nx=3, ny=3)).set_graph(True)


def test_graph_steps_when_a_set_outgrows_its_grid():
    """Batched instances, the first one at rest until step 4, when a stimulus
    sets all its nodes: that step's later sweeps cover about 44 map entries
    against 13 the step before (the oracle's sets), beyond the grids captured
    from it (a quarter more and 16), so the graph step is redone by the
    synchronous loop and the graphs captured again; the states stay bitwise
    equal to host-launched steps."""
    P = config4(n_inst=3, sizes=(64, 96), n_steps=8)
    (t0, nodes, val), = P.stimuli
    first = nodes < P.node_off[1]
    whole = np.arange(P.node_off[0], P.node_off[1]).astype(np.int32)
    P.stimuli = [(t0, nodes[~first], val), (4 * P.dt, whole, val)]
    ref = _solver(P)
    g = _solver(P)
    g.set_graph(True)
    rs, rst = _steps(P, ref, P.n_steps)
    gs, gst = _steps(P, g, P.n_steps)
    info = g.info()
    print(f"[graph, set growth] sweep-2 rows per step {[x[1][0] for x in rst]}; graph steps "
          f"{info['graph_steps']}, captures {info['graph_captures']}, redone {info['graph_redone']}", flush=True)
    for q in range(P.n_steps):
        assert np.array_equal(rs[q][0], gs[q][0]) and np.array_equal(rs[q][1], gs[q][1]), q
        assert rst[q] == gst[q], q
    assert info["graph_redone"] >= 1 and info["graph_captures"] >= 2
