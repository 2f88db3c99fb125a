"""A step whose time does not continue the last step begun (a window run
again from a saved state, a restart from a checkpoint) takes the
synchronous CG loop at once: the iteration budgets predicted from the last
step's counts belong to another time.  Such a step is never counted as
redone and never runs as graph-captured sweeps, and the window run again
reproduces the first run bitwise, step by step (host-launched and
graph-captured sweeps)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from workloads import config1, config4  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", ["2d", "batched"])
def test_window_run_again_matches_and_is_not_redone(case, graph):
    from paper_2311_07206_amd import Solver
    P = config1(n=48, theta=1e-7) if case == "2d" else config4(n_inst=4, sizes=(24, 40))
    n0, n1 = 3, 9
    print(f"[restart {case}, graph {graph}] N={P.N}, steps {n0}..{n1 - 1} run twice", flush=True)
    s = Solver.from_problem(P, small_set_rows=-1)
    if graph:
        s.set_graph(True)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    first, saved = [], None
    for n in range(n1):
        if n == n0:
            saved = (v.clone(), w.clone())
        s.step(v, w, n * P.dt)
        if n >= n0:
            first.append((v.cpu().numpy().copy(), w.cpu().numpy().copy()))
    v, w = saved[0].clone(), saved[1].clone()
    g0 = s.info()["graph_steps"]
    for n in range(n0, n1):
        i0 = s.info()
        s.step(v, w, n * P.dt)
        i1 = s.info()
        if n == n0:
            # the step back in time: synchronous loop, no redo, no graph
            assert i1["redone_steps"] == i0["redone_steps"]
            assert i1["graph_redone"] == i0["graph_redone"]
            assert i1["graph_steps"] == i0["graph_steps"]
        assert np.array_equal(v.cpu().numpy(), first[n - n0][0]), n
        assert np.array_equal(w.cpu().numpy(), first[n - n0][1]), n
    if graph:   # the steps after the one back in time replay graphs again
        assert s.info()["graph_steps"] - g0 >= n1 - n0 - 2
    s.close()
