"""GPU parity of the energy-norm SDC termination (Sec. 3.2) against the oracle.

The library decides on the device, per instance, after each sweep; the
oracle replays the GPU's active sets and takes its own decisions, which must
agree (the test prints the energies against the threshold).  States within
1e-10 relative; the step entry point equals the sweep-by-sweep loop bitwise.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.sdc import build, run  # noqa: E402
from workloads import config1, config4  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _solver(P, **kw):
    from paper_2311_07206_amd import Solver
    return Solver.from_problem(P, **kw)


def _gpu_steps(P, s, n_steps, K):
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    sets, counts, energies = [], [], []
    for n in range(n_steps):
        s.begin_step(v, w, n * P.dt)
        step_sets = [None]
        es = []
        for k in range(K):
            st = s.sweep()
            es.append(st["energy"])
            s._counts.append(s.cg_iters())
            if st["n_stopped"] == P.n_inst or k + 1 == K:
                break
            step_sets.append(s.active().cpu().numpy().astype(np.int64))
        s.end_step(v, w)
        sets.append(step_sets)
        counts.append(k + 1)
        energies.append(es)
    return v.cpu().numpy(), w.cpu().numpy(), sets, counts, energies


@pytest.mark.parametrize("case", ["single", "batched"])
def test_energy_termination_matches_oracle(case):
    K, rho, tol = 8, 0.3, 3e-6
    if case == "single":
        P = config1(n=33, theta=1e-7, n_steps=4)
    else:
        P = config4(n_inst=3, sizes=(10, 18), n_steps=3)
        lo1 = P.node_off[1]   # instance 0 without stimulus: at rest, stops after one sweep
        P.stimuli = [(t, nodes[nodes >= lo1], val) for t, nodes, val in P.stimuli]
    s = _solver(P, K=K, tol_sdc=tol, rho=rho, K_min=1)
    s._counts = []
    gv, gw, sets, counts, energies = _gpu_steps(P, s, P.n_steps, K)
    thr = ((1 - rho) / rho * tol) ** 2
    print(f"[termination {case}] sweeps per step {counts}, threshold {thr:.3e}", flush=True)
    for es in energies:
        print("   energies " + " ".join(f"{e:.3e}" for e in es), flush=True)
    orc = build(P, tol_sdc=tol, rho=rho, K_min=1)
    ov, ow, log = run(orc, P.v_init, P.w_init, P.n_steps, K, P.stimuli, idx_replay=sets)
    assert [len(st) for st in log] == counts
    assert any(c < K for c in counts)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
    assert np.abs(gv - ov).max() <= 1e-10 * np.abs(ov).max()
    # per node and instance, every solve's CG step count within one of the oracle's
    oc = [np.stack(i["cg_iters_inst"]) for st in log for i in st]
    assert len(oc) == len(s._counts) and all(np.abs(g - o).max() <= 1 for g, o in zip(s._counts, oc))
    # the step entry point takes the same decisions
    s2 = _solver(P, K=K, tol_sdc=tol, rho=rho, K_min=1)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    for n in range(P.n_steps):
        stats = s2.step(v, w, n * P.dt, stats=True)
        assert len(stats) == counts[n]
    assert np.array_equal(v.cpu().numpy(), gv) and np.array_equal(w.cpu().numpy(), gw)


def test_energy_termination_rejected_with_reverse_pass():
    from paper_2311_07206_amd import SDCError
    P = config1(n=12, theta=1e-7)
    s = _solver(P, tol_sdc=1e-6, rho=0.3)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    with pytest.raises(SDCError, match="STATE"):
        s.adjoint_record(0, v, w, 0.0)
