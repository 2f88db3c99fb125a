"""GPU parity of the a-priori drop tolerance (Sec. 4.1, eq. drop-tolerance)
against the oracle.

The library computes each instance's TOL_drop on the device after the
step's first sweep; the oracle replays the GPU's active sets and computes
its own tolerances from its own first sweep.  Compared: the integer r
exactly, TOL_drop, c and eta to rounding (they come from max / min
reductions of corrections and states that agree to the CG tolerance), the
states within 1e-10 relative, and the selected sets row by row wherever the
oracle's correction is not within 1e-9 of the GPU's tolerance.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.sdc import apply_stimuli, build  # noqa: E402
from workloads import config1, config3, config4  # noqa: E402

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


def _problem(case):
    if case == "single":
        return config1(n=40, theta=1e-7, n_steps=3)
    P = config4(n_inst=3, sizes=(10, 20), n_steps=2)
    lo1 = P.node_off[1]   # instance 0 without stimulus: at rest
    P.stimuli = [(t, nodes[nodes >= lo1], val) for t, nodes, val in P.stimuli]
    return P


@pytest.mark.parametrize("case", ["single", "batched"])
def test_apriori_drop_tolerance_matches_oracle(case):
    P = _problem(case)
    K, tol, rho = 5, 1e-5, 0.3
    s = _solver(P, K=K, tol_sdc=tol, rho=rho, K_min=K, drop="apriori")
    orc = build(P, tol_sdc=tol, rho=rho, K_min=K, drop="apriori")
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    ov, ow = P.v_init.copy(), P.w_init.copy()
    for n in range(P.n_steps):
        t = n * P.dt
        print(f"[drop {case}] step {n}", flush=True)
        s.begin_step(v, w, t)
        sets, drop = [None], None
        counts = []
        for k in range(K):
            s.sweep()
            counts.append(s.cg_iters())
            if k == 0:
                drop = s.drop_tolerance()
            if k + 1 < K:
                sets.append(s.active().cpu().numpy().astype(np.int64))
        s.end_step(v, w)
        apply_stimuli(ov, t, P.dt, P.stimuli)
        ov, ow, infos = orc.step(ov, ow, K, idx_replay=sets, keep=True)
        od = infos[0]
        print(f"   TOL_drop gpu {drop['tol_drop']} oracle {od['drop_tol']}; r {drop['r']} / {od['drop_r']}",
              flush=True)
        assert np.array_equal(drop["r"], od["drop_r"])
        assert np.allclose(drop["tol_drop"], od["drop_tol"], rtol=1e-10, atol=0)
        assert np.allclose(drop["c"], od["drop_c"], rtol=1e-9, atol=1e-300)
        assert np.allclose(drop["eta"], od["drop_eta"], rtol=1e-9, atol=1e-12)
        # the second set: rows of the first with max |dv| >= the instance's TOL_drop
        amax, idx0 = od["amax"], np.arange(P.N)
        th = drop["tol_drop"][orc.inst_of[idx0]]
        clear = np.abs(amax - th) > 1e-9 * th
        keep = amax >= th
        got = np.zeros(P.N, dtype=bool)
        got[sets[1]] = True
        assert np.array_equal(got[clear], keep[clear])
        assert 0 < sets[1].size < P.N
        assert rel(v.cpu().numpy(), ov) < 1e-10 and rel(w.cpu().numpy(), ow) < 1e-10
        assert np.abs(v.cpu().numpy() - ov).max() <= 1e-10 * np.abs(ov).max()
        # per node and instance, every solve's CG step count within one of the oracle's
        assert all(np.abs(g - np.stack(i["cg_iters_inst"])).max() <= 1 for g, i in zip(counts, infos))
        if case == "batched":
            # the instance at rest: c = 0, r = 0, eta = 0, so exactly (1 - rho) tol; none of its rows stays
            assert drop["tol_drop"][0] == (1.0 - rho) / 1 * tol and drop["r"][0] == 0
            assert not np.any(sets[1] < P.node_off[1])


def test_apriori_drop_rejected_for_cell_by_cell_and_queried_without_it():
    from paper_2311_07206_amd import SDCError
    P = config3(nc=2, nr=1, nx=3, ny=3)
    with pytest.raises(SDCError, match="monodomain"):
        _solver(P, tol_sdc=1e-4, rho=0.3, drop="apriori")
    Q = config1(n=12, theta=1e-7)
    with pytest.raises(SDCError, match="tol_sdc"):
        _solver(Q, drop="apriori")
    s = _solver(Q)
    with pytest.raises(SDCError, match="STATE|not enabled"):
        s.drop_tolerance()
