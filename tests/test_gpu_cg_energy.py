"""GPU parity of the optional energy-error CG stop (Sec. 5.1's estimated
energy-error reduction, the estimator a reading; see oracle.pcg).

The GPU's solves run the single-reduction CG (and, for small sets, the
one-workgroup plain PCG); the oracle's run textbook PCG.  Their step terms
alpha_j gamma_j agree to rounding, so each solve stops after the same number
of steps unless the estimate lands within rounding of the threshold, which
these seeded cases do not.  Checked: every solve's step count equals the
oracle's own decision on the same index sets, and the states agree within
1e-10; a vanishing tolerance gives the default run bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.sdc import apply_stimuli, build  # noqa: E402
from workloads import config0, config1, config2, config3, config4  # noqa: E402

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


def _run_gpu(P, s, n_steps, K):
    """Steps sweep by sweep: the sets after the first sweep and every
    sweep's per-node step counts (largest over instances)."""
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    sets, iters = [], []
    for n in range(n_steps):
        s.begin_step(v, w, n * P.dt)
        step_sets, step_iters = [None], []
        for k in range(K):
            st = s.sweep()
            step_iters.append(list(st["cg_iters_max"]))
            if k + 1 < K:
                step_sets.append(s.active().cpu().numpy().astype(np.int64))
        s.end_step(v, w)
        sets.append(step_sets)
        iters.append(step_iters)
    return v.cpu().numpy(), w.cpu().numpy(), sets, iters


def _run_oracle(P, orc, n_steps, K, sets):
    v, w = P.v_init.copy(), P.w_init.copy()
    iters = []
    for n in range(n_steps):
        apply_stimuli(v, n * P.dt, P.dt, P.stimuli)
        v, w, infos = orc.step(v, w, K, idx_replay=sets[n])
        iters.append([list(i["cg_iters"]) for i in infos])
    return v, w, iters


@pytest.mark.parametrize("case", ["1d", "2d", "3d", "batched", "2d_small_sets", "2d_linearized"])
def test_energy_stop_matches_oracle(case):
    tol, delay, kw, okw = 1e-3, 4, {}, {}
    if case == "1d":
        P, n_steps = config0(theta=1e-6), 30
    elif case in ("2d", "2d_small_sets", "2d_linearized"):
        P, n_steps = config1(n=41, theta=1e-7), 8
        if case == "2d":
            kw["small_set_rows"] = -1      # every solve one launch per iteration
        if case == "2d_linearized":
            kw["scheme"] = okw["scheme"] = "linearized"
    elif case == "3d":
        P, n_steps = config2(n=11, theta=1e-7), 3
        tol, delay = 1e-4, 3
    else:
        P, n_steps = config4(n_inst=3, sizes=(10, 18)), 4
    s = _solver(P, cg_energy_tol=tol, cg_delay=delay, **kw)
    print(f"[cg energy {case}] N={P.N} tol={tol} d={delay}", flush=True)
    gv, gw, sets, giters = _run_gpu(P, s, n_steps, P.K)
    orc = build(P, cg_energy_tol=tol, cg_delay=delay, **okw)
    ov, ow, oiters = _run_oracle(P, orc, n_steps, P.K, sets)
    print(f"   steps per solve {giters[-1]}; rel v {rel(gv, ov):.2e} w {rel(gw, ow):.2e}", flush=True)
    assert giters == oiters
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
    # the stop shortens the solves against the residual stop on the same sets
    full = build(P, **okw)
    _, _, fiters = _run_oracle(P, full, n_steps, P.K, sets)
    assert sum(map(sum, sum(giters, []))) < sum(map(sum, sum(fiters, [])))


def test_vanishing_tolerance_is_the_default_run_bitwise():
    P = config0(n=96, theta=1e-6, n_steps=20)
    a = _solver(P, cg_energy_tol=1e-300, cg_delay=8)
    b = _solver(P)
    va, wa, _, ia = _run_gpu(P, a, P.n_steps, P.K)
    vb, wb, _, ib = _run_gpu(P, b, P.n_steps, P.K)
    assert ia == ib and np.array_equal(va, vb) and np.array_equal(wa, wb)


def test_energy_stop_rejections():
    from paper_2311_07206_amd import SDCError
    with pytest.raises(SDCError, match="monodomain"):
        _solver(config3(nc=2, nr=1, nx=3, ny=3), cg_energy_tol=1e-3)
    with pytest.raises(SDCError, match="cg_delay"):
        _solver(config0(n=16), cg_energy_tol=1e-3, cg_delay=9)
    with pytest.raises(SDCError, match="cg_energy_tol"):
        _solver(config0(n=16), cg_energy_tol=-1.0)
    P = config0(n=32, theta=1e-6)
    s = _solver(P, cg_energy_tol=1e-3)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    with pytest.raises(SDCError, match="STATE"):
        s.adjoint_record(0, v, w, 0.0)


@pytest.mark.parametrize("n,n_steps", [(512, 3), (600, 1)])
def test_energy_stop_at_full_size(n, n_steps):
    """The 512 x 512 workload with the paper's tolerance (1e-3) over three
    steps from the stimulus, and 600 x 600 (over 1024 map entries per
    instance: the separate totals pass) for one step."""
    P = config1(n=n, theta=1e-7, n_steps=n_steps)
    s = _solver(P, cg_energy_tol=1e-3, cg_delay=4)
    print(f"[cg energy full] N={P.N}", flush=True)
    gv, gw, sets, giters = _run_gpu(P, s, n_steps, P.K)
    print(f"[cg energy full] steps per solve {giters}; oracle replay", flush=True)
    ov, ow, oiters = _run_oracle(P, build(P, cg_energy_tol=1e-3, cg_delay=4), n_steps, P.K, sets)
    print(f"[cg energy full] rel v {rel(gv, ov):.2e} w {rel(gw, ow):.2e}", flush=True)
    assert giters == oiters
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
