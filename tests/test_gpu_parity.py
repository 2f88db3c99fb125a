"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerances: floating-point results within 1e-10 relative L2 of the oracle
(FP64 on both sides; differences come from summation order and fused
multiply-adds, amplified at most by the CG tolerance 1e-12 and the SDC
contraction), CG solutions within 1e-11 relative, index sets bit-exact when
both sides see the same correction maxima.  Full runs replay the GPU's
active sets in the oracle, so a threshold comparison that rounding could
flip cannot make the two runs diverge; the free-running sets are compared
separately.
"""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.assembly import lumped_mass, stiffness  # noqa: E402
from oracle.pcg import jacobi_pcg  # noqa: E402
from oracle.sdc import apply_stimuli, build, run, select  # noqa: E402
from workloads import config0, config1, config2, config4  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(P, **kw):
    from paper_2311_07206_amd import Solver
    return Solver.from_problem(P, **kw)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu_run(P, n_steps, s=None, t0=0.0, v=None, w=None):
    """Free-running GPU steps in parts; returns final state, per-step sets and stats."""
    s = s or _solver(P)
    v = torch.tensor(P.v_init if v is None else v, device=DEV)
    w = torch.tensor(P.w_init if w is None else w, device=DEV)
    sets, stats = [], []
    for n in range(n_steps):
        t = t0 + n * P.dt
        print(f"[gpu_run] {P.name} N={P.N} step {n}", flush=True)
        s.begin_step(v, w, t)
        step_sets = [None]
        step_stats = []
        for k in range(P.K):
            step_stats.append(s.sweep())
            step_stats[-1]["iters_inst"] = s.cg_iters()
            if k + 1 < P.K:
                step_sets.append(s.active().cpu().numpy().astype(np.int64))
        s.end_step(v, w)
        sets.append(step_sets)
        stats.append(step_stats)
    torch.cuda.synchronize()
    return v.cpu().numpy(), w.cpu().numpy(), sets, stats, s


# ---------------------------------------------------------------- assembly

@pytest.mark.parametrize("P", [config0(n=37), config1(n=19), config2(n=6), config4(n_inst=3, sizes=(9, 14))],
                         ids=["1d", "2d", "3d", "batch"])
def test_assembly_matches_oracle(P):
    s = _solver(P)
    rp, col, val, ml = s.system()
    A = stiffness(P.coords, P.elems, P.elem_tensor, P.node_sigma, P.N)
    A.eliminate_zeros()
    G = sp.csr_matrix((val, col, rp), shape=(P.N, P.N))
    assert abs(G - A).max() <= 1e-14 * abs(A).max()
    assert (G != G.T).nnz == 0          # exactly symmetric (the diagonal storage keeps offsets >= 0)
    assert np.allclose(ml, lumped_mass(P.coords, P.elems, P.N), rtol=1e-14, atol=0)
    for i in range(P.N):   # sorted columns, diagonal present
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c


# ---------------------------------------------------------------- components

@pytest.mark.parametrize("M,m", [(3, 0), (3, 1), (4, 3)])
def test_restricted_pcg_matches_oracle(M, m):
    P = config1(n=41)
    P.M = M
    s = _solver(P)
    orc = build(P)
    rng = np.random.default_rng(m)
    for trial, frac in enumerate((1.0, 0.5, 0.05, 0.003)):
        n = max(1, int(frac * P.N))
        idx = np.sort(rng.choice(P.N, size=n, replace=False)) if frac < 1 else np.arange(P.N)
        b = rng.standard_normal(P.N)
        print(f"[pcg] M={M} m={m} n={n}", flush=True)
        x, iters = s.solve(m, torch.tensor(idx, dtype=torch.int32, device=DEV), torch.tensor(b, device=DEV))
        xo, ito = jacobi_pcg(orc.H[m], b, idx, P.cg_rtol)
        xg = x.cpu().numpy()
        assert rel(xg, xo) < 1e-11
        mask = np.ones(P.N, bool)
        mask[idx] = False
        assert np.all(xg[mask] == 0.0)
        assert abs(iters[0] - ito) <= 1


def test_pcg_on_instance_larger_than_in_kernel_reduction():
    # more than 1024 blocks of 256 rows: the partial sums go through the
    # per-instance totals pass
    P = config1(n=700)
    s = _solver(P)
    orc = build(P)
    rng = np.random.default_rng(11)
    for frac in (1.0, 0.6):
        n = int(frac * P.N)
        idx = np.arange(P.N) if frac == 1.0 else np.sort(rng.choice(P.N, size=n, replace=False))
        assert (n + 255) // 256 > 1024
        b = rng.standard_normal(P.N)
        print(f"[pcg large] n={n}", flush=True)
        x, iters = s.solve(2, torch.tensor(idx, dtype=torch.int32, device=DEV), torch.tensor(b, device=DEV))
        xo, ito = jacobi_pcg(orc.H[2], b, idx, P.cg_rtol)
        assert rel(x.cpu().numpy(), xo) < 1e-11
        assert abs(iters[0] - ito) <= 1


def test_pcg_edge_cases():
    P = config0(n=50)
    s = _solver(P)
    empty = torch.zeros(0, dtype=torch.int32, device=DEV)
    b = torch.ones(P.N, dtype=torch.float64, device=DEV)
    x, it = s.solve(0, empty, b)
    assert it == [0] and torch.all(x == 0)
    allrows = torch.arange(P.N, dtype=torch.int32, device=DEV)
    x, it = s.solve(1, allrows, torch.zeros(P.N, dtype=torch.float64, device=DEV))
    assert it == [0] and torch.all(x == 0)
    one = torch.tensor([17], dtype=torch.int32, device=DEV)
    x, it = s.solve(2, one, b)
    orc = build(P)
    assert it == [1] and abs(x[17].item() - 1.0 / orc.H[2][17, 17]) < 1e-15


def test_selection_bit_exact():
    P = config4(n_inst=3, sizes=(30, 60))
    s = _solver(P)
    rng = np.random.default_rng(3)
    amax = np.abs(rng.standard_normal(P.N)) * 1e-6
    theta = 1e-6
    amax[rng.choice(P.N, 50, replace=False)] = theta          # ties are kept
    amax[rng.choice(P.N, 5, replace=False)] = np.nan          # NaN is dropped
    amax_d = torch.tensor(amax, device=DEV)
    for frac in (1.0, 0.4, 0.01, 0.0):
        idx = np.sort(rng.choice(P.N, size=int(frac * P.N), replace=False)).astype(np.int64)
        got = s.select(amax_d, torch.tensor(idx, dtype=torch.int32, device=DEV), theta).cpu().numpy()
        assert np.array_equal(got, select(idx, amax, theta))
        got0 = s.select(amax_d, torch.tensor(idx, dtype=torch.int32, device=DEV), 0.0).cpu().numpy()
        assert np.array_equal(got0, idx)


# ---------------------------------------------------------------- sweeps and steps

def test_one_sweep_matches_oracle_node_by_node():
    P = config1(n=45, theta=1e-7)
    s = _solver(P)
    orc = build(P)
    v0 = P.v_init.copy()
    apply_stimuli(v0, 0.0, P.dt, P.stimuli)
    st = orc.spread(v0, P.w_init.copy())
    nxt, _ = orc.sweep(st, np.arange(P.N))
    s.begin_step(torch.tensor(P.v_init, device=DEV), torch.tensor(P.w_init, device=DEV), 0.0)
    s.sweep()
    for m in range(P.M):
        vm, wm = s.node(m)
        assert rel(vm.cpu().numpy(), st["v"][m]) < 1e-12
        assert rel(wm.cpu().numpy(), st["w"][m]) < 1e-12
    got = s.active().cpu().numpy()
    # membership can differ only where the maximum correction lies within rounding of theta
    diff = np.setxor1d(got, nxt)
    assert diff.size <= 2


@pytest.mark.parametrize("theta", [0.0, 1e-6])
def test_config0_full_run_matches_oracle(theta):
    P = config0(theta=theta)
    gv, gw, sets, stats, _ = gpu_run(P, P.n_steps)
    ov, ow, log = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
    for n in range(P.n_steps):
        for k in range(P.K):
            assert stats[n][k]["n_active"] == log[n][k]["n_active"]
    if theta > 0:
        assert any(st[-1]["n_active"] < P.N for st in stats)


def test_config0_free_running_sets_match_oracle():
    P = config0(theta=1e-6, n_steps=120)
    _, _, sets, _, _ = gpu_run(P, P.n_steps)
    _, _, log = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    flips = sum(np.setxor1d(sets[n][k], log[n][k]["idx"]).size
                for n in range(P.n_steps) for k in range(1, P.K))
    assert flips <= 4


def test_step_entry_equals_sweep_by_sweep():
    P = config0(n=128, theta=1e-6, n_steps=40)
    s1, s2 = _solver(P), _solver(P)
    v1 = torch.tensor(P.v_init, device=DEV)
    w1 = torch.tensor(P.w_init, device=DEV)
    for n in range(P.n_steps):
        s1.step(v1, w1, n * P.dt)
    v2, w2, _, _, _ = gpu_run(P, P.n_steps, s=s2)
    assert np.array_equal(v1.cpu().numpy(), v2) and np.array_equal(w1.cpu().numpy(), w2)


def test_pinned_all_rows_equals_nonadaptive_bitwise():
    P = config0(n=100, theta=1e-6, n_steps=30)
    P0 = config0(n=100, theta=0.0, n_steps=30)
    s = _solver(P)
    allrows = torch.arange(P.N, dtype=torch.int32, device=DEV)
    for k in range(1, P.K):
        s.set_active(k, allrows)
    a = gpu_run(P, P.n_steps, s=s)
    b = gpu_run(P0, P0.n_steps)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    s.set_active(0, None)


@pytest.mark.parametrize("density", [0.2, 0.01])
def test_pinned_front_shell_sets_match_oracle(density):
    """Sweeps 1..K-1 pinned to a front-shell mask (the sets the sweep latency
    measurement times) compute what the oracle computes on those sets."""
    import bench
    P = config1(n=41, theta=1e-7, n_steps=3)
    v = P.v_init.copy()
    apply_stimuli(v, 0.0, P.dt, P.stimuli)
    mask = bench.front_shell_masks(P.coords, P.elems, v, (density,))[0]
    assert 0 < mask.size < P.N
    s = _solver(P)
    pin = torch.tensor(mask, dtype=torch.int32, device=DEV)
    for k in range(1, P.K):
        s.set_active(k, pin)
    gv, gw, sets, _, _ = gpu_run(P, P.n_steps, s=s)
    s.set_active(0, None)
    assert all(np.array_equal(st, mask) for step in sets for st in step[1:])
    ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli,
                    idx_replay=[[None] + [mask.astype(np.int64)] * (P.K - 1)] * P.n_steps)
    print(f"[pinned shell] density {density}: {mask.size} rows, rel v {rel(gv, ov):.2e}", flush=True)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10


@pytest.mark.parametrize("P", [config0(n=200, theta=1e-6, n_steps=10), config1(n=33, theta=1e-7, n_steps=4),
                               config2(n=10, theta=1e-7, n_steps=3)], ids=["1d", "2d", "3d"])
def test_small_sets_are_solved_in_one_launch(P):
    """Sets of one workgroup's size run the whole solve in one launch (no
    per-iteration launches in the kernel timing); with that path off, one
    launch per iteration.  Both match the oracle on their own sets."""
    for rows, per_iteration in ((0, False), (-1, True)):
        s = _solver(P, small_set_rows=rows)
        s.profile(True)
        gv, gw, sets, _, _ = gpu_run(P, P.n_steps, s=s)
        launches = s.profile_read()["cg_launches"]
        s.profile(False)
        print(f"[small sets] {P.name} N={P.N} small_set_rows={rows}: {launches} CG launches", flush=True)
        assert (launches > 0) == per_iteration
        assert np.abs(gv).max() > 1e-3   # a stimulated run, not the rest state
        ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
        assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10


def test_solve_path_switches_within_a_step():
    """A threshold between the all-rows set and the later sets: the first
    sweep launches per iteration, smaller sweeps solve in one launch."""
    P = config0(n=200, theta=1e-6, n_steps=12)
    s = _solver(P, small_set_rows=150)
    s.profile(True)
    gv, gw, sets, stats, _ = gpu_run(P, P.n_steps, s=s)
    assert s.profile_read()["cg_launches"] > 0
    s.profile(False)
    assert any(0 < len(st) <= 150 for step in sets for st in step[1:])
    ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
    # the synchronous and the asynchronous sweeps agree bitwise across the switch
    s2 = _solver(P, small_set_rows=150)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    for n in range(P.n_steps):
        s2.step(v, w, n * P.dt)
    assert np.array_equal(v.cpu().numpy(), gv) and np.array_equal(w.cpu().numpy(), gw)


@pytest.mark.parametrize("P", [config0(n=300, theta=0.0, n_steps=6), config1(n=40, theta=0.0, n_steps=3),
                               config2(n=11, theta=0.0, n_steps=2)], ids=["1d", "2d", "3d"])
def test_rows_per_thread_of_all_rows_launches_agree_bitwise(P):
    """Every sweep on all rows (theta = 0, one launch per CG iteration): one
    and two rows per thread give the same bits, and the oracle's result."""
    runs = []
    for rpt in (1, 2):
        s = _solver(P, rows_per_thread=rpt, small_set_rows=-1)
        assert s.info()["format"] == "dia" and s.info()["rows_per_thread"] == rpt
        runs.append(gpu_run(P, P.n_steps, s=s)[:2])
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    assert rel(runs[0][0], ov) < 1e-10 and rel(runs[0][1], ow) < 1e-10


def test_rows_per_thread_timed_at_setup():
    # timed on maps of 2048 blocks and more; smaller ones keep two rows
    info = _solver(config1(n=800, theta=1e-7)).info()
    assert info["format"] == "dia" and info["rows_per_thread"] in (1, 2)
    assert info["t_rows1_us"] > 0 and info["t_rows2_us"] > 0
    small = _solver(config1(n=64, theta=1e-7)).info()
    assert small["rows_per_thread"] == 2 and small["t_rows1_us"] == 0
    csr = _solver(config1(n=64, theta=1e-7), fmt=1).info()
    assert csr["rows_per_thread"] == 1 and csr["t_rows1_us"] == 0


def test_ragged_2d_adaptive_run():
    P = config1(n=23, theta=1e-7, n_steps=12)
    gv, gw, sets, _, _ = gpu_run(P, P.n_steps)
    ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10


def test_3d_adaptive_steps():
    P = config2(n=11, theta=1e-7, n_steps=6)   # the smallest grids miss the stimulus balls
    assert all(len(nodes) > 0 for _, nodes, _ in P.stimuli)
    gv, gw, sets, _, _ = gpu_run(P, P.n_steps)
    assert np.abs(gv).max() > 1e-3
    ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10


def assert_counts(stats, log, slack=1):
    """Every restricted solve's CG step count, per node and instance, within
    `slack` of the oracle's (the library's single-reduction recurrences round
    differently from textbook PCG near the stopping test)."""
    for gs, os_ in zip(stats, log):
        for g, o in zip(gs, os_):
            got = np.asarray(g["iters_inst"])
            want = np.stack([np.asarray(c) for c in o["cg_iters_inst"]])
            assert got.shape == want.shape and np.abs(got - want).max() <= slack, (got, want)


def test_batched_instances_match_oracle_per_instance():
    P = config4(n_inst=3, sizes=(16, 24), n_steps=8)
    gv, gw, sets, stats, _ = gpu_run(P, P.n_steps)
    orc = build(P)
    ov, ow, log = run(orc, P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
    assert np.abs(gv - ov).max() <= 1e-10 * np.abs(ov).max()
    assert_counts(stats, log)
    # the instances' solves stop at different step counts
    assert any(len(set(st["iters_inst"][m].tolist())) > 1 for step in stats for st in step for m in range(P.M))
    # each instance alone in the oracle (own mesh, own CG stopping test)
    for i in range(P.n_inst):
        lo, hi = P.node_off[i], P.node_off[i + 1]
        sub = _instance(P, i)
        osub = build(sub)
        rep = [[None] + [s_[(s_ >= lo) & (s_ < hi)] - lo for s_ in st[1:]] for st in sets]
        ov, ow, _ = run(osub, sub.v_init, sub.w_init, P.n_steps, P.K, sub.stimuli, idx_replay=rep)
        assert rel(gv[lo:hi], ov) < 1e-10 and rel(gw[lo:hi], ow) < 1e-10
    assert orc.model.N == P.N


def test_batched_chunked_xcd_order_matches_oracle():
    """A batch whose work map spans full rounds of XCD chunks and a shorter
    tail in eighths: every row is processed once, the result matches the
    oracle (the order changes no arithmetic)."""
    P = config4(n_inst=8, sizes=(40, 56), n_steps=3)
    s = _solver(P)
    chunk = s.info()["xcd_chunk"]
    nblk = int(sum((np.diff(P.node_off) + 255) // 256))
    reach = max(int(n) + 2 for n in np.sqrt(np.diff(P.node_off)).round())   # 2D grid: (side + 1) + 1
    print(f"[xcd order] {nblk} blocks, chunk {chunk}, reach {reach}", flush=True)
    assert chunk == max(4, 1 << int(np.ceil(np.log2((8 * reach + 255) // 256))))
    assert 8 * chunk <= nblk and nblk % (8 * chunk) != 0
    gv, gw, sets, stats, _ = gpu_run(P, P.n_steps, s=s)
    ov, ow, log = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
    assert np.abs(gv - ov).max() <= 1e-10 * np.abs(ov).max()
    assert_counts(stats, log)


def _instance(P, i):
    from workloads.configs import Problem
    lo, hi = int(P.node_off[i]), int(P.node_off[i + 1])
    e0, e1 = int(P.elem_off[i]), int(P.elem_off[i + 1])
    stim = [(t, nodes[(nodes >= lo) & (nodes < hi)] - lo, val) for t, nodes, val in P.stimuli]
    return Problem(name="inst", dim=P.dim, coords=P.coords[lo:hi], elems=P.elems[e0:e1] - lo,
                   elem_tensor=P.elem_tensor[e0:e1], node_sigma=P.node_sigma[lo:hi],
                   node_off=np.array([0, hi - lo]), elem_off=np.array([0, e1 - e0]),
                   ionic=P.ionic[i:i + 1], M=P.M, K=P.K, dt=P.dt, n_steps=P.n_steps, theta=P.theta,
                   cg_rtol=P.cg_rtol, cg_maxit=P.cg_maxit, stimuli=stim,
                   v_init=P.v_init[lo:hi], w_init=P.w_init[lo:hi])


def test_rest_state_and_everything_dropped():
    P = config1(n=20, theta=1e-7)
    s = _solver(P)
    v = torch.zeros(P.N, dtype=torch.float64, device=DEV)
    w = torch.zeros(P.N, dtype=torch.float64, device=DEV)
    st = s.step(v, w, 5.0, stats=True)   # no stimulus at t = 5
    assert torch.all(v == 0) and torch.all(w == 0)
    assert st[0]["n_active"] == P.N and st[1]["n_active"] == 0 and st[0]["cg_iters_max"] == [0] * P.M
    # a huge threshold drops every row after the first sweep
    P2 = config1(n=20, theta=1e10, n_steps=3)
    gv, gw, sets, stats, _ = gpu_run(P2, 3)
    ov, ow, _ = run(build(P2), P2.v_init, P2.w_init, 3, P2.K, P2.stimuli, idx_replay=sets)
    assert all(st_[1]["n_active"] == 0 for st_ in stats)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10


def test_full_size_2d_steps():
    # the 512 x 512 workload at full size: two steps from the stimulus
    P = config1(theta=1e-7, n_steps=2)
    gv, gw, sets, stats, _ = gpu_run(P, P.n_steps)
    ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
    assert stats[0][0]["n_active"] == 512 * 512


def test_full_size_3d_steps():
    # the 128^3 workload at full size: two steps from the stimulus, the first
    # sweeps on all 2.1 M rows (about a minute of oracle work on the host)
    P = config2(theta=1e-7, n_steps=2)
    gv, gw, sets, stats, _ = gpu_run(P, P.n_steps)
    print("[3d full steps] oracle replay", flush=True)
    ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli, idx_replay=sets)
    print(f"[3d full steps] rel v {rel(gv, ov):.2e} w {rel(gw, ow):.2e}", flush=True)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10
    assert stats[0][0]["n_active"] == P.N and all(len(st) < P.N for st in sets[1][1:])


def test_large_2d_step():
    # one adaptive step on 600 x 600 (over 1024 blocks per sweep at the start)
    P = config1(n=600, theta=1e-7, n_steps=1)
    gv, gw, sets, stats, _ = gpu_run(P, 1)
    ov, ow, _ = run(build(P), P.v_init, P.w_init, 1, P.K, P.stimuli, idx_replay=sets)
    assert rel(gv, ov) < 1e-10 and rel(gw, ow) < 1e-10


def test_errors_are_reported():
    from paper_2311_07206_amd import SDCError
    P = config0(n=40)
    s = _solver(P, cg_maxit=2)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    with pytest.raises(SDCError, match="CG_MAXIT"):
        s.step(v, w, 0.0)
    s2 = _solver(P)
    vn = v.clone()
    vn[5] = float("nan")
    with pytest.raises(SDCError, match="NONFINITE"):
        s2.step(vn, w, 1.0)
    with pytest.raises(SDCError, match="STATE"):
        s2.sweep()


# sizes with map entries whose stencil stays inside the instance, so that the
# all-rows iteration's two-rows-per-thread path is compared with CSR too
@pytest.mark.parametrize("P", [config0(n=1100, theta=1e-6, n_steps=20), config1(n=33, theta=1e-7, n_steps=6),
                               config2(n=16, theta=1e-7, n_steps=4), config4(n_inst=3, sizes=(12, 20), n_steps=5)],
                         ids=["1d", "2d", "3d", "batch"])
def test_diagonal_and_csr_storage_agree_bitwise(P):
    runs = []
    for fmt in (1, 2):
        s = _solver(P, fmt=fmt)
        assert s.info()["format"] == {1: "csr", 2: "dia"}[fmt]
        v = torch.tensor(P.v_init, device=DEV)
        w = torch.tensor(P.w_init, device=DEV)
        for n in range(P.n_steps):
            s.step(v, w, n * P.dt)
        runs.append((v.cpu().numpy(), w.cpu().numpy()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    ov, ow, _ = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    assert rel(runs[1][0], ov) < 1e-8   # free-running sets: flips near theta perturb by ~theta


def test_invalid_index_lists_are_rejected():
    from paper_2311_07206_amd import SDCError
    P = config0(n=60)
    s = _solver(P)
    b = torch.ones(P.N, dtype=torch.float64, device=DEV)
    for bad in ([3, 2, 5], [0, 60], [-1, 4], [7, 7]):
        idx = torch.tensor(bad, dtype=torch.int32, device=DEV)
        with pytest.raises(SDCError, match="ARG"):
            s.solve(0, idx, b)
        with pytest.raises(SDCError, match="ARG"):
            s.select(b, idx, 0.5)
    # a good call still works afterwards
    x, it = s.solve(0, torch.arange(P.N, dtype=torch.int32, device=DEV), b)
    assert it[0] > 0 and torch.isfinite(x).all()


def test_list_maps_count_stored_entries_and_reject_bad_lists():
    """Work maps built from a device list (pinned sets, restricted solves):
    the stored entries of a pinned sweep are those of the listed rows of A,
    with lists whose 256-entry blocks span several instances and instances
    without entries; a list out of order, with a repeated entry, or with an
    entry outside [0, N) is rejected."""
    from paper_2311_07206_amd import SDCError
    P = config4(n_inst=7, sizes=(12, 30))
    s = _solver(P)
    rp = s.system()[0]
    rng = np.random.default_rng(3)
    parts = []
    for i in (0, 2, 3, 6):
        lo, hi = int(P.node_off[i]), int(P.node_off[i + 1])
        parts.append(np.sort(rng.choice(np.arange(lo, hi), size=min(90, hi - lo), replace=False)))
    idx = np.concatenate(parts).astype(np.int32)
    print(f"[list maps] {idx.size} rows over instances 0, 2, 3, 6", flush=True)
    s.set_active(1, torch.tensor(idx, device=DEV))
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    st = s.step(v, w, 0.0, stats=True)
    s.set_active(0, None)
    assert st[1]["n_active"] == idx.size
    assert st[1]["nnz_active"] == int(np.sum(rp[idx + 1] - rp[idx]))
    b = torch.ones(P.N, dtype=torch.float64, device=DEV)
    x, _ = s.solve(0, torch.tensor(idx, device=DEV), b)
    assert torch.all(x[torch.tensor(idx, device=DEV).long()] != 0)
    for bad in (idx[::-1], np.r_[idx[:5], idx[4], idx[5:]], np.r_[idx, P.N], np.r_[-1, idx]):
        with pytest.raises(SDCError, match="ascending"):
            s.solve(0, torch.tensor(bad.astype(np.int32), device=DEV), b)
    s.close()
