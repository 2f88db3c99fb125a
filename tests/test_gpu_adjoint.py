"""GPU reverse step against the oracle's tangent-linear model and central differences.

The dot-product identity <lam, TLM(e)> = <ADJ(lam), e> holds for the exact
derivative of the step with frozen active sets; both sides use the sets the
GPU forward produced.  Tolerance 1e-8 relative: the GPU solves to CG rtol
1e-12 while the oracle tangent uses direct solves.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import tlm  # noqa: E402
from oracle.sdc import build, run  # noqa: E402
from workloads import config1, config4  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(P, **kw):
    from paper_2311_07206_amd import Solver
    return Solver.from_problem(P, **kw)


def _gpu_sets(s, P, v, w, t):
    """Active sets of one GPU step from (v, w) at t (the step is not kept)."""
    vv = torch.tensor(v, device=DEV)
    ww = torch.tensor(w, device=DEV)
    s.begin_step(vv, ww, t)
    sets = [np.arange(P.N)]
    for k in range(P.K):
        s.sweep()
        if k + 1 < P.K:
            sets.append(s.active().cpu().numpy().astype(np.int64))
    s.end_step(vv, ww)
    return sets


def _mid_state(P, n):
    v, w, _ = run(build(P), P.v_init, P.w_init, n, P.K, P.stimuli)
    return v, w


@pytest.mark.parametrize("direction", ["state", "sigma", "a"])
@pytest.mark.parametrize("case", ["batch", "2d"])
def test_adjoint_dot_product_against_oracle_tlm(case, direction):
    P = config4(n_inst=3, sizes=(12, 18), theta=1e-6) if case == "batch" else config1(n=21, theta=1e-6)
    n0 = 3
    v0, w0 = _mid_state(P, n0)
    t = n0 * P.dt
    s = _solver(P)
    sets = _gpu_sets(s, P, v0, w0, t)
    assert any(len(x) < P.N for x in sets[1:])
    rng = np.random.default_rng(17)
    lam_v = rng.standard_normal(P.N)
    lam_w = rng.standard_normal(P.N)
    ds = rng.standard_normal(P.N) * P.node_sigma if direction == "sigma" else np.zeros(P.N)
    da = rng.standard_normal(P.n_inst) if direction == "a" else np.zeros(P.n_inst)
    dv = rng.standard_normal(P.N) if direction == "state" else np.zeros(P.N)
    dw = rng.standard_normal(P.N) if direction == "state" else np.zeros(P.N)
    tp = tlm.TLMProblem(P)
    a = P.ionic[:, 1].copy()
    _, _, vt, wt = tlm.step(tp, P.node_sigma, a, v0, w0, sets, ds, da, dv, dw)
    lhs = lam_v @ vt + lam_w @ wt
    Lv = torch.tensor(lam_v, device=DEV)
    Lw = torch.tensor(lam_w, device=DEV)
    gs = torch.zeros(P.N, dtype=torch.float64, device=DEV)
    ga = torch.zeros(P.n_inst, dtype=torch.float64, device=DEV)
    s.adjoint_step(torch.tensor(v0, device=DEV), torch.tensor(w0, device=DEV), t, Lv, Lw, gs, ga)
    rhs = (Lv.cpu().numpy() @ dv + Lw.cpu().numpy() @ dw + gs.cpu().numpy() @ ds + ga.cpu().numpy() @ da)
    scale = abs(lam_v) @ abs(vt) + abs(lam_w) @ abs(wt)
    assert abs(lhs - rhs) <= 1e-8 * scale, (lhs, rhs)


def test_adjoint_sigma_gradient_against_central_differences():
    # loss 0.5 ||v1 - target||^2 over one step, active sets pinned to the base run's
    P = config1(n=17, theta=1e-6)
    v0, w0 = _mid_state(P, 4)
    t = 4 * P.dt
    s = _solver(P)
    sets = _gpu_sets(s, P, v0, w0, t)
    rng = np.random.default_rng(5)
    target = rng.uniform(0, 1, P.N)

    def loss(sig):
        s.set_coefficients(sig)
        for k in range(1, P.K):
            s.set_active(k, torch.tensor(sets[k], dtype=torch.int32, device=DEV))
        v = torch.tensor(v0, device=DEV)
        w = torch.tensor(w0, device=DEV)
        s.step(v, w, t)
        s.set_active(0, None)
        r = v.cpu().numpy() - target
        return 0.5 * r @ r, v.cpu().numpy()

    L0, v1 = loss(P.node_sigma)
    s.set_coefficients(P.node_sigma)
    gs = torch.zeros(P.N, dtype=torch.float64, device=DEV)
    ga = torch.zeros(1, dtype=torch.float64, device=DEV)
    Lv = torch.tensor(v1 - target, device=DEV)
    Lw = torch.zeros(P.N, dtype=torch.float64, device=DEV)
    s.adjoint_step(torch.tensor(v0, device=DEV), torch.tensor(w0, device=DEV), t, Lv, Lw, gs, ga)
    ds = rng.standard_normal(P.N) * P.node_sigma
    h = 1e-5
    fd = (loss(P.node_sigma + h * ds)[0] - loss(P.node_sigma - h * ds)[0]) / (2 * h)
    assert abs(gs.cpu().numpy() @ ds - fd) <= 1e-6 * abs(fd)


def test_autograd_function_multi_step_against_oracle_tlm():
    from paper_2311_07206_amd.autograd import SDCRun
    P = config4(n_inst=2, sizes=(10, 14), theta=1e-6)
    n0, nsteps = 2, 4
    v0, w0 = _mid_state(P, n0)
    t0 = n0 * P.dt
    s = _solver(P)
    # GPU sets of each of the steps (free-running from the same state)
    sets_all = []
    v, w = v0.copy(), w0.copy()
    for n in range(nsteps):
        sets_all.append(_gpu_sets(s, P, v, w, t0 + n * P.dt))
        vv, ww = torch.tensor(v, device=DEV), torch.tensor(w, device=DEV)
        s.step(vv, ww, t0 + n * P.dt)
        v, w = vv.cpu().numpy(), ww.cpu().numpy()
    rng = np.random.default_rng(9)
    target = rng.uniform(0, 1, P.N)
    sigma = torch.tensor(P.node_sigma, device=DEV, requires_grad=True)
    a = torch.tensor(P.ionic[:, 1].copy(), device=DEV, requires_grad=True)
    v0t = torch.tensor(v0, device=DEV, requires_grad=True)
    w0t = torch.tensor(w0, device=DEV, requires_grad=True)
    vT, wT = SDCRun.apply(sigma, a, v0t, w0t, s, nsteps, t0, 2)
    loss = 0.5 * ((vT - torch.tensor(target, device=DEV)) ** 2).sum()
    loss.backward()
    tp = tlm.TLMProblem(P)
    for seed in range(2):
        r = np.random.default_rng(100 + seed)
        ds = r.standard_normal(P.N) * P.node_sigma
        da = r.standard_normal(P.n_inst)
        dv = r.standard_normal(P.N)
        dw = r.standard_normal(P.N)
        vT_o, _, vt, _ = tlm.run(tp, P.node_sigma, P.ionic[:, 1].copy(), v0, w0, nsteps, sets_all, (), t0,
                                 ds, da, dv, dw)
        lhs = (vT_o - target) @ vt
        rhs = (sigma.grad.cpu().numpy() @ ds + a.grad.cpu().numpy() @ da + v0t.grad.cpu().numpy() @ dv
               + w0t.grad.cpu().numpy() @ dw)
        assert abs(lhs - rhs) <= 1e-7 * (abs(lhs) + 1e-12), (lhs, rhs)


def test_checkpoint_interval_does_not_change_gradients():
    from paper_2311_07206_amd.autograd import SDCRun
    P = config4(n_inst=2, sizes=(9, 13), theta=1e-6)
    v0, w0 = _mid_state(P, 2)
    s = _solver(P)
    grads = []
    for ck in (1, 3, 5):
        sigma = torch.tensor(P.node_sigma, device=DEV, requires_grad=True)
        a = torch.tensor(P.ionic[:, 1].copy(), device=DEV, requires_grad=True)
        v = torch.tensor(v0, device=DEV, requires_grad=True)
        w = torch.tensor(w0, device=DEV, requires_grad=True)
        vT, wT = SDCRun.apply(sigma, a, v, w, s, 5, 2 * P.dt, ck)
        (vT.square().sum() + 0.5 * wT.sum()).backward()
        grads.append([x.grad.cpu().numpy() for x in (sigma, a, v, w)])
    for g in grads[1:]:
        for x, y in zip(grads[0], g):
            assert np.array_equal(x, y)


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


def test_adjoint_full_size_batched_sampled_instances():
    """The full 48-instance workload (3.7 M dofs): the reverse step of the
    whole context with the adjoint seeded on one instance, against the
    oracle's tangent-linear model of that instance alone (its smallest and
    its largest), all directions at once."""
    P = config4()
    s = _solver(P)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    for n in range(2):
        s.step(v, w, n * P.dt)
    t = 2 * P.dt
    v0, w0 = v.cpu().numpy(), w.cpu().numpy()
    sets = _gpu_sets(s, P, v0, w0, t)
    sizes = np.diff(P.node_off)
    rng = np.random.default_rng(23)
    for i in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        lo, hi = int(P.node_off[i]), int(P.node_off[i + 1])
        n = hi - lo
        print(f"[adjoint full] instance {i} ({n} dofs)", flush=True)
        lam_v, lam_w = np.zeros(P.N), np.zeros(P.N)
        lam_v[lo:hi] = rng.standard_normal(n)
        lam_w[lo:hi] = rng.standard_normal(n)
        ds, dv, dw = rng.standard_normal(n) * P.node_sigma[lo:hi], rng.standard_normal(n), rng.standard_normal(n)
        da = rng.standard_normal()
        Lv = torch.tensor(lam_v, device=DEV)
        Lw = torch.tensor(lam_w, device=DEV)
        gs = torch.zeros(P.N, dtype=torch.float64, device=DEV)
        ga = torch.zeros(P.n_inst, dtype=torch.float64, device=DEV)
        s.adjoint_step(torch.tensor(v0, device=DEV), torch.tensor(w0, device=DEV), t, Lv, Lw, gs, ga)
        Lv, Lw, gs, ga = (x.cpu().numpy() for x in (Lv, Lw, gs, ga))
        # the other instances see no adjoint
        assert not np.any(Lv[:lo]) and not np.any(Lv[hi:]) and not np.any(gs[:lo]) and not np.any(gs[hi:])
        sub = _instance(P, i)
        sub_sets = [np.arange(n)] + [x[(x >= lo) & (x < hi)] - lo for x in sets[1:]]
        tp = tlm.TLMProblem(sub)
        _, _, vt, wt = tlm.step(tp, sub.node_sigma, sub.ionic[:, 1].copy(), v0[lo:hi], w0[lo:hi], sub_sets,
                                ds, np.array([da]), dv, dw)
        lhs = lam_v[lo:hi] @ vt + lam_w[lo:hi] @ wt
        rhs = Lv[lo:hi] @ dv + Lw[lo:hi] @ dw + gs[lo:hi] @ ds + ga[i] * da
        scale = abs(lam_v[lo:hi]) @ abs(vt) + abs(lam_w[lo:hi]) @ abs(wt)
        print(f"[adjoint full] instance {i}: lhs {lhs:.6e} rhs {rhs:.6e} rel {abs(lhs - rhs) / scale:.2e}",
              flush=True)
        assert abs(lhs - rhs) <= 1e-8 * scale, (lhs, rhs)


def test_adjoint_elementwise_against_oracle_tlm_basis():
    """Every component of the reverse step's outputs against the oracle: on
    three instances of 7^2, 8^2 and 8^2 nodes, the oracle's tangent-linear model is
    run in every basis direction (each node's v0, w0 and sigma, each
    instance's a), which gives each component of J^T lam as <lam, J e>.  The
    library's lam_v, lam_w (adjoints of v0, w0), g_sigma and g_a must match
    component by component within 1e-8 of that component's scale
    s_q = sum |lam| |J e_q|, with the scale floored at 1e-3 of the largest
    scale of its kind: the library's solves stop at rtol 1e-12 relative to
    the whole vector (the oracle's are direct), so a component a million
    times below the largest carries that absolute rounding."""
    P = config4(n_inst=3, sizes=(4, 8), theta=1e-6)
    n0 = 3
    v0, w0 = _mid_state(P, n0)
    t = n0 * P.dt
    s = _solver(P)
    sets = _gpu_sets(s, P, v0, w0, t)
    assert any(len(x) < P.N for x in sets[1:])
    rng = np.random.default_rng(23)
    lam_v = rng.standard_normal(P.N)
    lam_w = rng.standard_normal(P.N)
    Lv = torch.tensor(lam_v, device=DEV)
    Lw = torch.tensor(lam_w, device=DEV)
    gs = torch.zeros(P.N, dtype=torch.float64, device=DEV)
    ga = torch.zeros(P.n_inst, dtype=torch.float64, device=DEV)
    s.adjoint_step(torch.tensor(v0, device=DEV), torch.tensor(w0, device=DEV), t, Lv, Lw, gs, ga)
    got = {"v": Lv.cpu().numpy(), "w": Lw.cpu().numpy(), "sigma": gs.cpu().numpy(), "a": ga.cpu().numpy()}
    tp = tlm.TLMProblem(P)
    a = P.ionic[:, 1].copy()
    zN, zI = np.zeros(P.N), np.zeros(P.n_inst)
    print(f"[adjoint elementwise] N={P.N}, {3 * P.N + P.n_inst} tangent directions", flush=True)
    for name, size in (("v", P.N), ("w", P.N), ("sigma", P.N), ("a", P.n_inst)):
        want, scale = np.zeros(size), np.zeros(size)
        for q in range(size):
            e = np.zeros(size)
            e[q] = 1.0
            dv, dw, ds, da = (e if name == "v" else zN, e if name == "w" else zN,
                              e if name == "sigma" else zN, e if name == "a" else zI)
            _, _, vt, wt = tlm.step(tp, P.node_sigma, a, v0, w0, sets, ds, da, dv, dw)
            want[q] = lam_v @ vt + lam_w @ wt
            scale[q] = abs(lam_v) @ abs(vt) + abs(lam_w) @ abs(wt)
        err = np.abs(got[name] - want)
        floor = np.maximum(scale, 1e-3 * scale.max())
        print(f"   {name}: largest |component| {np.abs(want).max():.3e}, worst err/scale "
              f"{(err / np.maximum(scale, 1e-300)).max():.2e}, worst err/floored scale {(err / floor).max():.2e}",
              flush=True)
        assert np.all(err <= 1e-8 * floor), name
