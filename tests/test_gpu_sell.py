"""Sliced ELL storage (sdc_params.format 3): slices of 64 rows (one
wavefront), entries column by column in each row's CSR order, padded with
exact zeros, so every sum is the CSR loop's.  Checked: steps bitwise equal
to CSR storage on 1D, 2D, 3D, batched and cell-by-cell problems (including
the one-workgroup solves of small sets), graph-captured steps, the reverse
step, restricted solves against the oracle, the timed storage choice and the
rejection with the linearized scheme.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.pcg import jacobi_pcg  # noqa: E402
from oracle.sdc import build  # noqa: E402
from workloads import config0, config1, config2, config3, config4  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(P, **kw):
    from paper_2311_07206_amd import Solver
    return Solver.from_problem(P, **kw)


def _run(P, s, n_steps, graph=False):
    if graph:
        s.set_graph(True)
    v = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    stats = []
    for n in range(n_steps):
        st = s.step(v, w, n * P.dt, stats=True)
        stats.append([(x["n_active"], x["cg_iters_max"]) for x in st])
    return v.cpu().numpy(), w.cpu().numpy(), stats


@pytest.mark.parametrize("case", ["1d", "2d", "3d", "batched", "emi"])
def test_sell_steps_equal_csr_bitwise(case):
    if case == "1d":
        P, n = config0(n=200, theta=1e-6), 10
    elif case == "2d":
        P, n = config1(n=45, theta=1e-7), 6
    elif case == "3d":
        P, n = config2(n=12, theta=1e-7), 3
    elif case == "batched":
        P, n = config4(n_inst=4, sizes=(12, 30)), 5
    else:
        P, n = config3(nc=3, nr=2, nx=9, ny=5), 3
    a = _solver(P, fmt=3)
    b = _solver(P, fmt=1)
    assert a.info()["format"] == "sell" and b.info()["format"] == "csr"
    print(f"[sell {case}] N={P.N}", flush=True)
    va, wa, sa = _run(P, a, n)
    vb, wb, sb = _run(P, b, n)
    assert sa == sb
    assert np.array_equal(va, vb) and np.array_equal(wa, wb)


def test_sell_graph_steps_and_reverse_step_equal_csr():
    P = config4(n_inst=3, sizes=(16, 40), theta=1e-6)
    a = _solver(P, fmt=3, small_set_rows=-1)
    b = _solver(P, fmt=1, small_set_rows=-1)
    va, wa, _ = _run(P, a, 6, graph=True)
    vb, wb, _ = _run(P, b, 6)
    assert a.info()["graph_steps"] >= 4
    assert np.array_equal(va, vb) and np.array_equal(wa, wb)
    out = []
    for s in (a, b):
        s.set_graph(False)
        rng = np.random.default_rng(3)
        Lv = torch.tensor(rng.standard_normal(P.N), device=DEV)
        Lw = torch.tensor(rng.standard_normal(P.N), device=DEV)
        gs = torch.zeros(P.N, dtype=torch.float64, device=DEV)
        ga = torch.zeros(P.n_inst, dtype=torch.float64, device=DEV)
        s.adjoint_step(torch.tensor(va, device=DEV), torch.tensor(wa, device=DEV), 6 * P.dt, Lv, Lw, gs, ga)
        out.append([x.cpu().numpy() for x in (Lv, Lw, gs, ga)])
    assert all(np.array_equal(x, y) for x, y in zip(*out))


def test_sell_restricted_solve_matches_oracle():
    P = config2(n=14, theta=1e-7)
    s = _solver(P, fmt=3)
    orc = build(P)
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(P.N, P.N // 3, replace=False)).astype(np.int32)
    b = rng.standard_normal(P.N)
    x, it = s.solve(1, torch.tensor(idx, device=DEV), torch.tensor(b, device=DEV))
    xo, ito = jacobi_pcg(orc.H[1], b, idx, P.cg_rtol)
    rel = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
    print(f"[sell solve] iters {it[0]} / {ito}, rel {rel:.2e}", flush=True)
    assert rel < 1e-11 and abs(it[0] - ito) <= 1


def test_timed_choice_considers_sell_and_rejections():
    from paper_2311_07206_amd import SDCError
    P = config3(nc=4, nr=2, nx=9, ny=5)
    s = _solver(P)
    info = s.info()
    print(f"[sell choice] cell-by-cell: {info['format']}, csr {info['t_csr_us']:.1f} us, "
          f"sell {info['t_sell_us']:.1f} us", flush=True)
    assert info["format"] in ("csr", "sell") and info["t_sell_us"] > 0 and info["t_csr_us"] > 0
    with pytest.raises(SDCError, match="sliced ELL"):
        _solver(config1(n=12, theta=1e-7), fmt=3, scheme="linearized")
    lin = _solver(config1(n=12, theta=1e-7), scheme="linearized")
    assert lin.info()["format"] in ("csr", "dia") and lin.info()["t_sell_us"] == 0.0
