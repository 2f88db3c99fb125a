"""GPU parity of the cell-by-cell model on the 3D cell array (P1 tetrahedra)
against the oracle: the assembled system, restricted solves (raw on a set,
mean-free and to the conditioning bound on all rows, as in 2D), adaptive and
non-adaptive steps with the oracle replaying the GPU's active sets, and the
full-size workload's system and restricted solves.  Tolerances as in 2D:
transmembrane voltage, gating and mean-free potential within 1e-10.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.emi import EMI, build, run  # noqa: E402
from oracle.pcg import jacobi_pcg  # noqa: E402
from workloads.emi import config5  # noqa: E402

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _solver(P, **kw):
    from paper_2311_07206_amd import Solver
    return Solver.from_problem(P, **kw)


def small(**kw):
    base = dict(nc=3, nr=2, nl=1, nx=6, ny=4, nz=4)
    base.update(kw)
    return config5(**base)


def mean_free(u):
    return u - u.mean()


def test_emi3d_assembly_matches_oracle():
    import scipy.sparse as sp
    P = small()
    s = _solver(P)
    rp, col, val, ml = s.system()
    mod = EMI(P)
    G = sp.csr_matrix((val, col, rp), shape=(P.N, P.N))
    assert abs(G - mod.A).max() <= 1e-14 * abs(mod.A).max()
    assert abs(G - G.T).max() == 0.0          # the library's assembly is exactly symmetric
    # the oracle sums facet shares whose lengths come from coordinate
    # differences (coordinates up to ~2000 segment lengths: ~3 digits lost);
    # the library takes the workload's closed-form arrays: equal to 1e-12
    assert np.allclose(ml, mod.M.diagonal(), rtol=1e-12, atol=0)


@pytest.mark.parametrize("m", [0, 2])
def test_emi3d_restricted_pcg_matches_oracle(m):
    P = small()
    s = _solver(P)
    orc = build(P)
    ev = np.linalg.eigvalsh(orc.H[m].toarray())
    raw_bound = 2.0 * P.cg_rtol * np.sqrt(ev[-1] / ev[0])
    rng = np.random.default_rng(17 + m)
    for frac in (1.0, 0.4):
        n = int(frac * P.N)
        idx = np.arange(P.N) if frac == 1.0 else np.sort(rng.choice(P.N, size=n, replace=False))
        b = rng.standard_normal(P.N) * 1e-4
        print(f"[emi3d pcg] m={m} n={n}", flush=True)
        x, iters = s.solve(m, torch.tensor(idx, dtype=torch.int32, device=DEV), torch.tensor(b, device=DEV))
        xo, ito = jacobi_pcg(orc.H[m], b, idx, P.cg_rtol, maxit=P.cg_maxit)
        d = x.cpu().numpy() - xo
        scale = np.abs(xo).max()
        print(f"  iters gpu {iters[0]} oracle {ito}; raw {np.abs(d).max() / scale:.3e}, "
              f"mean-free {np.abs(d - d.mean()).max() / scale:.3e}", flush=True)
        if frac == 1.0:
            assert np.abs(d - d.mean()).max() <= 1e-10 * scale
            assert np.abs(d).max() <= raw_bound * scale
        else:
            assert np.abs(d).max() <= 1e-10 * scale


@pytest.mark.parametrize("theta", [0.0, 1e-6])
def test_emi3d_steps_match_oracle(theta):
    P = small(theta=theta)
    s = _solver(P)
    u = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    n_steps = 3
    sets = []
    for n in range(n_steps):
        print(f"[emi3d steps] theta={theta} step {n}", flush=True)
        s.begin_step(u, w, n * P.dt)
        step_sets = [None]
        for k in range(P.K):
            s.sweep()
            if k + 1 < P.K:
                step_sets.append(s.active().cpu().numpy().astype(np.int64))
        s.end_step(u, w)
        sets.append(step_sets)
    ug, wg = u.cpu().numpy(), w.cpu().numpy()
    uo, wo, _ = run(build(P), P.v_init, P.w_init[P.mem_intra], n_steps, P.K, P.stimuli, idx_replay=sets)
    si, se = P.mem_intra, P.mem_extra
    vg, vo = ug[si] - ug[se], uo[si] - uo[se]
    print(f"  v rel {np.abs(vg - vo).max() / np.abs(vo).max():.3e}  w {np.abs(wg[si] - wo).max():.3e}  "
          f"u mean-free {np.abs(mean_free(ug) - mean_free(uo)).max() / np.abs(uo).max():.3e}", flush=True)
    if theta > 0:
        assert any(len(st_) < P.N for step in sets for st_ in step[1:])
    assert np.linalg.norm(vg - vo) <= 1e-10 * np.linalg.norm(vo)
    assert np.abs(wg[si] - wo).max() <= 1e-10 * max(np.abs(wo).max(), 1e-3)
    assert np.linalg.norm(mean_free(ug) - mean_free(uo)) <= 1e-10 * np.linalg.norm(uo)
    assert np.linalg.norm(ug - uo) <= 1e-6 * np.linalg.norm(uo)


def test_emi3d_full_size_assembly_and_restricted_pcg():
    import scipy.sparse as sp
    P = config5()
    s = _solver(P)
    print(f"[emi3d full] N={P.N}, oracle assembly", flush=True)
    mod = EMI(P)
    rp, col, val, ml = s.system()
    G = sp.csr_matrix((val, col, rp), shape=(P.N, P.N))
    assert abs(G - mod.A).max() <= 1e-14 * abs(mod.A).max()
    # the oracle sums facet shares whose lengths come from coordinate
    # differences (coordinates up to ~2000 segment lengths: ~3 digits lost);
    # the library takes the workload's closed-form arrays: equal to 1e-12
    assert np.allclose(ml, mod.M.diagonal(), rtol=1e-12, atol=0)
    orc = build(P)
    # the nodes of the first two cell columns and their surroundings: no constant mode
    first = np.nonzero(P.coords[:, 0] <= 2 * (100e-4 + 2e-4) + 1e-12)[0]
    rng = np.random.default_rng(29)
    for m in (0, 2):
        b = rng.standard_normal(P.N) * 1e-4
        print(f"[emi3d full] solve m={m} n={first.size}", flush=True)
        x, it = s.solve(m, torch.tensor(first, dtype=torch.int32, device=DEV), torch.tensor(b, device=DEV))
        xo, ito = jacobi_pcg(orc.H[m], b, first, P.cg_rtol, maxit=P.cg_maxit)
        rel = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
        print(f"  iters gpu {it[0]} oracle {ito}; rel {rel:.2e}", flush=True)
        assert rel < 1e-11


def test_emi3d_full_size_step_matches_oracle():
    """The 3D cell-by-cell workload at full size (209,672 potential dofs):
    the step from the stimulus, the oracle replaying the GPU's sets (about a
    minute and a half of oracle work on the host)."""
    P = config5()
    s = _solver(P)
    u = torch.tensor(P.v_init, device=DEV)
    w = torch.tensor(P.w_init, device=DEV)
    s.begin_step(u, w, 0.0)
    sets = [None]
    for k in range(P.K):
        print(f"[emi3d full step] sweep {k}", flush=True)
        s.sweep()
        if k + 1 < P.K:
            sets.append(s.active().cpu().numpy().astype(np.int64))
    s.end_step(u, w)
    ug, wg = u.cpu().numpy(), w.cpu().numpy()
    print("[emi3d full step] oracle replay", flush=True)
    uo, wo, _ = run(build(P), P.v_init, P.w_init[P.mem_intra], 1, P.K, P.stimuli, idx_replay=[sets])
    si, se = P.mem_intra, P.mem_extra
    vg, vo = ug[si] - ug[se], uo[si] - uo[se]
    print(f"[emi3d full step] v rel {np.linalg.norm(vg - vo) / np.linalg.norm(vo):.2e}", flush=True)
    assert np.linalg.norm(vg - vo) <= 1e-10 * np.linalg.norm(vo)
    assert np.abs(wg[si] - wo).max() <= 1e-10 * max(np.abs(wo).max(), 1e-3)
    assert np.linalg.norm(mean_free(ug) - mean_free(uo)) <= 1e-10 * np.linalg.norm(uo)
    assert np.linalg.norm(ug - uo) <= 1e-6 * np.linalg.norm(uo)
