"""Pins for the oracle's tangent-linear model: values agree with the forward
oracle, tangents agree with central finite differences (frozen active sets)."""
import numpy as np
import pytest

from oracle import tlm
from oracle.sdc import build, run
from workloads import config4


@pytest.fixture(scope="module")
def setup():
    P = config4(n_inst=2, sizes=(7, 10), n_steps=4, theta=1e-5)
    v, w, log = run(build(P), P.v_init, P.w_init, P.n_steps, P.K, P.stimuli)
    sets = [[info["idx"] for info in infos] for infos in log]
    assert any(len(s[-1]) < P.N for s in sets)        # adaptivity is active
    tp = tlm.TLMProblem(P)
    a = P.ionic[:, 1].copy()
    return P, tp, a, sets, v, w


def test_tlm_forward_values_match_oracle(setup):
    P, tp, a, sets, v_ref, w_ref = setup
    v, w, _, _ = tlm.run(tp, P.node_sigma, a, P.v_init, P.w_init, P.n_steps, sets, P.stimuli)
    assert np.linalg.norm(v - v_ref) <= 1e-10 * np.linalg.norm(v_ref)
    assert np.linalg.norm(w - w_ref) <= 1e-10 * np.linalg.norm(w_ref)


@pytest.mark.parametrize("which", ["sigma", "a", "state", "all"])
def test_tlm_matches_central_differences(setup, which):
    P, tp, a, sets, _, _ = setup
    rng = np.random.default_rng({"sigma": 1, "a": 2, "state": 3, "all": 4}[which])
    ds = rng.standard_normal(P.N) * P.node_sigma if which in ("sigma", "all") else np.zeros(P.N)
    da = rng.standard_normal(P.n_inst) * 0.1 if which in ("a", "all") else np.zeros(P.n_inst)
    dv = rng.standard_normal(P.N) * 0.1 if which in ("state", "all") else np.zeros(P.N)
    dw = rng.standard_normal(P.N) * 0.1 if which in ("state", "all") else np.zeros(P.N)
    # start from a mid-run state so that the state direction has no stimulus overwrite
    v0, w0, _ = run(build(P), P.v_init, P.w_init, 2, P.K, P.stimuli)
    sub = sets[2:]
    _, _, vt, wt = tlm.run(tp, P.node_sigma, a, v0, w0, 2, sub, (), t0=2 * P.dt,
                           dsigma=ds, da=da, dv=dv, dw=dw)
    h = 1e-6

    def f(sgn):
        v, w, _, _ = tlm.run(tp, P.node_sigma + sgn * h * ds, a + sgn * h * da, v0 + sgn * h * dv,
                             w0 + sgn * h * dw, 2, sub, (), t0=2 * P.dt)
        return v, w

    (vp, wp), (vm, wm) = f(1), f(-1)
    fv, fw = (vp - vm) / (2 * h), (wp - wm) / (2 * h)
    assert np.linalg.norm(vt - fv) <= 1e-6 * np.linalg.norm(fv)
    assert np.linalg.norm(wt - fw) <= 1e-6 * max(np.linalg.norm(fw), 1e-12)
