"""Pins for the oracle's Aliev-Panfilov model (Sec. 5.1)."""
import numpy as np

from oracle import ionic
from workloads import AP_PARAMS


def _paper_params(root):
    vals = {}
    with open(f"{root}/tests/golden/paper_constants.txt") as f:
        for line in f:
            line = line.split("#")[0].split()
            if len(line) == 2:
                vals[line[0]] = float(line[1])
    return vals


def test_paper_constants_fixture(root):
    c = _paper_params(root)
    assert c["ap_ga"] == c["ap_gs"] == 8.0
    assert c["ap_rate_factor"] == 0.25
    assert c["radau_order"] == 2 * c["radau_points"] - 1


def test_current_structure():
    p = ionic.as_params(AP_PARAMS)
    k, a = p[0], p[1]
    # cubic with roots 0, a, 1 at w = 0 and leading coefficient k
    for v0 in (0.0, a, 1.0):
        assert ionic.current(v0, 0.0, p) == 0.0
    assert np.isclose(ionic.current(2.0, 0.0, p), k * 2.0 * (2.0 - a) * 1.0)
    # linear in w with slope v
    assert np.isclose(ionic.current(0.3, 0.7, p) - ionic.current(0.3, 0.2, p), 0.3 * 0.5)


def test_rate_structure():
    p = ionic.as_params(AP_PARAMS)
    k, a, eps0, mu1, mu2, s = p
    v = np.linspace(0, 1, 11)
    # zero on the nullcline w = -k v (v - a - 1)
    w_null = -k * v * (v - a - 1)
    assert np.allclose(ionic.rate(v, w_null, p), 0.0, atol=1e-15)
    # at v = 0: s (eps0 + mu1 w/mu2)(-w)
    assert np.isclose(ionic.rate(0.0, 0.4, p), s * (eps0 + mu1 * 0.4 / mu2) * (-0.4))
    # rest state is an equilibrium
    assert ionic.rate(0.0, 0.0, p) == 0.0 and ionic.current(0.0, 0.0, p) == 0.0


def test_paper_parameter_set_scaling(root):
    c = _paper_params(root)
    p = np.array([c["ap_ga"], c["ap_a"], c["ap_eps1"], c["ap_mu1"], c["ap_mu2"], c["ap_rate_factor"]])
    q = p.copy()
    q[5] = 1.0
    # the printed factor 1/4 scales the rate only
    assert np.isclose(ionic.rate(0.3, 0.1, p), 0.25 * ionic.rate(0.3, 0.1, q))
    assert ionic.current(0.3, 0.1, p) == ionic.current(0.3, 0.1, q)


def test_partials_vs_central_differences():
    rng = np.random.default_rng(0)
    p = ionic.as_params(AP_PARAMS)
    v = rng.uniform(-0.1, 1.1, 50)
    w = rng.uniform(0.0, 2.5, 50)
    h = 1e-6
    dIv, dIw, dIa = ionic.current_partials(v, w, p)
    dRv, dRw, dRa = ionic.rate_partials(v, w, p)
    pa = p.copy(); pa[1] += h
    pb = p.copy(); pb[1] -= h
    fd = {
        "Iv": (ionic.current(v + h, w, p) - ionic.current(v - h, w, p)) / (2 * h),
        "Iw": (ionic.current(v, w + h, p) - ionic.current(v, w - h, p)) / (2 * h),
        "Ia": (ionic.current(v, w, pa) - ionic.current(v, w, pb)) / (2 * h),
        "Rv": (ionic.rate(v + h, w, p) - ionic.rate(v - h, w, p)) / (2 * h),
        "Rw": (ionic.rate(v, w + h, p) - ionic.rate(v, w - h, p)) / (2 * h),
        "Ra": (ionic.rate(v, w, pa) - ionic.rate(v, w, pb)) / (2 * h),
    }
    got = {"Iv": dIv, "Iw": dIw, "Ia": dIa, "Rv": dRv, "Rw": dRw, "Ra": dRa}
    for key in got:
        assert np.allclose(got[key], fd[key], rtol=1e-7, atol=1e-8), key
