"""Pins of the stimulus schedule: a stimulus overwrites v at the start of the
step whose interval [t, t + dt) contains its time t_on (the experiments of
Sec. 5.1 start an excitation by setting v).  In exact arithmetic that is step
floor(t_on / dt); the expected indices below are worked out by hand from
that, for step start times formed as n * dt and as a running sum t += dt
(which lands just above a boundary: 0.1 + 0.1 + 0.1 = 0.30000000000000004).

Plausible mistakes these cases catch (checked by planting each): no
downward shift of the interval (a boundary stimulus reached by an
accumulated t fires one step early), a strict lower end (a stimulus on a
step boundary, t = 0 included, never fires), the shift applied with the
wrong sign.
"""
import numpy as np
import pytest

from oracle.sdc import apply_stimuli, build, run, stimulus_applies, stimulus_nodes
from workloads import config0, config2

# (t_on, dt, step index worked out by hand)
CASES = [
    (0.0, 0.25, 0),       # the first stimulus of every workload
    (120.0, 0.25, 480),   # the 3D workload's second ball: 120 / 0.25
    (119.9, 0.25, 479),   # inside step 479 = [119.75, 120)
    (0.3, 0.1, 3),        # a boundary that the running sum overshoots
    (0.7, 0.1, 7),
    (0.35, 0.1, 3),       # strictly inside [0.3, 0.4)
    (5.0, 0.2, 25),
    (1.0, 0.2, 5),
    (0.05, 0.05, 1),
    (2.5, 0.05, 50),
]


def _fired(t_on, dt, n_max, accumulate):
    out, t = [], 0.0
    for n in range(n_max):
        tn = t if accumulate else n * dt
        if stimulus_applies(t_on, tn, dt):
            out.append(n)
        t += dt
    return out


@pytest.mark.parametrize("accumulate", [False, True])
@pytest.mark.parametrize("t_on,dt,n", CASES)
def test_stimulus_fires_once_in_the_step_that_contains_it(t_on, dt, n, accumulate):
    assert _fired(t_on, dt, n + 40, accumulate) == [n]


def test_running_sum_overshoots_the_boundary():
    """The premise of the boundary cases: without the shift, the step that
    starts at the accumulated 0.3 would miss a stimulus at 0.3."""
    t = 0.0
    for _ in range(3):
        t += 0.1
    assert t > 0.3


def test_stimulus_overwrites_the_state_at_that_step_of_a_run():
    """Through run(): a 1D workload with a second stimulus at t_on = 0.3
    (dt = 0.1) on the rightmost nodes: those nodes are still near rest after
    steps 0..2 (the pulse from the left has not reached them) and take the
    value at the start of step 3."""
    P = config0(n=64, theta=1e-6, n_steps=4)
    right = np.arange(P.N - 4, P.N, dtype=np.int32)
    stimuli = list(P.stimuli) + [(0.3, right, 0.9)]
    orc = build(P)
    v, w, _ = run(orc, P.v_init, P.w_init, 3, P.K, stimuli)
    assert np.abs(v[right]).max() < 1e-3
    v3 = apply_stimuli(v.copy(), 3 * P.dt, P.dt, stimuli)
    assert np.all(v3[right] == 0.9) and np.array_equal(np.delete(v3, right), np.delete(v, right))
    assert [a.tolist() for a in stimulus_nodes(3 * P.dt, P.dt, stimuli)] == [right.tolist()]


def test_workload_3d_second_stimulus_step():
    """The 3D workload's stimuli fire at steps 0 and 480 only."""
    P = config2(n=9)
    fired = [n for n in range(600) for t_on, _, _ in P.stimuli if stimulus_applies(t_on, n * P.dt, P.dt)]
    assert fired == [0, 480]
