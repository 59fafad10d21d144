"""Pins of the landmark-reward oracle (oracle/landmarks.py) against what Sec.
II-C fixes: the first landmark is the next MPC step and the last the end of
the horizon; the reward lies in (0, 1] and is 1 exactly when every available
landmark is met; the two limiting schedules of the paper's remark (next-step
supervision, time-averaged tracking); landmarks that were never predicted are
omitted."""
import math

import numpy as np
import pytest

from oracle import landmarks


@pytest.mark.parametrize("N,L", [(10, 5), (20, 5), (60, 7), (11, 3), (2, 2), (37, 4)])
def test_offsets_span_next_step_to_horizon_end(N, L):
    n = landmarks.landmark_offsets(N, L)
    assert n[0] == 1 and n[-1] == N
    assert all(a <= b for a, b in zip(n, n[1:]))
    # the uniform reading s_l = l / (L - 1), worked by hand for N = 10, L = 5:
    # floor(0, 2.25, 4.5, 6.75, 9) + 1
    assert landmarks.landmark_offsets(10, 5) == [1, 3, 5, 7, 10]
    # exact rationals: 1/3 of 9 is 3, not 2.999...
    assert landmarks.landmark_offsets(10, 4) == [1, 4, 7, 10]


def _traj(rng, N):
    x = rng.normal(0, 1, (N + 1, 13))
    return x


def test_limiting_schedules_of_the_remark():
    rng = np.random.default_rng(5)
    N, L, sigma = 10, 5, 0.3
    qc = np.array([1.0, 2.0, 0.5])
    st = landmarks.LandmarkStore(L)
    trajs = {}
    for T in range(12):
        trajs[T] = _traj(rng, N)
        st.push(0, T, trajs[T], N)
    t = 11
    com = rng.normal(0, 1, 3)
    # alpha = (1, 0, ...): strict next-step supervision
    r, used = st.reward(0, t, com, [1, 0, 0, 0, 0], qc, sigma)
    e = com - trajs[t - 1][1][3:6]
    assert math.isclose(r, math.exp(-(e @ (qc * e)) / sigma ** 2), rel_tol=1e-13)
    # alpha = 1 / L: the average of the weighted squared errors of every
    # landmark predicted for t (offsets 1, 3, 5, 7, 10)
    r, used = st.reward(0, t, com, [1 / L] * L, qc, sigma)
    errs = [com - trajs[t - n][n][3:6] for n in (1, 3, 5, 7, 10)]
    assert used == set(range(L))
    want = math.exp(-np.mean([e @ (qc * e) for e in errs]) / sigma ** 2)
    assert math.isclose(r, want, rel_tol=1e-13)


def test_reward_bounds_and_exact_match():
    rng = np.random.default_rng(6)
    st = landmarks.LandmarkStore(3)
    x = _traj(rng, 8)
    st.push(2, 0, x, 8)
    # offsets 1, 4 (1 + floor(3.5)), 8
    for n, l in ((1, 0), (4, 1), (8, 2)):
        r, used = st.reward(2, n, x[n][3:6], [0.5, 0.3, 0.2], np.ones(3), 0.1)
        assert r == 1.0 and used == {l}
        r, _ = st.reward(2, n, x[n][3:6] + 10.0, [0.5, 0.3, 0.2], np.ones(3), 0.1)
        assert 0.0 <= r < 1.0


def test_missing_landmarks_are_omitted_and_episodes_reset():
    rng = np.random.default_rng(7)
    st = landmarks.LandmarkStore(5, ticks_per_step=2)
    r, used = st.reward(0, 0, np.zeros(3), [0.5, 0.25, 0.15, 0.07, 0.03], np.ones(3), 1.0)
    assert r == 1.0 and used == set()            # nothing predicted yet
    x = _traj(rng, 10)
    st.push(0, 4, x, 10)                          # targets 4 + 2 n
    _, used = st.reward(0, 6, x[1][3:6], [1] * 5, np.ones(3), 1.0)
    assert used == {0}
    _, used = st.reward(0, 7, x[1][3:6], [1] * 5, np.ones(3), 1.0)
    assert used == set()                          # odd ticks: no MPC step lands there
    st.clear(0)
    _, used = st.reward(0, 6, x[1][3:6], [1] * 5, np.ones(3), 1.0)
    assert used == set()


def test_planted_mistake_next_step_offset():
    """An off-by-one offset (n_0 = 0, the current state) would make the
    next-step limit compare with the wrong prediction: the pin above relies on
    x[1] of the solve one step earlier."""
    rng = np.random.default_rng(8)
    st = landmarks.LandmarkStore(2)
    x0, x1 = _traj(rng, 4), _traj(rng, 4)
    st.push(0, 0, x0, 4)
    st.push(0, 1, x1, 4)
    r, _ = st.reward(0, 1, x0[1][3:6], [1, 0], np.ones(3), 1.0)
    assert r == 1.0
    r, _ = st.reward(0, 1, x1[0][3:6], [1, 0], np.ones(3), 1.0)
    assert r < 1.0
