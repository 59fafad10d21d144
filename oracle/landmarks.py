"""MPC landmark guidance reward (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. II-C of the paper: every MPC solve at time t stores a few predicted CoM
positions ("landmarks") from its trajectory, at prediction offsets
delta_l = n_l dt with n_l = 1 + floor(s_l (N - 1)), l = 0..N_L-1, s_0 = 0 and
s_{N_L-1} = 1 (so delta_0 is the next MPC step and the last landmark is the end
of the horizon).  When the rollout reaches time t, the realised CoM c_t is
compared with every landmark that an earlier solve predicted for this same
time, e_l(t) = c_t - c_hat^{t - delta_l}(delta_l), landmarks that do not exist
(early in an episode) being left out, and the reward is

    r_t = exp( - sum_l alpha_l |e_l(t)|_Qc^2 / sigma^2 )   in (0, 1].

Readings where the paper is silent: s_l = l / (N_L - 1) (uniform; N_L = 1 means
the single landmark s_0 = 0); time is counted in integer ticks of the reward
loop with d ticks per MPC step dt (a solve at tick T predicts for ticks
T + n_l d); Qc is diagonal; the trajectory's CoM at prediction offset n is the
CoM block (entries 3..5) of the predicted state x_n of the 13-state model.

The store is a plain dictionary from (environment, target step, landmark) to
the predicted CoM, filled in the order the solves happen; a later solve that
predicts the same (target step, landmark) replaces the earlier one.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

COM = slice(3, 6)


def landmark_offsets(N, n_landmarks):
    """n_l = 1 + floor(s_l (N - 1)) with s_l = l / (N_L - 1), in exact
    rational arithmetic (a floating-point s_l can land just below an integer)."""
    if n_landmarks == 1:
        return [1]
    return [1 + math.floor(Fraction(l, n_landmarks - 1) * (N - 1)) for l in range(n_landmarks)]


class LandmarkStore:
    """Landmarks of many environments, keyed by the step they predict."""

    def __init__(self, n_landmarks, ticks_per_step=1):
        self.L = n_landmarks
        self.d = ticks_per_step
        self.table = {}

    def clear(self, env):
        """Forget an environment's landmarks (a new episode starts)."""
        self.table = {k: v for k, v in self.table.items() if k[0] != env}

    def push(self, env, step, x, N):
        """Store the landmarks of the solve made at tick `step` (x: predicted
        states x_0..x_N of that solve, N its horizon)."""
        for l, n in enumerate(landmark_offsets(N, self.L)):
            self.table[(env, step + n * self.d, l)] = np.array(x[n][COM], dtype=np.float64)

    def reward(self, env, step, com, alpha, qc, sigma):
        """r_t of Sec. II-C for environment `env` at tick `step` with realised
        CoM `com`: landmarks not predicted for this tick are omitted.  Returns
        the reward and the set of landmark indices that entered it."""
        total = 0.0
        used = set()
        for l in range(self.L):
            pred = self.table.get((env, step, l))
            if pred is None:
                continue
            e = np.asarray(com, dtype=np.float64) - pred
            total += alpha[l] * float(e @ (np.asarray(qc, dtype=np.float64) * e)) / sigma ** 2
            used.add(l)
        return math.exp(-total), used
