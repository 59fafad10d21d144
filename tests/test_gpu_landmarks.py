"""The landmark guidance reward (Sec. II-C) on the device against the oracle,
through the C ABI: a rollout of ticks with solves every MPC step, uneven
horizons, episode resets of some environments; which landmarks entered each
reward must match exactly (integer work) and the reward within FP32 rounding
of at most five weighted squared errors and one exponential (relative 2e-5)."""
import numpy as np
import pytest

import mpcgen
from oracle import landmarks

pytestmark = pytest.mark.gpu

ALPHA = [0.5, 0.25, 0.15, 0.07, 0.03]   # the paper's horizon-tapered schedule


def test_landmark_reward_matches_oracle():
    import torch
    from paper_2606_05687_amd import binding
    E, n_max, L, d = 777, 60, 5, 2
    rng = np.random.default_rng(2024)
    N = mpcgen.make_batch("uneven_b16384", indices=range(E), n_max=n_max)["N"]
    ring = binding.LandmarkRing(E, L, n_max * d + 1, ticks_per_step=d)
    ring.clear()
    store = landmarks.LandmarkStore(L, ticks_per_step=d)
    alpha = torch.tensor(ALPHA, dtype=torch.float32).cuda()
    qc = np.array([1.0, 2.0, 0.5], dtype=np.float32)
    sigma = 0.2
    Nd = torch.from_numpy(N).cuda()
    last = {}
    used_total = 0
    for tick in range(3 * d * 12):
        if tick == 40:
            reset = (rng.uniform(size=E) < 0.3).astype(np.uint8)
            ring.clear(torch.from_numpy(reset).cuda())
            for e in np.nonzero(reset)[0]:
                store.clear(int(e))
        if tick % d == 0:
            x = rng.normal(0, 1, (E, n_max + 1, 13)).astype(np.float32)
            ring.push(torch.from_numpy(x).cuda(), Nd, tick)
            for e in range(E):
                store.push(e, tick, x[e].astype(np.float64), int(N[e]))
            last[tick] = x
        # realised CoM near what the solve one MPC step earlier predicted
        base = last[max(k for k in last if k <= tick)][:, 1, 3:6]
        com = (base + rng.normal(0, 0.05, (E, 3))).astype(np.float32)
        r, used = ring.reward(torch.from_numpy(com).cuda(), tick, alpha,
                              torch.from_numpy(qc).cuda(), sigma)
        torch.cuda.synchronize()
        r, used = r.cpu().numpy(), used.cpu().numpy()
        for e in range(0, E, 7):
            want, wused = store.reward(e, tick, com[e].astype(np.float64), ALPHA,
                                       qc.astype(np.float64), sigma)
            assert used[e] == sum(1 << l for l in wused), (tick, e, used[e], wused)
            assert abs(r[e] - want) <= 2e-5 * want + 1e-30, (tick, e, r[e], want)
            used_total += len(wused)
    assert used_total > 0


def test_landmark_calls_reject_bad_sizes():
    import ctypes
    import torch
    from paper_2606_05687_amd import binding
    lib = binding.load()
    ring = binding.LandmarkRing(4, 5, 11)
    x = torch.zeros((4, 11, 13), dtype=torch.float32).cuda()
    st = ring.st
    # ring (11) must exceed n_max * ticks_per_step: 10 is accepted, 11 is not
    assert lib.pinmpc_landmarks_push(ctypes.byref(st), 11, None, ctypes.c_void_p(x.data_ptr()),
                                     0, None) == -1
    assert lib.pinmpc_landmarks_push(ctypes.byref(st), 10, None, ctypes.c_void_p(x.data_ptr()),
                                     0, None) == 0
    torch.cuda.synchronize()
    assert lib.pinmpc_landmarks_push(ctypes.byref(st), 9, None, ctypes.c_void_p(x.data_ptr()),
                                     -1, None) == -1
    bad = binding.Landmarks(4, 32, 11, 1, st.com, st.tag)
    assert lib.pinmpc_landmarks_clear(ctypes.byref(bad), None, None) == -1
    assert lib.pinmpc_landmark_reward(ctypes.byref(st), None, 0, None, None, 0.0, None, None,
                                      None) == -1
