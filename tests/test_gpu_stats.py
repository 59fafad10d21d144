"""Measurement calls of the C ABI: the algorithmic-traffic figure of
pinmpc_stats_traffic follows its documented byte model with the refinement
work counted on the device (checked against the per-problem work outputs),
and its rate uses the solve's own measured time."""
import ctypes
import re
import os

import numpy as np
import pytest

import mpcgen

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _model():
    text = open(os.path.join(ROOT, "include", "pinmpc.h")).read()
    return {k: int(re.search(rf"#define PINMPC_{k}_BYTES (\d+)", text).group(1))
            for k in ("SETUP", "SWEEP", "REFINE")}


@pytest.mark.parametrize("graph", [0, 1])
def test_traffic_follows_the_byte_model(graph):
    import torch
    from paper_2606_05687_amd import binding
    m = _model()
    batch = mpcgen.make_batch("uneven_b16384", indices=range(300), n_max=60)
    dev = binding.to_device(batch)
    solver = binding.Solver(0, iters=5, refine_passes=8, first_passes=2, graph=graph)
    try:
        out = solver.alloc_out(dev)
        for _ in range(2):                        # the second replays a graph
            solver.solve(dev, out)
        torch.cuda.synchronize()
        tr = solver.traffic()
        st = solver.stats()
    finally:
        solver.close()
    det = out["detail"].cpu().numpy().astype(np.int64)
    N = batch["N"].astype(np.int64)
    pass_stages = int((N * (det[:, 0] + det[:, 1])).sum())
    stages = 300 * 60
    want = stages * (m["SETUP"] + 5 * m["SWEEP"]) + pass_stages * m["REFINE"]
    assert tr["bytes"] == pytest.approx(want, rel=1e-12)
    assert tr["gbs"] == pytest.approx(want / (st["total_ms"] * 1e6), rel=1e-3)


def test_traffic_rejects_context_without_solve():
    from paper_2606_05687_amd import binding
    solver = binding.Solver(0)
    try:
        b, g = ctypes.c_double(), ctypes.c_double()
        assert binding.load().pinmpc_stats_traffic(solver._h, ctypes.byref(b), ctypes.byref(g)) == -1
    finally:
        solver.close()
