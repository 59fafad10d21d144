"""The refinement's backward recursion as an associative scan over the
horizon (setting ``scan``: chunks of the horizon, one wave each), through the
C ABI.

* Parity with the FP64 oracle at N = 20 and N = 64 (every problem certified,
  sampled problems at the oracle's exact optimum) and at long horizons
  (100 to 400 stages: certified, optimal by the oracle's KKT measure).
* The scan and the sequential recursion reach the same certified solutions
  (the same QP optimum, to rounding), also when interior-point Newton steps
  run through the scan.
* Horizons too short to cut (under 8 stages) run the sequential recursion
  inside the scanning workgroup: bitwise the sequential result.
* A captured graph of a scanning solve replays bitwise equal to the eager
  solve, and the allocation-free entry point gives the same result.
"""
import numpy as np
import pytest

import mpcgen
from oracle import kkt
from gpu_common import ACT_TOL_FP32, TOL_KKT, _check_invariants, _compare, _solve

pytestmark = pytest.mark.gpu

# Two certified solutions of the same strictly convex QP differ only by the
# certificate's accuracy: measured below 2e-8 relative between the scan and
# the sequential recursion on every workload
AGREE = 1e-6


def _agree(a, b):
    ua, ub = a["u"].astype(np.float64), b["u"].astype(np.float64)
    scale = np.maximum(np.abs(ub).max(axis=(1, 2)), 1e-30)
    rel = np.abs(ua - ub).max(axis=(1, 2)) / scale
    return float(rel.max())


def test_scan_n20_matches_oracle_and_sequential(solver):
    batch = mpcgen.make_batch("plain_b4096_n20", indices=range(192))
    seq = _solve(solver, batch, iters=2, rho=1.0, refine_passes=12, first_passes=0)
    for w in (2, 4, 8):
        out = _solve(solver, batch, iters=2, rho=1.0, refine_passes=12, first_passes=0, scan=w)
        assert (out["status"] == 0).all(), (w, np.bincount(out["status"]))
        assert _agree(out, seq) <= AGREE, w
        _check_invariants(batch, out, range(0, 192, 16))
    _compare(batch, out, [0, 37, 101, 190])


def test_scan_n64_matches_oracle(solver):
    cfg = dict(mpcgen.CONFIGS["plain_b4096_n20"], horizons=(64,), batch=48, seed=31)
    batch = mpcgen.make_batch(cfg, indices=range(48))
    seq = _solve(solver, batch)
    out = _solve(solver, batch, scan=8)
    assert (out["status"] == 0).all(), np.bincount(out["status"])
    assert _agree(out, seq) <= AGREE
    _compare(batch, out, [3, 29])


def test_scan_through_interior_point_steps(solver):
    """Two active-set passes leave most problems to the interior point, whose
    factored Newton steps then run through the scan."""
    batch = mpcgen.make_batch("uneven_b16384", indices=range(160))
    seq = _solve(solver, batch, refine_passes=2)
    out = _solve(solver, batch, refine_passes=2, scan=4)
    assert (out["status"] == 0).all()
    assert out["detail"][:, 1].mean() > 1.0          # interior-point iterations ran
    assert _agree(out, seq) <= AGREE
    _check_invariants(batch, out, range(0, 160, 20))


LONG = dict(iters=3, refine_passes=16, first_passes=0, ipm_iters=150, polish_passes=20,
            kkt_tol=1e-10)


def test_scan_long_horizons_certified_and_optimal(solver):
    batch = mpcgen.make_batch("long_b64_n400", indices=range(12))
    seq = _solve(solver, batch, **LONG)
    out = _solve(solver, batch, scan=8, **LONG)
    assert (out["status"] == 0).all(), out["status"]
    assert np.all(out["res"] <= TOL_KKT)
    assert _agree(out, seq) <= AGREE
    for b in range(12):
        p = mpcgen.problem_fp64(batch, b)
        N = p["N"]
        r = kkt.residuals(p, out["u"][b, :N].astype(np.float64),
                          out["x"][b, :N + 1].astype(np.float64), act_tol=ACT_TOL_FP32)
        assert r["kkt"] <= TOL_KKT, (b, N, r)


def test_short_horizons_stay_sequential_bitwise(solver):
    cfg = dict(mpcgen.CONFIGS["plain_b4096_n20"], horizons=(3, 5, 7), batch=64, seed=32)
    batch = mpcgen.make_batch(cfg, indices=range(64), n_max=7)
    seq = _solve(solver, batch)
    out = _solve(solver, batch, scan=8)
    for k in seq:
        assert np.array_equal(seq[k], out[k]), k
    assert (out["status"] == 0).all()


def test_scan_graph_replay_and_noalloc(solver):
    import torch
    from paper_2606_05687_amd import binding
    batch = mpcgen.make_batch("uneven_b16384", indices=range(96), n_max=60)
    eager = _solve(solver, batch, scan=4, graph=0)
    dev = binding.to_device(batch)
    solver.set(graph=1)
    out = solver.alloc_out(dev)
    for rep in range(3):
        for v in out.values():
            v.zero_()
        solver.solve(dev, out)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        for k in eager:
            assert np.array_equal(eager[k], got[k]), (rep, k)
    solver.set(graph=0)
    na = solver.alloc_out(dev)
    solver.solve_noalloc(dev, na)
    torch.cuda.synchronize()
    for k in eager:
        assert np.array_equal(eager[k], na[k].cpu().numpy()), k
