"""GPU solves with four contacts per stage (feet and hands, loco-manipulation
of Sec. II-A: 24 inputs) through the C ABI.

  * ADMM iterates after 1 and 3 sweeps against the FP64 ADMM reference;
  * solutions against the FP64 oracle's certified optimum (rel-err <= 1e-4 in
    u and x, KKT <= 1e-5 by the library and by the oracle's measure), on the
    loco-manipulation workload, with affine terms, and at ragged horizons with
    hands and feet in and out of contact;
  * the forms of the sweep (one launch per sweep, all sweeps in one launch),
    a captured graph's replays and the entry point that allocates nothing all
    give bitwise the same results;
  * bad input in one problem sets only that problem's status.
"""
import numpy as np
import pytest

import mpcgen
from gpu_common import _check_invariants, _compare, _solve, reset_settings

pytestmark = pytest.mark.gpu

HANDS = "hands_b4096_n20"


def test_hands_admm_iterates(solver):
    import torch
    from oracle import admm
    from paper_2606_05687_amd import binding
    batch = mpcgen.make_batch(HANDS, indices=range(4), offsets=True)
    reset_settings(solver)
    solver.set()
    dev = binding.to_device(batch)
    for K, tol in ((1, 1e-4), (3, 1e-3)):
        z = solver.admm(dev, K)
        torch.cuda.synchronize()
        z = z.cpu().numpy().astype(np.float64)
        assert z.shape[-1] == 37
        for b in range(4):
            p = mpcgen.problem_fp64(batch, b)
            ref = admm.solve(p, iters=K, rho=10.0, scaling=True, accel=True)
            zr = ref["iterates"]["z"].copy()
            zr[:, 13:] *= ref["setup"]["S"]
            N = p["N"]
            scale = np.concatenate([np.ones(13), np.full(24, p["weight"])])
            d = np.max(np.abs(z[b, :N] - zr) / scale) / max(1.0, np.max(np.abs(zr) / scale))
            print(f"K={K} b={b} scaled max diff {d:.2e}")
            assert d <= tol, (K, b, d)


def test_hands_parity(solver):
    batch = mpcgen.make_batch(HANDS, indices=range(64))
    out = _solve(solver, batch, iters=20)
    assert out["u"].shape[-1] == 24
    _check_invariants(batch, out, range(64))
    _compare(batch, out, range(64))
    det = out["detail"].astype(np.int64)
    its, fact, n = det[:, 1], det[:, 2], np.asarray(batch["N"], dtype=np.int64)
    assert np.all(its > 0)                      # interior-point iterations
    assert np.all(det[:, 0] == 0) and np.all(det[:, 3] == 1)
    # stages of the factoring recursions: every predictor, some correctors
    assert np.all(fact % n == 0)
    assert np.all(fact >= its * n) and np.all(fact < 2 * its * n)
    print("interior-point iterations", np.bincount(its),
          "factorisations per iteration", (fact / n).sum() / its.sum())


def test_hands_parity_offsets_ragged(solver):
    cfg = dict(mpcgen.CONFIGS[HANDS], horizons=(3, 9, 20, 37, 64), duty=None, seed=71)
    batch = mpcgen.make_batch(cfg, indices=range(40), offsets=True)
    N = batch["N"]
    assert N.min() < N.max() and batch["B"].shape[1] == 64
    hands_off = ~batch["contact"][:, :, 2:].any(axis=(1, 2))
    print("horizons", np.bincount(N), "problems without hand contact", int(hands_off.sum()))
    out = _solve(solver, batch, iters=10)
    _check_invariants(batch, out, range(40))
    _compare(batch, out, range(40))


def test_hands_forms_graph_and_noalloc_bitwise(solver):
    import torch
    from paper_2606_05687_amd import binding
    batch = mpcgen.make_batch(HANDS, indices=range(96), offsets=True)
    ref = _solve(solver, batch, iters=6, form=0, graph=0)
    for form in (1, -1, 2):
        out = _solve(solver, batch, iters=6, form=form, graph=0)
        for k in ("u", "x", "res", "status", "iters"):
            assert np.array_equal(out[k], ref[k]), (form, k)
    reset_settings(solver)
    solver.set(iters=6, graph=1)
    dev = binding.to_device(batch)
    out = solver.solve(dev)
    for rep in range(3):
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        for k in ("u", "x", "res", "status"):
            assert np.array_equal(got[k], ref[k]), (rep, k)
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        del junk
        out = solver.solve(dev, out)
    reset_settings(solver)
    solver.set(iters=6)
    out2 = solver.alloc_out(dev)
    solver.solve_noalloc(dev, out2)
    torch.cuda.synchronize()
    for k in ("u", "x", "res", "status"):
        assert np.array_equal(out2[k].cpu().numpy(), ref[k]), k


def test_hands_bad_input_is_isolated(solver):
    batch = mpcgen.make_batch(HANDS, indices=range(8))
    bad = {k: v.copy() for k, v in batch.items()}
    bad["mu"][2] = 0.0
    bad["B"][5, 3, 7, 15] = np.nan
    out = _solve(solver, bad, iters=10)
    ref = _solve(solver, batch, iters=10)
    assert out["status"][2] == 4 and out["status"][5] == 3
    keep = [b for b in range(8) if b not in (2, 5)]
    for k in ("u", "x", "status"):
        assert np.array_equal(out[k][keep], ref[k][keep]), k
    assert np.all(out["u"][[2, 5]] == 0)
