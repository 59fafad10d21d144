"""Long single horizons (up to 512 stages) with the horizon split across
workgroups, through the C ABI.

* The split ADMM (a chain of stage-parallel launches per sweep) computes the
  same arithmetic in the same order as the one-workgroup-per-problem kernels:
  bitwise-equal iterates and solutions at horizons those kernels also handle.
* The refinement's long-horizon variant (stage buffers in the scratch block
  instead of LDS) is bitwise equal to the short one on the same problems.
* Long horizons (100, 200, 400 stages at small batch): every problem
  certified by the library, every result optimal by the oracle's own KKT
  measure (an independent check that needs no QP solve: by convexity a point
  with KKT residuals below the bar is the optimum to that accuracy), and the
  oracle's exact optimum matched on problems of each horizon.
"""
import numpy as np
import pytest

import mpcgen
from oracle import kkt
from oracle_refs import solve_many
from gpu_common import ACT_TOL_FP32, TOL_ERR, TOL_KKT, _check_invariants, _solve, reset_settings

pytestmark = pytest.mark.gpu


def test_split_admm_matches_one_workgroup_kernels(solver):
    import torch
    from paper_2606_05687_amd import binding
    for n_max, cfg in ((20, "plain_b4096_n20"), (60, "uneven_b16384")):
        batch = mpcgen.make_batch(cfg, indices=range(120), n_max=n_max)
        dev = binding.to_device(batch)
        reset_settings(solver)
        for sweeps in (1, 2, 37):
            zs = []
            for form in (0, 2):
                solver.set(form=form)
                z = solver.admm(dev, sweeps)
                torch.cuda.synchronize()
                zs.append(z.cpu().numpy())
            assert np.array_equal(zs[0], zs[1]), (n_max, sweeps)
        plain = _solve(solver, batch, form=0)
        split = _solve(solver, batch, form=2)
        for k in plain:
            assert np.array_equal(plain[k], split[k]), (n_max, k)
        assert (split["status"] == 0).all()


def _pad(batch, n_max):
    """The same problems with their stage arrays padded to n_max stages."""
    out = dict(batch)
    n0 = batch["A"].shape[1]
    extra = n_max - n0
    Bn = batch["A"].shape[0]
    out["A"] = np.concatenate([batch["A"], np.tile(np.eye(13, dtype=np.float32), (Bn, extra, 1, 1))], 1)
    for k in ("B", "e", "x_ref", "u_ref", "contact", "yaw_k", "c_ref", "feet"):
        pad = np.zeros((Bn, extra) + batch[k].shape[2:], batch[k].dtype)
        out[k] = np.concatenate([batch[k], pad], 1)
    return {k: np.ascontiguousarray(v) for k, v in out.items()}


def test_long_refinement_variant_matches_short(solver):
    """Horizons up to 60 padded to 72 stages run the long-horizon refinement
    (stage buffers in the scratch block) and the split ADMM; padded to 60 with
    the split ADMM forced they run the short refinement: bitwise the same
    results on the real stages."""
    batch = mpcgen.make_batch("uneven_b16384", indices=range(96), n_max=60)
    short = _solve(solver, batch, form=2)
    longb = _pad(batch, 72)
    lng = _solve(solver, longb, form=0)
    assert (lng["status"] == 0).all()
    assert np.array_equal(short["u"], lng["u"][:, :60])
    assert np.array_equal(short["x"], lng["x"][:, :61])
    for k in ("res", "iters", "status", "detail"):
        assert np.array_equal(short[k], lng[k]), k
    assert np.all(lng["u"][:, 60:] == 0)


# The interior-point fallback needs more iterations at hundreds of stages
# (measured: up to 117 at 200 stages from the ADMM point) than the default
# cap of 40 sized for horizons up to 64; and the certificate needs kkt_tol
# 1e-10: the multiplier-sign residual is normalised by the largest term of the
# stationarity condition, which grows with the costates over a long horizon,
# so at 1e-9 one 400-stage problem was accepted on a face with a multiplier of
# normalised size -4.6e-10 (rel-err 1.9e-4); at 1e-10 it goes on to the right
# face (rel-err 3.4e-8).
LONG = dict(iters=3, refine_passes=16, first_passes=0, ipm_iters=150, polish_passes=20,
            kkt_tol=1e-10)


def test_long_horizons_certified_and_optimal(solver):
    batch = mpcgen.make_batch("long_b64_n400", indices=range(24))
    out = _solve(solver, batch, **LONG)
    assert (out["status"] == 0).all(), out["status"]
    assert np.all(out["res"] <= TOL_KKT)
    _check_invariants(batch, out, range(24))
    for b in range(24):
        p = mpcgen.problem_fp64(batch, b)
        N = p["N"]
        r = kkt.residuals(p, out["u"][b, :N].astype(np.float64),
                          out["x"][b, :N + 1].astype(np.float64), act_tol=ACT_TOL_FP32)
        assert r["kkt"] <= TOL_KKT, (b, N, r)
    # the oracle's exact optimum for one problem of each horizon
    pick = [int(np.argmax(batch["N"] == n)) for n in (100, 200, 400)]
    refs = solve_many(batch, pick, workers=1)   # in-process: multithreaded BLAS
    for b, ref in zip(pick, refs):
        p = mpcgen.problem_fp64(batch, b)
        N = p["N"]
        eu, ex = kkt.rel_err(out["u"][b, :N].astype(np.float64), ref["u"],
                             out["x"][b, :N + 1].astype(np.float64), ref["x"], p["weight"])
        print("N", N, "rel-err", eu, ex, "passes", out["detail"][b])
        assert eu <= TOL_ERR and ex <= TOL_ERR, (b, N, eu, ex)


def test_longest_horizon_and_padding(solver):
    """The largest horizon (512) beside shorter ones padded to it."""
    cfg = dict(mpcgen.CONFIGS["long_b64_n400"], horizons=(512, 150, 65), batch=6)
    batch = mpcgen.make_batch(cfg, indices=range(6), n_max=512)
    out = _solve(solver, batch, **LONG)
    assert (out["status"] == 0).all(), out["status"]
    for b in range(6):
        p = mpcgen.problem_fp64(batch, b)
        N = p["N"]
        r = kkt.residuals(p, out["u"][b, :N].astype(np.float64),
                          out["x"][b, :N + 1].astype(np.float64), act_tol=ACT_TOL_FP32)
        assert r["kkt"] <= TOL_KKT, (b, N, r)
        assert np.all(out["u"][b, N:] == 0)


def test_split_form_with_bf16_operators_and_graph_replay(solver):
    """The split sweeps read BF16 operators like the other forms (bitwise the
    plain form's BF16 result), and a captured graph of a long-horizon solve
    replays bitwise equal to the eager solve."""
    import torch
    from paper_2606_05687_amd import binding
    batch = mpcgen.make_batch("uneven_b16384", indices=range(64), n_max=60)
    a = _solve(solver, batch, form=0, precision=1)
    b = _solve(solver, batch, form=2, precision=1)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    cfg = dict(mpcgen.CONFIGS["long_b64_n400"], horizons=(100, 200), batch=8)
    lb = mpcgen.make_batch(cfg, indices=range(8), n_max=200)
    eager = _solve(solver, lb, graph=0, **LONG)
    reset_settings(solver)
    solver.set(graph=1, **LONG)
    dev = binding.to_device(lb)
    out = solver.alloc_out(dev)
    bs = binding.make_batch_struct(dev)
    for rep in range(3):
        for v in out.values():
            v.fill_(-7)
        solver.solve(dev, out, batch_struct=bs)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        for k in eager:
            assert np.array_equal(got[k], eager[k]), (rep, k)
    assert (got["status"] == 0).all()
