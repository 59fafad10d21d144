"""Helpers shared by the GPU parity tests (solve through the C ABI, compare
with the FP64 oracle, check the invariants every result must satisfy)."""
import numpy as np

import mpcgen
from oracle import kkt
from oracle_refs import solve_many

TOL_ERR = 1e-4
TOL_KKT = 1e-5
# Activity threshold (in units of m g) for the oracle's multiplier refit on
# FP32 outputs: rounding u to FP32 moves a friction row's slack mu f_z - f_x by
# up to 2^-24 (|f_x| + mu |f_z|) <= 2^-24 * 2 * 0.9 * 1000 N = 1.1e-4 N, which
# is 3.7e-7 m g at the lightest robot (30 kg); a truly active row must not fall
# outside the refit, so the threshold sits above that bound.
ACT_TOL_FP32 = 1e-6


def reset_settings(solver):
    """Put the library defaults back into a solver's settings."""
    from paper_2606_05687_amd import binding
    base = binding.default_settings()
    for f, _ in binding.Settings._fields_:
        setattr(solver.settings, f, getattr(base, f))


def _solve(solver, batch, **settings):
    import torch
    from paper_2606_05687_amd import binding
    reset_settings(solver)
    if settings:
        solver.set(**settings)
    else:
        solver.set()
    dev = binding.to_device(batch)
    out = solver.solve(dev)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _check_invariants(batch, out, idx):
    for b in idx:
        p = mpcgen.problem_fp64(batch, b)
        N = p["N"]
        u = out["u"][b, :N].astype(np.float64)
        x = out["x"][b, :N + 1].astype(np.float64)
        sw = ~p["contact"]
        for i in range(p["contact"].shape[1]):
            assert np.all(out["u"][b, :N, 6 * i:6 * i + 6][sw[:, i]] == 0.0)
        assert np.all(out["u"][b, N:] == 0)
        r = kkt.residuals(p, u, x)
        assert r["r_ineq"] <= 1e-6, (b, r)
        assert r["r_dyn"] <= 1e-6, (b, r)


def _compare(batch, out, idx, refs=None):
    idx = [int(b) for b in idx]
    if refs is None:
        refs = solve_many(batch, idx)
    worst = dict(eu=0.0, ex=0.0, kkt_lib=0.0, kkt_oracle=0.0)
    for j, b in enumerate(idx):
        p = mpcgen.problem_fp64(batch, b)
        ref = refs[j]
        N = p["N"]
        u = out["u"][b, :N].astype(np.float64)
        x = out["x"][b, :N + 1].astype(np.float64)
        assert out["status"][b] == 0, (b, out["status"][b], out["res"][b])
        eu, ex = kkt.rel_err(u, ref["u"], x, ref["x"], p["weight"])
        r = kkt.residuals(p, u, x, act_tol=ACT_TOL_FP32)
        worst["eu"] = max(worst["eu"], eu)
        worst["ex"] = max(worst["ex"], ex)
        worst["kkt_lib"] = max(worst["kkt_lib"], float(np.max(out["res"][b])))
        worst["kkt_oracle"] = max(worst["kkt_oracle"], r["kkt"])
        assert eu <= TOL_ERR and ex <= TOL_ERR, (b, eu, ex)
        assert np.max(out["res"][b]) <= TOL_KKT, (b, out["res"][b])
        assert r["kkt"] <= TOL_KKT, (b, r)
    print("worst", {k: f"{v:.2e}" for k, v in worst.items()})
    return worst


