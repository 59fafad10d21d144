"""ADMM iterates of every sweep form on uneven horizons: one launch per
sweep (global stride 60, two (stage, row) pairs per thread), fused with
horizon-class packing, and fused on a tighter padding, against each other
(bitwise) and against the FP64 reference of Sec. III."""
import numpy as np
import pytest

import mpcgen

pytestmark = pytest.mark.gpu


def _admm(solver, batch, K, **settings):
    import torch
    from paper_2606_05687_amd import binding
    base = binding.default_settings()
    for f, _ in binding.Settings._fields_:
        setattr(solver.settings, f, getattr(base, f))
    solver.set(**settings)
    z = solver.admm(binding.to_device(batch), K)
    torch.cuda.synchronize()
    return z.cpu().numpy()


def test_sweep_forms_agree_on_uneven_horizons():
    from oracle import admm
    from paper_2606_05687_amd import binding
    solver = binding.Solver(0)
    full = mpcgen.make_batch("uneven_b16384", indices=range(40), n_max=60)
    short = np.where(full["N"] <= 40)[0]
    for K in (1, 3, 20):
        zp = _admm(solver, full, K, form=0)
        za = _admm(solver, full, K, form=-1)
        diffs = []
        for b in range(40):
            N = int(full["N"][b])
            d = np.max(np.abs(zp[b, :N] - za[b, :N]))
            diffs.append(d)
        bad = [(b, int(full["N"][b]), diffs[b]) for b in range(40) if diffs[b] != 0]
        # FP64 reference for two short-horizon problems
        for b in short[:2]:
            p = mpcgen.problem_fp64(full, int(b))
            ref = admm.solve(p, iters=K, rho=10.0, scaling=True, accel=True)
            zr = ref["iterates"]["z"].copy()
            zr[:, 13:] *= ref["setup"]["S"]
            N = p["N"]
            sc = np.concatenate([np.ones(13), np.full(12, p["weight"])])
            dp = np.max(np.abs(zp[b, :N] - zr) / sc)
            da = np.max(np.abs(za[b, :N] - zr) / sc)
            print(f"K={K} b={b} N={N} plain-vs-fp64 {dp:.2e} packed-vs-fp64 {da:.2e}")
        print(f"K={K} differing problems (b, N, maxdiff): {bad[:8]}")
        assert not bad, bad
    solver.close()
